"""The rule behind the batch and serving kernels' lazy mirror, checked on the
CPU: if every merge step writes only its survivor's row and remembers the
step that last wrote each row, then reading a pair (a, b) from whichever of
its two rows was written later (row a on equal steps) always gives the
current Lance-Williams distance.  The reference keeps the matrix fully
symmetric (both halves written), as Section 4 step 3 updates the merged row
and column.  Single-linkage (min) and average-linkage updates over the merge
lists of the oracle, tie-heavy input included."""
import numpy as np
import pytest

import oracle
import synth


def _pair(lazy, step, a, b):
    return lazy[b, a] if step[b] > step[a] else lazy[a, b]


@pytest.mark.parametrize("link", ["single", "average"])
@pytest.mark.parametrize("make", [lambda: synth.mixture_8192(seed=31, n=90),
                                  lambda: synth.quantized_matrix(80, 37, levels=3)])
def test_later_written_row_holds_the_pair(link, make):
    d = np.array(make(), dtype=np.float64)
    n = d.shape[0]
    iu = np.triu_indices(n, 1)
    full = np.zeros((n, n))
    full[iu] = d[iu]
    full = full + full.T
    lazy = full.copy()            # the set-up mirrors the input: both halves hold it
    step = np.zeros(n, np.int64)  # 0: the input
    size = np.ones(n)
    live = np.ones(n, bool)
    merges = oracle.run_f64(d.astype(np.float32), link)
    for s, (i, j) in enumerate(zip(merges["i"], merges["j"])):
        i, j = int(i), int(j)
        live[j] = False
        others = [k for k in range(n) if live[k] and k != i]
        for k in others:
            dik, djk = _pair(lazy, step, i, k), _pair(lazy, step, j, k)
            assert dik == full[i, k] and djk == full[j, k], (s, i, j, k)
            if link == "single":
                v = min(dik, djk)
            else:
                v = (size[i] * dik + size[j] * djk) / (size[i] + size[j])
            full[i, k] = full[k, i] = v  # symmetric storage: row and column
            lazy[i, k] = v               # lazy mirror: the survivor's row only
        step[i] = s + 1
        size[i] += size[j]
        # Every live pair reads back its current value.
        alive = np.flatnonzero(live)
        for x in range(len(alive)):
            for y in range(x + 1, len(alive)):
                a, b = int(alive[x]), int(alive[y])
                assert _pair(lazy, step, a, b) == full[a, b], (s, a, b)
