"""The oracle's pins must catch plausible mistakes.

Each case copies oracle/lw_oracle.c, plants one mistake by a textual edit,
builds it into a temporary library and runs the fp32 pins (hand-worked cases,
brute force over member sets, tie-break on constant matrices, Prim MST,
library weighted-average clustering)
against it.  At least one pin must fail for every planted mistake, and the
unmodified source must pass all of them.
"""
import json
import os
import tempfile

import numpy as np
import pytest

import oracle
import synth
from conftest import matrix_from_upper

HERE = os.path.dirname(os.path.abspath(__file__))
LINKS = ["single", "complete", "average", "ward", "weighted", "centroid"]
BRUTE = ["single", "complete", "average", "ward", "centroid"]

MUTANTS = {
    "ward_beta_sign": ("float b = (float)(-(double)nk / t);", "float b = (float)((double)nk / t);"),
    "ward_alpha_drops_nk": ("float ai = (float)((double)(ni + nk) / t);",
                            "float ai = (float)((double)(ni) / t);"),
    "average_swapped_weights": ("float ai = (float)((double)ni / s);",
                                "float ai = (float)((double)nj / s);"),
    "complete_uses_min": ("v = fmaxf(dki, dkj);", "v = fminf(dki, dkj);"),
    "tie_prefers_later_row": ("if (a != ba) return a < ba;", "if (a != ba) return a > ba;"),
    "tie_prefers_later_col": ("return b < bb;", "return b > bb;"),
    "update_reads_i_twice": ("w[UPPER(k, i)], w[UPPER(k, j)], h,", "w[UPPER(k, i)], w[UPPER(k, i)], h,"),
    "size_not_accumulated": ("sz[i] += sz[j];", "sz[i] += 1;"),
    "scan_skips_neighbour": ("for (int64_t b = a + 1; b < n; b++)\n                    if (alive[b]",
                             "for (int64_t b = a + 2; b < n; b++)\n                    if (alive[b]"),
    "survivor_keeps_j_alive": ("alive[j] = 0;", "alive[i] = 0;"),
    "centroid_beta_sign": ("float b = (float)(-((double)ni * (double)nj) / (s * s));",
                           "float b = (float)(((double)ni * (double)nj) / (s * s));"),
    "centroid_beta_not_squared": ("float b = (float)(-((double)ni * (double)nj) / (s * s));",
                                  "float b = (float)(-((double)ni * (double)nj) / s);"),
    "centroid_drops_beta": ("v = u + t3;", "v = u;"),
    "weighted_reads_i_twice": ("float t2 = 0.5f * dkj;", "float t2 = 0.5f * dki;"),
    "weighted_uses_sizes": ("float t1 = 0.5f * dki;\n        float t2 = 0.5f * dkj;",
                            "float t1 = (float)((double)ni / (double)(ni + nj)) * dki;\n"
                            "        float t2 = (float)((double)nj / (double)(ni + nj)) * dkj;"),
}


def _pins_fail(lib) -> list:
    """Run the fp32 pins against ``lib``; return the names of failing pins."""
    failed = []
    with open(os.path.join(HERE, "golden", "hand_worked.json")) as f:
        cases = json.load(f)["cases"]
    try:
        for case in cases:
            d = matrix_from_upper(case["n"], case["upper"])
            for link in LINKS:
                got = oracle.run_f32(d, link, lib=lib)
                exp = case["expected"][link]
                if [(int(g["i"]), int(g["j"]), float(g["h"]), int(g["size"])) for g in got] != \
                        [(e[0], e[1], float(np.float32(e[2])), e[3]) for e in exp]:
                    failed.append("hand_worked")
                    break
        for seed in range(3):
            for d in (synth.uniform_matrix(10, seed), synth.quantized_matrix(10, seed, 4)):
                for link in BRUTE:
                    m = oracle.run_f32(d, link, lib=lib)
                    if oracle.brute_force_check(d, m, link, rtol=2e-6, atol=1e-6,
                                                exact_ties=link in ("single", "complete")):
                        failed.append("brute_force")
        d = np.full((12, 12), 2.0, np.float32)
        for link in ("single", "complete"):
            m = oracle.run_f32(d, link, lib=lib)
            if not (np.all(m["i"] == 0) and np.array_equal(m["j"], np.arange(1, 12))):
                failed.append("constant")
        d = synth.uniform_matrix(60, 4)
        m = oracle.run_f32(d, "single", lib=lib)
        if not np.array_equal(np.sort(m["h"]), np.sort(oracle.prim_mst_weights(d))):
            failed.append("mst")
        from scipy.cluster.hierarchy import linkage as sp_linkage
        from scipy.spatial.distance import squareform
        d = synth.uniform_matrix(40, 6)
        d64 = np.triu(d, 1).astype(np.float64)
        ref = sp_linkage(squareform(d64 + d64.T, checks=False), method="weighted")[:, 2]
        got = oracle.run_f32(d, "weighted", lib=lib)["h"].astype(np.float64)
        if not np.allclose(np.sort(got), np.sort(ref), rtol=1e-5, atol=0):
            failed.append("library_weighted")
    except Exception as e:  # a crash or an error code also counts as caught
        failed.append("error:%s" % type(e).__name__)
    return failed


def _build_variant(tmpdir, name, edit):
    with open(oracle.SRC) as f:
        src = f.read()
    if edit is not None:
        old, new = edit
        assert src.count(old) >= 1, name
        src = src.replace(old, new, 1)
    path = os.path.join(tmpdir, name + ".c")
    with open(path, "w") as f:
        f.write(src)
    return oracle.load_variant(oracle.build(force=True, src=path,
                                            out=os.path.join(tmpdir, name + ".so")))


def test_unmodified_passes_pins():
    with tempfile.TemporaryDirectory() as tmp:
        assert _pins_fail(_build_variant(tmp, "clean", None)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_variant(tmp, name, MUTANTS[name])
        assert _pins_fail(lib), "planted mistake %s was not caught" % name
