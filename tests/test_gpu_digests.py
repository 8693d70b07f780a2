"""Full merge lists of the large workloads against the oracle, byte for byte.

The oracle needs minutes to hours at these sizes, so its lists were written
once, as SHA-256 digests, by tests/golden/make_digests.py (which calls only
oracle/ and synth/).  The inputs are regenerated here from the same seeds; the
digest of each input's strict upper triangle is checked first, so that a
different input is reported as such and not as a wrong result.

  * n=32768 RMSD-like, complete linkage (the benchmark's instance): the whole
    32767-record list, through the default path (rounds of merges) and
    through the one-merge-per-step engine (64 workgroups, deferred rescans).
  * the 1024-instance batch: every instance's list from one hac_batch call.
  * n=65536 mixture, average linkage (HAC_MAX_N): the first 512 records,
    plus the structure of the whole list and monotone heights.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import paper_1709_06816_amd as hac
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")


def _golden(key):
    with open(GOLDEN) as f:
        doc = json.load(f)
    if key not in doc:
        pytest.fail("%s holds no digest for %s (run tests/golden/make_digests.py)" % (GOLDEN, key))
    return doc[key]


def _upper_sha(d):
    h = hashlib.sha256()
    n = d.shape[0]
    for a in range(n - 1):
        h.update(d[a, a + 1:].tobytes())
    return h.hexdigest()


def _say(msg):
    print("[gpu-digest] " + msg, flush=True)


def _structure(m, n):
    i = m["i"].astype(np.int64)
    j = m["j"].astype(np.int64)
    assert len(m) == n - 1 and np.all(i < j) and np.all(i >= 0) and np.all(j < n)
    alive = np.ones(n, bool)
    size = np.ones(n, np.int64)
    for a, b, s in zip(i, j, m["size"]):
        assert alive[a] and alive[b]
        size[a] += size[b]
        assert size[a] == s
        alive[b] = False


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    with hac.Context(0) as c:
        c.set_option(hac.OPT_TIMEOUT_MS, 60000)
        yield c


def test_rmsd_like_32768_complete_full_list(ctx):
    import torch
    g = _golden("rmsd_like_n32768_complete")
    _say("rmsd_like n=32768: generating")
    d = synth.rmsd_like(seed=g["seed"], n=g["n"])
    assert _upper_sha(d) == g["input_upper_sha256"], "the regenerated input differs from the oracle's"
    src = torch.from_numpy(d).cuda()
    del d
    out = torch.empty((g["n"] - 1) * 16, dtype=torch.uint8, device="cuda")
    for rounds in (1, 0):
        ctx.set_option(hac.OPT_ROUNDS, rounds)
        try:
            _say("rmsd_like n=32768: %s engine" % ("round" if rounds else "one-merge-per-step"))
            ctx.run(src, "complete", preserve=True, out=out)
            ctx.sync()
            st = ctx.stats()
        finally:
            ctx.set_option(hac.OPT_ROUNDS, 1)
        rec = out.cpu().numpy().tobytes()
        assert (st["rounds"] > 0) == bool(rounds)
        if not rounds:
            assert st["workgroups"] == 64 and st["deferred"] == 1
        assert len(rec) == 16 * g["merges"]
        assert hashlib.sha256(rec).hexdigest() == g["records_sha256"]


def test_batch_1024_every_instance(ctx):
    import torch
    g = _golden("batch_1024")
    spec = synth.batch_spec(count=g["count"], n_lo=64, n_hi=4096)
    assert [int(x) for x in spec.ns] == g["ns"]
    offs, total = synth.pack_offsets(spec.ns)
    _say("batch of %d: generating" % g["count"])
    host = np.empty(total, np.float32)
    for k, (n, s) in enumerate(zip(spec.ns, spec.seeds)):
        m = synth.batch_instance(int(n), int(s))
        assert _upper_sha(m) == g["input_upper_sha256"][k], k
        host[offs[k]:offs[k] + m.size] = m.ravel()
    _say("batch of %d: hac_batch" % g["count"])
    res = ctx.batch(torch.from_numpy(host).cuda(), offs, spec.ns, spec.linkages)
    moff, _ = synth.merge_offsets(spec.ns)
    bad = [k for k, n in enumerate(spec.ns)
           if hashlib.sha256(res[moff[k]:moff[k] + int(n) - 1].tobytes()).hexdigest() != g["records_sha256"][k]]
    assert not bad, "instances differing from the oracle: %s" % bad[:20]


def test_mixture_65536_average_prefix(ctx):
    import torch
    g = _golden("mixture_n65536_average_p512")
    n = g["n"]
    _say("mixture n=65536: generating (16 GiB)")
    src = torch.empty((n, n), dtype=torch.float32).pin_memory()
    synth.mixture_65536(seed=g["seed"], n=n, out=src.numpy())
    assert _upper_sha(src.numpy()) == g["input_upper_sha256"]
    dev = src.cuda()
    del src
    _say("mixture n=65536: hac_run average")
    got = ctx.run(dev, "average")
    del dev
    torch.cuda.empty_cache()
    k = g["merges"]
    assert hashlib.sha256(got[:k].tobytes()).hexdigest() == g["records_sha256"]
    _structure(got, n)
    h = got["h"].astype(np.float64)
    assert np.all(h[1:] >= h[:-1] * (1 - 1e-6))
