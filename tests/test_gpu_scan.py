"""Scan engine (HAC_MODE_SCAN): the paper's own closest-pair step -- the whole
live upper triangle scanned before every merge (Section 5.3 step 1) -- over
every CU, with the live items compacted as they retire, must give the
oracle's merge list byte for byte for every Table 1 linkage."""
import numpy as np
import pytest

import oracle
import paper_1709_06816_amd as hac
import synth

pytestmark = pytest.mark.gpu

LINKS = ["single", "complete", "average", "ward", "weighted", "centroid"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    with hac.Context(0) as c:
        c.set_option(hac.OPT_TIMEOUT_MS, 20000)
        yield c


def _scan(ctx, d, link, wgs=0):
    import torch
    ctx.set_option(hac.OPT_WORKGROUPS, wgs)
    try:
        got = ctx.run(torch.from_numpy(np.ascontiguousarray(d)).cuda(), link, scan=True)
        st = ctx.stats()
    finally:
        ctx.set_option(hac.OPT_WORKGROUPS, 0)
    return got, st


@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("n", [2, 3, 4, 5, 63, 64, 65, 67, 130, 301])
def test_scan_small_sizes(ctx, link, n):
    d = synth.mixture_8192(seed=500 + n, n=n)
    print("scan: n=%d %s" % (n, link), flush=True)
    got, _ = _scan(ctx, d, link)
    assert got.tobytes() == oracle.run_f32(d, link).tobytes()


@pytest.mark.parametrize("link", LINKS)
def test_scan_compacts_and_matches(ctx, link):
    # n=2051 (not a multiple of 4): the live width is compacted many times.
    d = synth.mixture_8192(seed=77, n=2051)
    print("scan: n=2051 %s" % link, flush=True)
    got, st = _scan(ctx, d, link)
    assert st["compactions"] >= 10
    assert got.tobytes() == oracle.run_f32(d, link).tobytes()


@pytest.mark.parametrize("name,gen", [("quantized", lambda: synth.quantized_matrix(900, seed=78, levels=3)),
                                      ("rmsd_like", lambda: synth.rmsd_like(seed=79, n=1200)),
                                      ("constant", lambda: np.where(np.eye(300, dtype=bool), 0, 1.5).astype(np.float32))])
@pytest.mark.parametrize("link", ["single", "complete", "average"])
def test_scan_ties(ctx, name, gen, link):
    d = gen()
    print("scan: %s %s" % (name, link), flush=True)
    got, _ = _scan(ctx, d, link)
    assert got.tobytes() == oracle.run_f32(d, link).tobytes()


@pytest.mark.parametrize("wgs", [1, 3, 40])
def test_scan_any_workgroup_count(ctx, wgs):
    d = synth.mixture_8192(seed=80, n=1500)
    print("scan: n=1500 ward on %d workgroups" % wgs, flush=True)
    got, st = _scan(ctx, d, "ward", wgs)
    assert st["workgroups"] == wgs
    assert got.tobytes() == oracle.run_f32(d, "ward").tobytes()


def test_scan_noalloc_keeps_its_path(ctx):
    # The allocation-free entry point has no room for the compacted copy and
    # keeps the per-workgroup scan; same bytes.
    import torch
    d = synth.mixture_8192(seed=81, n=1800)
    out = torch.zeros(1799 * 16, dtype=torch.uint8, device="cuda")
    ctx.run_noalloc(torch.from_numpy(d).cuda().data_ptr(), 1800, "complete", out.data_ptr(), scan=True)
    got = np.frombuffer(out.cpu().numpy().tobytes(), dtype=hac.MERGE_DTYPE)
    assert got.tobytes() == oracle.run_f32(d, "complete").tobytes()
