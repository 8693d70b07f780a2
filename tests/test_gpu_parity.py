"""GPU parity: the HIP library, called through its C-ABI, against the CPU
oracle on the same seeded inputs.  Merge lists must be byte-identical
(indices, fp32 heights and sizes): single/complete are exact; average,
weighted average, centroid and Ward follow the same fixed fp32 recipe on both
sides.

At the full n=32768 RMSD-like size the oracle cannot run to the end in a
test, so there the GPU list is checked on its first merges against the
oracle's, and as a whole through an fp64 replay (heights within 1e-5
relative, sampled optimality) and structural invariants.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

# Table 1 rows; "weighted" is the Weighted Average row.
LINKS = ["single", "complete", "average", "ward", "weighted", "centroid"]


def _say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    # This file covers the one-merge-per-step engine (every linkage, batch,
    # serving); single and complete linkage merged in rounds are covered by
    # test_gpu_rounds.py and test_gpu_digests.py.
    import paper_1709_06816_amd as hac
    c = hac.Context(0)
    c.set_option(hac.OPT_ROUNDS, 0)
    yield c
    c.close()


_OPTS = {"workgroups": ("OPT_WORKGROUPS", 0), "single_wg_n": ("OPT_SINGLE_WG_N", 0), "defer": ("OPT_DEFER", 1)}


def _gpu_run(ctx, torch, d, link, **opts):
    import paper_1709_06816_amd as hac
    for k, v in opts.items():
        ctx.set_option(getattr(hac, _OPTS[k][0]), v)
    try:
        t = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda()
        res = ctx.run(t, link)
        torch.cuda.synchronize()
        return res
    finally:
        for k in opts:
            ctx.set_option(getattr(hac, _OPTS[k][0]), _OPTS[k][1])


def _same(a, b):
    return a.dtype.itemsize == b.dtype.itemsize == 16 and a.tobytes() == b.tobytes()


def _diff(a, b):
    for s in range(min(len(a), len(b))):
        if a[s].tobytes() != b[s].tobytes():
            return "first difference at merge %d: gpu %r oracle %r" % (s, a[s], b[s])
    return "lengths %d vs %d" % (len(a), len(b))


# ---------------------------------------------------------------------------
# Small and edge sizes, single workgroup and multi-workgroup paths
# ---------------------------------------------------------------------------

EDGE_NS = [2, 3, 5, 63, 64, 65, 127, 129, 300, 1000]


@pytest.mark.parametrize("defer", [1, 2])
@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("n", EDGE_NS)
def test_edge_sizes_single_wg(ctx, torch, n, link, defer):
    """One workgroup: immediate rescans (defer = 1, the default there) and
    deferred rescans on request (defer = 2)."""
    d = synth.mixture_8192(seed=1000 + n, n=n)
    _say("edge single-wg n=%d %s defer=%d" % (n, link, defer))
    got = _gpu_run(ctx, torch, d, link, defer=defer)
    exp = oracle.run_f32(d, link)
    assert _same(got, exp), _diff(got, exp)


@pytest.mark.parametrize("defer", [1, 0])
@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("n,wgs", [(65, 2), (129, 3), (300, 5), (1000, 7), (1000, 16), (2500, 40)])
def test_edge_sizes_multi_wg(ctx, torch, n, wgs, link, defer):
    """Groups of workgroups with deferred rescans (defer = 1, the default)
    and on one workgroup and groups with immediate rescans (defer = 0)."""
    d = synth.mixture_8192(seed=2000 + n, n=n)
    _say("edge multi-wg n=%d wgs=%d %s defer=%d" % (n, wgs, link, defer))
    got = _gpu_run(ctx, torch, d, link, single_wg_n=1, workgroups=wgs, defer=defer)
    exp = oracle.run_f32(d, link)
    assert _same(got, exp), _diff(got, exp)


@pytest.mark.parametrize("link", LINKS)
def test_tie_heavy(ctx, torch, link):
    """Quantised and constant matrices: ties everywhere, resolved to the
    smallest (i, j) on both sides."""
    for n, d in ((400, synth.quantized_matrix(400, 5, levels=3)),
                 (257, np.full((257, 257), 1.5, np.float32)),
                 (700, synth.rmsd_like(seed=77, n=700))):
        for opts in ({}, {"single_wg_n": 1, "workgroups": 9}):
            _say("ties n=%d %s %r" % (n, link, opts))
            got = _gpu_run(ctx, torch, d, link, **opts)
            exp = oracle.run_f32(d, link)
            assert _same(got, exp), _diff(got, exp)


def test_hand_worked_cases(ctx, torch):
    import json
    from conftest import matrix_from_upper
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "hand_worked.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        d = matrix_from_upper(case["n"], case["upper"], fill_lower=0.0)
        for link in LINKS:
            got = _gpu_run(ctx, torch, d, link)
            exp = case["expected"][link]
            assert [(int(g["i"]), int(g["j"]), float(g["h"]), int(g["size"])) for g in got] == \
                [(e[0], e[1], float(np.float32(e[2])), e[3]) for e in exp], (case["name"], link)


def test_mixture_512_complete(ctx, torch):
    """n=512 complete linkage, 8 isotropic Gaussians in R^8."""
    d = synth.mixture_512()
    _say("mixture_512")
    got = _gpu_run(ctx, torch, d, "complete")
    exp = oracle.run_f32(d, "complete")
    assert _same(got, exp), _diff(got, exp)


def test_workgroup_sweep_identical(ctx, torch):
    """The merge list does not depend on how many workgroups share the work."""
    d = synth.rmsd_like(seed=91, n=3000)
    ref = oracle.run_f32(d, "complete")
    for wgs in (1, 2, 8, 32, 47, 0):
        opts = {"single_wg_n": 1, "workgroups": wgs} if wgs != 1 else {"single_wg_n": 4096}
        _say("sweep wgs=%d" % wgs)
        got = _gpu_run(ctx, torch, d, "complete", **opts)
        assert _same(got, ref), (wgs, _diff(got, ref))


def test_input_conventions(ctx, torch):
    """Lower triangle ignored, -0 read as +0, non-finite rejected."""
    import paper_1709_06816_amd as hac
    d = synth.quantized_matrix(200, 4)
    d[3, 10] = -0.0
    junk = d.copy()
    il = np.tril_indices(200, 0)
    junk[il] = np.nan
    exp = oracle.run_f32(d, "average")
    assert _same(_gpu_run(ctx, torch, junk, "average"), exp)
    bad = d.copy()
    bad[5, 150] = np.inf
    with pytest.raises(hac.HacError) as e:
        _gpu_run(ctx, torch, bad, "average")
    assert e.value.code == hac.HAC_EINPUT
    bad[5, 150] = 2.0 ** 101
    with pytest.raises(hac.HacError) as e:
        _gpu_run(ctx, torch, bad, "average", single_wg_n=1, workgroups=4)
    assert e.value.code == hac.HAC_EINPUT
    # the context still works after an input error
    assert _same(_gpu_run(ctx, torch, d, "average"), exp)


def test_preserve_and_determinism(ctx, torch):
    d = synth.mixture_8192(seed=5, n=1500)
    t = torch.from_numpy(d).cuda()
    a = ctx.run(t, "ward", preserve=True)
    assert torch.equal(t.cpu(), torch.from_numpy(d))
    b = ctx.run(t, "ward", preserve=True)
    assert _same(a, b)
    assert _same(a, oracle.run_f32(d, "ward"))


def test_n1_and_errors(ctx, torch):
    import paper_1709_06816_amd as hac
    t = torch.zeros((1, 1), device="cuda")
    assert len(ctx.run(t, "single")) == 0
    with pytest.raises(hac.HacError) as e:
        ctx.run(torch.zeros((4, 4), device="cuda"), 9)
    assert e.value.code == hac.HAC_EINVAL


@pytest.mark.parametrize("link", LINKS)
def test_scan_mode_matches_oracle(ctx, torch, link):
    """HAC_MODE_SCAN (the paper's full rescan before every merge, Section 5.3
    step 1) gives the same bytes as the oracle and as the cached path, on
    one workgroup and on groups of workgroups, including a tie-heavy
    matrix."""
    import paper_1709_06816_amd as hac
    cases = [(synth.batch_instance(300, 301), 0), (synth.batch_instance(1000, 1001), 0),
             (synth.batch_instance(1000, 1002), 4), (synth.quantized_matrix(700, 703), 8),
             (synth.batch_instance(2500, 2501), 16)]
    for d, wgs in cases:
        n = d.shape[0]
        _say("scan mode n=%d wgs=%d %s" % (n, wgs, link))
        if wgs:
            ctx.set_option(hac.OPT_SINGLE_WG_N, 1)
            ctx.set_option(hac.OPT_WORKGROUPS, wgs)
        try:
            t = torch.from_numpy(np.ascontiguousarray(d)).cuda()
            got = ctx.run(t, link, preserve=True, scan=True)
            cached = ctx.run(t, link, preserve=True)
        finally:
            ctx.set_option(hac.OPT_SINGLE_WG_N, 0)
            ctx.set_option(hac.OPT_WORKGROUPS, 0)
        exp = oracle.run_f32(d, link)
        assert _same(got, exp), (n, wgs, _diff(got, exp))
        assert _same(cached, exp), (n, wgs)


@pytest.mark.parametrize("link", LINKS)
def test_deferred_rescans_match_oracle(ctx, torch, link):
    """Multi-workgroup hac_run with deferred rescans (stale rows keep lower
    bounds and are rescanned only when a bound wins an argmin) in automatic
    (the default: any group) and forced (HAC_OPT_DEFER = 2) mode, and with
    immediate rescans (HAC_OPT_DEFER = 0), gives the oracle's bytes.  Stale
    bounds win argmins on every input here, so the forced rounds run too."""
    import paper_1709_06816_amd as hac
    cases = [(synth.batch_instance(1000, 1001), 7), (synth.quantized_matrix(700, 703), 8),
             (synth.rmsd_like(seed=77, n=700), 9), (synth.quantized_matrix(1500, 1507, levels=4), 24),
             (synth.batch_instance(2500, 2501), 40)]
    forced = {}
    for d, wgs in cases:
        n = d.shape[0]
        exp = oracle.run_f32(d, link)
        t = torch.from_numpy(np.ascontiguousarray(d)).cuda()
        ctx.set_option(hac.OPT_SINGLE_WG_N, 1)
        ctx.set_option(hac.OPT_WORKGROUPS, wgs)
        try:
            for defer in (2, 1, 0):
                _say("deferred rescans n=%d wgs=%d %s defer=%d" % (n, wgs, link, defer))
                ctx.set_option(hac.OPT_DEFER, defer)
                got = ctx.run(t, link, preserve=True)
                st = ctx.stats()
                assert st["workgroups"] == wgs
                assert st["deferred"] == (defer == 2 or (defer == 1 and wgs >= 2))
                assert _same(got, exp), (n, wgs, defer, _diff(got, exp))
                if defer == 2:
                    forced[n] = st["forced_rounds"]
                elif not st["deferred"]:
                    assert st["forced_rounds"] == 0
        finally:
            ctx.set_option(hac.OPT_DEFER, 1)
            ctx.set_option(hac.OPT_SINGLE_WG_N, 0)
            ctx.set_option(hac.OPT_WORKGROUPS, 0)
    _say("forced rounds %s: %r" % (link, forced))
    if link == "complete":
        assert forced[700] > 0


# ---------------------------------------------------------------------------
# Batched launch
# ---------------------------------------------------------------------------

def test_batch_matches_oracle_and_run(ctx, torch):
    spec = synth.batch_spec(count=48, n_lo=64, n_hi=900, seed=4242)
    mats = [synth.batch_instance(n, s) for n, s in zip(spec.ns, spec.seeds)]
    offs, total = synth.pack_offsets(spec.ns)
    packed = np.zeros(total, np.float32)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k] + m.size] = m.ravel()
    _say("batch 48")
    t = torch.from_numpy(packed).cuda()
    res = ctx.batch(t, offs, spec.ns, spec.linkages, preserve=True)
    moff, _ = synth.merge_offsets(spec.ns)
    for k, m in enumerate(mats):
        n = int(spec.ns[k])
        got = res[moff[k]:moff[k] + n - 1]
        exp = oracle.run_f32(m, int(spec.linkages[k]))
        assert _same(got, exp), (k, n, _diff(got, exp))
        if k % 8 == 0:
            single = _gpu_run(ctx, torch, m, int(spec.linkages[k]))
            assert _same(got, single)


def test_batch_ragged_edges(ctx, torch):
    ns = np.array([1, 2, 3, 64, 65, 5, 130, 1], np.int64)
    links = np.array([0, 1, 2, 3, 0, 1, 2, 3], np.int32)
    mats = [synth.uniform_matrix(int(n), 50 + k) for k, n in enumerate(ns)]
    offs, total = synth.pack_offsets(ns)
    packed = np.zeros(total, np.float32)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k] + m.size] = m.ravel()
    res = ctx.batch(torch.from_numpy(packed).cuda(), offs, ns, links)
    moff, _ = synth.merge_offsets(ns)
    for k, m in enumerate(mats):
        n = int(ns[k])
        exp = oracle.run_f32(m, int(links[k]))
        assert _same(res[moff[k]:moff[k] + n - 1], exp), k


def test_batch_all_linkages(ctx, torch):
    """One batch holding every linkage, with instances large enough for
    groups of workgroups, on the tuned plan and on fixed plans with and
    without groups: every instance byte-identical to the oracle."""
    ns = np.array([2300, 2100, 700, 650, 300, 257, 130, 129, 65, 64, 33, 5, 3, 2], np.int64)
    links = np.array([5, 4, 4, 5, 0, 1, 2, 3, 4, 5, 5, 4, 5, 4], np.int32)
    mats = [synth.batch_instance(int(n), 6100 + k) for k, n in enumerate(ns)]
    offs, total = synth.pack_offsets(ns)
    packed = np.zeros(total, np.float32)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k] + m.size] = m.ravel()
    t = torch.from_numpy(packed).cuda()
    moff, _ = synth.merge_offsets(ns)
    exps = [oracle.run_f32(m, int(links[k])) for k, m in enumerate(mats)]
    for block, group in [(0, 0), (256, 1), (1024, 4)]:
        _say("batch all linkages block=%d group=%d" % (block, group))
        res, st = _batch_with_plan(ctx, torch, t, offs, ns, links, block, group)
        if group:
            assert st["group"] == group
        for k in range(len(ns)):
            n = int(ns[k])
            got = res[moff[k]:moff[k] + n - 1]
            assert _same(got, exps[k]), (block, group, k, n, int(links[k]), _diff(got, exps[k]))


def test_batch_lazy_mirror(ctx, torch):
    """The lazy mirror (the update writes only the survivor's row; each pair
    is read from whichever of its rows was written last) against writing
    both halves: identical records for every linkage, on one workgroup and on
    groups, with n a multiple of four (16-byte row scans) and not; both equal
    the oracle."""
    import paper_1709_06816_amd as hac
    ns = np.array([2100, 2051, 515, 512, 257, 130, 99, 64, 7, 2], np.int64)  # the first two get groups
    links = np.array([0, 1, 2, 3, 4, 5, 3, 2, 1, 0], np.int32)
    mats = [synth.batch_instance(int(n), 7300 + k) for k, n in enumerate(ns)]
    mats[1] = synth.quantized_matrix(2051, 7301, levels=6)  # many ties
    offs, total = synth.pack_offsets(ns)
    packed = np.zeros(total, np.float32)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k] + m.size] = m.ravel()
    t = torch.from_numpy(packed).cuda()
    moff, _ = synth.merge_offsets(ns)
    exps = [oracle.run_f32(m, int(links[k])) for k, m in enumerate(mats)]
    try:
        for block, group in [(1024, 1), (1024, 4), (256, 1)]:
            got = {}
            for lazy in (1, 0):
                _say("batch lazy=%d block=%d group=%d" % (lazy, block, group))
                ctx.set_option(hac.OPT_LAZY_MIRROR, lazy)
                got[lazy], st = _batch_with_plan(ctx, torch, t, offs, ns, links, block, group)
                assert st["group"] == group and st["deferred"] == 1
            assert _same(got[1], got[0]), (block, group)
            for k in range(len(ns)):
                n = int(ns[k])
                assert _same(got[1][moff[k]:moff[k] + n - 1], exps[k]), (block, group, k, n)
    finally:
        ctx.set_option(hac.OPT_LAZY_MIRROR, 1)


def test_batch_largest_instances(ctx, torch):
    """Instances of the batch's largest size (HAC_MAX_BATCH_N = 8192, the
    most LDS the lazy mirror's step table needs on one workgroup) beside
    small ones, with and without the lazy mirror and on one workgroup and
    on groups: each equals hac_run on the same matrix."""
    import paper_1709_06816_amd as hac
    ns = np.array([8192, 8191, 300, 5, 2], np.int64)
    links = np.array([1, 3, 2, 0, 4], np.int32)
    mats = [synth.batch_instance(int(n), 8800 + k) for k, n in enumerate(ns)]
    offs, total = synth.pack_offsets(ns)
    packed = np.zeros(total, np.float32)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k] + m.size] = m.ravel()
    t = torch.from_numpy(packed).cuda()
    moff, _ = synth.merge_offsets(ns)
    refs = [_gpu_run(ctx, torch, m, int(links[k])) for k, m in enumerate(mats)]
    try:
        for lazy in (1, 0):
            ctx.set_option(hac.OPT_LAZY_MIRROR, lazy)
            for block, group in [(1024, 1), (1024, 4)]:
                _say("batch largest lazy=%d block=%d group=%d" % (lazy, block, group))
                res, st = _batch_with_plan(ctx, torch, t, offs, ns, links, block, group)
                for k in range(len(ns)):
                    n = int(ns[k])
                    assert _same(res[moff[k]:moff[k] + n - 1], refs[k]), (lazy, block, group, k, n)
    finally:
        ctx.set_option(hac.OPT_LAZY_MIRROR, 1)


def _batch_with_plan(ctx, torch, t, offs, ns, links, block, group, upd=0):
    import paper_1709_06816_amd as hac
    ctx.set_option(hac.OPT_BATCH_BLOCK, block)
    ctx.set_option(hac.OPT_BATCH_GROUP, group)
    ctx.set_option(hac.OPT_BATCH_UPDATE, upd)
    try:
        res = ctx.batch(t, offs, ns, links, preserve=True)
        return res, ctx.stats()
    finally:
        ctx.set_option(hac.OPT_BATCH_BLOCK, 0)
        ctx.set_option(hac.OPT_BATCH_GROUP, 0)
        ctx.set_option(hac.OPT_BATCH_UPDATE, 0)


def test_batch_plans_identical(ctx, torch):
    """Every launch plan (threads per workgroup, workgroups per large
    instance) and the autotuned one give the same bytes; the instances that
    ran on groups of workgroups match the oracle."""
    spec = synth.batch_spec(count=40, n_lo=64, n_hi=4096, seed=777)
    ns = spec.ns.copy()
    ns[:3] = [4096, 2500, 2048]  # instances that qualify for groups
    mats = [synth.batch_instance(int(n), int(s)) for n, s in zip(ns, spec.seeds)]
    offs, total = synth.pack_offsets(ns)
    packed = np.zeros(total, np.float32)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k] + m.size] = m.ravel()
    t = torch.from_numpy(packed).cuda()
    ref = None
    for block, group, upd in [(256, 1, 0), (1024, 1, 0), (1024, 1, 2), (256, 4, 0), (1024, 8, 0), (1024, 2, 2),
                              (256, 16, 0)]:
        _say("batch plan block=%d group=%d update=%d" % (block, group, upd))
        res, st = _batch_with_plan(ctx, torch, t, offs, ns, spec.linkages, block, group, upd)
        assert st["block"] == block
        assert st["group"] == group
        assert st["plan_update"] == (8 if block == 256 else upd or 4)
        if ref is None:
            ref = res
        else:
            assert _same(res, ref), (block, group)
    _say("batch autotuned")
    res = ctx.batch(t, offs, ns, spec.linkages, preserve=True)
    assert _same(res, ref)
    st = ctx.stats()
    assert st["block"] in (256, 1024) and st["plan_source"] == 1
    assert st["plan_update"] in ((8,) if st["block"] == 256 else (2, 4))
    assert st["plan_share"] in ((1, 2, 3) if st["group"] > 1 else (0,))
    res = ctx.batch(t, offs, ns, spec.linkages, preserve=True)  # cached plan
    assert _same(res, ref)
    st2 = ctx.stats()
    assert st2["plan_source"] == 2 and (st2["block"], st2["group"]) == (st["block"], st["group"])
    assert np.array_equal(t.cpu().numpy(), packed)
    moff, _ = synth.merge_offsets(ns)
    for k in range(3):
        n = int(ns[k])
        exp = oracle.run_f32(mats[k], int(spec.linkages[k]))
        assert _same(ref[moff[k]:moff[k] + n - 1], exp), (k, n)


def test_batch_graph_replays(ctx, torch):
    """The batch as one HIP graph: built once per layout, relaunched with new
    inputs; every replay, with eager work in between, equals the stream
    launch on the same input.  Also with groups (cooperative kernel node)."""
    import paper_1709_06816_amd as hac
    ns = np.array([2600, 900, 700, 300, 64, 65, 130, 33, 5, 2], np.int64)
    links = np.array([1, 3, 2, 0, 1, 2, 3, 0, 1, 3], np.int32)
    offs, total = synth.pack_offsets(ns)
    inputs = []
    for rep in range(3):
        packed = np.zeros(total, np.float32)
        for k, n in enumerate(ns):
            packed[offs[k]:offs[k] + n * n] = synth.batch_instance(int(n), 9000 + 100 * rep + k).ravel()
        inputs.append(torch.from_numpy(packed).cuda())
    for group in (1, 4):
        ctx.set_option(hac.OPT_BATCH_BLOCK, 256)
        ctx.set_option(hac.OPT_BATCH_GROUP, group)
        try:
            ctx.set_option(hac.OPT_GRAPH, 0)
            eager = [ctx.batch(t, offs, ns, links, preserve=True) for t in inputs]
            assert ctx.stats()["graph"] == 0
            ctx.set_option(hac.OPT_GRAPH, 1)
            for rep in range(6):
                k = rep % 3
                _say("graph group=%d replay %d" % (group, rep))
                res = ctx.batch(inputs[k], offs, ns, links, preserve=True)
                st = ctx.stats()
                assert st["graph"] == (2 if rep == 0 else 1), st["graph"]
                assert st["group"] == group
                assert _same(res, eager[k]), (group, rep)
                # eager work between replays
                m = synth.uniform_matrix(70, 300 + rep)
                assert _same(_gpu_run(ctx, torch, m, "average"), oracle.run_f32(m, "average"))
        finally:
            ctx.set_option(hac.OPT_GRAPH, 1)
            ctx.set_option(hac.OPT_BATCH_BLOCK, 0)
            ctx.set_option(hac.OPT_BATCH_GROUP, 0)
    moff, _ = synth.merge_offsets(ns)
    packed = inputs[0].cpu().numpy()
    for k, n in enumerate(ns):
        m = packed[offs[k]:offs[k] + n * n].reshape(n, n)
        assert _same(eager[0][moff[k]:moff[k] + n - 1], oracle.run_f32(m, int(links[k]))), k


def test_batch_config_sample_vs_oracle(ctx, torch):
    """The 1024-instance batch configuration's first 256 instances (same seeds
    and size law, n log-uniform on [64, 4096], single, complete, average and Ward) in one
    launch with the default (tuned) plan: every instance with n <= 1536 and a
    sample of the larger ones byte-identical to the oracle, run on host
    threads in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    full = synth.batch_spec()  # the benchmark's batch: 1024 instances
    count = 256
    ns, links, seeds = full.ns[:count], full.linkages[:count], full.seeds[:count]
    offs, total = synth.pack_offsets(ns)
    packed = np.zeros(total, np.float32)
    mats = []
    for k in range(count):
        m = synth.batch_instance(int(ns[k]), int(seeds[k]))
        packed[offs[k]:offs[k] + m.size] = m.ravel()
        mats.append(m)
    _say("batch config sample: %d instances, %.2f GB" % (count, total * 4 / 1e9))
    res = ctx.batch(torch.from_numpy(packed).cuda(), offs, ns, links)
    moff, _ = synth.merge_offsets(ns)
    big = [k for k in range(count) if ns[k] > 1536]
    rng = np.random.default_rng(3)
    check = [k for k in range(count) if ns[k] <= 1536] + sorted(rng.choice(big, size=min(12, len(big)), replace=False))
    workers = min(16, os.cpu_count() or 4)

    def one(k):
        return k, oracle.run_f32(mats[k], int(links[k]), threads=1)

    with ThreadPoolExecutor(workers) as ex:
        for k, exp in ex.map(one, check):
            n = int(ns[k])
            got = res[moff[k]:moff[k] + n - 1]
            assert _same(got, exp), (k, n, int(links[k]), _diff(got, exp))
    _say("checked %d of %d instances against the oracle" % (len(check), count))


# ---------------------------------------------------------------------------
# Larger sizes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("link", LINKS)
def test_mixture_8192(ctx, torch, link):
    """n=8192, 32 Gaussians in R^16: full list byte-identical to the oracle."""
    d = synth.mixture_8192()
    _say("mixture_8192 %s" % link)
    got = _gpu_run(ctx, torch, d, link)
    exp = oracle.run_f32(d, link)
    assert _same(got, exp), _diff(got, exp)
    h64, _ = oracle.replay_f64(d, link, got)
    assert np.all(np.abs(got["h"].astype(np.float64) - h64) <= 1e-5 * np.abs(h64) + 1e-30)


def _check_structure(m, n):
    """Merge-list invariants: n-1 merges, i < j, j retired exactly once and
    never used again, sizes add up, survivor is the smallest member."""
    assert len(m) == n - 1
    alive = np.ones(n, bool)
    size = np.ones(n, np.int64)
    for r in m:
        i, j = int(r["i"]), int(r["j"])
        assert 0 <= i < j < n and alive[i] and alive[j]
        size[i] += size[j]
        assert int(r["size"]) == size[i]
        alive[j] = False
    assert alive.sum() == 1 and alive[0]


def test_rmsd_like_32768_complete(ctx, torch):
    """n=32768 RMSD-like complete linkage: first 40 merges byte-identical to
    the oracle's, complete-linkage heights non-decreasing, structure valid,
    fp64 replay heights within 1e-5 and sampled optimality."""
    n = 32768
    d = synth.rmsd_like()
    _say("rmsd_like 32768 gpu")
    got = _gpu_run(ctx, torch, d, "complete")
    _check_structure(got, n)
    assert np.all(np.diff(got["h"]) >= 0)
    _say("rmsd_like 32768 oracle prefix")
    exp = oracle.run_f32(d, "complete", max_merges=40)
    assert _same(got[:40], exp), _diff(got[:40], exp)
    _say("rmsd_like 32768 replay")
    h64, min64 = oracle.replay_f64(d, "complete", got, opt_stride=4096)
    assert np.all(np.abs(got["h"].astype(np.float64) - h64) <= 1e-5 * np.abs(h64))
    sel = ~np.isnan(min64)
    assert np.all(h64[sel] <= min64[sel])
