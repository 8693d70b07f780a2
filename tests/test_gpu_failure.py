"""Failure path of the persistent kernels: a wait that never ends is cut
short by the kernels' own watchdog.  HAC_OPT_INJECT_STALL makes workgroup 0
of a multi-workgroup hac_run keep its first exchange to itself (a flag set
from the host, no fault), so every other workgroup's bounded wait expires
after HAC_OPT_TIMEOUT_MS; every kernel must then leave, the call must return
HAC_ETIMEDOUT in about that time, and the context must work normally
afterwards."""
import time

import numpy as np
import pytest

import oracle
import paper_1709_06816_amd as hac
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    with hac.Context(0) as c:
        yield c


@pytest.mark.parametrize("rounds,link", [(0, "complete"), (0, "average"), (1, "single"), (1, "complete"),
                                         (2, "complete")])
def test_stalled_exchange_times_out_and_recovers(ctx, rounds, link):
    import torch
    d = synth.mixture_8192(seed=91, n=3000)
    t = torch.from_numpy(d).cuda()
    ctx.set_option(hac.OPT_ROUNDS, rounds)
    ctx.set_option(hac.OPT_TIMEOUT_MS, 100)
    ctx.set_option(hac.OPT_INJECT_STALL, 1)
    try:
        print("failure: stalled exchange, rounds=%d %s" % (rounds, link), flush=True)
        t0 = time.perf_counter()
        with pytest.raises(hac.HacError) as e:
            ctx.run(t, link, preserve=True)
        took = time.perf_counter() - t0
        assert e.value.code == hac.HAC_ETIMEDOUT
        assert took < 10.0
    finally:
        ctx.set_option(hac.OPT_INJECT_STALL, 0)
        ctx.set_option(hac.OPT_TIMEOUT_MS, 0)
    try:
        got = ctx.run(t, link, preserve=True)
        assert got.tobytes() == oracle.run_f32(d, link).tobytes()
    finally:
        ctx.set_option(hac.OPT_ROUNDS, 1)


def test_autotune_never_picks_a_failing_plan(ctx):
    """hac_batch's autotuner reads every candidate's status words: with the
    first exchange of every group withheld (HAC_OPT_INJECT_STALL) and a short
    watchdog, each plan with groups ends in a timeout, so the tuner must pick
    a plan without groups; the call then succeeds with the oracle's lists."""
    import torch
    spec = synth.batch_spec(count=12, n_lo=64, n_hi=1024, seed=515)
    ns = spec.ns.copy()
    ns[:2] = [2600, 2100]  # instances that qualify for groups
    mats = [synth.batch_instance(int(n), int(s)) for n, s in zip(ns, spec.seeds)]
    offs, total = synth.pack_offsets(ns)
    packed = np.zeros(total, np.float32)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k] + m.size] = m.ravel()
    t = torch.from_numpy(packed).cuda()
    ctx.set_option(hac.OPT_TIMEOUT_MS, 50)
    ctx.set_option(hac.OPT_INJECT_STALL, 1)
    try:
        print("failure: autotuning with stalled group exchanges", flush=True)
        res = ctx.batch(t, offs, ns, spec.linkages, preserve=True)
        st = ctx.stats()
    finally:
        ctx.set_option(hac.OPT_INJECT_STALL, 0)
        ctx.set_option(hac.OPT_TIMEOUT_MS, 0)
    assert st["plan_source"] == 1 and st["group"] == 1
    moff, _ = synth.merge_offsets(ns)
    for k in range(len(ns)):
        n = int(ns[k])
        assert res[moff[k]:moff[k] + n - 1].tobytes() == oracle.run_f32(mats[k], int(spec.linkages[k])).tobytes(), k
