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
