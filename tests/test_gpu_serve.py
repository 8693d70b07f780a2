"""GPU tests of the serving layer (hac_server_*), through the C-ABI: every
job's merge list is byte-identical to hac_run on the same matrix and to the
oracle, alone or in a mix, with groups of workgroups, under an arena budget
that makes jobs wait, across kernel stops and relaunches, and with job slots
reused.  References are computed before a server exists (or after it is
closed), so no other kernel competes with the persistent one."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

LINKS = ["single", "complete", "average", "ward", "weighted", "centroid"]


def _say(*a):
    print("[gpu-serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def hac():
    import paper_1709_06816_amd as h
    return h


@pytest.fixture(scope="module")
def ctx(torch, hac):
    c = hac.Context(0)
    c.set_option(hac.OPT_TIMEOUT_MS, 20000)  # server watchdog and idle self-stop
    yield c
    c.close()


def _run_ref(ctx, torch, d, link):
    t = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda()
    res = ctx.run(t, link)
    torch.cuda.synchronize()
    return res


def _drain(server, tickets, deadline_s=90.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for k, t in tickets.items():
            if k not in out:
                r = server.poll(t)
                if r is not None:
                    out[k] = r
        if time.time() - t0 > deadline_s:
            raise AssertionError("jobs not done after %.0f s: %d of %d" % (deadline_s, len(out), len(tickets)))
        time.sleep(0.001)
    return out


def _jobs():
    ns = [2, 3, 64, 65, 300, 1000, 2049, 2500, 4100, 5000, 1, 777, 8192, 129]
    jobs = []
    for k, n in enumerate(ns):
        d = synth.batch_instance(n, 5150 + k) if n > 1 else np.zeros((1, 1), np.float32)
        jobs.append((n, LINKS[k % len(LINKS)], d))
    return jobs


def test_server_matches_run_and_oracle(ctx, torch, hac):
    jobs = _jobs()
    refs = [_run_ref(ctx, torch, d, l) for n, l, d in jobs]
    for (n, l, d), r in zip(jobs, refs):
        if n <= 1000:
            assert r.tobytes() == oracle.run_f32(d, l).tobytes(), (n, l)
    # Some jobs as views of a larger array (leading dimension > n).
    host = []
    for k, (n, l, d) in enumerate(jobs):
        if k % 3 == 1 and n > 1:
            big = np.full((n + 5, n + 37), np.nan, np.float32)
            big[:n, :n] = d
            host.append(big[:n, :n])
        else:
            host.append(np.ascontiguousarray(d))
    with hac.Server(ctx, budget_bytes=1 << 30, max_jobs=64, max_n=8192) as srv:
        for rep in range(3):  # job slots are reused across rounds
            _say("round", rep)
            tickets = {k: srv.submit(host[k], l) for k, (n, l, d) in enumerate(jobs)}
            got = _drain(srv, tickets)
            for k, (n, l, d) in enumerate(jobs):
                assert got[k].tobytes() == refs[k].tobytes(), (rep, n, l)
        st = srv.stats()
        assert st["completed"] == st["submitted"] == 3 * len(jobs)
        assert st["peak_bytes"] <= 1 << 30 and st["bytes_in_use"] == 0
        _say("stats", st)


def test_server_without_lazy_mirror(ctx, torch, hac):
    """A server created with HAC_OPT_LAZY_MIRROR = 0 (every update writes
    both halves, as a job whose step table does not fit the LDS does): the
    same records as hac_run."""
    jobs = _jobs()
    refs = [_run_ref(ctx, torch, d, l) for n, l, d in jobs]
    ctx.set_option(hac.OPT_LAZY_MIRROR, 0)
    try:
        with hac.Server(ctx, budget_bytes=1 << 30, max_jobs=64, max_n=8192) as srv:
            tickets = {k: srv.submit(np.ascontiguousarray(d), l) for k, (n, l, d) in enumerate(jobs)}
            got = _drain(srv, tickets)
    finally:
        ctx.set_option(hac.OPT_LAZY_MIRROR, 1)
    for k, (n, l, d) in enumerate(jobs):
        assert got[k].tobytes() == refs[k].tobytes(), (n, l)


def test_server_mix_matches_run(ctx, torch, hac):
    """160 jobs submitted at once (n log-uniform on [64, 6000], all linkages,
    about a fifth of them on groups of two workgroups) from page-locked
    pools, twice: every job byte-identical to hac_run alone."""
    N, count = 6000, 160
    pool = [torch.empty((N, N), dtype=torch.float32).pin_memory() for _ in range(2)]
    synth.serve_pool(2, N, out=[p.numpy() for p in pool])
    rng = np.random.default_rng(5)
    ns = np.minimum(synth.log_uniform_int(rng, 64, N, size=count), N)
    links = rng.integers(0, 6, size=count)
    refs = [_run_ref(ctx, torch, pool[k % 2][:int(ns[k]), :int(ns[k])].numpy(), int(links[k]))
            for k in range(count)]
    with hac.Server(ctx, budget_bytes=8 << 30, max_jobs=256, max_n=N) as srv:
        for rnd in range(2):
            _say("mix round", rnd)
            tickets = {k: srv.submit(pool[k % 2][:int(ns[k]), :int(ns[k])], int(links[k]))
                       for k in range(count)}
            got = _drain(srv, tickets)
            bad = [(k, int(ns[k]), int(links[k])) for k in range(count)
                   if got[k].tobytes() != refs[k].tobytes()]
            assert not bad, bad


def test_server_saturated_groups_match_run(ctx, torch, hac):
    """Group jobs under saturation: 240 jobs of n in [2049, 5000] (every one
    on a group of workgroups, so every merge exchanges minima between
    workgroups on different XCDs), kept at the job limit for two rounds; every
    merge list byte-identical to hac_run.  A release that lets the exchange
    flag out before the L2 write-back of the data it publishes shows up here
    as a few merge heights read from values one update old."""
    N, count = 5000, 240
    pool = [torch.empty((N, N), dtype=torch.float32).pin_memory() for _ in range(2)]
    synth.serve_pool(2, N, seed=77, out=[p.numpy() for p in pool])
    rng = np.random.default_rng(11)
    ns = np.minimum(synth.log_uniform_int(rng, 2049, N, size=count), N)
    links = rng.integers(0, 4, size=count)
    refs = [_run_ref(ctx, torch, pool[k % 2][:int(ns[k]), :int(ns[k])].numpy(), int(links[k]))
            for k in range(count)]
    with hac.Server(ctx, budget_bytes=16 << 30, max_jobs=48, max_n=N) as srv:
        for rnd in range(2):
            _say("saturated groups round", rnd)
            tickets, got, k = {}, {}, 0
            t0 = time.time()
            while len(got) < count:
                while k < count:
                    try:
                        tickets[k] = srv.submit(pool[k % 2][:int(ns[k]), :int(ns[k])], int(links[k]))
                    except hac.HacError as e:
                        assert e.code == hac.HAC_EBUSY
                        break
                    k += 1
                for q in [q for q in tickets if q not in got]:
                    r = srv.poll(tickets[q])
                    if r is not None:
                        got[q] = r
                assert time.time() - t0 < 90, "jobs not done after 90 s"
                time.sleep(0.0005)
            bad = [(q, int(ns[q]), int(links[q])) for q in range(count) if got[q].tobytes() != refs[q].tobytes()]
            assert not bad, bad


def test_server_budget_makes_jobs_wait(ctx, torch, hac):
    n, count = 1200, 24
    mats = [synth.batch_instance(n, 7300 + k) for k in range(count)]
    refs = [_run_ref(ctx, torch, m, LINKS[k % 4]) for k, m in enumerate(mats)]
    budget = 40 << 20  # about six jobs at a time
    with hac.Server(ctx, budget_bytes=budget, max_jobs=count, max_n=n) as srv:
        tickets = {k: srv.submit(m, LINKS[k % 4]) for k, m in enumerate(mats)}
        got = _drain(srv, tickets)
        st = srv.stats()
    for k in range(count):
        assert got[k].tobytes() == refs[k].tobytes(), k
    assert 4 * n * n <= st["peak_bytes"] <= budget


def test_server_errors_and_restart(ctx, torch, hac):
    good = synth.batch_instance(500, 99)
    ref = _run_ref(ctx, torch, good, "average")
    bad = good.copy()
    bad[3, 7] = np.nan
    with hac.Server(ctx, budget_bytes=64 << 20, max_jobs=2, max_n=2048) as srv:
        with pytest.raises(hac.HacError) as e:
            srv.submit(np.zeros((3000, 3000), np.float32), "single")
        assert e.value.code == hac.HAC_EINVAL
        t1 = srv.submit(bad, "average")
        t2 = srv.submit(good, "average")
        with pytest.raises(hac.HacError) as e:
            srv.submit(good, "average")
        assert e.value.code == hac.HAC_EBUSY
        got = _drain(srv, {2: t2})
        assert got[2].tobytes() == ref.tobytes()
        t0 = time.time()
        while True:
            try:
                r = srv.poll(t1)
            except hac.HacError as err:
                assert err.code == hac.HAC_EINPUT
                break
            assert r is None and time.time() - t0 < 60
            time.sleep(0.001)
        # Idle long enough for the kernel to stop; the next job relaunches it.
        time.sleep(0.2)
        launches = srv.stats()["kernel_launches"]
        got = _drain(srv, {0: srv.submit(good, "average")})
        assert got[0].tobytes() == ref.tobytes()
        assert srv.stats()["kernel_launches"] == launches + 1
    with hac.Server(ctx, budget_bytes=1 << 20, max_jobs=2, max_n=2048) as srv:
        with pytest.raises(hac.HacError) as e:
            srv.submit(synth.batch_instance(600, 98), "single")  # 1.44 MB > 1 MiB budget
        assert e.value.code == hac.HAC_ENOMEM
