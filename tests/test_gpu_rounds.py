"""Round engine (HAC_OPT_ROUNDS): single and complete linkage merged in rounds
of reciprocal nearest neighbours must give the oracle's merge list byte for
byte (Section 4's loop, lexicographic ties), whatever the number of
workgroups, on tie-heavy inputs too, and at the workload sizes."""
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
        c.set_option(hac.OPT_ROUNDS, 2)
        c.set_option(hac.OPT_TIMEOUT_MS, 20000)
        yield c


def _run(ctx, d, link, wgs=0):
    import torch
    ctx.set_option(hac.OPT_WORKGROUPS, wgs)
    try:
        got = ctx.run(torch.from_numpy(np.ascontiguousarray(d)).cuda(), link)
        st = ctx.stats()
    finally:
        ctx.set_option(hac.OPT_WORKGROUPS, 0)
    return got, st


def _lattice(n, seed, side=4):
    rng = np.random.default_rng(seed)
    return synth.euclidean_matrix(rng.integers(0, side, size=(n, 2)).astype(np.float64))


CASES = [
    ("mixture", lambda n, s: synth.mixture_8192(seed=s, n=n)),
    ("rmsd_like", lambda n, s: synth.rmsd_like(seed=s, n=n)),
    ("quantized3", lambda n, s: synth.quantized_matrix(n, seed=s, levels=3)),
    ("quantized7", lambda n, s: synth.quantized_matrix(n, seed=s, levels=7)),
    ("uniform", lambda n, s: synth.uniform_matrix(n, seed=s)),
    ("lattice", _lattice),
]


@pytest.mark.parametrize("link", ["single", "complete"])
@pytest.mark.parametrize("name,gen", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("n", [2, 3, 5, 64, 65, 131, 700])
def test_rounds_match_oracle(ctx, link, name, gen, n):
    d = gen(n, 1000 + n)
    print("rounds: %s n=%d %s" % (name, n, link), flush=True)
    got, st = _run(ctx, d, link)
    exp = oracle.run_f32(d, link)
    assert got.tobytes() == exp.tobytes()
    assert st["rounds"] >= 1 and st["handed_over"] == 0


@pytest.mark.parametrize("wgs", [1, 2, 7, 33])
@pytest.mark.parametrize("link", ["single", "complete"])
def test_rounds_any_workgroup_count(ctx, link, wgs):
    d = synth.rmsd_like(seed=77, n=1500)
    print("rounds: rmsd_like n=1500 %s on %d workgroups" % (link, wgs), flush=True)
    got, st = _run(ctx, d, link, wgs)
    assert st["workgroups"] == wgs
    assert got.tobytes() == oracle.run_f32(d, link).tobytes()


@pytest.mark.parametrize("link", ["single", "complete"])
def test_rounds_constant_matrix(ctx, link):
    # Every pair tied: single linkage falls back to one merge per round.
    n = 300
    d = np.full((n, n), 2.5, np.float32)
    np.fill_diagonal(d, 0)
    print("rounds: constant n=300 %s" % link, flush=True)
    got, st = _run(ctx, d, link)
    assert got.tobytes() == oracle.run_f32(d, link).tobytes()


@pytest.mark.parametrize("link", ["single", "complete"])
def test_rounds_more_pairs_than_one_round_takes(ctx, link):
    # 4096 tight pairs of points far apart (n=8192): the first round offers
    # 4096 reciprocal pairs, more than a round merges (2048); the rest wait
    # for the next round.  Then the n=8192 mixture.
    rng = np.random.default_rng(5)
    centres = rng.uniform(-100.0, 100.0, size=(4096, 16))
    pts = np.repeat(centres, 2, axis=0) + rng.normal(0.0, 0.01, size=(8192, 16))
    # Past the first rounds the tight-pairs input is 4096 points spread
    # uniformly, on which single linkage chains (few reciprocal pairs per
    # round): the round bound is looser there.
    for name, d, bound in (("tight pairs", synth.euclidean_matrix(pts), 8191 // 2),
                           ("mixture", synth.mixture_8192(seed=5, n=8192), 8191 // 8)):
        print("rounds: %s n=8192 %s" % (name, link), flush=True)
        got, st = _run(ctx, d, link)
        assert got.tobytes() == oracle.run_f32(d, link).tobytes()
        assert st["rounds"] < bound, (name, st["rounds"])


def test_rounds_input_errors_and_flags(ctx):
    import torch
    d = synth.mixture_8192(seed=6, n=1200)
    t = torch.from_numpy(d).cuda()
    exp = oracle.run_f32(d, "complete")
    print("rounds: preserve / device output / rejected input", flush=True)
    got = ctx.run(t, "complete", preserve=True)
    assert got.tobytes() == exp.tobytes()
    assert torch.equal(t.cpu(), torch.from_numpy(d))
    out = torch.zeros(1199 * 16, dtype=torch.uint8, device="cuda")
    ctx.run(t.clone(), "complete", out=out)
    ctx.sync()
    assert out.cpu().numpy().tobytes() == exp.tobytes()
    bad = d.copy()
    bad[3, 900] = np.nan
    before = np.zeros(1199, hac.MERGE_DTYPE)
    with pytest.raises(hac.HacError) as e:
        ctx.run(torch.from_numpy(bad).cuda(), "single")
    assert e.value.code == hac.HAC_EINPUT
    del before


def test_rounds_not_used_for_other_linkages(ctx):
    import torch
    d = synth.mixture_8192(seed=8, n=1100)
    got = ctx.run(torch.from_numpy(d).cuda(), "average")
    assert ctx.stats()["rounds"] == 0
    assert got.tobytes() == oracle.run_f32(d, "average").tobytes()


def test_single_linkage_hands_over_part_way(ctx):
    """Automatic mode: rounds stop once they merge few pairs each and the
    one-merge-per-step kernel queued behind resumes from that state (early for
    single linkage on input with many equal values); every result is the
    oracle's, on several workgroup counts."""
    import torch
    ctx.set_option(hac.OPT_ROUNDS, 1)
    try:
        for name, d, handed in (("quantized", synth.quantized_matrix(2000, seed=31, levels=6), True),
                                ("rmsd_like", synth.rmsd_like(seed=33, n=3000), True),
                                # n <= 1536: the resuming kernel is one workgroup
                                ("quantized", synth.quantized_matrix(1200, seed=34, levels=4), True),
                                ("mixture", synth.mixture_8192(seed=32, n=2000), False)):
            for wgs in (0, 5):
                ctx.set_option(hac.OPT_WORKGROUPS, wgs)
                print("rounds: automatic single %s n=%d wgs=%d" % (name, d.shape[0], wgs), flush=True)
                got = ctx.run(torch.from_numpy(d).cuda(), "single")
                st = ctx.stats()
                if handed:
                    # Ties force it early (untied input may hand over only the tail).
                    assert st["handed_over"] == 1 and st["rounds"] < 200, (name, st)
                assert st["rounds"] > 0
                assert got.tobytes() == oracle.run_f32(d, "single").tobytes()
            ctx.set_option(hac.OPT_WORKGROUPS, 0)
            got = ctx.run(torch.from_numpy(d).cuda(), "complete")
            assert ctx.stats()["rounds"] > 0
            assert got.tobytes() == oracle.run_f32(d, "complete").tobytes()
    finally:
        ctx.set_option(hac.OPT_ROUNDS, 2)
        ctx.set_option(hac.OPT_WORKGROUPS, 0)
