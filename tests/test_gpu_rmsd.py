"""GPU parity of the input producer (hac_rmsd): the RMSD matrix of n
conformations against the fp64 Kabsch oracle (oracle/rmsd.py), through the
C-ABI.

Tolerance, derived from the arithmetic.  The device rounds centred
coordinates to fp32 (u = 2^-24), sums the nine cross-covariances
M_pq = sum_i a_ip b_iq in fp32 (recursive-summation bound
|dM_pq| <= (m-1) u sum_i |a_ip b_iq| <= (m-1) u sqrt(G_A G_B), G the squared
norms), and finds lambda_max of the key matrix K(M) in fp64.  |d lambda| <=
||dK||_2 <= 2 ||dM||_F <= 6 (m-1) u sqrt(G_A G_B), and RMSD^2 =
(G_A + G_B - 2 lambda) / m, so
    |r_gpu^2 - r^2| <= 12 u sqrt(G_A G_B) + 2 r u (sqrt(G_A/m) + sqrt(G_B/m))
                       + 2^-22 r^2 + 1e-6 (G_A + G_B) / m,
the next two terms for the coordinate rounding and the fp32 result, the last
for Newton's method at a multiple largest root (two atoms, collinear or
planar conformations), where the quartic's value near the root is rounding
noise below about sqrt(eps64) relative (measured on the host build of the
epilogue: <= 1.2e-7 (G_A + G_B) / m).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import rmsd as R

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _say(*a):
    print("[gpu-rmsd]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_1709_06816_amd as hac
    c = hac.Context(0)
    yield c
    c.close()


def _norms(coords):
    x = coords.astype(np.float64)
    x = x - x.mean(axis=1, keepdims=True)
    return (x * x).sum(axis=(1, 2))


def _bound(g, rows, cols, ref, m):
    ga, gb = g[rows], g[cols]
    return (12 * U * np.sqrt(ga * gb) + 2 * ref * U * (np.sqrt(ga / m) + np.sqrt(gb / m))
            + 2.0 ** -22 * ref * ref + 1e-6 * (ga + gb) / m + 1e-30)


def _gpu(ctx, torch, coords, sentinel=True):
    n = coords.shape[0]
    t = torch.from_numpy(np.ascontiguousarray(coords, dtype=np.float32)).cuda()
    out = torch.full((n, n), float("nan"), device="cuda") if sentinel else None
    res = ctx.rmsd(t, out=out)
    torch.cuda.synchronize()
    return res.cpu().numpy()


def _check_full(got, coords, exact_zero_diag=True):
    n, m = coords.shape[0], coords.shape[1]
    ref = R.rmsd_matrix(coords)
    rows, cols = np.triu_indices(n, 1)
    err = np.abs(got[rows, cols].astype(np.float64) ** 2 - ref[rows, cols] ** 2)
    bound = _bound(_norms(coords), rows, cols, ref[rows, cols], m)
    assert np.all(err <= bound), (n, m, float(np.max(err / bound)))
    if exact_zero_diag:
        assert np.all(np.diag(got) == 0)
    lower = np.tril_indices(n, -1)
    assert np.all(np.isnan(got[lower])), "lower triangle was written"
    return float(np.max(err / bound)) if len(err) else 0.0


@pytest.mark.parametrize("n,m", [(1, 5), (2, 1), (2, 2), (3, 3), (31, 7), (33, 64), (64, 65), (65, 128),
                                 (100, 2), (129, 33), (257, 129), (300, 300)])
def test_matches_oracle(ctx, torch, n, m):
    """Sizes around the 32- and 64-conformation tiles and odd atom counts
    (padding atom), every pair against the oracle."""
    coords = synth.conformations(n, m, seed=1000 + 7 * n + m)
    _say("rmsd n=%d m=%d" % (n, m))
    worst = _check_full(_gpu(ctx, torch, coords), coords)
    _say("worst error / bound %.3g" % worst)


def test_special_conformations(ctx, torch):
    """Rigid copies give ~0, one atom gives exactly 0, mirror images of a
    chiral conformation stay apart, collinear conformations."""
    rng = np.random.default_rng(5)
    base = synth.conformations(1, 40, seed=77)[0].astype(np.float64)
    confs = [base]
    for _ in range(5):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        confs.append(base @ q.T + rng.uniform(-30, 30, size=3))
    confs.append(base * np.array([1.0, 1.0, -1.0]))            # mirror image
    line = np.outer(np.arange(40.0), [0.5, 1.0, -1.0])
    confs += [line, line * 1.3 + 4.0]                           # collinear
    coords = np.array(confs, np.float32)
    got = _gpu(ctx, torch, coords)
    _check_full(got, coords)
    scale = np.sqrt(_norms(coords[:1])[0] / 40)
    assert np.all(got[0, 1:6] <= 1e-3 * scale)
    assert got[0, 6] > 0.1 * scale
    one = synth.conformations(40, 1, seed=3)
    g1 = _gpu(ctx, torch, one)
    assert np.all(g1[np.triu_indices(40)] == 0)


def test_input_rejected(ctx, torch):
    import paper_1709_06816_amd as hac
    coords = synth.conformations(50, 20, seed=9)
    for bad in (np.nan, np.inf, 2.0 ** 41):
        c = coords.copy()
        c[17, 3, 1] = bad
        t = torch.from_numpy(c).cuda()
        out = torch.full((50, 50), 7.0, device="cuda")
        with pytest.raises(hac.HacError) as e:
            ctx.rmsd(t, out=out)
        assert e.value.code == hac.HAC_EINPUT
        assert bool(torch.all(out == 7.0)), "output written despite rejected input"
    with pytest.raises(hac.HacError) as e:
        ctx.rmsd(torch.zeros((4, 0, 3), device="cuda"))
    assert e.value.code == hac.HAC_EINVAL
    # the context still works
    _check_full(_gpu(ctx, torch, coords), coords)


def test_feeds_clustering(ctx, torch):
    """The produced matrix is the clustering input: hac_run on it gives the
    same merge list as the oracle on the same (device-produced) matrix."""
    import oracle
    coords = synth.conformations(700, 96, seed=31)
    t = torch.from_numpy(coords).cuda()
    d = ctx.rmsd(t)
    torch.cuda.synchronize()
    got = ctx.run(d, "complete", preserve=True)
    host = d.cpu().numpy()
    exp = oracle.run_f32(host, "complete")
    assert got.tobytes() == exp.tobytes()
    _check_full(np.triu(host) + np.tril(np.full_like(host, np.nan), -1), coords)


def test_full_size_sampled(ctx, torch):
    """The benchmark's size, 32768 conformations of 128 atoms (a 4 GiB
    matrix), in the launch configuration bench.py times: 3000 sampled pairs
    (including the first and last rows and columns) against the oracle, the
    diagonal zero, and the matrix finite."""
    n, m = 32768, 128
    coords = synth.conformations(n, m)
    _say("full size: producing")
    t = torch.from_numpy(coords).cuda()
    d = ctx.rmsd(t)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    rows = rng.integers(0, n, size=3000)
    cols = rng.integers(0, n, size=3000)
    rows[:4] = [0, 0, n - 2, 5]
    cols[:4] = [n - 1, 1, n - 1, n - 1]
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    keep = lo < hi
    lo, hi = lo[keep], hi[keep]
    got = d[torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()].cpu().numpy().astype(np.float64)
    ref = R.rmsd_pairs(coords, lo, hi)
    g = _norms(coords)
    err = np.abs(got ** 2 - ref ** 2)
    bound = _bound(g, lo, hi, ref, m)
    assert np.all(err <= bound), float(np.max(err / bound))
    assert bool(torch.all(torch.diagonal(d) == 0))
    upper = torch.triu(d, 1)
    assert bool(torch.isfinite(upper).all())
    _say("full size: worst error / bound %.3g, max rmsd %.3f" % (np.max(err / bound), float(upper.max())))


def test_maximum_size_sampled(ctx, torch):
    """n = HAC_MAX_N = 65536 conformations (a 17 GB matrix, 2.1 M
    workgroups) of 32 atoms: sampled pairs including the last rows and
    columns against the oracle, and a sample of the diagonal."""
    import paper_1709_06816_amd as hac
    n, m = hac.MAX_N, 32
    coords = synth.conformations(n, m, seed=4242)
    _say("maximum size: producing")
    t = torch.from_numpy(coords).cuda()
    d = ctx.rmsd(t)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    lo = rng.integers(0, n - 1, size=1500)
    hi = rng.integers(0, n, size=1500)
    lo[:3] = [0, n - 2, 65535 - 16]
    hi[:3] = [n - 1, n - 1, n - 1]
    keep = lo < hi
    lo, hi = lo[keep], hi[keep]
    got = d[torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()].cpu().numpy().astype(np.float64)
    ref = R.rmsd_pairs(coords, lo, hi)
    err = np.abs(got ** 2 - ref ** 2)
    bound = _bound(_norms(coords), lo, hi, ref, m)
    assert np.all(err <= bound), float(np.max(err / bound))
    diag = torch.from_numpy(rng.integers(0, n, size=200)).cuda()
    assert bool(torch.all(d[diag, diag] == 0))
    del d, t
    torch.cuda.empty_cache()
