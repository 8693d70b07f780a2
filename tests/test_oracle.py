"""Pins for the CPU oracle (oracle/), checked against what the paper and the
mathematics fix rather than against the oracle itself.

  hand-worked merge lists (Section 4 steps 1-4, Table 1)   test_hand_worked
  brute force over raw member sets (Section 2.1 defs)      test_brute_force_*
  Ward's member formula vs centroid closed form            test_ward_member_formula
  single linkage == Prim's MST (Section 2.1)               test_single_is_prim_mst
  threshold-graph components (single linkage)              test_single_threshold_components
  Prim vs a library MST                                     test_prim_matches_scipy
  monotone heights (reducible linkages)                     test_monotone_heights
  constant / ultrametric special cases                      test_constant_matrix, test_ultrametric
  relabeling invariance                                     test_relabel_invariance
  fp64 replay error bound and optimality                    test_fp64_replay_bounds
  library hierarchical clustering cross-check               test_scipy_cross_check
  input conventions (upper triangle, -0, non-finite)        test_input_*
  centroid: member formula vs |c_A - c_B|^2, brute force    test_centroid_*
  weighted average: exact fp32 special cases, library       test_weighted_*, test_scipy_cross_check
  centroid bound on extreme inputs                          test_centroid_extreme_inputs_finite
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import matrix_from_upper

HERE = os.path.dirname(os.path.abspath(__file__))
LINKS = ["single", "complete", "average", "ward"]
# Table 1 rows Weighted Average and Centroid.
EXTRA = ["weighted", "centroid"]
ALL = LINKS + EXTRA


def _golden():
    with open(os.path.join(HERE, "golden", "hand_worked.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
@pytest.mark.parametrize("link", ALL)
def test_hand_worked(case, link):
    d = matrix_from_upper(case["n"], case["upper"])
    got = oracle.run_f32(d, link)
    exp = case["expected"][link]
    assert len(got) == len(exp)
    for g, e in zip(got, exp):
        assert (int(g["i"]), int(g["j"]), int(g["size"])) == (e[0], e[1], e[3])
        assert g["h"] == np.float32(e[2]), (link, g, e)
    got64 = oracle.run_f64(d, link)
    for g, e in zip(got64, exp):
        assert (int(g["i"]), int(g["j"]), int(g["size"])) == (e[0], e[1], e[3])
        assert abs(g["h"] - e[2]) <= 1e-7 * abs(e[2])


def test_n1_no_merges():
    d = np.zeros((1, 1), np.float32)
    assert len(oracle.run_f32(d, "complete")) == 0
    assert len(oracle.run_f64(d, "ward")) == 0


def _small_inputs():
    out = []
    for seed in range(6):
        out.append(("uniform", seed, synth.uniform_matrix(9 + seed % 4, seed)))
        out.append(("quantized", seed, synth.quantized_matrix(10 + seed % 3, seed, levels=4)))
        rng = np.random.default_rng(seed)
        pts = synth.gaussian_mixture(rng, 11, 3, 3)
        out.append(("mixture", seed, synth.euclidean_matrix(pts)))
    return out


@pytest.mark.parametrize("link", LINKS + ["centroid"])
def test_brute_force_f32(link):
    """Every fp32 merge height equals the linkage recomputed from raw member
    sets; every chosen pair is minimal; single/complete ties resolve to the
    smallest (i, j)."""
    for kind, seed, d in _small_inputs():
        m = oracle.run_f32(d, link)
        # centroid values can cancel towards zero on non-Euclidean input:
        # the absolute slack scales with the input's magnitude
        atol = 1e-6 if link != "centroid" else 2e-6 * float(np.abs(d).max())
        errs = oracle.brute_force_check(d, m, link, rtol=2e-6, atol=atol,
                                        exact_ties=link in ("single", "complete"))
        assert not errs, (kind, seed, errs[:3])


@pytest.mark.parametrize("link", LINKS + ["centroid"])
def test_brute_force_f64(link):
    for kind, seed, d in _small_inputs():
        m = oracle.run_f64(d, link)
        errs = oracle.brute_force_check(d, m, link, rtol=1e-12, atol=1e-12,
                                        exact_ties=link in ("single", "complete"))
        assert not errs, (kind, seed, errs[:3])


def test_ward_member_formula():
    """The member-set Ward formula used by the brute-force checker equals the
    textbook merge cost 2|A||B|/(|A|+|B|) |c_A - c_B|^2 on squared Euclidean
    distances (closed form from centroids)."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal((9, 4))
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    for a, b in ([[0, 1, 2], [3, 4]], [[5], [6, 7, 8]], [[1], [2]]):
        ca, cb = x[a].mean(0), x[b].mean(0)
        want = 2.0 * len(a) * len(b) / (len(a) + len(b)) * ((ca - cb) ** 2).sum()
        got = oracle.linkage_from_members(d2, a, b, "ward")
        assert abs(got - want) <= 1e-12 * want


def test_centroid_member_formula():
    """The member-set centroid formula used by the brute-force checker equals
    the squared distance between the two clusters' centroids on squared
    Euclidean distances (closed form from the points)."""
    rng = np.random.default_rng(8)
    x = rng.standard_normal((9, 4))
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    for a, b in ([[0, 1, 2], [3, 4]], [[5], [6, 7, 8]], [[1], [2]]):
        want = ((x[a].mean(0) - x[b].mean(0)) ** 2).sum()
        got = oracle.linkage_from_members(d2, a, b, "centroid")
        assert abs(got - want) <= 1e-12 * want
    with pytest.raises(ValueError):
        oracle.linkage_from_members(d2, [0], [1], "weighted")


def test_centroid_heights_are_centroid_distances():
    """On squared Euclidean input every fp64 centroid height is the squared
    distance between the centroids of the two member sets, recomputed from
    the points (not from the matrix)."""
    rng = np.random.default_rng(31)
    x = synth.gaussian_mixture(rng, 120, 4, 5).astype(np.float64)
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    m = oracle.run_f64(d2, "centroid")
    members = {k: [k] for k in range(len(x))}
    for r in m:
        a, b = members[int(r["i"])], members[int(r["j"])]
        want = ((x[a].mean(0) - x[b].mean(0)) ** 2).sum()
        assert abs(r["h"] - want) <= 1e-10 * want + 1e-12
        members[int(r["i"])] = a + b
        del members[int(r["j"])]


def test_centroid_extreme_inputs_finite():
    """The merged pair holds the minimum, so a negative minimum never grows in
    magnitude and one merge adds at most a quarter of it to any entry: inputs
    at the accepted limit 2^100 of either sign stay finite in fp32."""
    rng = np.random.default_rng(5)
    n = 300
    d = (rng.choice([-1.0, 1.0], size=(n, n)) * 2.0 ** 100).astype(np.float32)
    m = oracle.run_f32(d, "centroid")
    assert len(m) == n - 1 and np.all(np.isfinite(m["h"]))
    assert np.all(np.abs(m["h"].astype(np.float64)) <= 2.0 ** 100 * (1 + (n - 1) / 4))


def test_single_is_prim_mst():
    """Single linkage heights, sorted, equal the sorted MST edge weights
    bit-for-bit (Section 2.1: single linkage mimics Prim's MST)."""
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        d = synth.euclidean_matrix(synth.gaussian_mixture(rng, 300, 5, 6))
        m = oracle.run_f32(d, "single")
        mst = oracle.prim_mst_weights(d)
        assert np.array_equal(np.sort(m["h"]), np.sort(mst))
    d = synth.quantized_matrix(200, 3, levels=5)
    m = oracle.run_f32(d, "single")
    assert np.array_equal(np.sort(m["h"]), np.sort(oracle.prim_mst_weights(d)))


def test_single_threshold_components():
    for d in (synth.quantized_matrix(120, 4, levels=6), synth.uniform_matrix(90, 5)):
        m = oracle.run_f32(d, "single")
        assert not oracle.threshold_partition_check(d, m)


def test_prim_matches_scipy():
    from scipy.sparse.csgraph import minimum_spanning_tree
    d = synth.uniform_matrix(150, 9, lo=0.5, hi=1.5).astype(np.float64)
    ref = minimum_spanning_tree(np.triu(d, 1)).toarray()
    assert np.allclose(np.sort(ref[ref > 0]), np.sort(oracle.prim_mst_weights(d)))


@pytest.mark.parametrize("link", LINKS + ["weighted"])
def test_monotone_heights(link):
    """For the five reducible linkages heights never decrease: exactly for
    single/complete and for weighted average (halving is exact and a rounded
    sum of two halves lies between them), up to 1e-6 relative for fp32
    average/Ward (fp32 coefficients need not sum to one)."""
    for seed in range(3):
        d = synth.mixture_8192(seed=seed, n=400)
        m = oracle.run_f32(d, link)
        rel = 0.0 if link in ("single", "complete", "weighted") else 1e-6
        assert oracle.monotone_violations(m, rel) == 0
        m64 = oracle.run_f64(d, link)
        assert oracle.monotone_violations(m64, 0.0 if link != "ward" else 1e-12) == 0


@pytest.mark.parametrize("link", ["single", "complete", "weighted"])
def test_constant_matrix(link):
    """All distances equal c: every step is a tie, the smallest (i, j) wins,
    so the list is (0, k, c, k+1) (weighted average: 0.5c + 0.5c is exactly c
    in fp32)."""
    n, c = 37, np.float32(2.5)
    d = np.full((n, n), c, np.float32)
    m = oracle.run_f32(d, link)
    assert np.array_equal(m["i"], np.zeros(n - 1))
    assert np.array_equal(m["j"], np.arange(1, n))
    assert np.all(m["h"] == c)
    assert np.array_equal(m["size"], np.arange(2, n + 1))


@pytest.mark.parametrize("link", ["average", "ward"])
def test_constant_matrix_f64(link):
    """In exact arithmetic average and Ward keep every distance at c
    (coefficients sum to 1 with beta*c included for Ward)."""
    n, c = 25, 3.0
    d = np.full((n, n), c)
    m = oracle.run_f64(d, link)
    assert np.allclose(m["h"], c, rtol=1e-13)
    assert np.array_equal(m["size"][-1:], [n])


@pytest.mark.parametrize("link", ["single", "complete", "average", "weighted"])
def test_ultrametric(link):
    """On an ultrametric, all cross distances between two clusters that are
    merged are equal, so single, complete, average and weighted average
    reproduce its levels: the sorted heights are the sorted distinct levels
    (weighted average exactly in fp32: the mean of two equal values)."""
    for seed in range(3):
        d = synth.ultrametric_matrix(40, seed)
        levels = np.unique(d[np.triu_indices(40, 1)])
        m = oracle.run_f32(d, link) if link != "average" else oracle.run_f64(d, link)
        assert len(levels) == 39
        tol = 0 if link != "average" else 1e-12
        assert np.allclose(np.sort(m["h"]), levels, rtol=tol, atol=0)


@pytest.mark.parametrize("link", ALL)
def test_relabel_invariance(link):
    """Permuting the items leaves the set of (member set, height) merges
    unchanged on tie-free input: every recipe is symmetric in i <-> j and uses
    commutative operations."""
    n = 60
    d = synth.uniform_matrix(n, 11, lo=1.0, hi=2.0)
    perm = np.random.default_rng(12).permutation(n)
    dp = d[np.ix_(perm, perm)]
    a = oracle.members_after(oracle.run_f32(d, link), n)
    b = oracle.members_after(oracle.run_f32(dp, link), n)
    b = [(tuple(sorted(perm[list(u)])), h) for u, h in b]
    assert sorted(a) == sorted(b)


@pytest.mark.parametrize("link", ALL)
def test_fp64_replay_bounds(link):
    """Replaying the fp32 list in fp64: heights within 1e-5 relative, and each
    chosen pair within 1e-5 relative of the fp64 minimum over live pairs."""
    for d in (synth.mixture_8192(seed=5, n=500), synth.rmsd_like(seed=6, n=400)):
        m = oracle.run_f32(d, link)
        h64, min64 = oracle.replay_f64(d, link, m, opt_stride=1)
        h32 = m["h"].astype(np.float64)
        assert np.all(np.abs(h32 - h64) <= 1e-5 * np.abs(h64) + 1e-30)
        assert np.all(h64 <= min64 + 1e-5 * np.abs(min64))


@pytest.mark.parametrize("link", ALL)
def test_scipy_cross_check(link):
    """Library hierarchical clustering on tie-free input: same heights.  For
    Ward and centroid, Table 1 applied to D o D gives the squared
    minimum-variance costs and squared centroid distances, so sqrt of our
    heights on D o D equals the library's heights (which it computes from
    Euclidean distances)."""
    from scipy.cluster.hierarchy import linkage as sp_linkage
    from scipy.spatial.distance import squareform
    n = 200
    rng = np.random.default_rng(21)
    x = rng.standard_normal((n, 6))
    d64 = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d64, 0)
    sq = link in ("ward", "centroid")
    if sq:
        ours = np.sqrt(oracle.run_f64(d64 * d64, link)["h"])
    else:
        ours = oracle.run_f64(d64, link)["h"]
    ref = sp_linkage(squareform(d64, checks=False), method=link)[:, 2]
    assert np.allclose(np.sort(ours), np.sort(ref), rtol=1e-10, atol=0)
    ours32 = oracle.run_f32(d64.astype(np.float32) if not sq
                            else (d64 * d64).astype(np.float32), link)["h"].astype(np.float64)
    if sq:
        ours32 = np.sqrt(ours32)
    assert np.allclose(np.sort(ours32), np.sort(ref), rtol=2e-5, atol=0)


def test_input_lower_triangle_ignored():
    d = synth.uniform_matrix(30, 2)
    junk = d.copy()
    il = np.tril_indices(30, 0)
    junk[il] = np.random.default_rng(0).uniform(-5, 5, size=len(il[0])).astype(np.float32)
    junk[5, 2] = np.nan
    junk[7, 1] = np.inf
    for link in LINKS:
        assert oracle.run_f32(d, link).tobytes() == oracle.run_f32(junk, link).tobytes()


def test_input_negative_zero():
    d = synth.quantized_matrix(20, 3)
    d[0, 5] = 0.0
    d[2, 9] = -0.0
    d[3, 4] = -0.0
    m = oracle.run_f32(d, "complete")
    assert not np.any(np.signbit(m["h"]) & (m["h"] == 0))
    d2 = d.copy()
    d2[2, 9] = 0.0
    d2[3, 4] = 0.0
    assert m.tobytes() == oracle.run_f32(d2, "complete").tobytes()
    assert (int(m[0]["i"]), int(m[0]["j"])) == (0, 5)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf, 2.0 ** 101, -(2.0 ** 101)])
def test_input_rejected(bad):
    d = synth.uniform_matrix(10, 1)
    d[3, 7] = bad
    with pytest.raises(oracle.OracleError) as e:
        oracle.run_f32(d, "average")
    assert e.value.code == oracle.EINPUT
    # the same value below the diagonal is ignored
    d = synth.uniform_matrix(10, 1)
    d[7, 3] = bad
    assert len(oracle.run_f32(d, "average")) == 9


def test_input_limits_accepted():
    d = synth.uniform_matrix(10, 1)
    d[0, 1] = 2.0 ** 100
    d[0, 2] = -(2.0 ** 100)
    assert len(oracle.run_f32(d, "ward")) == 9


def test_bad_arguments():
    with pytest.raises(oracle.OracleError):
        oracle.run_f32(np.zeros((3, 3), np.float32), 7)
    with pytest.raises(oracle.OracleError):
        oracle.run_f32(np.zeros((0, 0), np.float32), 0)


def test_max_merges_prefix():
    d = synth.uniform_matrix(50, 3)
    full = oracle.run_f32(d, "average")
    part = oracle.run_f32(d, "average", max_merges=17)
    assert part.tobytes() == full[:17].tobytes()


def test_thread_count_invariance():
    d = synth.quantized_matrix(150, 8, levels=3)
    a = oracle.run_f32(d, "ward", threads=1)
    b = oracle.run_f32(d, "ward", threads=7)
    assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("link", ALL)
def test_replay_reproduces_fp64_oracle(link):
    """The fp64 replay checker, fed the fp64 oracle's own merge list, must
    return exactly the oracle's heights, and every listed pair must be the
    fp64 minimum at its step (optimality with no slack)."""
    d = synth.rmsd_like(seed=8, n=300)
    m = oracle.run_f64(d.astype(np.float64), link)
    h64, min64 = oracle.replay_f64(d, link, m, opt_stride=1)
    assert np.array_equal(h64, m["h"])
    assert np.array_equal(h64, min64)


def test_replay_rejects_invalid_lists():
    d = synth.uniform_matrix(8, 2)
    m = oracle.run_f32(d, "single")
    bad = m.copy()
    bad[3]["j"] = bad[1]["j"]  # a slot retired twice
    with pytest.raises(oracle.OracleError):
        oracle.replay_f64(d, "single", bad)
