"""Pins for the RMSD oracle (oracle/rmsd.py), checked against what the
definition and the mathematics fix rather than against the oracle itself.

  rigid motions give zero                              test_rigid_motion_is_zero
  library Wahba/Kabsch solver (SciPy align_vectors)    test_matches_library_alignment
  direct minimisation over rotations                   test_matches_direct_minimisation
  two atoms: |d_A - d_B| / 2                           test_two_atoms_closed_form
  mirror images: chiral > 0, planar = 0                test_mirror_images
  metric: symmetry, zero diagonal, triangle inequality test_metric_properties
  one atom, permuted atoms, translated input           test_special_cases
  matrix and pair routines agree                       test_matrix_and_pairs_agree
  planted mistakes are caught                          test_planted_mistake_caught
"""
import os
import types

import numpy as np
import pytest

import synth
from oracle import rmsd as R


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _chain(rng, m):
    return np.cumsum(rng.standard_normal((m, 3)) * 2.0, axis=0)


def test_rigid_motion_is_zero():
    rng = np.random.default_rng(1)
    for m in (3, 10, 100):
        a = _chain(rng, m)
        b = a @ _rotation(rng).T + rng.uniform(-40, 40, size=3)
        scale = np.sqrt(((a - a.mean(0)) ** 2).sum() / m)
        assert R.rmsd(a, b) <= 1e-6 * scale  # sqrt of an fp64 cancellation


def test_matches_library_alignment():
    """SciPy's Rotation.align_vectors solves the same minimum (Wahba's
    problem with unit weights) on centred inputs: its root sum of squared
    distances / sqrt(m) is the RMSD."""
    from scipy.spatial.transform import Rotation
    c = synth.conformations(12, 37, seed=5)
    for i in range(12):
        for j in range(i + 1, 12):
            a = c[i].astype(np.float64)
            b = c[j].astype(np.float64)
            a = a - a.mean(0)
            b = b - b.mean(0)
            _, rssd = Rotation.align_vectors(a, b)
            want = rssd / np.sqrt(len(a))
            assert abs(R.rmsd(c[i], c[j]) - want) <= 1e-9 * want


def test_matches_direct_minimisation():
    """Minimise the definition's objective over unit quaternions from many
    starts (no SVD): the minimum equals the oracle's value, and no sampled
    rotation does better."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(2)
    for trial in range(4):
        m = 6
        a = _chain(rng, m)
        b = _chain(rng, m)
        ac = a - a.mean(0)
        bc = b - b.mean(0)

        def obj(q):
            w, x, y, z = q / np.linalg.norm(q)
            rot = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
            return ((ac @ rot.T - bc) ** 2).sum() / m

        best = min(minimize(obj, rng.standard_normal(4), method="Nelder-Mead",
                            options={"xatol": 1e-12, "fatol": 1e-14, "maxiter": 20000}).fun
                   for _ in range(12))
        want = R.rmsd(a, b) ** 2
        assert abs(best - want) <= 1e-7 * max(want, 1e-12)
        for _ in range(200):
            q = rng.standard_normal(4)
            assert obj(q) >= want - 1e-12 * max(want, 1.0)


def test_two_atoms_closed_form():
    """Two atoms: centred, each conformation is +-half its bond; the best
    rotation aligns the bonds, leaving |d_A - d_B| / 2 per atom."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        a = rng.standard_normal((2, 3)) * 3
        b = rng.standard_normal((2, 3)) * 3
        da = np.linalg.norm(a[0] - a[1])
        db = np.linalg.norm(b[0] - b[1])
        assert abs(R.rmsd(a, b) - abs(da - db) / 2) <= 1e-12 * (da + db)


def test_mirror_images():
    """Only proper rotations count: a chiral structure and its mirror image
    stay apart, a planar one coincides with its mirror image."""
    chiral = np.array([[0.0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3]])
    mirror = chiral * np.array([1.0, 1.0, -1.0])
    assert R.rmsd(chiral, mirror) > 0.1
    planar = np.array([[0.0, 0, 0], [1, 0, 0], [0, 2, 0], [3, 1, 0]])
    assert R.rmsd(planar, planar * np.array([1.0, 1.0, -1.0])) <= 1e-7


def test_metric_properties():
    c = synth.conformations(40, 25, seed=9)
    d = R.rmsd_matrix(c)
    assert np.array_equal(d, d.T) or np.allclose(d, d.T, rtol=1e-12, atol=1e-12)
    assert np.all(np.diag(d) == 0)
    assert np.all(d[np.triu_indices(40, 1)] > 0)
    lhs = d[:, None, :]
    rhs = d[:, :, None] + d[None, :, :]
    assert np.all(lhs <= rhs + 1e-9)


def test_special_cases():
    rng = np.random.default_rng(4)
    a = _chain(rng, 1)
    b = _chain(rng, 1) + 5
    assert R.rmsd(a, b) == 0.0  # one atom: the translation is free
    a = _chain(rng, 20)
    b = _chain(rng, 20)
    perm = rng.permutation(20)
    assert abs(R.rmsd(a[perm], b[perm]) - R.rmsd(a, b)) <= 1e-12 * R.rmsd(a, b)
    assert abs(R.rmsd(a + 7.0, b - 3.0) - R.rmsd(a, b)) <= 1e-12 * R.rmsd(a, b)


def test_matrix_and_pairs_agree():
    c = synth.conformations(70, 13, seed=6)
    d = R.rmsd_matrix(c, block=16)
    rows, cols = np.triu_indices(70, 1)
    assert np.allclose(R.rmsd_pairs(c, rows, cols), d[rows, cols], rtol=1e-12, atol=0)


MUTANTS = {
    "no_centring": ("return x - x.mean(axis=-2, keepdims=True)", "return x"),
    "reflection_allowed": ("best = s[..., 0] + s[..., 1] + d * s[..., 2]",
                           "best = s[..., 0] + s[..., 1] + s[..., 2]"),
    "cross_term_halved": ("r2 = (ga + gb - 2.0 * best) / m", "r2 = (ga + gb - best) / m"),
    "mean_over_m_minus_1": ("r2 = (ga + gb - 2.0 * best) / m", "r2 = (ga + gb - 2.0 * best) / (m - 1)"),
    "largest_value_dropped": ("best = s[..., 0] + s[..., 1] + d * s[..., 2]",
                              "best = s[..., 1] + s[..., 1] + d * s[..., 2]"),
}


def _variant(edit):
    path = os.path.join(os.path.dirname(R.__file__), "rmsd.py")
    with open(path) as f:
        src = f.read()
    if edit is not None:
        assert src.count(edit[0]) == 1
        src = src.replace(edit[0], edit[1])
    mod = types.ModuleType("rmsd_variant")
    exec(compile(src, "rmsd_variant", "exec"), mod.__dict__)
    return mod


def _pins_fail(mod) -> list:
    from scipy.spatial.transform import Rotation
    failed = []
    rng = np.random.default_rng(11)
    a = _chain(rng, 10)
    if mod.rmsd(a, a @ _rotation(rng).T + 9.0) > 1e-6:
        failed.append("rigid")
    c = synth.conformations(6, 17, seed=12)
    for i in range(1, 6):
        x = c[0].astype(np.float64) - c[0].mean(0)
        y = c[i].astype(np.float64) - c[i].mean(0)
        want = Rotation.align_vectors(x, y)[1] / np.sqrt(17)
        if abs(mod.rmsd(c[0], c[i]) - want) > 1e-9 * want:
            failed.append("library")
            break
    chiral = np.array([[0.0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3]])
    if not mod.rmsd(chiral, chiral * np.array([1.0, 1.0, -1.0])) > 0.1:
        failed.append("mirror")
    two = rng.standard_normal((2, 2, 3))
    da, db = (np.linalg.norm(t[0] - t[1]) for t in two)
    if abs(mod.rmsd(two[0], two[1]) - abs(da - db) / 2) > 1e-9:
        failed.append("two_atoms")
    return failed


def test_unmodified_passes_pins():
    assert _pins_fail(_variant(None)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_caught(name):
    assert _pins_fail(_variant(MUTANTS[name])), name
