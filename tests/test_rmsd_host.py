"""The RMSD producer's per-pair epilogue (paper_1709_06816_amd/csrc/hac_qcp.h:
largest eigenvalue of the quaternion key matrix by Newton's method on its
characteristic polynomial), built for the host and checked against the
Kabsch oracle (oracle/rmsd.py, singular values) on the same fp64
cross-covariances, including degenerate conformations (collinear, planar,
identical, two atoms, one atom) whose largest root is multiple."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import rmsd as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cases():
    """(A, B, degenerate): degenerate pairs have a multiple largest root."""
    rng = np.random.default_rng(17)
    out = []
    c = synth.conformations(30, 57, seed=21)
    for i in range(30):
        out.append((c[i], c[(i + 1) % 30], False))
        out.append((c[i], c[i], False))  # identical
    line = np.outer(np.arange(7.0), [1.0, -2.0, 0.5])
    out.append((line, line * 1.7, True))                # collinear
    out.append((line, line[::-1].copy(), True))
    pl = rng.standard_normal((9, 3))
    pl[:, 2] = 0
    out.append((pl, pl * np.array([1, 1, -1.0]), True))  # planar mirror
    out.append((pl, rng.standard_normal((9, 3)), True))
    for _ in range(10):
        out.append((rng.standard_normal((2, 3)), rng.standard_normal((2, 3)), True))  # two atoms
    out.append((rng.standard_normal((1, 3)), rng.standard_normal((1, 3)), True))      # one atom
    chiral = np.array([[0.0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3]])
    out.append((chiral, chiral * np.array([1, 1, -1.0]), False))
    for _ in range(40):
        m = int(rng.integers(3, 40))
        a = rng.standard_normal((m, 3)) * 5
        out.append((a, a @ np.linalg.qr(rng.standard_normal((3, 3)))[0].T + 1e-3 * rng.standard_normal((m, 3)),
                    False))
    return out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_qcp_epilogue_matches_kabsch(tmp_path):
    exe = str(tmp_path / "qcp_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I",
                    os.path.join(ROOT, "paper_1709_06816_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "qcp_check.cpp"), "-o", exe], check=True)
    lines, want, scale, tol, lam = [], [], [], [], []
    for a, b, degenerate in _cases():
        a = np.asarray(a, np.float64) - np.mean(a, axis=0)
        b = np.asarray(b, np.float64) - np.mean(b, axis=0)
        m9 = (a.T @ b).ravel()
        ga, gb = (a * a).sum(), (b * b).sum()
        lines.append("%d %.17g %.17g %s" % (len(a), ga, gb, " ".join("%.17g" % v for v in m9)))
        want.append(R.rmsd(a, b))
        scale.append((ga + gb) / len(a))
        tol.append(1e-6 if degenerate else 1e-9)
        sv = np.linalg.svd(a.T @ b, compute_uv=False)
        lam.append(sv[0] + sv[1] + np.sign(np.linalg.det(a.T @ b)) * sv[2])
    res = subprocess.run([exe], input="\n".join(lines) + "\n", stdout=subprocess.PIPE, text=True, check=True)
    got = np.array([[float(v) for v in l.split()] for l in res.stdout.strip().split("\n")])
    assert len(got) == len(want)
    r = got[:, 1]
    want = np.array(want)
    scale = np.array(scale)
    # RMSD^2 agrees to 1e-9 of the conformations' mean squared radius, plus
    # the fp32 rounding of the result.  Where the largest root is multiple
    # (two atoms, collinear or planar conformations) the quartic's value near
    # the root is rounding noise below a distance of about sqrt(eps) = 1.5e-8
    # relative, so those pairs get 1e-6; fp32 cross-covariances already carry
    # errors of order 1e-6 relative on the device.
    err = np.abs(r.astype(np.float64) ** 2 - want ** 2)
    bound = np.array(tol) * scale + 2.0 ** -22 * want ** 2
    assert np.all(err <= bound), np.max(err / np.maximum(scale, 1e-300))
    # lambda_max itself (fp64, before the fp32 result) on the generic pairs
    generic = np.array(tol) == 1e-9
    norm = np.maximum(scale * np.array([len(a) for a, _, _ in _cases()]), 1e-300)
    lam_err = np.abs(got[:, 0] - np.array(lam)) / norm
    assert np.max(lam_err[generic]) < 1e-12
