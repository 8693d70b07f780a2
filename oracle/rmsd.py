"""CPU oracle for the RMSD matrix that feeds the clustering (test
infrastructure: only tests/, the package's smoke check and bench.py's CPU leg
use it; the product never imports it).

The paper's input is an n x n matrix of RMSDs between protein structures:
chains of one sequence in different conformations (Section 2.1's protein
example), computed by a parallel RMSD step before the clustering (Section
5.1).  The paper does not define RMSD further; the standard definition for
two conformations A, B of the same m atoms (atom i of A corresponds to atom i
of B) is the root mean square deviation after the best rigid superposition:

    RMSD(A, B) = min over rotations R (det R = +1) and translations t of
                 sqrt( (1/m) * sum_i |R a_i + t - b_i|^2 ).

Steps (Kabsch's solution of that minimum), all in fp64:
  1. centre both conformations on their centroids (the best t);
  2. H = sum_i a_i b_i^T, a 3 x 3 matrix (a library matmul);
  3. the best rotation attains s1 + s2 + d*s3 of tr(R H), with s1 >= s2 >= s3
     the singular values of H (a library SVD) and d the sign of det H
     (d = -1 would need a reflection, so the smallest term is subtracted);
  4. RMSD^2 = (|A|^2 + |B|^2 - 2 (s1 + s2 + d*s3)) / m, clamped at 0.
"""
from __future__ import annotations

import numpy as np


def _centred(coords: np.ndarray) -> np.ndarray:
    x = np.asarray(coords, dtype=np.float64)
    return x - x.mean(axis=-2, keepdims=True)


def _rmsd_from(a: np.ndarray, b: np.ndarray, ga: np.ndarray, gb: np.ndarray, m: int) -> np.ndarray:
    """Steps 2-4 for centred a (..., m, 3), b (..., m, 3) and their squared norms."""
    h = np.einsum("...ip,...iq->...pq", a, b)
    s = np.linalg.svd(h, compute_uv=False)
    d = np.sign(np.linalg.det(h))
    best = s[..., 0] + s[..., 1] + d * s[..., 2]
    r2 = (ga + gb - 2.0 * best) / m
    return np.sqrt(np.maximum(r2, 0.0))


def rmsd(a: np.ndarray, b: np.ndarray) -> float:
    """Superposed RMSD of two conformations (m, 3) of the same m atoms."""
    a = _centred(a)
    b = _centred(b)
    m = a.shape[0]
    return float(_rmsd_from(a, b, (a * a).sum(), (b * b).sum(), m))


def rmsd_matrix(coords: np.ndarray, block: int = 64) -> np.ndarray:
    """N x N fp64 matrix of superposed RMSDs of the conformations
    coords (N, m, 3); zero diagonal, symmetric.  Computed in row blocks so
    that memory stays at block * N * 9 doubles."""
    x = _centred(coords)
    n, m = x.shape[0], x.shape[1]
    g = (x * x).sum(axis=(1, 2))
    out = np.zeros((n, n))
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        a = x[r0:r1, None]
        b = x[None, :]
        out[r0:r1] = _rmsd_from(np.broadcast_to(a, (r1 - r0, n, m, 3)),
                                np.broadcast_to(b, (r1 - r0, n, m, 3)),
                                g[r0:r1, None], g[None, :], m)
    np.fill_diagonal(out, 0.0)
    return out


def rmsd_pairs(coords: np.ndarray, rows, cols) -> np.ndarray:
    """Superposed RMSDs of the listed pairs (rows[k], cols[k]), fp64: the
    sampled check at sizes where the whole matrix is too large."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    a = _centred(np.asarray(coords)[rows])
    b = _centred(np.asarray(coords)[cols])
    m = a.shape[1]
    return _rmsd_from(a, b, (a * a).sum(axis=(1, 2)), (b * b).sum(axis=(1, 2)), m)
