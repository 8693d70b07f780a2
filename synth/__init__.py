"""Seeded synthetic inputs for the clustering hot path.

This module only draws points and turns them into distance matrices.  It holds
none of the clustering arithmetic, and both the CPU oracle (test side) and the
GPU library (product side) consume what it produces.

Every matrix is fp32, n x n, row-major, zero diagonal.  Only the strict upper
triangle is meaningful to the algorithm (Section 5.2: a distance matrix needs
only its upper or lower half); the lower triangle produced here is its exact
mirror and is ignored by every consumer.  The fp64 arithmetic that turns
points into distances runs in a small C helper (_gen.c) with every sum in a
fixed order, so a seeded matrix is the same bytes on every host.

Workload recipes follow the paper's setting (Section 6: complete linkage on
protein-structure RMSD matrices, average n about 1968) with synthetic
Gaussian-mixture points standing in for the protein data, which is not
available.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

BASE_SEED = 170906816

LINKAGES = ("single", "complete", "average", "ward")


_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "_gen.c")
_GEN_LIB = os.path.join(_HERE, "_gen.so")
_gen_lock = threading.Lock()
_gen = None


def build(force: bool = False) -> str:
    """Compile the fixed-order fp64 helper (_gen.c) with gcc."""
    if force or not os.path.exists(_GEN_LIB) or os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
        tmp = _GEN_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-std=gnu11", "-Wall", "-o", tmp, _GEN_SRC, "-lm"])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _lib():
    global _gen
    with _gen_lock:
        if _gen is None:
            build()
            lib = ctypes.CDLL(_GEN_LIB)
            dp, fp, lp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float), \
                ctypes.POINTER(ctypes.c_int64)
            lib.synth_euclid.argtypes = [dp, ctypes.c_int64, ctypes.c_int, fp, ctypes.c_double, ctypes.c_int]
            lib.synth_euclid.restype = ctypes.c_int
            lib.synth_orthonormal.argtypes = [dp, ctypes.c_int, dp]
            lib.synth_orthonormal.restype = ctypes.c_int
            lib.synth_rotate.argtypes = [dp, lp, ctypes.c_int64, ctypes.c_int, dp, dp, dp, dp]
            lib.synth_rotate.restype = None
            _gen = lib
    return _gen


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def gaussian_mixture(rng: np.random.Generator, n: int, dim: int, k: int,
                     sigma_lo: float = 1.0, sigma_hi: float = 1.0,
                     anisotropic: bool = False, box: float = 10.0) -> np.ndarray:
    """Draw n points in R^dim from a mixture of k Gaussians (float64).

    Centres ~ U[-box, box]^dim, labels uniform over clusters.  Isotropic
    clusters use one sigma per cluster ~ U[sigma_lo, sigma_hi]; anisotropic
    clusters use x = c + R diag(s) z with R a random orthogonal matrix (the
    Q factor, with positive diagonal of R, of a Gaussian matrix, by modified
    Gram-Schmidt in fixed order) and s_d ~ U[0.3, 3].
    """
    centres = rng.uniform(-box, box, size=(k, dim))
    labels = rng.integers(0, k, size=n)
    z = rng.standard_normal((n, dim))
    if not anisotropic:
        sig = rng.uniform(sigma_lo, sigma_hi, size=k)
        return centres[labels] + z * sig[labels, None]
    lib = _lib()
    pts = np.empty((n, dim))
    q = np.empty((dim, dim))
    for c in range(k):
        g = np.ascontiguousarray(rng.standard_normal((dim, dim)))
        if lib.synth_orthonormal(_p(g, ctypes.c_double), dim, _p(q, ctypes.c_double)) != 0:
            raise ValueError("singular Gaussian matrix")
        s = np.ascontiguousarray(rng.uniform(0.3, 3.0, size=dim))
        rows = np.ascontiguousarray(np.nonzero(labels == c)[0].astype(np.int64))
        cen = np.ascontiguousarray(centres[c])
        lib.synth_rotate(_p(z, ctypes.c_double), _p(rows, ctypes.c_int64), len(rows), dim,
                         _p(cen, ctypes.c_double), _p(s, ctypes.c_double), _p(q, ctypes.c_double),
                         _p(pts, ctypes.c_double))
    return pts


def euclidean_matrix(points: np.ndarray, scale_to: float | None = None,
                     round_decimals: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Full n x n fp32 Euclidean distance matrix of float64 points.

    Distances are sqrt(max(0, |x|^2 + |y|^2 - 2 x.y)) evaluated in float64
    with every sum taken in index order (so the matrix is bit-identical on
    any host), optionally rescaled so the largest distance equals
    ``scale_to`` and rounded (half to even) to ``round_decimals`` decimals,
    then rounded once to fp32.  The strict upper triangle is computed and
    mirrored; the diagonal is exactly zero.
    """
    x = np.ascontiguousarray(points, dtype=np.float64)
    n, dim = x.shape
    if out is None:
        out = np.empty((n, n), dtype=np.float32)
    assert out.shape == (n, n) and out.dtype == np.float32 and out.flags["C_CONTIGUOUS"]
    rc = _lib().synth_euclid(_p(x, ctypes.c_double), n, dim, _p(out, ctypes.c_float),
                             float(scale_to) if scale_to is not None else 0.0,
                             int(round_decimals) if round_decimals is not None else -1)
    if rc != 0:
        raise MemoryError("synth_euclid")
    return out


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def mixture_512(seed: int = BASE_SEED + 1) -> np.ndarray:
    """n=512 points in R^8, 8 isotropic clusters, sigma=1."""
    rng = np.random.default_rng(seed)
    return euclidean_matrix(gaussian_mixture(rng, 512, 8, 8))


def mixture_8192(seed: int = BASE_SEED + 2, n: int = 8192) -> np.ndarray:
    """n=8192 points in R^16, 32 clusters with sigma ~ U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    return euclidean_matrix(gaussian_mixture(rng, n, 16, 32, 0.5, 2.0))


def rmsd_like(seed: int = BASE_SEED + 3, n: int = 32768, out: np.ndarray | None = None) -> np.ndarray:
    """RMSD-like matrix: n points in R^30 from 64 anisotropic clusters,
    distances rescaled to [0, 20] and rounded to 1e-3 (many exact ties)."""
    rng = np.random.default_rng(seed)
    pts = gaussian_mixture(rng, n, 30, 64, anisotropic=True)
    return euclidean_matrix(pts, scale_to=20.0, round_decimals=3, out=out)


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int, size=None):
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


@dataclass
class BatchSpec:
    ns: np.ndarray          # int64[count]
    linkages: np.ndarray    # int32[count], 0..3
    seeds: np.ndarray       # int64[count]


def batch_spec(count: int = 1024, n_lo: int = 64, n_hi: int = 4096,
               seed: int = BASE_SEED + 4) -> BatchSpec:
    """Ragged batch: n log-uniform in [n_lo, n_hi], linkage uniform over 4."""
    rng = np.random.default_rng(seed)
    ns = np.minimum(log_uniform_int(rng, n_lo, n_hi, size=count), n_hi)
    links = rng.integers(0, 4, size=count).astype(np.int32)
    seeds = seed * 1000 + np.arange(count, dtype=np.int64)
    return BatchSpec(ns, links, seeds)


def batch_instance(n: int, seed: int) -> np.ndarray:
    """One batch instance: Gaussian mixture in R^16, K ~ U{2..32} clusters,
    sigma ~ U[0.5, 2]."""
    rng = np.random.default_rng(int(seed))
    k = int(rng.integers(2, 33))
    return euclidean_matrix(gaussian_mixture(rng, int(n), 16, k, 0.5, 2.0))


def pack_offsets(ns, align: int = 64):
    """Element offsets of n_k x n_k blocks packed back to back, each start
    aligned to ``align`` floats.  Returns (offsets int64[count], total)."""
    offs = np.empty(len(ns), dtype=np.int64)
    cur = 0
    for k, n in enumerate(ns):
        cur = (cur + align - 1) // align * align
        offs[k] = cur
        cur += int(n) * int(n)
    return offs, (cur + align - 1) // align * align


def merge_offsets(ns):
    """Merge-record offsets: instance k's n_k - 1 records start at
    sum_{l<k} (n_l - 1)."""
    ns = np.asarray(ns, dtype=np.int64)
    m = np.maximum(ns - 1, 0)
    offs = np.zeros(len(ns), dtype=np.int64)
    if len(ns) > 1:
        offs[1:] = np.cumsum(m)[:-1]
    return offs, int(m.sum())


@dataclass
class ServeTrace:
    arrivals: np.ndarray    # float64 seconds, increasing
    ns: np.ndarray
    linkages: np.ndarray
    seeds: np.ndarray


def serve_trace(count: int, rate: float = 200.0, n_lo: int = 256, n_hi: int = 16384,
                seed: int = BASE_SEED + 5) -> ServeTrace:
    """Poisson arrivals at ``rate`` per second; n log-uniform on [n_lo, n_hi];
    linkage uniform over the four."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    ns = np.minimum(log_uniform_int(rng, n_lo, n_hi, size=count), n_hi)
    links = rng.integers(0, 4, size=count).astype(np.int32)
    seeds = seed * 1000 + np.arange(count, dtype=np.int64)
    return ServeTrace(np.cumsum(gaps), ns, links, seeds)


def serve_pool(count: int = 2, n: int = 16384, seed: int = BASE_SEED + 5, out=None) -> list:
    """Matrices that serving requests are cut from: each is the distance
    matrix of n points of a Gaussian mixture in R^16 (K ~ U{2..32} centres,
    sigma ~ U[0.5, 2]), so its top-left m x m block is the matrix of m points
    drawn from that mixture.  ``out``: optional list of (n, n) float32
    arrays to fill (e.g. views of page-locked buffers)."""
    mats = []
    for p in range(count):
        rng = np.random.default_rng(seed * 1000 + 7919 + p)
        k = int(rng.integers(2, 33))
        pts = gaussian_mixture(rng, n, 16, k, 0.5, 2.0)
        mats.append(euclidean_matrix(pts, out=None if out is None else out[p]))
    return mats


def mixture_65536(seed: int = BASE_SEED + 6, n: int = 65536, out=None) -> np.ndarray:
    """n=65536 points in R^16, 64 clusters with sigma ~ U[0.5, 2] (16 GiB
    fp32 matrix; pass ``out`` to fill a preallocated (n, n) float32 array)."""
    rng = np.random.default_rng(seed)
    return euclidean_matrix(gaussian_mixture(rng, n, 16, 64, 0.5, 2.0), out=out)


# ---------------------------------------------------------------------------
# Small structured matrices for edge cases
# ---------------------------------------------------------------------------

def uniform_matrix(n: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Independent U[lo, hi) entries (not a metric), zero diagonal, symmetric."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(lo, hi, size=(n, n)).astype(np.float32)
    a = np.triu(a, 1)
    return a + a.T


def quantized_matrix(n: int, seed: int, levels: int = 7) -> np.ndarray:
    """Entries drawn from a handful of values: tie-heavy."""
    rng = np.random.default_rng(seed)
    a = rng.integers(1, levels + 1, size=(n, n)).astype(np.float32) * 0.5
    a = np.triu(a, 1)
    return a + a.T


def ultrametric_matrix(n: int, seed: int) -> np.ndarray:
    """Ultrametric from a random binary hierarchy with distinct levels:
    D[a][b] = level of the lowest common ancestor of leaves a and b."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    d = np.zeros((n, n), dtype=np.float64)
    levels = iter(np.sort(rng.uniform(1.0, 100.0, size=max(1, n - 1)))[::-1])

    def split(items):
        if len(items) <= 1:
            return
        cut = int(rng.integers(1, len(items)))
        left, right = items[:cut], items[cut:]
        lev = next(levels)
        d[np.ix_(left, right)] = lev
        d[np.ix_(right, left)] = lev
        split(left)
        split(right)

    split(list(perm))
    return d.astype(np.float32)


def conformations(count: int, atoms: int, seed: int = BASE_SEED + 7, states: int = 64) -> np.ndarray:
    """``count`` conformations of one chain of ``atoms`` atoms, as a
    (count, atoms, 3) fp32 array in angstrom: the shape of the paper's input
    before its RMSD step (chains of one sequence folded differently, Section
    2.1; RMSD computed in parallel, Section 5.1).

    Recipe: a base chain is a persistent random walk with 3.8 A steps (the
    C-alpha spacing of a protein backbone); ``states`` folding states each add
    a smooth displacement field to it (a sum of three random sinusoids along
    the chain, amplitude ~ U[1, 4] A); a conformation picks a state, adds
    isotropic noise sigma ~ U[0.2, 1.0] A per atom, and is placed by a random
    proper rotation and a translation ~ U[-50, 50]^3 A, so that the
    superposition matters.  Pure input generation: no RMSD arithmetic."""
    rng = np.random.default_rng(seed)
    step = rng.standard_normal((atoms, 3))
    for i in range(1, atoms):  # persistence: each step leans on the previous one
        step[i] = 0.6 * step[i - 1] + step[i]
    step *= 3.8 / np.maximum(np.linalg.norm(step, axis=1, keepdims=True), 1e-12)
    base = np.cumsum(step, axis=0)
    base -= base.mean(0)
    pos = np.arange(atoms, dtype=np.float64)[:, None]
    fields = np.zeros((states, atoms, 3))
    for c in range(states):
        amp = rng.uniform(1.0, 4.0)
        for _ in range(3):
            freq = rng.uniform(0.01, 0.2)
            phase = rng.uniform(0, 2 * np.pi, size=3)
            direc = rng.standard_normal(3)
            fields[c] += amp / 3.0 * np.sin(freq * pos + phase) * direc / np.linalg.norm(direc)
    label = rng.integers(0, states, size=count)
    sigma = rng.uniform(0.2, 1.0, size=count)
    out = np.empty((count, atoms, 3), np.float32)
    for k in range(count):
        x = base + fields[label[k]] + sigma[k] * rng.standard_normal((atoms, 3))
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        out[k] = (x @ q.T + rng.uniform(-50, 50, size=3)).astype(np.float32)
    return out
