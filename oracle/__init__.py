"""CPU oracle and checkers for Lance-Williams agglomerative clustering.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the GPU path; the only module both sides use is ``synth`` (seeded
inputs, no clustering arithmetic).

Contents
  run_f32 / run_f64   the plain O(n^3) loop of Section 4 (steps 1-4) with the
                      Table 1 coefficients, in C (lw_oracle.c)
  replay_f64          fp64 replay of a given merge list (heights, optimality)
  brute_force_check   linkage recomputed from raw member sets (definitions of
                      Section 2.1 / Table 1), for tiny n
  prim_mst_weights    Prim's MST (Section 2.1: single linkage can be solved by
                      an algorithm that mimics Prim's MST)
  threshold_partition_check, monotone_check, relabel helpers

Parity pins: every function here is pinned by tests under tests/ against
closed forms, brute force or textbook routines; see the test docstrings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lw_oracle.c")
LIB = os.path.join(HERE, "_lw_oracle.so")

# Table 1 rows; "weighted" is the Weighted Average row (WPGMA).
LINKAGES = {"single": 0, "complete": 1, "average": 2, "ward": 3, "weighted": 4, "centroid": 5}
MERGE_DTYPE = np.dtype([("i", "<i4"), ("j", "<i4"), ("h", "<f4"), ("size", "<i4")])
MERGE64_DTYPE = np.dtype([("i", "<i4"), ("j", "<i4"), ("h", "<f8"), ("size", "<i4")])

OK, EINVAL, EINPUT, ENOMEM, EINTERNAL = 0, -1, -2, -3, -4

_lock = threading.Lock()
_lib = None


def build(force: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile the C oracle with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-std=gnu11", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _bind(path):
    lib = ctypes.CDLL(path)
    i64, i32p, f32p, f64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), \
        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
    lib.lw_oracle_f32.argtypes = [f32p, i64, ctypes.c_int, i64, i32p, i32p, f32p,
                                  i32p, ctypes.c_int, ctypes.POINTER(i64)]
    lib.lw_oracle_f64.argtypes = [f64p, i64, ctypes.c_int, i64, i32p, i32p, f64p,
                                  i32p, ctypes.c_int, ctypes.POINTER(i64)]
    lib.lw_replay_f64.argtypes = [f32p, i64, ctypes.c_int, i64, i32p, i32p, f64p,
                                  f64p, i64, ctypes.c_int]
    for f in (lib.lw_oracle_f32, lib.lw_oracle_f64, lib.lw_replay_f64):
        f.restype = ctypes.c_int
    return lib


def _load(lib=None):
    """The compiled oracle (built on first use), or ``lib`` if given (a
    variant loaded with ``load_variant``)."""
    global _lib
    if lib is not None:
        return lib
    with _lock:
        if _lib is None:
            build()
            _lib = _bind(LIB)
    return _lib


def load_variant(path: str):
    """Load another build of lw_oracle.c (e.g. one with a planted mistake, for
    the tests that check that the pins catch mistakes)."""
    return _bind(path)


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle returned %d" % code)
        self.code = code


def _link(linkage) -> int:
    return LINKAGES[linkage] if isinstance(linkage, str) else int(linkage)


def run_f32(dist: np.ndarray, linkage, max_merges: int = -1, threads: int | None = None,
            lib=None):
    """fp32 Lance-Williams clustering.  Returns a structured array of
    MERGE_DTYPE records (i, j, height, size), one per merge."""
    d = np.ascontiguousarray(dist, dtype=np.float32)
    n = d.shape[0]
    assert d.shape == (n, n)
    cnt = max(n - 1, 0) if max_merges < 0 else min(max_merges, max(n - 1, 0))
    mi = np.zeros(max(cnt, 1), np.int32); mj = np.zeros_like(mi)
    mh = np.zeros(max(cnt, 1), np.float32); ms = np.zeros_like(mi)
    done = ctypes.c_int64(0)
    rc = _load(lib).lw_oracle_f32(_ptr(d, ctypes.c_float), n, _link(linkage), max_merges,
                                  _ptr(mi, ctypes.c_int32), _ptr(mj, ctypes.c_int32),
                                  _ptr(mh, ctypes.c_float), _ptr(ms, ctypes.c_int32),
                                  threads or default_threads(), ctypes.byref(done))
    if rc != OK:
        raise OracleError(rc)
    out = np.zeros(done.value, MERGE_DTYPE)
    out["i"], out["j"], out["h"], out["size"] = mi[:done.value], mj[:done.value], \
        mh[:done.value], ms[:done.value]
    return out


def run_f64(dist: np.ndarray, linkage, max_merges: int = -1, threads: int | None = None,
            lib=None):
    """fp64 Lance-Williams clustering (same loop, no fp32 rounding)."""
    d = np.ascontiguousarray(dist, dtype=np.float64)
    n = d.shape[0]
    cnt = max(n - 1, 0) if max_merges < 0 else min(max_merges, max(n - 1, 0))
    mi = np.zeros(max(cnt, 1), np.int32); mj = np.zeros_like(mi)
    mh = np.zeros(max(cnt, 1), np.float64); ms = np.zeros_like(mi)
    done = ctypes.c_int64(0)
    rc = _load(lib).lw_oracle_f64(_ptr(d, ctypes.c_double), n, _link(linkage), max_merges,
                                  _ptr(mi, ctypes.c_int32), _ptr(mj, ctypes.c_int32),
                                  _ptr(mh, ctypes.c_double), _ptr(ms, ctypes.c_int32),
                                  threads or default_threads(), ctypes.byref(done))
    if rc != OK:
        raise OracleError(rc)
    out = np.zeros(done.value, MERGE64_DTYPE)
    out["i"], out["j"], out["h"], out["size"] = mi[:done.value], mj[:done.value], \
        mh[:done.value], ms[:done.value]
    return out


def replay_f64(dist: np.ndarray, linkage, merges, opt_stride: int = 0,
               threads: int | None = None, lib=None):
    """Replay ``merges`` (fields i, j) in fp64.  Returns (h64, min64): the fp64
    distance of each listed pair when it is merged, and (every opt_stride-th
    merge, else NaN) the fp64 minimum over all live pairs at that moment."""
    d = np.ascontiguousarray(dist, dtype=np.float32)
    n = d.shape[0]
    mi = np.ascontiguousarray(merges["i"], dtype=np.int32)
    mj = np.ascontiguousarray(merges["j"], dtype=np.int32)
    cnt = len(mi)
    h64 = np.zeros(max(cnt, 1)); m64 = np.zeros(max(cnt, 1))
    rc = _load(lib).lw_replay_f64(_ptr(d, ctypes.c_float), n, _link(linkage), cnt,
                                  _ptr(mi, ctypes.c_int32), _ptr(mj, ctypes.c_int32),
                                  _ptr(h64, ctypes.c_double), _ptr(m64, ctypes.c_double),
                                  opt_stride, threads or default_threads())
    if rc != OK:
        raise OracleError(rc)
    return h64[:cnt], m64[:cnt]


# ---------------------------------------------------------------------------
# Checkers built from definitions rather than from the update formula
# ---------------------------------------------------------------------------

def linkage_from_members(d: np.ndarray, a, b, linkage) -> float:
    """Distance between clusters A and B from their raw members (fp64).

    single   : min over A x B (closest members, Section 2.1)
    complete : max over A x B (furthest members, Section 2.1)
    average  : mean over A x B (group average)
    ward     : 2|A||B|/(|A|+|B|) * (mean_{AxB} D - mean_{AxA} D / 2
               - mean_{BxB} D / 2), means over ordered pairs including the
               zero diagonal.  For squared Euclidean D this is the Ward
               merge cost 2|A||B|/(|A|+|B|) |c_A - c_B|^2.
    centroid : mean_{AxB} D - mean_{AxA} D / 2 - mean_{BxB} D / 2 (same
               means).  For squared Euclidean D this is |c_A - c_B|^2, the
               squared distance between the centroids (the centroid method
               named in Section 2.1); the Table 1 centroid row reproduces it
               for any symmetric D with zero diagonal.
    weighted : has no member-set form (it depends on the merge order) and is
               rejected here.
    """
    link = _link(linkage)
    ab = d[np.ix_(a, b)]
    if link == 0:
        return float(ab.min())
    if link == 1:
        return float(ab.max())
    if link == 2:
        return float(ab.mean())
    if link == 4:
        raise ValueError("weighted average has no member-set form")
    aa = d[np.ix_(a, a)]
    bb = d[np.ix_(b, b)]
    na, nb = len(a), len(b)
    f = ab.mean() - 0.5 * aa.mean() - 0.5 * bb.mean()
    if link == 5:
        return float(f)
    return 2.0 * na * nb / (na + nb) * f


def symmetric_from_upper(dist: np.ndarray) -> np.ndarray:
    """fp64 symmetric matrix from the strict upper triangle, zero diagonal."""
    u = np.triu(np.asarray(dist, dtype=np.float64), 1)
    return u + u.T


def brute_force_check(dist: np.ndarray, merges, linkage, rtol: float = 1e-5,
                      atol: float = 0.0, exact_ties: bool = False):
    """Walk ``merges`` keeping explicit member sets.  At every step verify
      * the listed height equals the linkage recomputed from members
        (within rtol * |value| + atol);
      * the listed pair minimises that linkage over all pairs of live
        clusters (within the same tolerance);
      * with ``exact_ties`` (single/complete, whose values are exact copies of
        input entries): the listed pair is the lexicographically smallest
        (slot a, slot b) among the pairs attaining the exact minimum;
      * slot i is the smallest member of the merged cluster, slot j the
        smallest member of the other, and size is |A| + |B|.
    Returns a list of error strings (empty = pass).  O(n^4): tiny n only."""
    d = symmetric_from_upper(dist)
    n = d.shape[0]
    members = {k: [k] for k in range(n)}
    errs = []
    for s, m in enumerate(merges):
        i, j, h, size = int(m["i"]), int(m["j"]), float(m["h"]), int(m["size"])
        if i not in members or j not in members or not i < j:
            errs.append("step %d: bad slots %d %d" % (s, i, j))
            break
        live = sorted(members)
        vals = {}
        for x in range(len(live)):
            for y in range(x + 1, len(live)):
                a, b = live[x], live[y]
                vals[(a, b)] = linkage_from_members(d, members[a], members[b], linkage)
        true_h = vals[(i, j)]
        scale = max(abs(true_h), 1e-30)
        if abs(h - true_h) > rtol * scale + atol:
            errs.append("step %d: height %r vs members %r" % (s, h, true_h))
        best = min(vals.values())
        if true_h > best + rtol * max(abs(best), 1e-30) + atol:
            errs.append("step %d: pair (%d,%d) at %r not minimal (%r)" % (s, i, j, true_h, best))
        if exact_ties:
            first = min(p for p, v in vals.items() if v == best)
            if first != (i, j):
                errs.append("step %d: tie-break chose (%d,%d), smallest is %r" % (s, i, j, first))
        if members[i][0] != i or min(members[j]) != j:
            errs.append("step %d: slot is not the smallest member" % s)
        if size != len(members[i]) + len(members[j]):
            errs.append("step %d: size %d" % (s, size))
        members[i] = sorted(members[i] + members[j])
        del members[j]
    return errs


def prim_mst_weights(dist: np.ndarray) -> np.ndarray:
    """Edge weights of a minimum spanning tree of the complete graph on the
    strict-upper-triangle distances (Prim's algorithm, O(n^2)), in the
    input's precision."""
    d = np.asarray(dist)
    u = np.triu(d, 1)
    full = u + u.T
    n = d.shape[0]
    if n <= 1:
        return np.zeros(0, dtype=d.dtype)
    in_tree = np.zeros(n, bool)
    in_tree[0] = True
    best = full[0].copy()
    best[0] = np.inf
    out = []
    for _ in range(n - 1):
        cand = np.where(in_tree, np.inf, best)
        v = int(np.argmin(cand))
        out.append(cand[v])
        in_tree[v] = True
        best = np.minimum(best, full[v])
    return np.array(out, dtype=d.dtype)


class _DSU:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        while self.p[x] != x:
            self.p[x] = self.p[self.p[x]]
            x = self.p[x]
        return x

    def union(self, a, b):
        a, b = self.find(a), self.find(b)
        if a != b:
            self.p[max(a, b)] = min(a, b)


def threshold_partition_check(dist: np.ndarray, merges) -> list:
    """Single linkage: for every distinct merge height t, the clusters after
    all merges with height <= t are the connected components of the graph
    {(a, b): D[a][b] <= t} (tie-independent).  Returns error strings."""
    d = np.asarray(dist)
    n = d.shape[0]
    iu, ju = np.triu_indices(n, 1)
    w = d[iu, ju]
    order = np.argsort(w, kind="stable")
    hs = np.asarray(merges["h"])
    errs = []
    dsu_m = _DSU(n)
    dsu_g = _DSU(n)
    e = 0
    s = 0
    while s < len(hs):
        t = hs[s]
        while s < len(hs) and hs[s] <= t:
            dsu_m.union(int(merges["i"][s]), int(merges["j"][s]))
            s += 1
        while e < len(order) and w[order[e]] <= t:
            dsu_g.union(int(iu[order[e]]), int(ju[order[e]]))
            e += 1
        a = [dsu_m.find(x) for x in range(n)]
        b = [dsu_g.find(x) for x in range(n)]
        if a != b:
            errs.append("threshold %r: partitions differ" % float(t))
            break
    return errs


def monotone_violations(merges, rel: float = 0.0) -> int:
    """Number of steps whose height is below the previous one by more than
    rel * |previous|."""
    h = np.asarray(merges["h"], dtype=np.float64)
    if len(h) < 2:
        return 0
    drop = h[:-1] - h[1:]
    return int(np.sum(drop > rel * np.abs(h[:-1])))


def members_after(merges, n: int):
    """Sorted member tuples of every merge (A u B), with heights: a
    label-free description of the dendrogram."""
    members = {k: (k,) for k in range(n)}
    out = []
    for m in merges:
        i, j = int(m["i"]), int(m["j"])
        u = tuple(sorted(members[i] + members[j]))
        out.append((u, float(m["h"])))
        members[i] = u
        del members[j]
    return out
