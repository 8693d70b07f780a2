"""Lance-Williams agglomerative clustering on one MI355X (gfx950).

Thin ctypes binding over the C-ABI library ``libhac.so`` (include/hac.h).
Every step of the clustering runs in the library's HIP kernels; this module
only marshals arguments.  PyTorch supplies device memory and streams.

    import paper_1709_06816_amd as hac
    merges = hac.run(dist_cuda_tensor, "complete")      # (n-1,) records
    z = hac.to_linkage_matrix(merges, n)                 # SciPy-style matrix

A merge record is (i, j, height, size): slot i keeps the merged cluster, slot
j is retired, height is D_ij when merged and size the merged cluster's member
count (Section 4 steps 1-4; Section 5.3 step 6).
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

__all__ = ["HacError", "Context", "Server", "run", "batch", "to_linkage_matrix", "MERGE_DTYPE",
           "LINKAGES", "library_path", "load_library"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhac.so")

# hac_linkage values; "weighted" is Table 1's Weighted Average row.
LINKAGES = {"single": 0, "complete": 1, "average": 2, "ward": 3, "weighted": 4, "centroid": 5}
MERGE_DTYPE = np.dtype([("i", "<i4"), ("j", "<i4"), ("h", "<f4"), ("size", "<i4")])

HAC_OK, HAC_EINVAL, HAC_EINPUT, HAC_ENOMEM, HAC_EDEVICE, HAC_ENODEV, HAC_EBUSY, \
    HAC_ETIMEDOUT, HAC_EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7, -8
PRESERVE_INPUT = 1
OUT_DEVICE = 2
MODE_SCAN = 4
OPT_WORKGROUPS, OPT_SINGLE_WG_N, OPT_TIMEOUT_MS, OPT_EXCHANGE, OPT_PROFILE, OPT_BLOCK = 1, 2, 3, 4, 5, 6
OPT_AUTOTUNE, OPT_BATCH_BLOCK, OPT_BATCH_GROUP, OPT_GRAPH = 7, 8, 9, 10
OPT_DEFER = 11
OPT_ROUNDS = 12
OPT_INJECT_STALL = 13
OPT_LAZY_MIRROR = 14
OPT_BATCH_UPDATE = 15
MAX_N = 65536
MAX_BATCH_N = 8192
NOALLOC_MAX_N = 65536
NOALLOC_MAX_WORKGROUPS = 64
NOALLOC_SCRATCH_BYTES = 1057280

_STATUS_NAMES = {
    HAC_EINVAL: "HAC_EINVAL", HAC_EINPUT: "HAC_EINPUT", HAC_ENOMEM: "HAC_ENOMEM",
    HAC_EDEVICE: "HAC_EDEVICE", HAC_ENODEV: "HAC_ENODEV", HAC_EBUSY: "HAC_EBUSY",
    HAC_ETIMEDOUT: "HAC_ETIMEDOUT", HAC_EINTERNAL: "HAC_EINTERNAL",
}

# Symbols the library must export (one per declaration in include/hac.h).
EXPORTS = ("hac_create", "hac_destroy", "hac_run", "hac_run_noalloc", "hac_batch", "hac_rmsd", "hac_sync", "hac_last_error",
           "hac_set_option", "hac_get_stats", "hac_server_create", "hac_submit", "hac_poll",
           "hac_server_get_stats", "hac_server_last_error", "hac_server_destroy")


class HacError(RuntimeError):
    def __init__(self, code: int, message: str = ""):
        name = _STATUS_NAMES.get(code, str(code))
        super().__init__("%s%s" % (name, (": " + message) if message else ""))
        self.code = code


class _Stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("init_ms", ctypes.c_double),
                ("rescans", ctypes.c_int64), ("rescan_elems", ctypes.c_int64),
                ("update_elems", ctypes.c_int64), ("workgroups", ctypes.c_int32),
                ("block", ctypes.c_int32), ("phase_avg_ms", ctypes.c_double * 5),
                ("phase_max_ms", ctypes.c_double * 5), ("group", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("forced_rounds", ctypes.c_int64),
                ("deferred", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("handed_over", ctypes.c_int32), ("compactions", ctypes.c_int32),
                ("rounds_ms", ctypes.c_double), ("rounds_rescan_elems", ctypes.c_int64),
                ("rounds_update_elems", ctypes.c_int64), ("plan_source", ctypes.c_int32),
                ("plan_share", ctypes.c_int32), ("plan_update", ctypes.c_int32)]


PHASES = ("setup", "exchange", "update", "rescan", "candidates")


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("waiting", ctypes.c_int64), ("running", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("kernel_launches", ctypes.c_int64), ("workgroups", ctypes.c_int32),
                ("block", ctypes.c_int32)]


_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libhac.so.  Raises ImportError if it has not been built: there is
    no fallback implementation."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libhac.so is missing at %s: build it with "
                              "`python paper_1709_06816_amd/build.py`" % _LIB_PATH)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i32, u32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
        lib.hac_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        lib.hac_destroy.argtypes = [vp]
        lib.hac_run.argtypes = [vp, vp, i32, i32, vp, u32, vp]
        lib.hac_run_noalloc.argtypes = [vp, vp, i32, i32, vp, u32, vp]
        lib.hac_batch.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, u32, vp]
        lib.hac_rmsd.argtypes = [vp, vp, i32, i32, vp, u32, vp]
        lib.hac_sync.argtypes = [vp]
        lib.hac_last_error.argtypes = [vp]
        lib.hac_last_error.restype = ctypes.c_char_p
        lib.hac_set_option.argtypes = [vp, i32, i64]
        lib.hac_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        lib.hac_server_create.argtypes = [vp, ctypes.c_size_t, i32, i32, ctypes.POINTER(vp)]
        lib.hac_submit.argtypes = [vp, vp, i64, i32, i32, ctypes.POINTER(ctypes.c_uint64)]
        lib.hac_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(i32)]
        lib.hac_server_get_stats.argtypes = [vp, ctypes.POINTER(_ServerStats)]
        lib.hac_server_last_error.argtypes = [vp]
        lib.hac_server_last_error.restype = ctypes.c_char_p
        lib.hac_server_destroy.argtypes = [vp]
        for name in EXPORTS:
            if name not in ("hac_last_error", "hac_server_last_error"):
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
        return lib


def _link(linkage) -> int:
    if isinstance(linkage, str):
        return LINKAGES[linkage]
    return int(linkage)


def _dev_ptr(x) -> int:
    """Device address of a torch tensor (or an int address)."""
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError("expected a device tensor")
    if not x.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return x.data_ptr()


def _stream_of(stream):
    if stream is not None:
        return int(stream) if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


class Context:
    """One library context (hac_create/hac_destroy) on a HIP device."""

    def __init__(self, device: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        rc = self._lib.hac_create(int(device), ctypes.byref(h))
        if rc != HAC_OK:
            raise HacError(rc, "hac_create(%d)" % device)
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hac_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc != HAC_OK:
            msg = self._lib.hac_last_error(self._h)
            raise HacError(rc, msg.decode() if msg else "")

    def set_option(self, option: int, value: int):
        self._check(self._lib.hac_set_option(self._h, int(option), int(value)))

    def stats(self) -> dict:
        s = _Stats()
        self._check(self._lib.hac_get_stats(self._h, ctypes.byref(s)))
        out = {f: getattr(s, f) for f, _ in _Stats._fields_
               if f not in ("phase_avg_ms", "phase_max_ms")}
        out["phase_avg_ms"] = dict(zip(PHASES, list(s.phase_avg_ms)))
        out["phase_max_ms"] = dict(zip(PHASES, list(s.phase_max_ms)))
        return out

    def run(self, dist, linkage, preserve: bool = False, out=None, stream=None, scan: bool = False) -> np.ndarray:
        """Cluster one n x n fp32 device matrix.  Returns MERGE_DTYPE[n-1].

        With ``out`` given as a device buffer (torch uint8/int32 tensor of
        16*(n-1) bytes, or an int address) the records are written there, the
        call returns after enqueueing, and ``sync()`` reports the status."""
        n = int(dist.shape[0]) if not isinstance(dist, int) else None
        if n is None:
            raise ValueError("pass a tensor (use run_ptr for raw addresses)")
        if tuple(dist.shape) != (n, n):
            raise ValueError("dist must be square")
        import torch
        if dist.dtype != torch.float32:
            raise ValueError("dist must be float32")
        return self.run_ptr(_dev_ptr(dist), n, linkage, preserve=preserve, out=out, stream=stream, scan=scan)

    def run_ptr(self, dist_ptr: int, n: int, linkage, preserve: bool = False, out=None, scan: bool = False,
                stream=None):
        flags = (PRESERVE_INPUT if preserve else 0) | (MODE_SCAN if scan else 0)
        s = _stream_of(stream)
        if out is None:
            res = np.zeros(max(n - 1, 0), MERGE_DTYPE)
            optr = res.ctypes.data if n > 1 else None
        else:
            flags |= OUT_DEVICE
            res = None
            optr = _dev_ptr(out)
        self._check(self._lib.hac_run(self._h, ctypes.c_void_p(dist_ptr), int(n), _link(linkage),
                                      ctypes.c_void_p(optr) if optr else None, flags,
                                      ctypes.c_void_p(s) if s else None))
        return res

    def run_noalloc(self, dist_ptr: int, n: int, linkage, out_ptr: int, scan: bool = False, wait: bool = True,
                    stream=None):
        """hac_run_noalloc: cluster the n x n fp32 device matrix at
        ``dist_ptr`` (overwritten) into the n-1 records at device address
        ``out_ptr``, with the library's static scratch and no allocation.
        ``wait=False`` returns once enqueued (``sync()`` reports the status)."""
        flags = (MODE_SCAN if scan else 0) | (0 if wait else OUT_DEVICE)
        s = _stream_of(stream)
        self._check(self._lib.hac_run_noalloc(self._h, ctypes.c_void_p(_dev_ptr(dist_ptr)), int(n), _link(linkage),
                                              ctypes.c_void_p(_dev_ptr(out_ptr)), flags,
                                              ctypes.c_void_p(s) if s else None))

    def rmsd(self, coords, out=None, stream=None):
        """RMSD matrix of n conformations (hac_rmsd): ``coords`` a contiguous
        float32 device tensor (n, atoms, 3).  Returns ``out`` (a float32
        device tensor (n, n), allocated if not given) with the strict upper
        triangle and the diagonal written."""
        import torch
        if coords.dtype != torch.float32 or coords.dim() != 3 or coords.shape[2] != 3:
            raise ValueError("coords must be a float32 tensor (n, atoms, 3)")
        if not coords.is_contiguous():
            raise ValueError("coords must be contiguous")
        n, atoms = int(coords.shape[0]), int(coords.shape[1])
        if out is None:
            out = torch.empty((n, n), dtype=torch.float32, device=coords.device)
        elif tuple(out.shape) != (n, n) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor (n, n)")
        s = _stream_of(stream)
        self._check(self._lib.hac_rmsd(self._h, ctypes.c_void_p(_dev_ptr(coords)), n, atoms,
                                       ctypes.c_void_p(_dev_ptr(out)), 0, ctypes.c_void_p(s) if s else None))
        return out

    def batch(self, packed, offsets, ns, linkages, preserve: bool = False, out=None,
              stream=None) -> np.ndarray:
        """Cluster many instances packed in one device buffer in one launch.

        Instance k is the n_k x n_k matrix at element offsets[k] of ``packed``.
        Returns the concatenated records; instance k's n_k-1 records start at
        sum_{l<k} (n_l - 1)."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        ns = np.ascontiguousarray(ns, dtype=np.int32)
        links = np.ascontiguousarray([_link(l) for l in linkages], dtype=np.int32)
        count = len(ns)
        if not (len(offsets) == len(links) == count):
            raise ValueError("offsets, ns and linkages must have the same length")
        m = np.maximum(ns.astype(np.int64) - 1, 0)
        out_off = np.zeros(count, np.int64)
        if count > 1:
            out_off[1:] = np.cumsum(m)[:-1]
        total = int(m.sum())
        flags = PRESERVE_INPUT if preserve else 0
        s = _stream_of(stream)
        if out is None:
            res = np.zeros(max(total, 1), MERGE_DTYPE)
            optr = res.ctypes.data
        else:
            flags |= OUT_DEVICE
            res = None
            optr = _dev_ptr(out)
        self._check(self._lib.hac_batch(
            self._h, ctypes.c_void_p(_dev_ptr(packed)), offsets.ctypes.data, ns.ctypes.data,
            links.ctypes.data, count, ctypes.c_void_p(optr), out_off.ctypes.data, flags,
            ctypes.c_void_p(s) if s else None))
        return res[:total] if res is not None else None

    def sync(self):
        self._check(self._lib.hac_sync(self._h))


class Server:
    """Continuous-batching server (hac_server_create ... hac_server_destroy).

    ``submit`` takes a host float32 matrix (2-D, rows contiguous; a view of
    the top-left n x n block of a larger array is fine) and returns a ticket;
    the array is kept referenced until the job is returned by ``poll``.
    ``poll`` returns None while the job runs, else its MERGE_DTYPE[n-1]
    records (raising HacError if the job failed)."""

    def __init__(self, ctx: Context, budget_bytes: int, max_jobs: int = 1024, max_n: int = 16384):
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        rc = self._lib.hac_server_create(ctx._h, int(budget_bytes), int(max_jobs), int(max_n),
                                         ctypes.byref(h))
        if rc != HAC_OK:
            raise HacError(rc, "hac_server_create")
        self._h = h
        self._held = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hac_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, what):
        if rc != HAC_OK:
            msg = self._lib.hac_server_last_error(self._h)
            raise HacError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    def submit(self, dist, linkage) -> int:
        """Queue the top-left n x n block of ``dist`` (host float32, 2-D)."""
        a = dist
        if isinstance(a, np.ndarray):
            if a.dtype != np.float32 or a.ndim != 2 or a.shape[0] != a.shape[1] or a.strides[1] != 4:
                raise ValueError("expected a square float32 array with contiguous rows")
            n, ld, ptr = a.shape[0], a.strides[0] // 4, a.ctypes.data
        else:  # torch CPU tensor (e.g. a pinned one or a view of it)
            import torch
            if a.dtype != torch.float32 or a.dim() != 2 or a.shape[0] != a.shape[1] or a.stride(1) != 1 \
                    or a.is_cuda:
                raise ValueError("expected a square float32 host tensor with contiguous rows")
            n, ld, ptr = a.shape[0], a.stride(0), a.data_ptr()
        t = ctypes.c_uint64()
        self._check(self._lib.hac_submit(self._h, ctypes.c_void_p(ptr), int(ld), int(n), _link(linkage),
                                         ctypes.byref(t)), "hac_submit")
        self._held[t.value] = (a, int(n))
        return t.value

    def poll(self, ticket: int):
        a, n = self._held[ticket]
        out = np.zeros(max(n - 1, 1), MERGE_DTYPE)
        done = ctypes.c_int32(0)
        rc = self._lib.hac_poll(self._h, ctypes.c_uint64(ticket), out.ctypes.data, ctypes.byref(done))
        if done.value:
            del self._held[ticket]
        self._check(rc, "hac_poll")
        return out[:n - 1] if done.value else None

    def stats(self) -> dict:
        st = _ServerStats()
        self._check(self._lib.hac_server_get_stats(self._h, ctypes.byref(st)), "hac_server_get_stats")
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}


_default = None


def _ctx() -> Context:
    global _default
    if _default is None:
        import torch
        _default = Context(torch.cuda.current_device())
    return _default


def run(dist, linkage, preserve: bool = False) -> np.ndarray:
    """Cluster one device matrix with the default context."""
    return _ctx().run(dist, linkage, preserve=preserve)


def batch(packed, offsets, ns, linkages, preserve: bool = False) -> np.ndarray:
    return _ctx().batch(packed, offsets, ns, linkages, preserve=preserve)


def to_linkage_matrix(merges: np.ndarray, n: int) -> np.ndarray:
    """Convert merge records to a SciPy-style (n-1) x 4 linkage matrix: rows
    [id_a, id_b, height, size] where ids < n are items and id n+s is the
    cluster formed at merge s.  Pure bookkeeping on the returned records."""
    z = np.zeros((len(merges), 4), dtype=np.float64)
    cid = np.arange(n, dtype=np.int64)
    for s, m in enumerate(merges):
        a, b = int(cid[m["i"]]), int(cid[m["j"]])
        z[s] = (min(a, b), max(a, b), float(m["h"]), int(m["size"]))
        cid[m["i"]] = n + s
    return z
