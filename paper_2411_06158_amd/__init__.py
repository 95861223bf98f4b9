"""MRQ approximate k-NN search on MI355X (gfx950): ctypes binding of libmrq.so.

The binding only marshals arguments: every step of index build and search runs in the library's
HIP kernels.  Arrays may be numpy arrays (host) or torch tensors on the GPU (device); torch streams
are passed through as hipStream_t.  The entry points keep the C names of include/mrq.h.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrq.so")

MRQ_OK, MRQ_EINVAL, MRQ_ENOMEM, MRQ_EDEVICE, MRQ_ESTATE, MRQ_EIO = range(6)
MRQ_BATCHED, MRQ_PER_QUERY = 0, 1
MRQ_METHOD_MRQ, MRQ_METHOD_MRSQ = 0, 1

EXPORTED = [
    "mrq_build_opts_default", "mrq_search_opts_default", "mrq_build", "mrq_search", "mrq_search_mixed",
    "mrq_index_info", "mrq_export", "mrq_save", "mrq_load", "mrq_free", "mrq_last_error", "mrq_timing",
    "mrq_timing_enable", "mrq_server_create", "mrq_server_submit", "mrq_server_poll", "mrq_server_drain",
    "mrq_server_destroy", "mrq_choose_dr", "mrq_tune", "mrq_search_noalloc", "mrq_search_trace",
    "mrq_stream_copy", "mrq_search_mixed_dev", "mrq_server_stats",
]
NOALLOC_BYTES = 128 << 20  # MRQ_NOALLOC_BYTES

# mrq_search_trace records (include/mrq.h)
TRACE_STAGE1, TRACE_EXT, TRACE_STAGE2, TRACE_EXACT = 1, 2, 3, 4
TRACE_PAIR_DTYPE = np.dtype([("phase", "<i4"), ("q", "<i4"), ("list", "<i4"), ("su", "<i4"), ("nq", "<f4"),
                             ("vl", "<f4"), ("delta", "<f4"), ("kr", "<f4"), ("ebc", "<f4"), ("er", "<f4"),
                             ("qn2", "<f4"), ("pad", "<f4")])
TRACE_CAND_DTYPE = np.dtype([("kind", "<i4"), ("phase", "<i4"), ("q", "<i4"), ("list", "<i4"), ("id", "<i8"),
                             ("ip", "<i4"), ("pc", "<i4"), ("v0", "<f4"), ("v1", "<f4"), ("v2", "<f4"),
                             ("v3", "<f4")])
assert TRACE_PAIR_DTYPE.itemsize == 48 and TRACE_CAND_DTYPE.itemsize == 48


class MRQError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mrq status {status}: {msg}")
        self.status = status


class BuildOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("kmeans_iters", C.c_int32), ("sq8", C.c_int32), ("reserved", C.c_int32 * 6)]


class SearchOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("bq", C.c_int32), ("eps0", C.c_float), ("m", C.c_float),
                ("stage2", C.c_int32), ("use_ext", C.c_int32), ("counters", C.c_void_p),
                ("group", C.c_int32), ("exact_cap", C.c_int32), ("method", C.c_int32), ("rerank", C.c_int32),
                ("phase_growth", C.c_int32), ("ncounters", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libmrq.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2411_06158_amd.build_lib.build()")
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.mrq_build_opts_default.argtypes = [C.POINTER(BuildOpts)]
        L.mrq_search_opts_default.argtypes = [C.POINTER(SearchOpts)]
        L.mrq_build.argtypes = [P, I64, I32, I32, I32, I32, C.POINTER(BuildOpts), P, C.POINTER(P)]
        L.mrq_search.argtypes = [P, P, I64, I32, I32, P, P, C.POINTER(SearchOpts), P]
        L.mrq_search_mixed.argtypes = [P, P, I64, P, P, P, P, P, C.POINTER(SearchOpts), P]
        L.mrq_search_noalloc.argtypes = [P, P, I64, I32, I32, P, P, C.POINTER(SearchOpts), P]
        L.mrq_stream_copy.argtypes = [P, P, C.c_size_t, P]
        L.mrq_search_mixed_dev.argtypes = [P, P, I64, P, P, P, I32, I32, P, P, P, C.POINTER(SearchOpts), P]
        L.mrq_search_trace.argtypes = [P, P, I64, I32, I32, C.POINTER(SearchOpts), P, I32, P, P, P, P, P, I64, P,
                                       P, I64, P]
        L.mrq_index_info.argtypes = [P, P, P, P, P, P, P]
        L.mrq_export.argtypes = [P, C.c_char_p]
        L.mrq_save.argtypes = [P, C.c_char_p]
        L.mrq_load.argtypes = [C.c_char_p, C.POINTER(P)]
        L.mrq_free.argtypes = [P]
        L.mrq_free.restype = None
        L.mrq_last_error.restype = C.c_char_p
        L.mrq_timing.argtypes = [P, C.c_char_p, C.c_size_t, P, P, C.c_int]
        L.mrq_timing.restype = C.c_int
        L.mrq_timing_enable.argtypes = [P, C.c_int, C.c_int]
        if hasattr(L, "mrq_server_create"):
            L.mrq_server_create.argtypes = [P, C.c_size_t, I32, C.POINTER(SearchOpts), C.POINTER(P)]
            L.mrq_server_submit.argtypes = [P, C.c_uint64, P, I32, I32]
            L.mrq_server_poll.argtypes = [P, P, P, P, P, I32, I32, P]
            L.mrq_server_poll.restype = C.c_int
            L.mrq_server_drain.argtypes = [P, I64]
            L.mrq_server_destroy.argtypes = [P]
            L.mrq_server_destroy.restype = None
            L.mrq_server_stats.argtypes = [P, P, P, P, P]
        L.mrq_choose_dr.argtypes = [P, I32]
        L.mrq_choose_dr.restype = I32
        L.mrq_tune.argtypes = [P, P, I64, I32, I32, P, P, P]
        _lib = L
    return _lib


def _check(status: int):
    if status != MRQ_OK:
        raise MRQError(status, lib().mrq_last_error().decode(errors="replace"))


def _ptr(a) -> int:
    """Raw pointer of a numpy array or a torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return a.data_ptr()
    raise TypeError(f"unsupported array type {type(a)}")


def _stream(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def search_opts(mode=MRQ_BATCHED, bq=4, eps0=1.9, m=3.0, stage2=True, use_ext=True, counters=None,
                group=0, exact_cap=0, method=MRQ_METHOD_MRQ, rerank=0, phase_growth=0) -> SearchOpts:
    """Search options; `counters` (int64 array / tensor) of 8 entries, or of 16 for the extended counters."""
    o = SearchOpts()
    lib().mrq_search_opts_default(C.byref(o))
    o.mode, o.bq, o.eps0, o.m = int(mode), int(bq), float(eps0), float(m)
    o.stage2, o.use_ext, o.group = int(bool(stage2)), int(bool(use_ext)), int(group)
    o.exact_cap = int(exact_cap)
    o.method, o.rerank, o.phase_growth = int(method), int(rerank), int(phase_growth)
    o.counters = _ptr(counters) if counters is not None else None
    o.ncounters = 16 if counters is not None and len(counters) >= 16 else 8
    return o


def stream_copy(dst, src, stream=None):
    """mrq_stream_copy of src into dst (device tensors of the same byte size)."""
    nb = src.numel() * src.element_size()
    _check(lib().mrq_stream_copy(_ptr(dst), _ptr(src), nb, _stream(stream)))


def choose_dr(lam) -> int:
    """Eq 8: the projection dimension for eigenvalues `lam` (descending)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    return int(lib().mrq_choose_dr(lam.ctypes.data, len(lam)))


class Index:
    """An MRQ index living in GPU memory (owned by the library)."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        N, D, d, B, L, nb = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().mrq_index_info(self._h, C.byref(N), C.byref(D), C.byref(d), C.byref(B), C.byref(L),
                                    C.byref(nb)))
        self.N, self.D, self.d, self.B, self.nlist, self.device_bytes = (
            N.value, D.value, d.value, B.value, L.value, nb.value)

    @classmethod
    def build(cls, X, d_r: int, bits: int, nlist: int, seed: int = 4001, kmeans_iters: int = 25,
              stream=None, sq8: bool = False) -> "Index":
        """sq8: also build the MR-SQ codes (search with method=MRQ_METHOD_MRSQ)."""
        o = BuildOpts()
        lib().mrq_build_opts_default(C.byref(o))
        o.seed, o.kmeans_iters, o.sq8 = seed, kmeans_iters, int(bool(sq8))
        h = C.c_void_p()
        N, D = int(X.shape[0]), int(X.shape[1])
        _check(lib().mrq_build(_ptr(X), N, D, d_r, bits, nlist, C.byref(o), _stream(stream), C.byref(h)))
        return cls(h)

    @classmethod
    def load(cls, path: str) -> "Index":
        h = C.c_void_p()
        _check(lib().mrq_load(path.encode(), C.byref(h)))
        return cls(h)

    def save(self, path: str):
        _check(lib().mrq_save(self._h, path.encode()))

    def export(self, path: str):
        _check(lib().mrq_export(self._h, path.encode()))

    def search(self, Q, k: int, nprobe: int, ids=None, dists=None, opts: Optional[SearchOpts] = None,
               stream=None, **kw):
        """Top-k ids (int64, -1 padded) and squared distances (float32, +inf padded) per query.

        Q, ids and dists are all numpy (host) or all torch CUDA tensors (device); with device
        tensors the call is asynchronous on `stream`."""
        nq = int(Q.shape[0])
        if ids is None or dists is None:
            if isinstance(Q, np.ndarray):
                ids = np.empty((nq, k), dtype=np.int64)
                dists = np.empty((nq, k), dtype=np.float32)
            else:
                import torch
                ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
                dists = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        o = opts if opts is not None else search_opts(**kw)
        _check(lib().mrq_search(self._h, _ptr(Q), nq, k, nprobe, _ptr(ids), _ptr(dists), C.byref(o),
                                _stream(stream)))
        return ids, dists

    def search_noalloc(self, Q, k: int, nprobe: int, ids, dists, opts: Optional[SearchOpts] = None, stream=None,
                       **kw):
        """mrq_search_noalloc: the search into caller-allocated device tensors ids (nq x k int64) and dists
        (nq x k float32), with the workspace in the library's fixed device buffer (no allocation)."""
        o = opts if opts is not None else search_opts(**kw)
        _check(lib().mrq_search_noalloc(self._h, _ptr(Q), int(Q.shape[0]), k, nprobe, _ptr(ids), _ptr(dists),
                                        C.byref(o), _stream(stream)))
        return ids, dists

    def search_trace(self, Q, k: int, nprobe: int, traced, max_pairs: int = 4096, max_cands: int = 1 << 20,
                     opts: Optional[SearchOpts] = None, **kw):
        """mrq_search_trace on host arrays: (ids, dists, pairs, qprime, levels, cands) with the per-stage
        records of the queries `traced` (indices into Q); raises if a buffer was too small."""
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        nq = Q.shape[0]
        tr = np.ascontiguousarray(traced, dtype=np.int32)
        ids = np.empty((nq, k), dtype=np.int64)
        dists = np.empty((nq, k), dtype=np.float32)
        pairs = np.empty(max_pairs, dtype=TRACE_PAIR_DTYPE)
        qp = np.empty((max_pairs, self.d), dtype=np.float32)
        lev = np.empty((max_pairs, self.d), dtype=np.uint8)
        cands = np.empty(max_cands, dtype=TRACE_CAND_DTYPE)
        npairs, ncands = C.c_int64(0), C.c_int64(0)
        o = opts if opts is not None else search_opts(**kw)
        _check(lib().mrq_search_trace(self._h, _ptr(Q), nq, k, nprobe, C.byref(o), _ptr(tr), len(tr), _ptr(ids),
                                      _ptr(dists), pairs.ctypes.data, _ptr(qp), _ptr(lev), max_pairs,
                                      C.byref(npairs), cands.ctypes.data, max_cands, C.byref(ncands)))
        if npairs.value > max_pairs or ncands.value > max_cands:
            raise MRQError(MRQ_ENOMEM, f"trace buffers too small ({npairs.value} pairs, {ncands.value} records)")
        n, m = npairs.value, ncands.value
        return ids, dists, pairs[:n], qp[:n], lev[:n], cands[:m]

    def search_mixed(self, Q, k, nprobe, opts: Optional[SearchOpts] = None, stream=None, **kw):
        """Per-query k[i] / nprobe[i]; returns (ids, dists, out_off) as flat host arrays."""
        k = np.ascontiguousarray(k, dtype=np.int32)
        nprobe = np.ascontiguousarray(nprobe, dtype=np.int32)
        off = np.zeros(len(k), dtype=np.int64)
        off[1:] = np.cumsum(k[:-1].astype(np.int64))
        tot = int(k.astype(np.int64).sum())
        ids = np.empty(tot, dtype=np.int64)
        dists = np.empty(tot, dtype=np.float32)
        o = opts if opts is not None else search_opts(**kw)
        _check(lib().mrq_search_mixed(self._h, _ptr(Q), len(k), _ptr(k), _ptr(nprobe), _ptr(off), _ptr(ids),
                                      _ptr(dists), C.byref(o), _stream(stream)))
        return ids, dists, off

    def search_mixed_dev(self, Q, k, nprobe, k_max: int, nprobe_max: int, ids, dists, out_off=None,
                         rejected=None, opts: Optional[SearchOpts] = None, stream=None, **kw):
        """mrq_search_mixed_dev: per-query k / nprobe as device int32 tensors (bounded by k_max / nprobe_max),
        results into device tensors ids / dists at out_off (device int64, or None: packed in query order);
        no host synchronisation (capturable)."""
        o = opts if opts is not None else search_opts(**kw)
        _check(lib().mrq_search_mixed_dev(self._h, _ptr(Q), int(Q.shape[0]), _ptr(k), _ptr(nprobe), _ptr(out_off),
                                          int(k_max), int(nprobe_max), _ptr(ids), _ptr(dists), _ptr(rejected),
                                          C.byref(o), _stream(stream)))
        return ids, dists

    def tune(self, Q, k: int, nprobe: int, stream=None):
        """Time the scan schedules (query group, phase growth) on queries Q and keep the fastest as this
        index's default; returns (group, phase_growth)."""
        g, p = C.c_int32(0), C.c_int32(0)
        _check(lib().mrq_tune(self._h, _ptr(Q), int(Q.shape[0]), k, nprobe, _stream(stream), C.byref(g),
                              C.byref(p)))
        return g.value, p.value

    def timing_enable(self, on: bool = True, reset: bool = True):
        _check(lib().mrq_timing_enable(self._h, int(on), int(reset)))

    def timing(self) -> dict:
        buf = C.create_string_buffer(4096)
        ms = (C.c_double * 64)()
        n = (C.c_int64 * 64)()
        cnt = lib().mrq_timing(self._h, buf, 4096, ms, n, 64)
        names = buf.value.decode().split("\n")[:cnt]
        return {nm: (ms[i], n[i]) for i, nm in enumerate(names)}

    def close(self):
        if getattr(self, "_h", None):
            lib().mrq_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
