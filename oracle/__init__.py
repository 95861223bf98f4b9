"""ctypes binding of the MRQ CPU oracle — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  The product library (``paper_2411_06158_amd``) never does: the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mrq_oracle.c")
LIB = os.path.join(HERE, "libmrq_oracle.so")

EXACT_IVF = 0
ALG2 = 1


def build(force: bool = True) -> str:
    """Compile the oracle: plain C99, -O2, no fused multiply-add contraction, no fast-math."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-o", tmp, SRC,
                               "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("eps0", C.c_double), ("m", C.c_double), ("bq", C.c_int32), ("stage2", C.c_int32),
                ("use_ext", C.c_int32), ("verify", C.c_int32)]


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in
                ("scanned", "pass1", "pass_ext", "pass2", "viol1", "viol_ext", "viol2")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.POINTER(C.c_uint64)]
        L.orc_gaussian.argtypes = [C.c_uint64, C.c_int64, P]
        L.orc_eigh.argtypes = [P, C.c_int, P, P]
        L.orc_haar.argtypes = [C.c_int, C.c_uint64, P]
        L.orc_encode_sign.argtypes = [P, C.c_int, P, P]
        L.orc_encode_ext.restype = C.c_double
        L.orc_encode_ext.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_ext_exhaustive.restype = C.c_double
        L.orc_ext_exhaustive.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_quantize_query_f32.argtypes = [P, C.c_int, C.c_int, P, P, P, P]
        L.orc_kmeans.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_uint64, C.c_int, P, P]
        L.orc_build.restype = P
        L.orc_build.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                C.c_int32]
        L.orc_import.restype = P
        L.orc_import.argtypes = [C.c_char_p, P, C.c_int64, C.c_int32]
        L.orc_attach.argtypes = [P, P, C.c_int64, C.c_int32]
        L.orc_free.argtypes = [P]
        L.orc_info.argtypes = [P, P, P, P, P, P]
        L.orc_get.argtypes = [P, C.c_char_p, P]
        L.orc_probe.argtypes = [P, P, C.c_int32, P, P]
        L.orc_search.argtypes = [P, P, C.c_int32, C.c_int32, C.POINTER(Params), C.c_int32, P, P,
                                 C.POINTER(Counters)]
        L.orc_pair_trace.argtypes = [P, P, C.c_int32, C.POINTER(Params), P, P, P, P, P]
        L.orc_topk_risk.argtypes = [P, P, C.c_int32, C.c_int32, C.POINTER(Params), C.c_double, P, P,
                                    P]
        L.orc_bruteforce.argtypes = [P, C.c_int64, C.c_int32, P, C.c_int64, C.c_int32, P, P]
        L.orc_sq8_range.argtypes = [P, C.c_int64, C.c_int, C.c_int, P, P]
        L.orc_sq8_encode.argtypes = [P, C.c_int, P, P, P]
        L.orc_sq8_build.argtypes = [P]
        L.orc_mrsq_estimates.argtypes = [P, P, C.c_int32, P, P, P]
        L.orc_mrsq_search.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def params(eps0=1.9, m=3.0, bq=4, stage2=True, use_ext=True, verify=False) -> Params:
    return Params(float(eps0), float(m), int(bq), int(bool(stage2)), int(bool(use_ext)),
                  int(bool(verify)))


# ---- building blocks --------------------------------------------------------------------------

def splitmix64_stream(seed: int, n: int) -> np.ndarray:
    s = C.c_uint64(seed)
    return np.array([lib().orc_splitmix64(C.byref(s)) for _ in range(n)], dtype=np.uint64)


def gaussian(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().orc_gaussian(seed, n, _p(out))
    return out


def eigh(A: np.ndarray):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n))
    if lib().orc_eigh(_p(A), n, _p(w), _p(V)) != 0:
        raise MemoryError
    return w, V


def haar(d: int, seed: int) -> np.ndarray:
    P = np.empty((d, d))
    lib().orc_haar(d, seed, _p(P))
    return P


def encode_sign(xprime: np.ndarray):
    x = np.ascontiguousarray(xprime, dtype=np.float64)
    bits = np.empty(x.size, dtype=np.uint8)
    xi = C.c_double()
    lib().orc_encode_sign(_p(x), x.size, _p(bits), C.byref(xi))
    return bits, xi.value


def encode_ext(xprime: np.ndarray, B: int):
    x = np.ascontiguousarray(xprime, dtype=np.float64)
    u = np.empty(x.size, dtype=np.uint8)
    xi = lib().orc_encode_ext(_p(x), x.size, B, _p(u))
    return u, xi


def ext_exhaustive(xprime: np.ndarray, B: int):
    x = np.ascontiguousarray(xprime, dtype=np.float64)
    u = np.empty(x.size, dtype=np.uint8)
    c = lib().orc_ext_exhaustive(_p(x), x.size, B, _p(u))
    return u, c


def quantize_query_f32(qprime: np.ndarray, bq: int = 4):
    q = np.ascontiguousarray(qprime, dtype=np.float32)
    u = np.empty(q.size, dtype=np.uint8)
    vl, dl, su = C.c_float(), C.c_float(), C.c_int32()
    lib().orc_quantize_query_f32(_p(q), q.size, bq, _p(u), C.byref(vl), C.byref(dl), C.byref(su))
    return u, np.float32(vl.value), np.float32(dl.value), su.value


def kmeans(P: np.ndarray, k: int, seed: int, iters: int = 25):
    P = np.ascontiguousarray(P, dtype=np.float64)
    n, dim = P.shape
    Cc = np.empty((k, dim))
    a = np.empty(n, dtype=np.int32)
    if lib().orc_kmeans(_p(P), n, dim, k, seed, iters, _p(Cc), _p(a)) != 0:
        raise ValueError("k-means arguments")
    return Cc, a


def bruteforce(X: np.ndarray, Q: np.ndarray, k: int):
    X = np.ascontiguousarray(X, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    ids = np.empty((Q.shape[0], k), dtype=np.int64)
    dd = np.empty((Q.shape[0], k))
    lib().orc_bruteforce(_p(X), X.shape[0], X.shape[1], _p(Q), Q.shape[0], k, _p(ids), _p(dd))
    return ids, dd


def sq8_range(xd: np.ndarray):
    """MR-SQ grid (readings S1, S2): per-coordinate lo and delta of FP32 rows."""
    x = np.ascontiguousarray(xd, dtype=np.float32)
    lo = np.empty(x.shape[1], dtype=np.float32)
    dl = np.empty(x.shape[1], dtype=np.float32)
    lib().orc_sq8_range(_p(x), x.shape[0], x.shape[1], x.shape[1], _p(lo), _p(dl))
    return lo, dl


def sq8_encode(x: np.ndarray, lo: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """MR-SQ 8-bit codes (reading S2) of FP32 rows."""
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float32)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    delta = np.ascontiguousarray(delta, dtype=np.float32)
    u = np.empty(x.shape, dtype=np.uint8)
    for i in range(x.shape[0]):
        lib().orc_sq8_encode(_p(x[i]), x.shape[1], _p(lo), _p(delta), _p(u[i]))
    return u


# ---- index ------------------------------------------------------------------------------------

class Index:
    """An oracle index: built here (Algorithm 1 in FP64) or imported from a device-library export."""

    def __init__(self, handle, X):
        if not handle:
            raise ValueError("oracle index could not be built / imported")
        self._h = C.c_void_p(handle)
        self._X = X  # the oracle reads the caller's original vectors for exact distances
        N, D, d, B, L = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        lib().orc_info(self._h, C.byref(N), C.byref(D), C.byref(d), C.byref(B), C.byref(L))
        self.N, self.D, self.d, self.B, self.nlist = N.value, D.value, d.value, B.value, L.value

    @classmethod
    def build(cls, X, d, B, nlist, seed=4001, kmeans_iters=25):
        X = np.ascontiguousarray(X, dtype=np.float32)
        h = lib().orc_build(_p(X), X.shape[0], X.shape[1], d, B, nlist, seed, kmeans_iters)
        return cls(h, X)

    @classmethod
    def load_export(cls, path, X=None):
        """Import a device export; with X every per-vector quantity is re-derived in FP64."""
        if X is not None:
            X = np.ascontiguousarray(X, dtype=np.float32)
            h = lib().orc_import(path.encode(), _p(X), X.shape[0], X.shape[1])
        else:
            h = lib().orc_import(path.encode(), None, 0, 0)
        return cls(h, X)

    def attach(self, X):
        """Use the stored per-vector summaries of an export, with X for the exact distances."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        if lib().orc_attach(self._h, _p(X), X.shape[0], X.shape[1]) != 0:
            raise ValueError("shape of X does not match the index")
        self._X = X
        return self

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().orc_free(self._h)
                self._h = None
        except Exception:
            pass

    def get(self, name):
        shapes = {"mu": (self.D,), "Pp": (self.D, self.D), "lam": (self.D,), "Pr": (self.d, self.d),
                  "C": (self.nlist, self.d), "off": (self.nlist + 1,), "lid": (self.N,),
                  "code": (self.N, self.d), "xd": (self.N, self.d), "sq_lo": (self.d,),
                  "sq_delta": (self.d,), "sq_code": (self.N, self.d)}
        dtypes = {"off": np.int64, "lid": np.int64, "code": np.uint8, "sq_lo": np.float32,
                  "sq_delta": np.float32, "sq_code": np.uint8}
        shp = shapes.get(name, (self.N,))
        out = np.empty(shp, dtype=dtypes.get(name, np.float64))
        if lib().orc_get(self._h, name.encode(), _p(out)) != 0:
            raise KeyError(name)
        return out

    def probe(self, q, nprobe):
        q = np.ascontiguousarray(q, dtype=np.float32)
        lists = np.empty(nprobe, dtype=np.int32)
        g = np.empty(nprobe)
        if lib().orc_probe(self._h, _p(q), nprobe, _p(lists), _p(g)) != 0:
            raise ValueError("nprobe")
        return lists, g

    def search(self, q, k, nprobe, mode=ALG2, prm=None, counters=False):
        q = np.ascontiguousarray(q, dtype=np.float32)
        prm = prm or params()
        ids = np.empty(k, dtype=np.int64)
        dd = np.empty(k)
        cnt = Counters()
        n = lib().orc_search(self._h, _p(q), k, nprobe, C.byref(prm), mode, _p(ids), _p(dd),
                             C.byref(cnt) if counters else None)
        if n < 0:
            raise ValueError("search arguments")
        return (ids, dd, cnt.as_dict()) if counters else (ids, dd)

    def search_many(self, Q, k, nprobe, mode=ALG2, prm=None):
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        ids = np.empty((Q.shape[0], k), dtype=np.int64)
        dd = np.empty((Q.shape[0], k))
        for i in range(Q.shape[0]):
            ids[i], dd[i] = self.search(Q[i], k, nprobe, mode, prm)
        return ids, dd

    def pair_trace(self, q, list_id, prm=None):
        q = np.ascontiguousarray(q, dtype=np.float32)
        prm = prm or params()
        off = self.get("off")
        n = int(off[list_id + 1] - off[list_id])
        qs = np.empty(8)
        qp = np.empty(self.d)
        u = np.empty(self.d, dtype=np.uint8)
        ids = np.empty(max(n, 1), dtype=np.int64)
        cand = np.empty((max(n, 1), 10))
        r = lib().orc_pair_trace(self._h, _p(q), list_id, C.byref(prm), _p(qs), _p(qp), _p(u),
                                 _p(ids), _p(cand))
        if r < 0:
            raise ValueError("list id")
        keys = ["nq", "Tq", "er", "qn2", "vl", "delta", "su", "sigma"]
        cols = ["dis1", "eb1", "lb1", "disB", "ebB", "lbB", "diso", "dis", "ip", "pc"]
        return (dict(zip(keys, qs)), qp, u, ids[:n], {c: cand[:n, i] for i, c in enumerate(cols)})

    def build_sq8(self):
        """MR-SQ codes from this index's own leading coordinates (readings S1, S2)."""
        if lib().orc_sq8_build(self._h) != 0:
            raise MemoryError
        return self

    def mrsq_estimates(self, q, nprobe):
        """Reading S3 for every candidate of the probed lists: (ids, estimates, exact distances)."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        lists, _ = self.probe(q, nprobe)
        off = self.get("off")
        n = int(sum(off[j + 1] - off[j] for j in lists))
        ids = np.empty(max(n, 1), dtype=np.int64)
        est = np.empty(max(n, 1))
        ex = np.empty(max(n, 1))
        r = lib().orc_mrsq_estimates(self._h, _p(q), nprobe, _p(ids), _p(est), _p(ex))
        if r < 0:
            raise ValueError("no MR-SQ codes or bad nprobe")
        return ids[:r], est[:r], ex[:r]

    def search_mrsq(self, q, k, nprobe, R=500):
        """MR-SQ search of one query (reading S4): ids (-1 padded) and FP64 distances."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        ids = np.empty(k, dtype=np.int64)
        dd = np.empty(k)
        if lib().orc_mrsq_search(self._h, _p(q), k, nprobe, R, _p(ids), _p(dd)) < 0:
            raise ValueError("MR-SQ search arguments")
        return ids, dd

    def topk_risk(self, q, k, nprobe, prm=None, margin=0.0):
        q = np.ascontiguousarray(q, dtype=np.float32)
        prm = prm or params()
        ids = np.empty(k, dtype=np.int64)
        dd = np.empty(k)
        risk = np.empty(k, dtype=np.uint8)
        lib().orc_topk_risk(self._h, _p(q), k, nprobe, C.byref(prm), margin, _p(ids), _p(dd),
                            _p(risk))
        return ids, dd, risk
