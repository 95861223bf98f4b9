"""Continuous-batching server on the GPU: every request's result equals the search of that query alone,
whatever mix it was batched with; admission by memory budget defers, never drops, requests."""
import ctypes as C
import time

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("no GPU", allow_module_level=True)

import torch  # noqa: E402

import paper_2411_06158_amd as mrq  # noqa: E402
from paper_2411_06158_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def env():
    print("\n[gpu] server: build N=20000 D=128 d=32 B=1 nlist=64", flush=True)
    X, Q, _ = synth.workload("small", N=20000, nq=240, cache=False)
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=32, bits=1, nlist=64)
    return dict(X=X, Q=Q, ix=ix)


def _serve(ix, Q, ks, nps, budget=0, max_slots=64, spacing_s=0.0):
    L = mrq.lib()
    srv = C.c_void_p()
    assert L.mrq_server_create(ix._h, budget, max_slots, None, C.byref(srv)) == mrq.MRQ_OK
    try:
        for i in range(Q.shape[0]):
            q = np.ascontiguousarray(Q[i])
            assert L.mrq_server_submit(srv, i, q.ctypes.data, int(ks[i]), int(nps[i])) == mrq.MRQ_OK
            if spacing_s:
                time.sleep(spacing_s)
        assert L.mrq_server_drain(srv, 60_000) == mrq.MRQ_OK
        row = int(max(ks))
        n = Q.shape[0]
        rid = np.zeros(n, np.uint64)
        kk = np.zeros(n, np.int32)
        ids = np.zeros((n, row), np.int64)
        dd = np.zeros((n, row), np.float32)
        lat = np.zeros(n, np.float64)
        got = L.mrq_server_poll(srv, rid.ctypes.data, kk.ctypes.data, ids.ctypes.data, dd.ctypes.data, row, n,
                                lat.ctypes.data)
        assert got == n
        return rid, kk, ids, dd, lat
    finally:
        L.mrq_server_destroy(srv)


def test_server_results_equal_search_alone(env):
    rng = np.random.default_rng(5)
    n = env["Q"].shape[0]
    ks = rng.choice([10, 50, 100], n).astype(np.int32)
    nps = rng.choice([4, 8, 16], n).astype(np.int32)
    rid, kk, ids, dd, lat = _serve(env["ix"], env["Q"], ks, nps, spacing_s=0.0005)
    assert sorted(rid.tolist()) == list(range(n))
    assert np.all(lat > 0)
    for j in range(n):
        i = int(rid[j])
        assert kk[j] == ks[i]
        a, b = env["ix"].search(env["Q"][i:i + 1].copy(), int(ks[i]), int(nps[i]))
        assert np.array_equal(a[0], ids[j, :ks[i]])
        assert np.array_equal(b[0].view(np.uint32), dd[j, :ks[i]].view(np.uint32))
    print(f"[gpu] server latency p50 {np.percentile(lat, 50):.2f} ms p99 {np.percentile(lat, 99):.2f} ms", flush=True)


def _stats(srv):
    L = mrq.lib()
    cur, peak, nb = C.c_int64(), C.c_int64(), C.c_int64()
    inflight = C.c_int32()
    assert L.mrq_server_stats(srv, C.byref(cur), C.byref(peak), C.byref(nb), C.byref(inflight)) == mrq.MRQ_OK
    return cur.value, peak.value, nb.value, inflight.value


def test_budget_bounds_device_memory_and_slots_overlap(env):
    """With a budget the server holds exactly it (half per slot, allocated at creation) and never more; a
    burst of requests keeps both slots' batches on the device at once."""
    L = mrq.lib()
    srv = C.c_void_p()
    budget = 64 << 20
    assert L.mrq_server_create(env["ix"]._h, budget, 32, None, C.byref(srv)) == mrq.MRQ_OK
    try:
        n = env["Q"].shape[0]
        for i in range(n):
            q = np.ascontiguousarray(env["Q"][i])
            assert L.mrq_server_submit(srv, i, q.ctypes.data, 100, 16) == mrq.MRQ_OK
        assert L.mrq_server_drain(srv, 60_000) == mrq.MRQ_OK
        cur, peak, nb, inflight = _stats(srv)
        print(f"[gpu] server stats: bytes {cur} peak {peak} batches {nb} max in flight {inflight}", flush=True)
        assert peak <= budget and cur <= budget
        assert nb >= (n + 31) // 32
        assert inflight == 2
    finally:
        L.mrq_server_destroy(srv)


def test_memory_admission_defers_requests(env):
    n = 40
    ks = np.full(n, 10, np.int32)
    nps = np.full(n, 8, np.int32)
    L = mrq.lib()
    # a budget just above one request: batches of one, still every request completes
    probe = C.c_void_p()
    assert L.mrq_server_create(env["ix"]._h, 1, 8, None, C.byref(probe)) == mrq.MRQ_OK
    q = np.ascontiguousarray(env["Q"][0])
    assert L.mrq_server_submit(probe, 0, q.ctypes.data, 10, 8) == mrq.MRQ_ENOMEM   # can never fit 1 byte
    assert L.mrq_server_submit(probe, 0, q.ctypes.data, 0, 8) == mrq.MRQ_EINVAL
    L.mrq_server_destroy(probe)
    rid, kk, ids, dd, lat = _serve(env["ix"], env["Q"][:n], ks, nps, budget=6 << 20, max_slots=64)
    for j in range(n):
        i = int(rid[j])
        a, _ = env["ix"].search(env["Q"][i:i + 1].copy(), 10, 8)
        assert np.array_equal(a[0], ids[j, :10])
