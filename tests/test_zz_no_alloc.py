"""The allocation-free search entry point (mrq_search_noalloc) against mrq_search, through the C ABI.

Both run the same kernels; the allocation-free one takes its workspace from the library's fixed device
buffer and runs the seed pass on the caller's stream.  Results must be identical: ids bit for bit, and
the distances bit for bit too (every distance is the same FP32 operation sequence on the same inputs).
Two calls in a row, the second with a smaller batch, check that nothing of the first call's buffer
contents leaks into the second.
"""
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
    print("\n[gpu] no-alloc: build N=20000 D=128 d=32 B=1 nlist=64", flush=True)
    X, Q, _ = synth.workload("small", N=20000, nq=300, cache=False)
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=32, bits=1, nlist=64)
    yield dict(X=X, Q=torch.from_numpy(Q).cuda(), ix=ix)
    ix.close()


def _pair(ix, Q, k, nprobe, **kw):
    ids_a, d_a = ix.search(Q, k, nprobe, **kw)
    ids_b = torch.full((Q.shape[0], k), -7, dtype=torch.int64, device=Q.device)
    d_b = torch.full((Q.shape[0], k), -7.0, dtype=torch.float32, device=Q.device)
    ix.search_noalloc(Q, k, nprobe, ids_b, d_b, **kw)
    torch.cuda.synchronize()
    return ids_a.cpu().numpy(), d_a.cpu().numpy(), ids_b.cpu().numpy(), d_b.cpu().numpy()


def test_noalloc_equals_search_twice_smaller_second(env):
    ix, Q = env["ix"], env["Q"]
    for nq, k, nprobe in ((300, 20, 12), (37, 10, 5)):
        print(f"[gpu] no-alloc nq={nq} k={k} nprobe={nprobe}", flush=True)
        ia, da, ib, db = _pair(ix, Q[:nq].contiguous(), k, nprobe)
        assert np.array_equal(ia, ib)
        assert np.array_equal(da.view(np.uint32), db.view(np.uint32))
        assert (ia[:, 0] >= 0).all()


def test_noalloc_counters_and_per_query_mode(env):
    ix, Q = env["ix"], env["Q"][:20].contiguous()
    ca = torch.zeros(8, dtype=torch.int64, device="cuda")
    cb = torch.zeros(8, dtype=torch.int64, device="cuda")
    ia, da, ib, db = _pair(ix, Q, 10, 8, counters=None)
    ix.search(Q, 10, 8, counters=ca)
    ix.search_noalloc(Q, 10, 8, torch.empty((20, 10), dtype=torch.int64, device="cuda"),
                      torch.empty((20, 10), dtype=torch.float32, device="cuda"), counters=cb)
    torch.cuda.synchronize()
    assert torch.equal(ca, cb)
    ipq = torch.empty((20, 10), dtype=torch.int64, device="cuda")
    dpq = torch.empty((20, 10), dtype=torch.float32, device="cuda")
    ix.search_noalloc(Q, 10, 8, ipq, dpq, mode=mrq.MRQ_PER_QUERY)
    torch.cuda.synchronize()
    assert np.array_equal(ipq.cpu().numpy(), ia)


def test_noalloc_rejects_host_buffers_and_oversized_batches(env):
    ix = env["ix"]
    Qh = env["Q"][:4].cpu().numpy()
    ids = torch.empty((4, 10), dtype=torch.int64, device="cuda")
    dd = torch.empty((4, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(mrq.MRQError) as e:
        ix.search_noalloc(Qh, 10, 8, ids, dd)
    assert e.value.status == mrq.MRQ_EINVAL
    # a batch whose workspace exceeds the fixed buffer is refused before any device work (the query rows
    # alone, nq x D floats twice, pass 128 MiB at nq = 2^18)
    nq = 1 << 18
    Qbig = torch.zeros((nq, 128), dtype=torch.float32, device="cuda")
    ib = torch.empty((nq, 1), dtype=torch.int64, device="cuda")
    db = torch.empty((nq, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(mrq.MRQError) as e:
        ix.search_noalloc(Qbig, 1, 1, ib, db)
    assert e.value.status == mrq.MRQ_EINVAL
    assert "workspace" in str(e.value)
