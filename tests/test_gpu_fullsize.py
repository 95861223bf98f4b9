"""Parity at the benchmark's full size (needs an MI355X).

The GIST-shaped workload (N = 1,000,000, D = 960, 10,000 queries, nlist = 4,096, d_r = 128) is built and
searched on the GPU exactly as the benchmark runs it (one batched call over all queries); the index is
exported and the CPU oracle checks a seeded sample of the result rows one by one against its plain
definition (EXACT-IVF over the probed lists, with the bound-risk / near-tie excuses of tests/parity.py).
"""
import os
import tempfile

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("no GPU", allow_module_level=True)

import torch  # noqa: E402

import oracle  # noqa: E402
import paper_2411_06158_amd as mrq  # noqa: E402
from paper_2411_06158_amd import synth  # noqa: E402
from parity import assert_rows, check_mrsq_rows, check_rows  # noqa: E402

# rows of a full-size batch checked against the oracle, one by one (seeded choice)
SAMPLE = 600


def _tmpdir():
    return "/dev/shm" if os.path.isdir("/dev/shm") else None


@pytest.fixture(scope="module")
def gist():
    print("\n[gpu] fullsize: generate gist1m N=1000000 D=960 nq=10000", flush=True)
    X, Q, _ = synth.workload("gist1m", cache=False)
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    out = dict(X=X, Q=Q, Xd=Xd, Qd=Qd, ix={}, orc={})
    yield out
    for ix in out["ix"].values():
        ix.close()


def _index(env, bits):
    if bits not in env["ix"]:
        print(f"[gpu] fullsize: build d=128 B={bits} nlist=4096", flush=True)
        ix = mrq.Index.build(env["Xd"], d_r=128, bits=bits, nlist=4096, sq8=bits == 1)
        with tempfile.TemporaryDirectory(dir=_tmpdir()) as td:
            path = os.path.join(td, "ix.mrqx")
            ix.export(path)
            env["orc"][bits] = oracle.Index.load_export(path).attach(env["X"])
        env["ix"][bits] = ix
    return env["ix"][bits], env["orc"][bits]


@pytest.mark.parametrize("bits,k,nprobe", [(1, 10, 32), (4, 10, 32), (1, 100, 64)])
def test_fullsize_sampled_rows_match_oracle(gist, bits, k, nprobe):
    ix, orc = _index(gist, bits)
    print(f"[gpu] fullsize: search nq=10000 k={k} nprobe={nprobe} B={bits}", flush=True)
    ids, dists = ix.search(gist["Qd"], k, nprobe)
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    assert np.all(ids[:, 0] >= 0)
    rows = np.random.default_rng(1000 + 7 * bits + k).choice(ids.shape[0], SAMPLE, replace=False)
    st = check_rows(orc, gist["X"], gist["Q"][rows], ids[rows], dists[rows], k, nprobe, oracle.params())
    assert_rows(st, f"fullsize gist1m B={bits} k={k} nprobe={nprobe}")


def test_fullsize_mrsq_sampled_rows_match_oracle(gist):
    """MR-SQ (Appendix A.2, Exp-5) at the same size: 10,000 queries, nprobe 64, R = 500; the estimates of
    the batch do not fit one buffer, so the queries run in several chunks."""
    ix, orc = _index(gist, 1)
    print("[gpu] fullsize: MR-SQ search nq=10000 k=10 nprobe=64 R=500", flush=True)
    ids, dists = ix.search(gist["Qd"], 10, 64, method=mrq.MRQ_METHOD_MRSQ, rerank=500)
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    rows = np.random.default_rng(3003).choice(ids.shape[0], SAMPLE, replace=False)
    st = check_mrsq_rows(orc, gist["X"], gist["Q"][rows], ids[rows], dists[rows], 10, 64, 500)
    print(f"[gpu] fullsize MR-SQ parity: {dict((a, b) for a, b in st.items() if a != 'failures')}", flush=True)
    assert not st["failures"], st["failures"][:5]
    assert st["boundary_excused"] + st["probe_tie"] <= max(2, 0.02 * SAMPLE)


def test_fullsize_rows_do_not_depend_on_batch(gist):
    ix, _ = _index(gist, 1)
    ids, dists = ix.search(gist["Qd"], 10, 32)
    rows = torch.tensor(np.random.default_rng(5).choice(10000, 257, replace=False), device="cuda")
    ids2, dists2 = ix.search(gist["Qd"][rows].contiguous(), 10, 32)
    torch.cuda.synchronize()
    assert torch.equal(ids[rows], ids2)
    assert torch.equal(dists[rows].view(torch.int32), dists2.view(torch.int32))


def test_fullsize_deep10m_sampled_rows_match_oracle():
    """DEEP-shaped: N = 10,000,000, D = 128, nlist = 16,384, d_r = 64, 1-bit codes, nprobe 16 and 64."""
    print("\n[gpu] fullsize: generate deep10m N=10000000 D=128 nq=10000", flush=True)
    X, Q, _ = synth.workload("deep10m", cache=False)
    Xd = torch.from_numpy(X).cuda()
    print("[gpu] fullsize: build d=64 B=1 nlist=16384", flush=True)
    ix = mrq.Index.build(Xd, d_r=64, bits=1, nlist=16384)
    try:
        with tempfile.TemporaryDirectory(dir=_tmpdir()) as td:
            path = os.path.join(td, "ix.mrqx")
            ix.export(path)
            orc = oracle.Index.load_export(path).attach(X)
        Qd = torch.from_numpy(Q).cuda()
        for nprobe in (16, 64):
            print(f"[gpu] fullsize: search deep10m nq=10000 k=10 nprobe={nprobe}", flush=True)
            ids, dists = ix.search(Qd, 10, nprobe)
            torch.cuda.synchronize()
            ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
            rows = np.random.default_rng(2000 + nprobe).choice(ids.shape[0], SAMPLE, replace=False)
            st = check_rows(orc, X, Q[rows], ids[rows], dists[rows], 10, nprobe, oracle.params())
            assert_rows(st, f"fullsize deep10m nprobe={nprobe}")
    finally:
        ix.close()


def test_fullsize_openai2m_mixed_k_nprobe_match_oracle():
    """Embedding-shaped: N = 2,000,000 unit vectors, D = 1,536, d_r = 256, 4-bit codes, nlist = 4,096;
    20,000 queries with per-query k in [10, 100] and nprobe in [8, 64] in one launch."""
    print("\n[gpu] fullsize: generate openai2m N=2000000 D=1536 nq=20000", flush=True)
    X, Q, _ = synth.workload("openai2m", cache=False)
    Xd = torch.from_numpy(X).cuda()
    print("[gpu] fullsize: build d=256 B=4 nlist=4096", flush=True)
    ix = mrq.Index.build(Xd, d_r=256, bits=4, nlist=4096)
    del Xd
    try:
        with tempfile.TemporaryDirectory(dir=_tmpdir()) as td:
            path = os.path.join(td, "ix.mrqx")
            ix.export(path)
            orc = oracle.Index.load_export(path).attach(X)
        rng = np.random.default_rng(4004)
        ks = rng.integers(10, 101, Q.shape[0]).astype(np.int32)
        nps = rng.integers(8, 65, Q.shape[0]).astype(np.int32)
        print("[gpu] fullsize: search openai2m mixed nq=20000", flush=True)
        ids, dists, off = ix.search_mixed(Q, ks, nps)
        rows = rng.choice(Q.shape[0], SAMPLE, replace=False)
        kmax = int(ks[rows].max())
        I = np.full((SAMPLE, kmax), -1, np.int64)
        Dd = np.full((SAMPLE, kmax), np.inf, np.float32)
        for j, r in enumerate(rows):
            I[j, :ks[r]] = ids[off[r]:off[r] + ks[r]]
            Dd[j, :ks[r]] = dists[off[r]:off[r] + ks[r]]
        st = check_rows(orc, X, Q[rows], I, Dd, kmax, 8, oracle.params(), ks=ks[rows], nprobes=nps[rows])
        assert_rows(st, "fullsize openai2m mixed k / nprobe")
    finally:
        ix.close()
