"""GPU parity of the MR-SQ search (Appendix A.2, Exp-5) with the CPU oracle (needs an MI355X).

The index is built on the device with its MR-SQ codes and exported; the oracle checks the codes
bit for bit against its own grid applied to the exported FP32 leading coordinates, and each device
result row against its own MR-SQ search (readings S1-S4) under the rules of tests/parity.py.
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
from parity import check_mrsq_rows  # noqa: E402

MRSQ = mrq.MRQ_METHOD_MRSQ


@pytest.fixture(scope="module")
def sq():
    print("\n[gpu] build small with MR-SQ codes: N=20000 D=128 d=32 nlist=64", flush=True)
    X, Q, _ = synth.workload("small", N=20000, nq=100, cache=False)
    Xd = torch.from_numpy(X).cuda()
    ix = mrq.Index.build(Xd, d_r=32, bits=1, nlist=64, sq8=True)
    path = os.path.join(tempfile.mkdtemp(), "ix.mrqx")
    ix.export(path)
    env = dict(X=X, Q=Q, Xd=Xd, Qd=torch.from_numpy(Q).cuda(), ix=ix, path=path,
               raw=oracle.Index.load_export(path), orc=oracle.Index.load_export(path, X))
    yield env
    ix.close()


def _search(env, k, nprobe, R, **kw):
    ids, dists = env["ix"].search(env["Qd"], k, nprobe, method=MRSQ, rerank=R, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dists.cpu().numpy()


def _assert_parity(env, ids, dists, k, nprobe, R, **kw):
    st = check_mrsq_rows(env["orc"], env["X"], env["Q"], ids, dists, k, nprobe, R, **kw)
    print(f"[gpu] MR-SQ parity k={k} nprobe={nprobe} R={R}: "
          f"{dict((a, b) for a, b in st.items() if a != 'failures')}", flush=True)
    assert not st["failures"], st["failures"][:5]
    assert st["boundary_excused"] + st["probe_tie"] <= 0.05 * st["queries"]


def test_codes_follow_the_grid_of_the_exported_coordinates(sq):
    raw = sq["raw"]
    xd = raw.get("xd").astype(np.float32)      # the device's FP32 leading coordinates, exactly
    lo, dl = oracle.sq8_range(xd)
    assert np.array_equal(raw.get("sq_lo"), lo) and np.array_equal(raw.get("sq_delta"), dl)
    assert np.array_equal(raw.get("sq_code"), oracle.sq8_encode(xd, lo, dl))


@pytest.mark.parametrize("k,nprobe,R", [(10, 8, 500), (10, 8, 50), (1, 4, 10), (50, 16, 200), (10, 64, 100)])
def test_mrsq_matches_oracle(sq, k, nprobe, R):
    ids, dists = _search(sq, k, nprobe, R)
    _assert_parity(sq, ids, dists, k, nprobe, R)


def test_reranking_every_candidate_gives_exact_ivf(sq):
    """R above every query's candidate count: the result is the plain definition (EXACT-IVF)."""
    ids, dists = _search(sq, 10, 4, 16384)
    _assert_parity(sq, ids, dists, 10, 4, 16384)
    for i in range(0, 100, 9):
        ex, _ = sq["orc"].search(sq["Q"][i], 10, 4, mode=oracle.EXACT_IVF)
        assert set(ex.tolist()) == set(ids[i].tolist())


def test_per_query_path_and_batch_composition_do_not_change_rows(sq):
    ids, dists = sq["ix"].search(sq["Qd"], 10, 8, method=MRSQ, rerank=100)
    ids1, dists1 = sq["ix"].search(sq["Qd"], 10, 8, method=MRSQ, rerank=100, mode=mrq.MRQ_PER_QUERY)
    rows = torch.tensor([3, 17, 18, 50, 99], device="cuda")
    ids2, dists2 = sq["ix"].search(sq["Qd"][rows].contiguous(), 10, 8, method=MRSQ, rerank=100)
    torch.cuda.synchronize()
    assert torch.equal(ids, ids1) and torch.equal(dists.view(torch.int32), dists1.view(torch.int32))
    assert torch.equal(ids[rows], ids2) and torch.equal(dists[rows].view(torch.int32), dists2.view(torch.int32))


def test_mixed_k_nprobe(sq):
    rng = np.random.default_rng(77)
    ks = rng.integers(1, 40, 100).astype(np.int32)
    nps = rng.integers(1, 24, 100).astype(np.int32)
    ids, dists, off = sq["ix"].search_mixed(sq["Q"], ks, nps, method=MRSQ, rerank=120)
    kmax = int(ks.max())
    I = np.full((100, kmax), -1, np.int64)
    Dd = np.full((100, kmax), np.inf, np.float32)
    for i in range(100):
        I[i, :ks[i]] = ids[off[i]:off[i] + ks[i]]
        Dd[i, :ks[i]] = dists[off[i]:off[i] + ks[i]]
    _assert_parity(sq, I, Dd, kmax, 1, 120, ks=ks, nprobes=nps)


def test_counters_count_scanned_candidates_and_exact_distances(sq):
    cnt = np.zeros(8, dtype=np.int64)
    sq["ix"].search(sq["Q"], 10, 8, method=MRSQ, rerank=50, counters=cnt)
    off = sq["orc"].get("off")
    scanned = 0
    for i in range(100):
        lists, _ = sq["orc"].probe(sq["Q"][i], 8)
        scanned += int(sum(off[j + 1] - off[j] for j in lists))
    assert cnt[0] == scanned
    assert cnt[3] == 100 * 50          # every query has more than R candidates here


def test_save_load_keeps_the_codes(sq):
    path = os.path.join(tempfile.mkdtemp(), "ix.mrqs")
    sq["ix"].save(path)
    ix2 = mrq.Index.load(path)
    try:
        a = sq["ix"].search(sq["Qd"], 10, 8, method=MRSQ, rerank=64)
        b = ix2.search(sq["Qd"], 10, 8, method=MRSQ, rerank=64)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    finally:
        ix2.close()


def test_invalid_requests_are_rejected(sq):
    with pytest.raises(mrq.MRQError) as e:
        sq["ix"].search(sq["Q"][:4], 20, 8, method=MRSQ, rerank=10)     # R < k
    assert e.value.status == mrq.MRQ_EINVAL
    with pytest.raises(mrq.MRQError) as e:
        sq["ix"].search(sq["Q"][:4], 10, 8, method=MRSQ, rerank=20000)  # R too large
    assert e.value.status == mrq.MRQ_EINVAL
    plain = mrq.Index.build(sq["Xd"][:5000].contiguous(), d_r=32, bits=1, nlist=16)
    try:
        with pytest.raises(mrq.MRQError) as e:
            plain.search(sq["Q"][:4], 10, 4, method=MRSQ)               # no MR-SQ codes
        assert e.value.status == mrq.MRQ_ESTATE
    finally:
        plain.close()
