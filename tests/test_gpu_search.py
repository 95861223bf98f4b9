"""GPU parity of the MRQ search path with the CPU oracle (needs an MI355X).

The device index is exported and the oracle imports it, re-deriving every per-vector quantity in
FP64 from the original vectors; the device results are then compared with the oracle's plain
definition of the result (EXACT-IVF over the probed lists) under the rules in tests/parity.py.
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
from parity import assert_rows, check_rows  # noqa: E402


def _mk(name, N, nq, d, B, nlist, spec_override=None):
    X, Q, spec = synth.workload(name, N=N, nq=nq, cache=False)
    Xd = torch.from_numpy(X).cuda()
    ix = mrq.Index.build(Xd, d_r=d, bits=B, nlist=nlist)
    tmp = tempfile.mkdtemp()
    path = os.path.join(tmp, "ix.mrqx")
    ix.export(path)
    orc = oracle.Index.load_export(path, X)
    return dict(X=X, Q=Q, Xd=Xd, Qd=torch.from_numpy(Q).cuda(), ix=ix, orc=orc, d=d, B=B, nlist=nlist)


@pytest.fixture(scope="module")
def small():
    print("\n[gpu] build small: N=20000 D=128 d=32 B=1 nlist=64", flush=True)
    return _mk("small", 20000, 100, 32, 1, 64)


@pytest.fixture(scope="module")
def small_ext():
    print("\n[gpu] build small ext: N=12000 D=128 d=64 B=4 nlist=48", flush=True)
    return _mk("small", 12000, 60, 64, 4, 48)


def _search(env, k, nprobe, **kw):
    ids, dists = env["ix"].search(env["Qd"], k, nprobe, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dists.cpu().numpy()


def _assert_parity(env, ids, dists, k, nprobe, prm=None):
    prm = prm or oracle.params()
    st = check_rows(env["orc"], env["X"], env["Q"], ids, dists, k, nprobe, prm)
    assert_rows(st, f"k={k} nprobe={nprobe}")
    return st


# ---- build parity -------------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["small", "small_ext"])
def test_build_matches_oracle(which, request):
    env = request.getfixturevalue(which)
    path = os.path.join(tempfile.mkdtemp(), "raw.mrqx")
    env["ix"].export(path)
    raw = oracle.Index.load_export(path)        # the device's own stored summaries
    orc = env["orc"]                             # the same index re-derived in FP64
    for name, tol in (("nx", 2e-5), ("tx", 2e-5), ("ax", 2e-6), ("xi1", 2e-5), ("xiB", 2e-5), ("yn", 1e-6)):
        a, b = raw.get(name), orc.get(name)
        scale = np.maximum(np.abs(b), 1e-3 * np.abs(b).max())
        err = np.abs(a - b) / scale
        assert err.max() <= tol, (name, float(err.max()))
    # sign bits: every disagreement with the FP64 rotated residual sits at a near-zero coordinate
    d = env["d"]
    Pr, Cc, off, lid, code = orc.get("Pr"), orc.get("C"), orc.get("off"), orc.get("lid"), orc.get("code")
    xd = orc.get("xd")
    B = env["B"]
    lists = np.searchsorted(off, np.arange(orc.N), side="right") - 1
    o = xd - Cc[lists]
    xp = (o @ Pr) / np.linalg.norm(o, axis=1, keepdims=True)
    sign = (code >> (B - 1)) & 1
    flips = sign != (xp >= 0)
    assert np.all(np.abs(xp[flips]) < 1e-5), np.abs(xp[flips]).max()
    if B > 1:  # the B-bit code reaches the best cosine up to FP32 input noise
        for r in range(0, orc.N, max(1, orc.N // 300)):
            _, best = oracle.encode_ext(xp[r], B)
            assert orc.get("xiB")[r] >= best - 1e-5


# ---- search parity --------------------------------------------------------------------------------

@pytest.mark.parametrize("k,nprobe", [(10, 8), (1, 4), (50, 16), (10, 64)])
def test_search_matches_oracle(small, k, nprobe):
    ids, dists = _search(small, k, nprobe)
    _assert_parity(small, ids, dists, k, nprobe)


def test_search_ext_bits_matches_oracle(small_ext):
    ids, dists = _search(small_ext, 10, 8)
    _assert_parity(small_ext, ids, dists, 10, 8)
    ids2, dists2 = _search(small_ext, 10, 8, use_ext=False)
    _assert_parity(small_ext, ids2, dists2, 10, 8, prm=oracle.params(use_ext=False))


def test_plain_mrq_without_stage2(small):
    ids, dists = _search(small, 10, 8, stage2=False)
    _assert_parity(small, ids, dists, 10, 8, prm=oracle.params(stage2=False))


def test_all_lists_is_exact_knn(small):
    """nprobe = nlist: the definition of the result is exact k-NN over the whole set (brute force)."""
    gt, gd = oracle.bruteforce(small["X"], small["Q"], 10)
    ids, dists = _search(small, 10, small["nlist"])
    st = _assert_parity(small, ids, dists, 10, small["nlist"])
    same = sum(set(a.tolist()) == set(b.tolist()) for a, b in zip(ids, gt))
    assert same >= st["exact_match"], (same, st)


def test_recall_against_ground_truth(small):
    gt, _ = oracle.bruteforce(small["X"], small["Q"], 10)
    ids, _ = _search(small, 10, 8)
    rec = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(ids, gt)])
    print(f"[gpu] recall@10 nprobe=8: {rec:.4f}", flush=True)
    assert rec >= 0.95


# ---- batch independence and the per-query path -----------------------------------------------------

def test_per_query_path_bit_identical(small):
    ids, dists = _search(small, 10, 8)
    ids1, dists1 = _search(small, 10, 8, mode=mrq.MRQ_PER_QUERY)
    assert np.array_equal(ids, ids1) and np.array_equal(dists.view(np.uint32), dists1.view(np.uint32))


def test_result_independent_of_batch(small):
    ids, dists = _search(small, 10, 8)
    sel = [3, 17, 42, 99]
    sub = small["Qd"][sel].contiguous()
    ids2, dists2 = small["ix"].search(sub, 10, 8)
    torch.cuda.synchronize()
    assert np.array_equal(ids[sel], ids2.cpu().numpy())
    assert np.array_equal(dists[sel].view(np.uint32), dists2.cpu().numpy().view(np.uint32))
    big = torch.cat([small["Qd"]] * 5)
    ids3, dists3 = small["ix"].search(big, 10, 8)
    torch.cuda.synchronize()
    assert np.array_equal(np.concatenate([ids] * 5), ids3.cpu().numpy())


def test_host_buffers(small):
    ids, dists = small["ix"].search(small["Q"][:7].copy(), 10, 8)
    ref, refd = _search(small, 10, 8)
    assert np.array_equal(ids, ref[:7]) and np.array_equal(dists, refd[:7])


def test_mixed_k_nprobe(small):
    rng = np.random.default_rng(0)
    n = small["Q"].shape[0]
    ks = rng.integers(1, 40, n).astype(np.int32)
    nps = rng.integers(1, 20, n).astype(np.int32)
    ids, dists, off = small["ix"].search_mixed(small["Qd"], ks, nps)
    rows_i = [ids[off[i]:off[i] + ks[i]] for i in range(n)]
    rows_d = [dists[off[i]:off[i] + ks[i]] for i in range(n)]
    for i in range(0, n, 9):  # each row equals the uniform search with that (k, nprobe)
        a, b = small["ix"].search(small["Qd"][i:i + 1].contiguous(), int(ks[i]), int(nps[i]))
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy()[0], rows_i[i])
        assert np.array_equal(b.cpu().numpy()[0].view(np.uint32), rows_d[i].view(np.uint32))
    st = check_rows(small["orc"], small["X"], small["Q"], rows_i, rows_d, None, None, oracle.params(),
                    ks=ks, nprobes=nps)
    assert_rows(st, "mixed k / nprobe")


def test_mixed_batch_on_the_device(small):
    """Per-query k / nprobe as device arrays (mrq_search_mixed_dev): the same rows as the host-metadata mixed
    search; entries outside the bounds are rejected and counted, the other rows are unchanged."""
    rng = np.random.default_rng(11)
    n = small["Q"].shape[0]
    ks = rng.integers(1, 40, n).astype(np.int32)
    nps = rng.integers(1, 20, n).astype(np.int32)
    ids, dists, off = small["ix"].search_mixed(small["Qd"], ks, nps)
    tot = int(ks.sum())
    kd, npd = torch.from_numpy(ks).cuda(), torch.from_numpy(nps).cuda()
    ib = torch.full((tot,), -7, dtype=torch.int64, device="cuda")
    db = torch.full((tot,), -7.0, dtype=torch.float32, device="cuda")
    rej = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    small["ix"].search_mixed_dev(small["Qd"], kd, npd, 40, 20, ib, db, rejected=rej)
    torch.cuda.synchronize()
    assert int(rej.item()) == 0
    assert np.array_equal(ib.cpu().numpy(), ids)
    assert np.array_equal(db.cpu().numpy().view(np.uint32), dists.view(np.uint32))
    # two bad entries: k = 0 and nprobe above the bound; rows at the caller's offsets
    ks2, nps2 = ks.copy(), nps.copy()
    ks2[3], nps2[5] = 0, 21
    offd = torch.from_numpy(off).cuda()
    ib.fill_(-7)
    db.fill_(-7.0)
    small["ix"].search_mixed_dev(small["Qd"], torch.from_numpy(ks2).cuda(), torch.from_numpy(nps2).cuda(), 40, 20,
                                 ib, db, out_off=offd, rejected=rej)
    torch.cuda.synchronize()
    assert int(rej.item()) == 2
    ih, dh = ib.cpu().numpy(), db.cpu().numpy()
    for i in range(n):
        sl = slice(int(off[i]), int(off[i] + ks[i]))
        if i in (3, 5):
            assert np.all(ih[sl] == -7)
        else:
            assert np.array_equal(ih[sl], ids[sl]) and np.array_equal(dh[sl].view(np.uint32), dists[sl].view(np.uint32))


def test_mixed_batch_replays_from_a_captured_graph(small):
    """A device-side mixed batch recorded into a HIP graph gives the eager rows on every replay, with eager
    searches between the replays."""
    rng = np.random.default_rng(12)
    Qd = small["Qd"]
    n = Qd.shape[0]
    ks = torch.from_numpy(rng.integers(1, 30, n).astype(np.int32)).cuda()
    nps = torch.from_numpy(rng.integers(1, 16, n).astype(np.int32)).cuda()
    tot = int(ks.sum().item())
    ib = torch.empty((tot,), dtype=torch.int64, device="cuda")
    db = torch.empty((tot,), dtype=torch.float32, device="cuda")
    opts = mrq.search_opts(group=16, phase_growth=4)
    s = torch.cuda.Stream()
    small["ix"].search_mixed_dev(Qd, ks, nps, 30, 16, ib, db, opts=opts, stream=s)  # sizes the workspace
    torch.cuda.synchronize()
    ref_i, ref_d = ib.clone(), db.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        small["ix"].search_mixed_dev(Qd, ks, nps, 30, 16, ib, db, opts=opts, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        ib.fill_(-7)
        db.fill_(-1.0)
        small["ix"].search(Qd[:6 + rep].contiguous(), 5, 4, opts=opts)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ib, ref_i), rep
        assert torch.equal(db.view(torch.int32), ref_d.view(torch.int32)), rep


@pytest.mark.parametrize("nlist", [256, 1500, 5000, 9000, 16000])
def test_probe_selection_kernels_agree(nlist):
    """The probe ranking has four forms: one wave per query for nprobe <= 64 and nlist <= 4096 (16, 32 or 64
    lists per lane in registers), one wave per query from the product's tile minima for nprobe <= 64 and
    nlist above 4096, and one block per query otherwise, which gathers the keys at or below the np-th
    smallest per-thread minimum when np <= 256 and takes a bitwise search of the np-th smallest pattern
    beyond.  All take the np smallest (g_j, j) in that order, so a row is the same under each (nlist 256
    and 1500: wave against block; 5000, 9000 and 16000: tiles against blocks of 4 and 8 waves), and rows at nprobe
    64 (tiles) and 300 (bitwise search) are checked against the oracle row by row."""
    print(f"\n[gpu] selection kernels agree: nlist={nlist}", flush=True)
    X, Q, _ = synth.workload("small", N=20000, nq=60, cache=False)
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=32, bits=1, nlist=nlist)
    try:
        Qd = torch.from_numpy(Q).cuda()
        for np_small in (1, 7, 20, 64):
            ks = np.full(60, 10, np.int32)
            nps = np.full(60, np_small, np.int32)
            nps[-1] = 100                                   # np_max 100: the block kernel for every row
            ids, dists, off = ix.search_mixed(Qd, ks, nps)
            a, b = ix.search(Qd[:59].contiguous(), 10, np_small)  # np_max <= 64: the wave kernel up to 4096
            torch.cuda.synchronize()
            assert np.array_equal(ids[:590].reshape(59, 10), a.cpu().numpy())
            assert np.array_equal(dists[:590].reshape(59, 10).view(np.uint32), b.cpu().numpy().view(np.uint32))
        if nlist > 4096:
            path = os.path.join(tempfile.mkdtemp(), "ix.mrqx")
            ix.export(path)
            env = dict(X=X, Q=Q, ix=ix, Qd=Qd, orc=oracle.Index.load_export(path, X))
            for nprobe in (64, 300):
                ids, dists = _search(env, 10, nprobe)
                _assert_parity(env, ids, dists, 10, nprobe)
    finally:
        ix.close()


def test_tile_selection_ties_and_hand_back():
    """Above 4096 lists and up to nprobe 64 the ranking starts from the product's per-tile minima (64 lists
    a tile): only the tiles whose minimum is at most the np-th smallest one are read.  Here the data repeats
    48 points, so most of the 6000 centroids coincide and the probe distances tie exactly: most queries have
    more than 64 tiles at that minimum and are handed to the block selection, the others rank ties inside
    the tile kernel (bitwise search of the pattern, then of the last list id taken).  Either way the rows
    equal those of the block selection run for the whole batch (nprobe_max 100)."""
    print("\n[gpu] tile selection with tied probe distances: N=24000 D=64 nlist=6000", flush=True)
    rng = np.random.default_rng(11)
    base = rng.standard_normal((48, 64)).astype(np.float32)
    X = np.ascontiguousarray(base[rng.integers(0, 48, 24000)])
    Q = np.ascontiguousarray(base[rng.integers(0, 48, 60)] + 0.05 * rng.standard_normal((60, 64)).astype(np.float32))
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=32, bits=1, nlist=6000)
    try:
        Qd = torch.from_numpy(Q).cuda()
        for np_small in (1, 10, 40, 64):
            ks = np.full(60, 10, np.int32)
            nps = np.full(60, np_small, np.int32)
            nps[-1] = 100
            ids, dists, _ = ix.search_mixed(Qd, ks, nps)
            a, b = ix.search(Qd[:59].contiguous(), 10, np_small)
            torch.cuda.synchronize()
            assert np.array_equal(ids[:590].reshape(59, 10), a.cpu().numpy()), np_small
            assert np.array_equal(dists[:590].reshape(59, 10).view(np.uint32), b.cpu().numpy().view(np.uint32))
    finally:
        ix.close()


@pytest.mark.parametrize("D", [100, 102, 2112])
def test_dimensions_off_the_tiles(D):
    """D = 100 (float4-aligned rows, not a multiple of 32: the query's tail coordinates come from the BF16
    product on zero-padded rows), D = 102 (rows not float4-aligned: the FP32 product of every axis) and
    D = 2112 (query rows too long to stage in the seed pass's LDS: its global-memory form) all give the
    oracle's results."""
    N = 8000 if D < 1000 else 3000
    print(f"\n[gpu] build N={N} D={D} d=32 B=1 nlist=32", flush=True)
    m = synth.build_model(synth.MixtureSpec(D=D, n_comp=32, decay=1.0, cluster_dims=8, model_seed=5))
    X, Q = synth.sample(m, N, 1), synth.sample(m, 40, 2)
    Xd = torch.from_numpy(X).cuda()
    ix = mrq.Index.build(Xd, d_r=32, bits=1, nlist=32)
    try:
        path = os.path.join(tempfile.mkdtemp(), "ix.mrqx")
        ix.export(path)
        env = dict(X=X, Q=Q, ix=ix, Qd=torch.from_numpy(Q).cuda(), orc=oracle.Index.load_export(path, X))
        ids, dists = _search(env, 10, 8)
        _assert_parity(env, ids, dists, 10, 8)
    finally:
        ix.close()


@pytest.mark.parametrize("D,d", [(128, 64), (64, 32), (48, 40)])
def test_short_exact_rows_match_oracle(D, d):
    """Tails no wider than the leading block: the exact stage takes dis_o' - 2 <x_r, q_r> from rows of D - d
    floats (64, 32 and 8 here), four candidates per lane group at a time; with stage 2 off it reads the whole
    rows (at most 64 floats at D = 64 and 48: the same short-row form).  Rows match the oracle, and the
    in-place form of the scan (exact_cap 1) and the per-query path give the same rows bit for bit."""
    N = 12000
    print(f"\n[gpu] short exact rows: build N={N} D={D} d={d} B=1 nlist=48", flush=True)
    m = synth.build_model(synth.MixtureSpec(D=D, n_comp=24, decay=1.0, cluster_dims=8, model_seed=17))
    X, Q = synth.sample(m, N, 1), synth.sample(m, 50, 2)
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=d, bits=1, nlist=48)
    try:
        path = os.path.join(tempfile.mkdtemp(), "ix.mrqx")
        ix.export(path)
        env = dict(X=X, Q=Q, ix=ix, Qd=torch.from_numpy(Q).cuda(), orc=oracle.Index.load_export(path, X))
        for k, nprobe, kw in ((10, 8, {}), (50, 16, {}), (10, 8, dict(stage2=False))):
            ids, dists = _search(env, k, nprobe, **kw)
            prm = oracle.params(**kw)
            _assert_parity(env, ids, dists, k, nprobe, prm)
            for alt in (dict(exact_cap=1), dict(mode=mrq.MRQ_PER_QUERY)):
                b_ids, b_d = _search(env, k, nprobe, **kw, **alt)
                assert np.array_equal(ids, b_ids), (k, nprobe, kw, alt)
                assert np.array_equal(dists.view(np.uint32), b_d.view(np.uint32)), (k, nprobe, kw, alt)
    finally:
        ix.close()


def test_counters_monotone(small):
    cnt = np.zeros(8, dtype=np.int64)
    small["ix"].search(small["Q"][:20].copy(), 10, 8, counters=cnt)
    for part in (cnt[:4], cnt[4:]):
        scanned, p1, pext, p2 = part
        assert scanned > 0 and scanned >= p1 >= pext >= p2 > 0


def test_extended_counters_count_scan_work(small):
    """16 counters: [0..7] as with 8; [8] scan work items, [9] row tiles whose x_d entered stage 2 (at most four
    per item, at least one per item with a stage-2 entrant)."""
    c8 = torch.zeros(8, dtype=torch.int64, device="cuda")
    c16 = torch.zeros(16, dtype=torch.int64, device="cuda")
    small["ix"].search(small["Qd"], 10, 16, counters=c8, group=16)
    small["ix"].search(small["Qd"], 10, 16, counters=c16, group=16)
    torch.cuda.synchronize()
    c8, c16 = c8.cpu().numpy(), c16.cpu().numpy()
    assert np.array_equal(c8, c16[:8])
    items, tiles = c16[8], c16[9]
    assert items > 0 and 0 < tiles <= 4 * items
    assert np.all(c16[10:] == 0)
    # every item is a 64-row block against at most 16 pairs: items * 64 * 16 >= candidates scanned
    assert items * 64 * 16 >= c16[0]


def test_stream_copy_moves_every_byte():
    src = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    mrq.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    with pytest.raises(mrq.MRQError) as e:
        mrq.lib()
        mrq._check(mrq.lib().mrq_stream_copy(dst.data_ptr() + 4, src.data_ptr(), 64, None))
    assert e.value.status == mrq.MRQ_EINVAL


# ---- edge cases -----------------------------------------------------------------------------------

def test_padding_when_k_exceeds_candidates():
    X, Q, _ = synth.workload("small", N=300, nq=5, cache=False)
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=16, bits=1, nlist=40)
    ids, dists = ix.search(torch.from_numpy(Q).cuda(), 64, 1)
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    path = os.path.join(tempfile.mkdtemp(), "p.mrqx")
    ix.export(path)
    orc = oracle.Index.load_export(path, X)
    for i in range(5):
        lists, _ = orc.probe(Q[i], 1)
        off = orc.get("off")
        n = int(off[lists[0] + 1] - off[lists[0]])
        assert np.all(ids[i, :n] >= 0) and np.all(ids[i, n:] == -1) and np.all(np.isinf(dists[i, n:]))
        assert set(ids[i, :n].tolist()) == set(orc.get("lid")[off[lists[0]]:off[lists[0] + 1]].tolist())


def test_full_dimension_rabitq_mode():
    """d_r = D: no residual terms (the IVF + RaBitQ special case)."""
    X, Q, _ = synth.workload("small", N=8000, nq=30, cache=False)
    env = dict(X=X, Q=Q, Qd=torch.from_numpy(Q).cuda(), nlist=32)
    env["ix"] = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=128, bits=1, nlist=32)
    path = os.path.join(tempfile.mkdtemp(), "f.mrqx")
    env["ix"].export(path)
    env["orc"] = oracle.Index.load_export(path, X)
    assert np.abs(oracle.Index.load_export(path).get("tx")).max() == 0
    ids, dists = _search(env, 10, 6)
    _assert_parity(env, ids, dists, 10, 6)


def test_invalid_arguments_rejected(small):
    with pytest.raises(mrq.MRQError) as e:
        small["ix"].search(small["Qd"], 0, 8)
    assert e.value.status == mrq.MRQ_EINVAL
    with pytest.raises(mrq.MRQError):
        small["ix"].search(small["Qd"], 10, small["nlist"] + 1)
    bad = small["X"][:500].copy()
    bad[7, 3] = np.nan
    with pytest.raises(mrq.MRQError) as e:
        mrq.Index.build(torch.from_numpy(bad).cuda(), d_r=16, bits=1, nlist=4)
    assert e.value.status == mrq.MRQ_EINVAL


def test_save_load_roundtrip(small):
    path = os.path.join(tempfile.mkdtemp(), "s.mrqs")
    small["ix"].save(path)
    ix2 = mrq.Index.load(path)
    a, b = _search(small, 10, 8)
    c, d = ix2.search(small["Qd"], 10, 8)
    torch.cuda.synchronize()
    assert np.array_equal(a, c.cpu().numpy()) and np.array_equal(b, d.cpu().numpy())


def test_exact_buffer_overflow_gives_same_results(small, small_ext):
    """Candidates that do not fit the exact-stage buffer are finished inside the scan with the same
    arithmetic, so a buffer of a single entry returns bit-identical results."""
    for env in (small, small_ext):
        ix, Q = env["ix"], env["Q"]
        a_ids, a_d = ix.search(Q, 10, 16)
        b_ids, b_d = ix.search(Q, 10, 16, opts=mrq.search_opts(exact_cap=1))
        assert np.array_equal(a_ids, b_ids)
        assert np.array_equal(a_d.view(np.uint32), b_d.view(np.uint32))


@pytest.mark.parametrize("growth", [2, 4, 8, 1024])
@pytest.mark.parametrize("group", [16, 32, 64])
def test_group_size_does_not_change_results(small, group, growth):
    ix, Q = small["ix"], small["Q"]
    a_ids, a_d = ix.search(Q, 10, 16, opts=mrq.search_opts(group=16, phase_growth=growth))
    b_ids, b_d = ix.search(Q, 10, 16, opts=mrq.search_opts(group=group, phase_growth=growth))
    assert np.array_equal(a_ids, b_ids)
    assert np.array_equal(a_d.view(np.uint32), b_d.view(np.uint32))


@pytest.mark.parametrize("growth", [2, 4, 8, 64, 1024])
def test_phase_growth_rows_match_oracle(small, growth):
    """Phases [1, g), [g, g^2), ...: any growth gives the oracle's result wherever the bounds hold (1024: one
    batched phase after the nearest list)."""
    ids, dists = _search(small, 10, 32, phase_growth=growth)
    _assert_parity(small, ids, dists, 10, 32)


def test_phase_growth_rejects_other_values(small):
    with pytest.raises(mrq.MRQError) as e:
        small["ix"].search(small["Q"][:2], 10, 8, phase_growth=3)
    assert e.value.status == mrq.MRQ_EINVAL
    with pytest.raises(mrq.MRQError) as e:
        small["ix"].search(small["Q"][:2], 10, 8, phase_growth=2048)
    assert e.value.status == mrq.MRQ_EINVAL


def test_eight_bit_codes_and_query_levels():
    """B = 8 extended codes and B_q = 8 query levels exceed the signed-byte range of the i8 matrix-core
    operands; the scan stores them with an offset and corrects the products exactly."""
    print("\n[gpu] build N=6000 D=128 d=32 B=8 nlist=24", flush=True)
    env = _mk("small", 6000, 40, 32, 8, 24)
    cnt = {}
    for bq in (4, 8):
        c = torch.zeros(8, dtype=torch.int64, device="cuda")
        ids, dists = _search(env, 10, 8, bq=bq, counters=c)
        _assert_parity(env, ids, dists, 10, 8, prm=oracle.params(bq=bq))
        cnt[bq] = c.cpu().numpy()
    # both query resolutions prune a similar share of candidates at stage 1 and with the B-bit codes
    for i in (1, 2):
        r4, r8 = cnt[4][i] / cnt[4][0], cnt[8][i] / cnt[8][0]
        assert 0.5 * r4 <= r8 <= 1.5 * r4 + 1e-3, (i, r4, r8)


def test_automatic_dr_follows_eq8():
    """d_r = 0 builds with the Eq 8 choice on the data's own eigenvalues."""
    print("\n[gpu] build N=8000 D=256 d_r=auto B=1 nlist=16", flush=True)
    X, Q, _ = synth.workload("small", N=8000, nq=20, cache=False)
    X = np.ascontiguousarray(np.concatenate([X, X[:, ::-1] * 0.5], axis=1))  # D = 256
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=0, bits=1, nlist=16)
    try:
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "ix.mrqx")
            ix.export(path)
            lam = oracle.Index.load_export(path).get("lam")
            orc = oracle.Index.load_export(path, X)
        assert ix.d == mrq.choose_dr(lam)
        assert 128 <= ix.d <= 256
        q = np.ascontiguousarray(np.concatenate([Q, Q[:, ::-1] * 0.5], axis=1))
        ids, dists = ix.search(q, 10, 4)
        assert np.all(ids[:, 0] >= 0)
        st = check_rows(orc, X, q, ids, dists, 10, 4, oracle.params())
        assert_rows(st, f"Eq 8 d_r={ix.d}")
    finally:
        ix.close()


def test_tuner_picks_a_schedule_and_keeps_results(small):
    ix, Q = small["ix"], small["Q"]
    g, p = ix.tune(Q, 10, 16)
    assert g in (16, 32, 64) and p in (2, 4, 8)
    a_ids, a_d = ix.search(Q, 10, 16, opts=mrq.search_opts(group=16, phase_growth=p))
    b_ids, b_d = ix.search(Q, 10, 16)  # the tuned defaults
    assert np.array_equal(a_ids, b_ids)
    assert np.array_equal(a_d.view(np.uint32), b_d.view(np.uint32))


def test_search_replays_from_a_captured_graph(small):
    """The search recorded into a HIP graph (stream capture) gives the eager result on every replay, with
    eager searches on the same index and synchronisations between the replays; a later search that grows
    the workspace keeps the captured one valid."""
    ix, Qd = small["ix"], small["Qd"]
    opts = mrq.search_opts(group=16, phase_growth=4)
    ids = torch.empty((Qd.shape[0], 10), dtype=torch.int64, device="cuda")
    dd = torch.empty((Qd.shape[0], 10), dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    ix.search(Qd, 10, 16, ids=ids, dists=dd, opts=opts, stream=s)  # sizes the workspace
    torch.cuda.synchronize()
    ref_i, ref_d = ids.clone(), dd.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        ix.search(Qd, 10, 16, ids=ids, dists=dd, opts=opts, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        ids.fill_(-7)
        dd.fill_(-1.0)
        ix.search(Qd[:5 + rep].contiguous(), 5, 4, opts=opts)  # eager work on the index between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ids, ref_i), rep
        assert torch.equal(dd.view(torch.int32), ref_d.view(torch.int32)), rep
    ix.search(torch.cat([Qd, Qd, Qd]).contiguous(), 20, 32, opts=opts)  # grows the workspace
    torch.cuda.synchronize()
    ids.fill_(-7)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(ids, ref_i)


def test_capture_refuses_host_buffers(small):
    ix, Q = small["ix"], small["Q"]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(mrq.MRQError) as e:
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            ix.search(Q, 10, 8, stream=s)  # host Q and outputs need copies: not capturable
    assert e.value.status == mrq.MRQ_ESTATE
