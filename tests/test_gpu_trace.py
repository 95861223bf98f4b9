"""Element-wise parity of the search's stages with the oracle (needs an MI355X).

mrq_search_trace runs the search kernels' tracing instantiations (the same device code and arithmetic as
mrq_search, plus stores) and returns, for a few queries of a batch, every (query, list) pair's query code
and every candidate's per-stage values.  Each is compared with the oracle's pair trace on the exported
index (Section 4.2 Eq 4-6; Algorithm 2's normalisation, rotation and quantisation of the query; Eq 7):
  * integers bit for bit: the levels u equal the oracle's quantiser applied to the device's own FP32 q';
    the stage-1 inner product ip = sum_i b_i u_i, popcount(b) and the B-bit ip = sum_i ux_i u_i equal the
    sums evaluated directly from the exported codes and the device's levels (brute force);
  * the device's q' against the oracle's FP64 q', and u against the oracle's own levels: equal except
    where the oracle's FP64-derived coordinate lies at a rounding edge of the FP32 quantiser (counted);
  * floating point within 1e-5 C1 (C1 = ||x_d - c||^2 + ||x_r||^2 + ||q_d - c||^2 + ||q_r||^2, the scale of
    the estimate): dis', eps_b and the lower bound without its eps_r term (dis' - eps_b) of stage 1 and of the
    B-bit stage, dis_o' (Eq 7), and the exact distance (1e-5 relative).  eps_r = 2 m sigma (Eq 6) is compared
    on its own, within 2e-3 relative: sigma comes from the query's tail coordinates, which the search takes
    from a BF16 matrix product (FP32 accumulation), 8 significant bits per operand;
  * decisions: in the batched phases a candidate goes on to the next stage exactly when its device bound
    is below the phase threshold, and wherever the oracle's bound is clear of that threshold by more than
    the tolerance, the oracle's bound takes the same decision.
"""
import os
import tempfile
from collections import defaultdict

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

TRACED = [0, 5, 11, 23]


def _env(D, d, B, N, nlist, nq=30, seed=21, name=None):
    print(f"\n[gpu] trace: build N={N} D={D} d={d} B={B} nlist={nlist}", flush=True)
    if name:
        X, Q, _ = synth.workload(name, N=N, nq=nq, cache=False)
    else:
        m = synth.build_model(synth.MixtureSpec(D=D, n_comp=32, decay=1.2, cluster_dims=16, model_seed=seed))
        X, Q = synth.sample(m, N, 1), synth.sample(m, nq, 2)
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=d, bits=B, nlist=nlist)
    path = os.path.join(tempfile.mkdtemp(), "ix.mrqx")
    ix.export(path)
    orc = oracle.Index.load_export(path, X)
    pos = np.empty(orc.N, dtype=np.int64)
    pos[orc.get("lid")] = np.arange(orc.N)
    return dict(X=X, Q=Q, ix=ix, orc=orc, d=d, B=B, code=orc.get("code"), off=orc.get("off"), pos=pos,
                nx=orc.get("nx"), tx=orc.get("tx"))


@pytest.fixture(scope="module")
def c1():
    env = _env(128, 32, 1, 20000, 64, name="small")
    yield env
    env["ix"].close()


@pytest.fixture(scope="module")
def gist_b1():
    env = _env(960, 128, 1, 10000, 32)
    yield env
    env["ix"].close()


@pytest.fixture(scope="module")
def gist_b4():
    env = _env(960, 128, 4, 10000, 32)
    yield env
    env["ix"].close()


def _compare(env, k, nprobe, prm_kw=None, check_values=True):
    """Run a traced search and compare every record with the oracle; returns statistics."""
    prm_kw = prm_kw or {}
    ix, orc, d, B = env["ix"], env["orc"], env["d"], env["B"]
    ids, dists, pairs, qp, lev, cands = ix.search_trace(env["Q"], k, nprobe, TRACED, **prm_kw)
    prm = oracle.params(**{a: b for a, b in prm_kw.items() if a in ("eps0", "m", "bq", "stage2", "use_ext")})
    bq = prm.bq
    st = defaultdict(int)
    worst = defaultdict(float)
    # ---- pairs: one record per (traced query, probed list), the oracle's probe lists ----
    by_pair = {}
    for t, p in enumerate(pairs):
        key = (int(p["q"]), int(p["list"]))
        if key in by_pair:
            # the nearest list's pair is coded by the seed pass (64 lanes) and by the pair preparation
            # (16 lanes per pair): the two codes are the same bit for bit
            u0 = by_pair[key]
            assert p["phase"] == 0 and pairs[u0]["phase"] == 0, key
            assert pairs[u0].tobytes() == p.tobytes(), key
            assert np.array_equal(qp[u0].view(np.uint32), qp[t].view(np.uint32)) and np.array_equal(lev[u0], lev[t])
            st["seed_pair_twice"] += 1
            continue
        by_pair[key] = t
    oref = {}
    for q in TRACED:
        lists, _ = orc.probe(env["Q"][q], nprobe)
        mine = sorted(j for (qq, j) in by_pair if qq == q)
        assert mine == sorted(lists.tolist()), (q, mine[:5], sorted(lists.tolist())[:5])
        for j in lists.tolist():
            oref[(q, j)] = orc.pair_trace(env["Q"][q], j, prm)
    same_u = {}
    for key, t in by_pair.items():
        p = pairs[t]
        qs, qp_o, u_o, lid, cand = oref[key]
        # the levels are the quantiser of the device's own FP32 q', bit for bit
        u_re, vl_re, dl_re, su_re = oracle.quantize_query_f32(qp[t], bq)
        assert np.array_equal(u_re, lev[t]), key
        assert np.float32(vl_re) == p["vl"] and np.float32(dl_re) == p["delta"] and su_re == p["su"], key
        # ... and close to the oracle's FP64 q'; any level that differs lies at a rounding edge
        err = np.abs(qp[t].astype(np.float64) - qp_o).max()
        worst["qprime"] = max(worst["qprime"], err)
        assert err <= 2e-5, (key, err)
        diff = lev[t].astype(int) != u_o.astype(int)
        st["dims"] += d
        st["level_flips"] += int(diff.sum())
        if diff.any():
            assert np.all(np.abs(lev[t].astype(int) - u_o.astype(int))[diff] == 1), key
            # the oracle's coordinate sits within 1e-5 (in level units) of a half-level boundary
            edge = (qp_o[diff] - float(p["vl"])) / float(p["delta"]) + 0.5
            assert np.all(np.abs(edge - np.round(edge)) <= 2e-5 * (2 ** bq)), (key, edge)
        same_u[key] = not diff.any()
        # the pair's scalars
        nq2 = qs["nq"] ** 2
        scale = nq2 + qs["Tq"] + qs["er"]
        assert abs(p["nq"] - qs["nq"]) <= 1e-5 * max(qs["nq"], 1e-12), key
        assert abs(p["kr"] - (nq2 + qs["Tq"] - float(p["er"]))) <= 1e-5 * scale, key
        assert abs(p["qn2"] - qs["qn2"]) <= 1e-5 * qs["qn2"], key
        assert abs(p["er"] - qs["er"]) <= 2e-3 * max(qs["er"], 1e-12) + 1e-5 * scale, key  # BF16 tail product
        worst["er_rel"] = max(worst["er_rel"], abs(p["er"] - qs["er"]) / max(qs["er"], 1e-12))
    # ---- candidates ----
    ev = defaultdict(dict)  # (kind, phase, q, id) -> record
    for c in cands:
        if c["id"] < 0:
            continue  # padding rows of a 64-row block (never pass)
        key = (int(c["kind"]), int(c["phase"]), int(c["q"]), int(c["id"]))
        assert key not in ev, f"candidate record {key} twice"
        ev[key] = c
    list_of = {}
    for (kind, ph, q, i), c in ev.items():
        if kind in (mrq.TRACE_STAGE1, mrq.TRACE_EXT, mrq.TRACE_STAGE2):
            list_of[(q, i)] = int(c["list"])
    # every candidate of every traced pair got exactly one stage-1 record
    for (q, j), t in by_pair.items():
        n1 = sum(1 for (kind, ph, qq, i) in ev if kind == mrq.TRACE_STAGE1 and qq == q and list_of[(qq, i)] == j)
        assert n1 == int(env["off"][j + 1] - env["off"][j]), (q, j, n1)
    for (kind, ph, q, i), c in ev.items():
        j = list_of.get((q, i))
        if j is None:  # an exact record whose candidate's list is known from its stage records
            continue
        qs, _, _, lid, cand = oref[(q, j)]
        r = int(np.nonzero(lid == i)[0][0])
        p = env["pos"][i]
        code = env["code"][p].astype(np.int64)
        u_dev = lev[by_pair[(q, j)]].astype(np.int64)
        C1 = env["nx"][p] ** 2 + env["tx"][p] + qs["nq"] ** 2 + qs["Tq"]
        tol = 1e-5 * C1
        er = float(pairs[by_pair[(q, j)]]["er"])
        if kind == mrq.TRACE_STAGE1:
            b = (code >> (B - 1)) & 1
            assert c["ip"] == int((b * u_dev).sum()) and c["pc"] == int(b.sum()), (q, i)
            assert c["pc"] == cand["pc"][r]
            st["stage1"] += 1
            if check_values and same_u[(q, j)]:
                for name, dev, ref in (("dis1", float(c["v0"]) + er, cand["dis1"][r]),
                                       ("eb1", c["v1"], cand["eb1"][r]),
                                       ("lb1+er", float(c["v2"]) + er, cand["lb1"][r] + qs["er"])):
                    e = abs(dev - ref) / C1
                    worst[name] = max(worst[name], e)
                    assert e <= 1e-5, (name, q, i, dev, ref, C1)
        elif kind == mrq.TRACE_EXT:
            assert c["ip"] == int((code * u_dev).sum()), (q, i)
            st["ext"] += 1
            if check_values and same_u[(q, j)]:
                for name, dev, ref in (("disB", float(c["v0"]) + er, cand["disB"][r]),
                                       ("ebB", c["v1"], cand["ebB"][r]),
                                       ("lbB+er", float(c["v2"]) + er, cand["lbB"][r] + qs["er"])):
                    e = abs(dev - ref) / C1
                    worst[name] = max(worst[name], e)
                    assert e <= 1e-5, (name, q, i, dev, ref, C1)
        elif kind == mrq.TRACE_STAGE2:
            st["stage2"] += 1
            e = abs(float(c["v0"]) - cand["diso"][r]) / C1
            worst["diso"] = max(worst["diso"], e)
            assert e <= 1e-5, ("diso", q, i, c["v0"], cand["diso"][r], C1)
        elif kind == mrq.TRACE_EXACT:
            st["exact"] += 1
            e = abs(float(c["v0"]) - cand["dis"][r]) / max(cand["dis"][r], 1e-30)
            worst["exact"] = max(worst["exact"], e)
            assert e <= 1e-5, ("exact", q, i, c["v0"], cand["dis"][r])
        # decisions in the batched phases: the next stage's record exists exactly when the bound passed
        nxt = None
        if kind == mrq.TRACE_STAGE1 and ph > 0:
            nxt = mrq.TRACE_EXT if (B > 1 and prm.use_ext) else (mrq.TRACE_STAGE2 if prm.stage2 else None)
        elif kind == mrq.TRACE_EXT and ph > 0:
            nxt = mrq.TRACE_STAGE2 if prm.stage2 else None
        if nxt is not None:
            tau = float(c["v3"])
            passed = (nxt, ph, q, i) in ev
            assert passed == (float(c["v2"]) < tau), (kind, ph, q, i)
            if check_values and same_u[(q, j)]:
                # the oracle's bound with the device's eps_r (its tail coordinates come from the BF16
                # product; eps_r is compared on its own above)
                ref = (cand["lb1"] if kind == mrq.TRACE_STAGE1 else cand["lbB"])[r] + qs["er"] - er
                if ref < tau - tol:
                    assert passed, (kind, q, i, ref, tau)
                elif ref > tau + tol:
                    assert not passed, (kind, q, i, ref, tau)
                else:
                    st["decision_at_edge"] += 1
                st["decisions"] += 1
    # the traced rows are the search's own rows
    for q in TRACED:
        a, b = ix.search(env["Q"][q:q + 1].copy(), k, nprobe, **prm_kw)
        assert np.array_equal(a[0], ids[q]) and np.array_equal(b[0].view(np.uint32), dists[q].view(np.uint32))
    print(f"[gpu] trace k={k} nprobe={nprobe} {prm_kw}: {dict(st)}; worst {dict(worst)}", flush=True)
    assert st["level_flips"] <= max(2, 1e-3 * st["dims"]), st
    return st


def test_trace_c1_default(c1):
    st = _compare(c1, 10, 8)
    assert st["stage1"] > 0 and st["stage2"] > 0 and st["exact"] > 0 and st["decisions"] > 0


def test_trace_c1_bq8_and_no_stage2(c1):
    _compare(c1, 10, 8, dict(bq=8))
    _compare(c1, 10, 8, dict(stage2=False))


def test_trace_c1_without_pruning_reaches_every_stage(c1):
    """Huge eps0 and m: every candidate passes every test, so every candidate's stage-2 value and exact
    distance are traced (the bound values themselves are then dominated by eps_r and not compared)."""
    st = _compare(c1, 10, 4, dict(eps0=1e6, m=1e6), check_values=False)
    assert st["stage2"] + st["exact"] >= st["stage1"]


@pytest.fixture(scope="module")
def deep_split():
    env = _env(128, 64, 1, 20000, 64)  # tail no wider than the leading block: the split exact stage
    yield env
    env["ix"].close()


def test_trace_split_exact_stage(deep_split):
    """d_r = D / 2: exact distances come from dis_o' - 2 <x_r, q_r> (FP32 tail coordinates); every exact record
    is within 1e-5 of the oracle's FP64 distance, and eps_r (from the FP32 tail now) within 1e-5 relative."""
    st = _compare(deep_split, 10, 8)
    assert st["exact"] > 0 and st["stage2"] > 0


def test_trace_d128_b1(gist_b1):
    st = _compare(gist_b1, 10, 6)
    assert st["stage1"] > 0 and st["stage2"] > 0


def test_trace_d128_b4(gist_b4):
    st = _compare(gist_b4, 10, 6)
    assert st["ext"] > 0 and st["stage2"] > 0
    _compare(gist_b4, 10, 6, dict(use_ext=False))
