"""Pins of the MR-SQ oracle (Appendix A.2, Exp-5; readings S1-S4 of the oracle header), CPU only.

The estimate is checked against a distance computed independently in the original space, the
selection against brute force over the oracle's own per-candidate values, and the method against its
special cases (re-ranking every candidate reduces it to the plain definition of the result).
"""
import numpy as np
import pytest

from paper_2411_06158_amd import synth


def _data(N=2500, D=40, nq=12, seed=21):
    spec = synth.MixtureSpec(D=D, n_comp=12, decay=1.0, cluster_dims=6, model_seed=seed)
    m = synth.build_model(spec)
    return synth.sample(m, N, 1), synth.sample(m, nq, 2)


@pytest.fixture(scope="module")
def sq_index(orc):
    X, Q = _data()
    ix = orc.Index.build(X, d=12, B=1, nlist=16).build_sq8()
    return ix, X, Q


def test_sq8_grid_endpoints_error_and_order(orc):
    """S1, S2: a uniform 8-bit grid per coordinate over its range: the minimum codes to 0, the maximum
    to 255, every value lies within half a step of its reconstruction, and codes follow value order."""
    rng = np.random.default_rng(3)
    x = (rng.standard_normal((4000, 6)) * np.array([1, 2, 5, 0.1, 30, 1])).astype(np.float32)
    x[:, 5] = 1.25                                      # a constant coordinate
    lo, dl = orc.sq8_range(x)
    assert np.array_equal(lo, x.min(0))
    assert np.all(dl[:5] == (x.max(0)[:5] - lo[:5]) / np.float32(255))
    assert dl[5] == 1.0                                 # hi == lo: step 1, every code 0
    u = orc.sq8_encode(x, lo, dl)
    assert np.all(u[:, 5] == 0)
    for i in range(5):
        assert u[np.argmin(x[:, i]), i] == 0 and u[np.argmax(x[:, i]), i] == 255
        rec = lo[i].astype(np.float64) + dl[i].astype(np.float64) * u[:, i]
        assert np.abs(rec - x[:, i]).max() <= 0.5 * dl[i] * (1 + 1e-5)
        o = np.argsort(x[:, i], kind="stable")
        assert np.all(np.diff(u[o, i].astype(int)) >= 0)


def test_sq8_codes_of_built_index_follow_the_grid(orc, sq_index):
    ix, _, _ = sq_index
    xd = ix.get("xd").astype(np.float32)
    lo, dl = orc.sq8_range(xd)
    assert np.array_equal(ix.get("sq_lo"), lo) and np.array_equal(ix.get("sq_delta"), dl)
    assert np.array_equal(ix.get("sq_code"), orc.sq8_encode(xd, lo, dl))


def _unproject(ix, lead, tail):
    """A point of the original space from its PCA coordinates (x = mu + P_p^T x_p, P_p orthogonal)."""
    return ix.get("mu") + np.concatenate([lead, tail]) @ ix.get("Pp")


def test_estimate_is_the_original_space_distance_when_the_query_tail_is_zero(orc, sq_index):
    """S3: with q_r = 0 the estimate is ||xtilde - q||^2 for xtilde = (reconstructed x_d, exact x_r),
    a distance evaluated here in the original space; zeroing the tail of any query lowers every estimate
    by exactly ||q_r||^2."""
    ix, X, Q = sq_index
    d = ix.d
    mu, Pp = ix.get("mu"), ix.get("Pp")
    lo, dl = ix.get("sq_lo").astype(np.float64), ix.get("sq_delta").astype(np.float64)
    code, lid = ix.get("sq_code"), ix.get("lid")
    pos_of = np.empty(ix.N, dtype=np.int64)
    pos_of[lid] = np.arange(ix.N)
    for qi in range(4):
        qp = Pp @ (Q[qi].astype(np.float64) - mu)
        q0 = _unproject(ix, qp[:d], np.zeros(ix.D - d)).astype(np.float32)
        ids, est0, _ = ix.mrsq_estimates(q0, 4)
        q0p = Pp @ (q0.astype(np.float64) - mu)
        r0 = np.linalg.norm(q0p[d:])  # what FP32 rounding of the query leaves of its tail
        for i in range(0, len(ids), 7):
            x = X[ids[i]].astype(np.float64)
            xp = Pp @ (x - mu)
            xt = _unproject(ix, lo + dl * code[pos_of[ids[i]]], xp[d:])
            ref = np.sum((xt - q0.astype(np.float64)) ** 2)
            # the two differ by the cross term -2 <x_r, q_r>, bounded by 2 ||x_r|| ||q_r||
            tol = 2.0 * np.linalg.norm(xp[d:]) * r0 + 1e-10 * max(ref, 1.0)
            assert abs(est0[i] - ref) <= tol, (qi, i)
        # the same lists, the full query: every estimate grows by the query's ||q_r||^2 (up to the
        # change of q_d that rounding the two queries to FP32 leaves, bounded by ||dq|| (2 ||xhat_d -
        # q_d|| + ||dq||) with ||xhat_d - q_d||^2 <= the estimate)
        qf = _unproject(ix, q0p[:d], qp[d:]).astype(np.float32)
        ids_f, est_f, _ = ix.mrsq_estimates(qf, 4)
        qfp = Pp @ (qf.astype(np.float64) - mu)
        dq = np.linalg.norm(qfp[:d] - q0p[:d])
        dt = np.sum(qfp[d:] ** 2) - np.sum(q0p[d:] ** 2)
        assert dt > 1.0 and np.array_equal(ids_f, ids)
        tol = dq * (2.0 * np.sqrt(est0) + dq) + 1e-10 * (est0 + dt)
        assert np.all(np.abs((est_f - est0) - dt) <= tol)


def test_reranking_every_candidate_is_the_plain_definition(orc, sq_index):
    """S4 with R >= the candidate count: the result is the exact k nearest members of the probed lists
    (EXACT-IVF), for any estimate."""
    ix, _, Q = sq_index
    for qi in range(len(Q)):
        ids, est, _ = ix.mrsq_estimates(Q[qi], 3)
        a = ix.search_mrsq(Q[qi], 10, 3, R=len(ids) + 5)
        b = ix.search(Q[qi], 10, 3, mode=orc.EXACT_IVF)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_result_is_the_exact_topk_of_the_r_best_estimates(orc, sq_index):
    """S4 by brute force: sort the candidates by (estimate, id), keep R, sort those by (distance, id)."""
    ix, _, Q = sq_index
    for qi in range(len(Q)):
        for R, k in ((10, 10), (25, 10), (60, 5)):
            ids, est, ex = ix.mrsq_estimates(Q[qi], 4)
            order = np.lexsort((ids, est))[:R]
            keep = order[np.lexsort((ids[order], ex[order]))][:k]
            got_ids, got_d = ix.search_mrsq(Q[qi], k, 4, R=R)
            assert np.array_equal(got_ids, ids[keep]) and np.allclose(got_d, ex[keep], rtol=0, atol=0)


def test_overlap_with_exact_ivf_never_falls_as_r_grows(orc, sq_index):
    """A larger re-ranking range keeps every candidate of a smaller one, so the share of the exact
    result it returns cannot fall (and reaches 1 once every candidate is re-ranked)."""
    ix, _, Q = sq_index
    for qi in range(len(Q)):
        exact = set(ix.search(Q[qi], 10, 4, mode=orc.EXACT_IVF)[0])
        n = len(ix.mrsq_estimates(Q[qi], 4)[0])
        prev = -1
        for R in (10, 12, 16, 24, 40, 80, n):
            got = len(exact & set(ix.search_mrsq(Q[qi], 10, 4, R=R)[0]))
            assert got >= prev
            prev = got
        assert prev == 10


def test_mrsq_rejects_bad_arguments(orc, sq_index):
    ix, _, Q = sq_index
    with pytest.raises(ValueError):
        ix.search_mrsq(Q[0], 10, 4, R=5)                # R < k
    plain = orc.Index.build(*_data(N=600, nq=1)[:1], d=12, B=1, nlist=8)
    with pytest.raises(ValueError):
        plain.mrsq_estimates(Q[0], 2)                   # no MR-SQ codes
