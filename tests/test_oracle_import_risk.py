"""Pins of the oracle's import path and of its risk flags (no GPU needed).

Every GPU parity test searches an index the device exported ("MRQX0001", layout in include/mrq.h) and the
oracle imported with the original vectors, re-deriving each per-vector quantity of Algorithm 1 in FP64
(Section 5.1: x_d, ||x_r||^2, the normalisation factors of Section 4.2).  The parity checker then excuses a
missing result only where the oracle flags one of the pruning bounds of Algorithm 2 as failing for it.
These tests pin both without the device: an index the oracle built itself is written in the export
layout with numpy and read back.
"""
import math
import os

import numpy as np
import pytest

from paper_2411_06158_amd import synth


def _data(N=2500, D=48, seed=17, nq=24, cluster_dims=8):
    spec = synth.MixtureSpec(D=D, n_comp=12, decay=1.0, cluster_dims=cluster_dims, model_seed=seed)
    m = synth.build_model(spec)
    return synth.sample(m, N, 1), synth.sample(m, nq, 2)


def write_export(path, ix):
    """The "MRQX0001" layout of include/mrq.h, field by field, from an oracle-built index (FP64 values
    stored as FP32 where the layout says f32)."""
    N, D, d, B, L = ix.N, ix.D, ix.d, ix.B, ix.nlist
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32).tobytes()  # noqa: E731
    with open(path, "wb") as f:
        f.write(b"MRQX0001")
        f.write(np.int64(N).tobytes())
        f.write(np.array([D, d, B, L], dtype=np.int32).tobytes())
        f.write(f32(ix.get("mu")))
        f.write(f32(ix.get("Pp")))
        f.write(np.ascontiguousarray(ix.get("lam"), dtype=np.float64).tobytes())
        f.write(f32(ix.get("Pr")))
        f.write(f32(ix.get("C")))
        f.write(np.ascontiguousarray(ix.get("off"), dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(ix.get("lid"), dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(ix.get("code"), dtype=np.uint8).tobytes())
        f.write(f32(ix.get("xd")))
        for name in ("nx", "tx", "ax", "xi1", "xiB", "yn"):
            f.write(f32(ix.get(name)))


def _defs_from_file_values(X, ix_file, B):
    """Algorithm 1's per-vector quantities from their definitions, in numpy FP64, on the FP32 matrices the
    file holds: x_p = P_p (x - mu) (Eq 1 with centring), x_d its leading d coordinates, ||x - mu||^2,
    ||x_r||^2 = ||x - mu||^2 - ||x_d||^2, n_x = ||x_d - c||, x' = P_r^T (x_d - c)/n_x (Section 4.2),
    <xbar, x'> for the sign code (xbar_i = (2 b_i - 1)/sqrt(d), b the top bit of the level index) and for
    the B-bit code (y = u - (2^B - 1)/2, xbar = y/||y||)."""
    d = ix_file.d
    mu, Pp, Pr, C = ix_file.get("mu"), ix_file.get("Pp"), ix_file.get("Pr"), ix_file.get("C")
    off, lid, code = ix_file.get("off"), ix_file.get("lid"), ix_file.get("code")
    lists = np.searchsorted(off, np.arange(ix_file.N), side="right") - 1
    xc = X[lid].astype(np.float64) - mu
    xd = xc @ Pp[:d].T
    ax = (xc ** 2).sum(1)
    tx = ax - (xd ** 2).sum(1)
    o = xd - C[lists]
    nx = np.linalg.norm(o, axis=1)
    xp = (o @ Pr) / nx[:, None]
    sign = (code >> (B - 1)) & 1
    xi1 = ((2.0 * sign - 1.0) * xp).sum(1) / math.sqrt(d)
    y = code.astype(np.float64) - ((1 << B) - 1) / 2.0
    yn = np.linalg.norm(y, axis=1)
    xiB = (y * xp).sum(1) / yn
    return dict(xd=xd, ax=ax, tx=tx, nx=nx, xi1=xi1, xiB=xiB, yn=yn)


@pytest.mark.parametrize("B", [1, 4])
def test_import_rederives_every_field(orc, tmp_path, B):
    """orc_import with X: (i) each re-derived field equals its definition evaluated independently on the
    file's own FP32 matrices to 1e-12; (ii) it agrees with the oracle's own FP64 build to the FP32 rounding
    of the stored matrices (a wrong sign bit, a swapped field or a dropped term moves a value by O(1));
    (iii) codes, lists and ids are taken over unchanged; (iv) Algorithm 2 returns the same rows on both."""
    X, Q = _data()
    d = 16
    built = orc.Index.build(X, d=d, B=B, nlist=12)
    path = os.path.join(tmp_path, "ix.mrqx")
    write_export(path, built)
    imp = orc.Index.load_export(path, X)
    for name in ("code", "off", "lid"):
        assert np.array_equal(imp.get(name), built.get(name)), name
    ref = _defs_from_file_values(X, imp, B)
    for name, want in ref.items():
        got = imp.get(name)
        scale = np.abs(ref["ax"]) if name in ("tx", "xd") else np.maximum(np.abs(want), 1e-300)
        if name == "xd":
            scale = np.sqrt(ref["ax"])[:, None]
        assert np.all(np.abs(got - want) <= 1e-12 * scale), (name, float(np.max(np.abs(got - want) / scale)))
    # against the FP64 build: a coordinate or a squared norm is compared on the scale of ||x - mu|| (or
    # its square), the normalisation factors relative to themselves
    rown = np.sqrt(built.get("ax"))
    for name, tol in (("xd", 2e-6), ("ax", 1e-6), ("tx", 2e-6), ("nx", 2e-6), ("xi1", 2e-6), ("xiB", 2e-6),
                      ("yn", 0.0)):
        a, b = imp.get(name), built.get(name)
        if name == "xd":
            scale = rown[:, None]
        elif name in ("ax", "tx"):
            scale = rown ** 2
        elif name == "nx":
            scale = rown
        else:
            scale = np.abs(b)
        err = np.abs(a - b) / scale
        assert err.max() <= tol, (name, float(err.max()))
    prm = orc.params(verify=True)
    for qi in range(Q.shape[0]):
        a, ad = built.search(Q[qi], 10, 4, mode=orc.ALG2, prm=prm)
        b, bd = imp.search(Q[qi], 10, 4, mode=orc.ALG2, prm=prm)
        assert np.array_equal(a, b) and np.array_equal(ad, bd), qi


def test_import_without_vectors_keeps_stored_summaries(orc, tmp_path):
    """Without X the importer takes the stored per-vector summaries as they are (Algorithm 2's precomputed
    inputs): the FP32 values written are the values read."""
    X, _ = _data(N=800)
    built = orc.Index.build(X, d=12, B=2, nlist=6)
    path = os.path.join(tmp_path, "ix.mrqx")
    write_export(path, built)
    raw = orc.Index.load_export(path)
    for name in ("xd", "nx", "tx", "ax", "xi1", "xiB", "yn"):
        assert np.array_equal(raw.get(name), built.get(name).astype(np.float32).astype(np.float64)), name


def test_import_rejects_wrong_shapes(orc, tmp_path):
    X, _ = _data(N=400)
    built = orc.Index.build(X, d=8, B=1, nlist=4)
    path = os.path.join(tmp_path, "ix.mrqx")
    write_export(path, built)
    with pytest.raises(ValueError):
        orc.Index.load_export(path, X[:300])
    with open(path, "r+b") as f:
        f.write(b"MRQX0002")
    with pytest.raises(ValueError):
        orc.Index.load_export(path)


@pytest.mark.parametrize("B,stage2", [(1, True), (4, True), (1, False)])
def test_every_member_missed_by_alg2_is_flagged(orc, B, stage2):
    """A member of the exact top-k of the probed lists that Algorithm 2 drops was pruned by a bound that
    reached tau, and tau never falls below that member's exact distance (tau is at least the final k-th
    distance, which is at least the member's), so one of its bounds is >= its distance: the risk flags
    with margin 0 must mark every such member.  Loose settings (eps0 = 0.25, m = 0.3) make bounds fail
    often enough to exercise this."""
    X, Q = _data(N=3000, nq=40)
    ix = orc.Index.build(X, d=16, B=B, nlist=16)
    prm = orc.params(eps0=0.25, m=0.3, stage2=stage2, verify=True)
    missed = 0
    for qi in range(Q.shape[0]):
        a, _, cnt = ix.search(Q[qi], 10, 5, mode=orc.ALG2, prm=prm, counters=True)
        ex, exd, risk = ix.topk_risk(Q[qi], 10, 5, prm, margin=0.0)
        e2, e2d = ix.search(Q[qi], 10, 5, mode=orc.EXACT_IVF)
        assert np.array_equal(ex, e2) and np.array_equal(exd, e2d)  # the flagged rows are EXACT-IVF's
        for j, m in enumerate(ex.tolist()):
            if m >= 0 and m not in set(a.tolist()):
                missed += 1
                assert risk[j] != 0, (qi, m)
        if cnt["viol1"] + cnt["viol_ext"] * (B > 1) + cnt["viol2"] * stage2 == 0:
            assert not (set(ex.tolist()) - set(a.tolist()))
    assert missed >= 5  # the settings do drop members


@pytest.mark.parametrize("B", [1, 4])
def test_risk_flags_follow_the_bounds(orc, B):
    """Each flag bit is exactly "this bound is >= the member's exact distance minus the margin": bit 1 the
    stage-1 lower bound, bit 2 the B-bit bound, bit 4 the Eq 7 value minus eps_r, read from the per-pair
    trace of the list that holds the member (whose stage values are pinned against Eq 4-7 elsewhere)."""
    X, Q = _data(N=2000, nq=12)
    ix = orc.Index.build(X, d=16, B=B, nlist=10)
    off = ix.get("off")
    lid = ix.get("lid")
    for eps0, m in ((1.9, 3.0), (0.25, 0.3)):
        prm = orc.params(eps0=eps0, m=m)
        for qi in range(Q.shape[0]):
            for margin in (0.0, 0.05):
                ex, exd, risk = ix.topk_risk(Q[qi], 10, 4, prm, margin=margin)
                for j, mid in enumerate(ex.tolist()):
                    if mid < 0:
                        assert risk[j] == 0
                        continue
                    p = int(np.nonzero(lid == mid)[0][0])
                    lst = int(np.searchsorted(off, p, side="right") - 1)
                    qs, _, _, tids, cand = ix.pair_trace(Q[qi], lst, prm)
                    t = int(np.nonzero(tids == mid)[0][0])
                    thr = exd[j] - margin
                    want = (1 if cand["lb1"][t] >= thr else 0)
                    if B > 1:
                        want |= 2 if cand["lbB"][t] >= thr else 0
                    want |= 4 if cand["diso"][t] - qs["er"] >= thr else 0
                    assert risk[j] == want, (qi, mid, risk[j], want)
