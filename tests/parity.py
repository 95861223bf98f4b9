"""Comparison of device search results with the CPU oracle (shared by the GPU tests and smoke).

A device result row for a query is accepted when
  * every returned id is a genuine vector and its distance equals the FP64 exact squared distance
    to within `rel` (relative), rows are sorted by (distance, id), and padding is -1 / +inf;
  * its id set equals the oracle's EXACT-IVF top-k (the plain definition of what the multi-stage
    search returns when its bounds hold), except for members the oracle flags as at risk (one of the
    pruning bounds is within a margin of, or above, the member's exact distance: any correct pruned
    search may drop them), near-ties at the k-th position, and queries whose probe set has a near-tie
    at the nprobe-th list (FP32 vs FP64 centroid distances may pick either list).
"""
from __future__ import annotations

import numpy as np


def exact_d64(X, q, ids):
    return ((X[ids].astype(np.float64) - q.astype(np.float64)) ** 2).sum(1)


def _row_basics(X, q, g, gd, rel):
    """Padding only at the tail, distinct genuine ids, exact FP64 distances within rel, (dis, id) order.
    Returns (ids, distances) of the valid part, or a failure string."""
    valid = g >= 0
    nv = int(valid.sum())
    if not (np.all(valid[:nv]) and np.all(~valid[nv:]) and np.all(np.isinf(gd[nv:]))):
        return "padding"
    gv = g[:nv]
    if len(set(gv.tolist())) != nv or np.any(gv >= X.shape[0]):
        return "duplicate or invalid id"
    d64 = exact_d64(X, q, gv)
    if not np.allclose(gd[:nv], d64, rtol=rel, atol=1e-30):
        return f"distance error {np.max(np.abs(gd[:nv] - d64) / np.maximum(d64, 1e-30)):.2e}"
    keys = list(zip(gd[:nv].tolist(), gv.tolist()))
    if keys != sorted(keys):
        return "not sorted"
    return gv, gd[:nv]


def _probe_tie(orc_ix, q, npi):
    _, gl = orc_ix.probe(q, min(npi + 1, orc_ix.nlist))
    return npi < orc_ix.nlist and abs(gl[npi] - gl[npi - 1]) <= 1e-4 * max(gl[npi - 1], 1e-30)


def check_rows(orc_ix, X, Q, ids, dists, k, nprobe, prm, rel=1e-5, risk_rel=1e-4, tie_rel=1e-5,
               ks=None, nprobes=None):
    stats = dict(queries=0, exact_match=0, risk_excused=0, tie_excused=0, probe_tie=0, failures=[])
    for i in range(Q.shape[0]):
        ki = k if ks is None else int(ks[i])
        npi = nprobe if nprobes is None else int(nprobes[i])
        g = np.asarray(ids[i])[:ki]
        gd = np.asarray(dists[i])[:ki]
        stats["queries"] += 1
        b = _row_basics(X, Q[i], g, gd, rel)
        if isinstance(b, str):
            stats["failures"].append((i, b))
            continue
        gv, _ = b
        nv = len(gv)
        probe_tie = _probe_tie(orc_ix, Q[i], npi)
        _, exd0, _ = orc_ix.topk_risk(Q[i], ki, npi, prm, margin=0.0)
        fin = exd0[np.isfinite(exd0)]
        margin = risk_rel * (float(fin.max()) if fin.size else 1.0)
        ex, exd, risk = orc_ix.topk_risk(Q[i], ki, npi, prm, margin=margin)
        exv = ex[ex >= 0]
        if set(exv.tolist()) == set(gv.tolist()):
            stats["exact_match"] += 1
            continue
        if probe_tie:
            stats["probe_tie"] += 1
            continue
        ex2, exd2 = orc_ix.search(Q[i], ki + 1, npi, mode=0)
        missing = [m for m in exv.tolist() if m not in set(gv.tolist())]
        pos = {int(m): j for j, m in enumerate(ex.tolist())}
        near_tie = len(exv) == ki and ex2[ki] >= 0 and abs(exd2[ki] - exd2[ki - 1]) <= tie_rel * exd2[ki - 1]
        ok = True
        used_risk = False
        for m in missing:
            j = pos[int(m)]
            if risk[j]:
                used_risk = True
            elif near_tie and j >= ki - 1:
                pass
            else:
                ok = False
        if not ok:
            stats["failures"].append((i, f"missing {missing} (risk {risk.tolist()})"))
            continue
        stats["risk_excused" if used_risk else "tie_excused"] += 1
    return stats


def check_mrsq_rows(orc_ix, X, Q, ids, dists, k, nprobe, R, rel=1e-5, est_rel=1e-5, tie_rel=1e-5, ks=None,
                    nprobes=None):
    """MR-SQ rows (re-ranking range R).  Besides the checks of every row (padding, genuine ids, exact
    distances, order), the id set must equal the oracle's (the k nearest by exact distance of the R
    candidates with the smallest (estimate, id)), unless the selection boundary is ambiguous at FP32
    precision: then every returned id has an oracle estimate at most est_rel * (largest estimate of the
    query) above the R-th smallest, and every candidate clearly inside the range (that much below it)
    whose exact distance is below the row's k-th is returned.  Queries with a near-tie at the nprobe-th
    list are excused (FP32 vs FP64 centroid distances)."""
    stats = dict(queries=0, exact_match=0, boundary_excused=0, probe_tie=0, failures=[])
    for i in range(Q.shape[0]):
        ki = k if ks is None else int(ks[i])
        npi = nprobe if nprobes is None else int(nprobes[i])
        g = np.asarray(ids[i])[:ki]
        gd = np.asarray(dists[i])[:ki]
        stats["queries"] += 1
        b = _row_basics(X, Q[i], g, gd, rel)
        if isinstance(b, str):
            stats["failures"].append((i, b))
            continue
        gv, gdv = b
        oid, _ = orc_ix.search_mrsq(Q[i], ki, npi, R)
        if set(oid[oid >= 0].tolist()) == set(gv.tolist()):
            stats["exact_match"] += 1
            continue
        if _probe_tie(orc_ix, Q[i], npi):
            stats["probe_tie"] += 1
            continue
        cid, est, ex = orc_ix.mrsq_estimates(Q[i], npi)
        order = np.lexsort((cid, est))
        e_r = est[order[min(R, len(cid)) - 1]]
        tol = est_rel * float(np.max(np.abs(est)))
        pos = {int(c): j for j, c in enumerate(cid.tolist())}
        if any(int(x) not in pos or est[pos[int(x)]] > e_r + tol for x in gv.tolist()):
            stats["failures"].append((i, "a returned id lies outside the re-ranking range"))
            continue
        kth = gdv[-1] if len(gv) == ki else np.inf
        must = cid[(est < e_r - tol) & (ex < kth * (1.0 - tie_rel))]
        if not set(must.tolist()) <= set(gv.tolist()):
            stats["failures"].append((i, f"missing {sorted(set(must.tolist()) - set(gv.tolist()))[:5]}"))
            continue
        stats["boundary_excused"] += 1
    return stats
