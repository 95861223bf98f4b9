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


def _check_one(orc_ix, X, q, g, gd, ki, npi, prm, rel, risk_rel, tie_rel):
    """One row: (category, detail); categories as in check_rows."""
    b = _row_basics(X, q, g, gd, rel)
    if isinstance(b, str):
        return "failure", b
    gv, _ = b
    _, exd0, risk0 = orc_ix.topk_risk(q, ki, npi, prm, margin=0.0)
    fin = exd0[np.isfinite(exd0)]
    margin = risk_rel * (float(fin.max()) if fin.size else 1.0)
    ex, exd, risk = orc_ix.topk_risk(q, ki, npi, prm, margin=margin)
    exv = ex[ex >= 0]
    if set(exv.tolist()) == set(gv.tolist()):
        return "exact_match", None
    if _probe_tie(orc_ix, q, npi):
        return "probe_tie", None
    ex2, exd2 = orc_ix.search(q, ki + 1, npi, mode=0)
    got = set(gv.tolist())
    missing = [m for m in exv.tolist() if m not in got]
    pos = {int(m): j for j, m in enumerate(ex.tolist())}
    near_tie = len(exv) == ki and ex2[ki] >= 0 and abs(exd2[ki] - exd2[ki - 1]) <= tie_rel * exd2[ki - 1]
    hard = margin_only = False
    for m in missing:
        j = pos[int(m)]
        if risk0[j]:
            hard = True        # an oracle bound of this member is at or above its exact distance
        elif risk[j]:
            margin_only = True  # a bound within the FP32 margin below its exact distance
        elif near_tie and j >= ki - 1:
            pass
        else:
            return "failure", f"missing {missing} (risk {risk.tolist()})"
    if hard:
        # the oracle's own Algorithm 2 with verification logs the same kind of bound failure for this query
        _, _, cnt = orc_ix.search(q, ki, npi, mode=1, prm=_verify(prm), counters=True)
        if cnt["viol1"] + cnt["viol_ext"] + cnt["viol2"] == 0:
            return "failure", f"missing {missing}: flagged at risk but the oracle logs no bound violation"
        return "risk_hard", None
    return ("risk_margin", None) if margin_only else ("tie_excused", None)


def _verify(prm):
    import ctypes

    v = type(prm)()
    ctypes.memmove(ctypes.addressof(v), ctypes.addressof(prm), ctypes.sizeof(prm))
    v.verify = 1
    return v


def check_rows(orc_ix, X, Q, ids, dists, k, nprobe, prm, rel=1e-5, risk_rel=1e-4, tie_rel=1e-5,
               ks=None, nprobes=None, threads=8):
    """Check every row (see the module docstring); rows run on `threads` host threads (the oracle's
    calls release the interpreter lock).  Returns counts per category:
      exact_match   the id set equals the oracle's EXACT-IVF top-k
      risk_hard     a missing member has an oracle bound (Eq 5 + Eq 6 stage 1, B-bit or Eq 7) at or above
                    its exact distance: a failure of the paper's bound, which the oracle's Algorithm 2 in
                    verification mode also logs for the query (checked)
      risk_margin   a missing member's bound is within risk_rel (relative) below its exact distance: FP32
                    vs FP64 rounding of the bound can put it on either side
      tie_excused   the only differences are at a near-tie of the k-th distance
      probe_tie     the nprobe-th and next lists are nearly equidistant (FP32 vs FP64 may take either)
    and `failures` [(row, message)]."""
    from concurrent.futures import ThreadPoolExecutor

    n = Q.shape[0]

    def one(i):
        ki = k if ks is None else int(ks[i])
        npi = nprobe if nprobes is None else int(nprobes[i])
        return _check_one(orc_ix, X, Q[i], np.asarray(ids[i])[:ki], np.asarray(dists[i])[:ki], ki, npi, prm,
                          rel, risk_rel, tie_rel)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        res = list(ex.map(one, range(n)))
    stats = dict(queries=n, exact_match=0, risk_hard=0, risk_margin=0, tie_excused=0, probe_tie=0, failures=[])
    for i, (cat, detail) in enumerate(res):
        if cat == "failure":
            stats["failures"].append((i, detail))
        else:
            stats[cat] += 1
    return stats


def soft_excuses(st) -> int:
    """Rows excused for rounding reasons rather than a failed bound (margin, k-th tie, probe tie)."""
    return st["risk_margin"] + st["tie_excused"] + st["probe_tie"]


def assert_rows(st, what=""):
    """No failures, and rounding excuses in at most max(2, 2 %) of the rows; bound failures (risk_hard) are
    the paper's own and are reported, not capped."""
    print(f"[parity] {what}: {dict((a, b) for a, b in st.items() if a != 'failures')}", flush=True)
    assert not st["failures"], st["failures"][:5]
    assert soft_excuses(st) <= max(2, 0.02 * st["queries"]), st


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
