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


def check_rows(orc_ix, X, Q, ids, dists, k, nprobe, prm, rel=1e-5, risk_rel=1e-4, tie_rel=1e-5,
               ks=None, nprobes=None):
    stats = dict(queries=0, exact_match=0, risk_excused=0, tie_excused=0, probe_tie=0, failures=[])
    for i in range(Q.shape[0]):
        ki = k if ks is None else int(ks[i])
        npi = nprobe if nprobes is None else int(nprobes[i])
        g = np.asarray(ids[i])[:ki]
        gd = np.asarray(dists[i])[:ki]
        stats["queries"] += 1
        valid = g >= 0
        # padding only at the tail
        nv = int(valid.sum())
        if not (np.all(valid[:nv]) and np.all(~valid[nv:]) and np.all(np.isinf(gd[nv:]))):
            stats["failures"].append((i, "padding"))
            continue
        gv = g[:nv]
        if len(set(gv.tolist())) != nv or np.any(gv >= X.shape[0]):
            stats["failures"].append((i, "duplicate or invalid id"))
            continue
        d64 = exact_d64(X, Q[i], gv)
        if not np.allclose(gd[:nv], d64, rtol=rel, atol=1e-30):
            stats["failures"].append((i, f"distance error {np.max(np.abs(gd[:nv] - d64) / np.maximum(d64, 1e-30)):.2e}"))
            continue
        keys = list(zip(gd[:nv].tolist(), gv.tolist()))
        if keys != sorted(keys):
            stats["failures"].append((i, "not sorted"))
            continue
        lists, gl = orc_ix.probe(Q[i], min(npi + 1, orc_ix.nlist))
        probe_tie = npi < orc_ix.nlist and abs(gl[npi] - gl[npi - 1]) <= 1e-4 * max(gl[npi - 1], 1e-30)
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
