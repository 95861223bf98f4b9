#!/usr/bin/env python3
"""Benchmark of the batched MRQ search on one MI355X.

Metric: queries per second of the batched search at the smallest nprobe whose recall@10 against
exact brute-force ground truth is >= 0.95, on the GIST-shaped synthetic workload (N = 1,000,000,
D = 960, 10,000 queries, nlist = 4,096, d_r = 128, 1-bit codes, k = 10).  A step is one batched
search of all queries (projection, probe, query codes, seed pass, phased scans, top-k) with the
index and the queries resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SEARCH_SOURCES = ["paper_2411_06158_amd/csrc/mrq_search.hip", "paper_2411_06158_amd/csrc/mrq_internal.h"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def ground_truth(torch, Xd, Qd, k, extra=32, chunk=1024):
    """Exact top-k (ties -> smaller id): FP32 distance tiles on the GPU pick k + extra candidates,
    which are re-scored in FP64.  A distance tile stays within 2^28 floats (1 GiB): tiles above 4 GiB
    (107 x 10M and larger) have returned wrong top-k rows on this stack."""
    xn = (Xd * Xd).sum(1)
    chunk = max(1, min(chunk, (1 << 28) // Xd.shape[0]))
    out = []
    for s in range(0, Qd.shape[0], chunk):
        q = Qd[s:s + chunk]
        d = xn[None, :] - 2.0 * (q @ Xd.T)
        cand = torch.topk(d, k + extra, dim=1, largest=False).indices
        cand, _ = torch.sort(cand, dim=1)
        dd = ((Xd[cand].double() - q.double()[:, None, :]) ** 2).sum(-1)
        order = torch.argsort(dd, dim=1, stable=True)
        out.append(torch.gather(cand, 1, order)[:, :k])
        del d, dd
    return torch.cat(out).cpu().numpy()


def counter_traffic(tag, kernel):
    """HBM bytes per launch of `kernel` on workload `tag` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summaries under profiles/, or None when there is none or the search sources have changed
    since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    for p in SEARCH_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    src = h.hexdigest()[:16]
    path = os.path.join(ROOT, "profiles", f"{kernel}_{tag}.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-record:"):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if kv.get("workload") == tag and kv.get("kernel") == kernel and kv.get("source") == src:
                    return float(kv["bytes_per_launch"])
    return None


def recall(ids, gt, k):
    import numpy as np
    hit = 0
    for a, b in zip(ids[:, :k], gt[:, :k]):
        hit += len(set(a.tolist()) & set(b.tolist()))
    return hit / (gt.shape[0] * k)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gist1m")
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--nlist", type=int, default=4096)
    ap.add_argument("--d", type=int, default=128)
    ap.add_argument("--bits", type=int, default=1)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--nprobe", type=int, default=0, help="fixed nprobe (0 = smallest reaching the recall)")
    ap.add_argument("--target-recall", type=float, default=0.95)
    ap.add_argument("--per-query", type=int, default=200, help="queries timed on the per-query path")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle CPU-baseline time budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true", help="skip GT/sweep/baselines (profiler runs)")
    ap.add_argument("--group", type=int, default=0,
                    help="queries per scan work item (16, 32 or 64); with --phase-growth skips the autotuner")
    ap.add_argument("--phase-growth", type=int, default=0,
                    help="probe-rank phase growth (2, 4 or 8); with --group skips the autotuner")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: Poisson arrivals on the embedding-shaped index")
    ap.add_argument("--rates", default="5000,10000,20000,50000", help="--serve: arrival rates (queries/s)")
    ap.add_argument("--requests", type=int, default=20000, help="--serve: requests per rate")
    ap.add_argument("--max-slots", type=int, default=512, help="--serve: queries per batch at most")
    ap.add_argument("--mem-budget", type=float, default=4.0, help="--serve: device GiB for the batch slots")
    ap.add_argument("--mrsq", default="",
                    help="comma-separated d_r values: MR-SQ (8-bit scalar codes of the leading d_r dims, exact "
                         "re-ranking of --rerank candidates; d_r = D is plain SQ) instead of the headline run")
    ap.add_argument("--rerank", type=int, default=500, help="--mrsq: candidates re-ranked per query")
    ap.add_argument("--sweep-d", default="",
                    help="comma-separated d_r values: QPS at the target recall per projection dimension "
                         "(Exp-4 grid) instead of the headline measurement")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this search path runs on a single MI355X "
              "and reports single-GPU throughput; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2411_06158_amd as mrq
    from paper_2411_06158_amd import synth

    torch.backends.cuda.matmul.allow_tf32 = False
    dev = torch.device("cuda:0")
    if args.serve:
        serve_main(args, np, torch, mrq, synth, dev)
        return
    if args.sweep_d:
        sweep_d_main(args, np, torch, mrq, synth, dev)
        return
    if args.mrsq:
        mrsq_main(args, np, torch, mrq, synth, dev)
        return
    t0 = time.time()
    X, Q, spec = synth.workload(args.workload, N=args.N, nq=args.nq)
    N, D = X.shape
    nq = Q.shape[0]
    log(f"data {N}x{D}, {nq} queries in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    torch.cuda.synchronize()
    t1 = time.time()
    ix = mrq.Index.build(Xd, d_r=args.d, bits=args.bits, nlist=args.nlist)
    build_s = time.time() - t1
    log(f"build {build_s:.1f}s, index {ix.device_bytes / 2**30:.2f} GiB")

    k = args.k
    ids_buf = torch.empty((nq, k), dtype=torch.int64, device=dev)
    d_buf = torch.empty((nq, k), dtype=torch.float32, device=dev)

    def run(nprobe, counters=None, mode=mrq.MRQ_BATCHED, Qs=None, ib=None, db=None):
        o = mrq.search_opts(mode=mode, counters=counters, group=args.group, phase_growth=args.phase_growth)
        Qs = Qd if Qs is None else Qs
        return ix.search(Qs, k, nprobe, ids=ids_buf if ib is None else ib, dists=d_buf if db is None else db,
                         opts=o)

    chosen, rec_at = args.nprobe, None
    sweep = []
    if not args.profile_only:
        t2 = time.time()
        gt = ground_truth(torch, Xd, Qd, k)
        log(f"ground truth {time.time() - t2:.1f}s")
        # the smallest nprobe reaching the target: a coarse grid, the autotuner at its first value reaching
        # the target, then (with the tuned schedule) every value between the last one below the target and
        # that one
        cands = [args.nprobe] if args.nprobe else [8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]

        def try_np(npb):
            run(npb)
            torch.cuda.synchronize()
            r = recall(ids_buf.cpu().numpy(), gt, k)
            sweep.append((npb, r))
            log(f"nprobe {npb}: recall@{k} {r:.4f}")
            return r

        prev = 0
        for npb in cands:
            if npb > args.nlist:
                break
            chosen, rec_at = npb, try_np(npb)
            if rec_at >= args.target_recall:
                break
            prev = npb
    if not chosen:
        chosen = 64

    if args.calib_copy:  # a copy kernel of known size: 1 GiB read + 1 GiB written
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the autotuner picks the scan schedule (query-group size, phase growth) on this batch; the group size
    # never changes a result, the phase growth only where an error bound fails
    if args.group and args.phase_growth:
        group, growth = args.group, args.phase_growth
        log(f"query group {group}, phase growth {growth}")
    else:
        group, growth = ix.tune(Qd, k, chosen)
        log(f"autotuned query group {group}, phase growth {growth}")
    if not args.profile_only:
        if chosen is not None and rec_at is not None and rec_at >= args.target_recall:
            for fine in list(range(prev + 1, chosen)) + [chosen] if not args.nprobe else [chosen]:
                rf = try_np(fine)
                if rf >= args.target_recall or fine == chosen:
                    chosen, rec_at = fine, rf
                    break

    # timed region: W warm-up steps, then K plain searches (the throughput); then K more searches, not
    # timed, with per-kernel HIP events and device counters (the kernel breakdown and the roofline)
    for _ in range(args.warmup):
        run(chosen)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        run(chosen)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    cnt = torch.zeros(8, dtype=torch.int64, device=dev)
    ix.timing_enable(True, reset=True)
    ti = time.perf_counter()
    for _ in range(args.steps):
        run(chosen, counters=cnt)
    torch.cuda.synchronize()
    ms_instr = 1e3 * (time.perf_counter() - ti) / args.steps
    ix.timing_enable(False, reset=False)
    kt = ix.timing()
    cnt = cnt.cpu().numpy() / args.steps
    qps = nq * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    log(f"batched: {qps:,.0f} QPS, {ms_step:.2f} ms/step at nprobe {chosen} "
        f"({ms_instr:.2f} ms/step with per-step events and device counters)")
    log("kernel ms/step: " + ", ".join(f"{n}={v[0] / args.steps:.3f}" for n, v in kt.items()))

    # roofline: algorithmic bytes (and multiply-add ops) per launch of each batched-phase kernel, from the
    # device stage counters; the kernel with the largest device time is reported as dominant
    d, B, bq = args.d, args.bits, 4
    d4 = (d + 3) // 4 * 4
    scanned, p1, pext, p2 = (float(x) for x in cnt[:4])
    pairs_scan = nq * (chosen - 1)
    KP = 64 * ((d + 63) // 64)
    kern = {
        # stage 1 (codes + factors per candidate, record + query bytes per pair), B-bit refinement per
        # stage-1 survivor, Eq 7 per refined survivor (x_d row + a_x), 8 B per exact-stage candidate written
        "scan": dict(bytes=scanned * (d / 8 + 12) + pairs_scan * (48 + KP)
                     + (p1 * ((B - 1) * d / 8 + 12) if B > 1 else 0) + pext * (4 * d4 + 4) + p2 * 8,
                     ops=scanned * 2 * d + pext * 2 * d),
        "exact": dict(bytes=p2 * (8 + 4 * D), ops=p2 * 3 * D),
    }
    rows = {}
    for name, kb in kern.items():
        ms_tot, launches = kt.get(name, (0.0, 0))
        if launches == 0 or ms_tot <= 0:
            continue
        per_ms = ms_tot / launches
        per_launch_bytes = kb["bytes"] / (launches / args.steps)
        per_launch_ops = kb["ops"] / (launches / args.steps)
        rows[name] = dict(ms_per_step=ms_tot / args.steps, launch_ms=per_ms,
                          gbs=per_launch_bytes / (per_ms * 1e-3) / 1e9,
                          tops=per_launch_ops / (per_ms * 1e-3) / 1e12,
                          bytes_per_launch=per_launch_bytes)
    dom = max(rows, key=lambda n: rows[n]["ms_per_step"]) if rows else None
    if dom:
        r = rows[dom]
        # both kernels stream per-candidate data: the HBM roof bounds them (the scan's matrix-core work,
        # int8 stage 1 and FP32 stage 2, is far below the int8 / FP32 MFMA peaks; see per_kernel TOP/s)
        roof = {"bound": "hbm", "achieved": round(r["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(r["gbs"] / HBM_PEAK_GBS, 4)}
        tag = f"{args.workload}_d{args.d}_b{args.bits}_np{chosen}_k{k}"
        kname = {"scan": "k_scan", "exact": "k_exact"}[dom]
        traffic = counter_traffic(tag, kname)
        roof.update({"kernel": kname, "traffic": None if traffic is None else round(traffic),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "algorithmic_bytes_per_launch": round(r["bytes_per_launch"]),
                     "launch_ms": round(r["launch_ms"], 4),
                     "per_kernel": {n: {"ms_per_step": round(v["ms_per_step"], 4), "GB/s": round(v["gbs"], 1),
                                        "TOP/s": round(v["tops"], 3)} for n, v in rows.items()}})
    else:
        roof = None

    out_extra = {}
    if not args.profile_only:
        # the plain per-query GPU path at the same nprobe
        npq = min(args.per_query, nq)
        Qs = Qd[:npq].contiguous()
        ib = torch.empty((npq, k), dtype=torch.int64, device=dev)
        db = torch.empty((npq, k), dtype=torch.float32, device=dev)
        run(chosen, mode=mrq.MRQ_PER_QUERY, Qs=Qs, ib=ib, db=db)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        run(chosen, mode=mrq.MRQ_PER_QUERY, Qs=Qs, ib=ib, db=db)
        torch.cuda.synchronize()
        pq_qps = npq / (time.perf_counter() - tp)
        same = bool(torch.equal(ib, ids_buf[:npq]))
        log(f"per-query path: {pq_qps:,.0f} QPS (ids identical to batched: {same})")
        out_extra.update({"per_query_qps": round(pq_qps, 1), "speedup_vs_per_query": round(qps / pq_qps, 1),
                          "per_query_matches_batched": same})

    cpu = None
    if not args.profile_only and not args.no_cpu_baseline:
        import oracle
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "bench.mrqx")
            ix.export(path)
            orc = oracle.Index.load_export(path).attach(X)
            prm = oracle.params()
            n, tc = 0, time.perf_counter()
            tot = {}
            while n < nq and time.perf_counter() - tc < args.cpu_seconds:
                _, _, c = orc.search(Q[n], k, chosen, mode=oracle.ALG2, prm=prm, counters=True)
                for key_, v in c.items():
                    tot[key_] = tot.get(key_, 0) + v
                n += 1
            el = time.perf_counter() - tc
            cpu = {"value": round(n / el, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
                   "sample": f"first {n} queries, single-threaded FP64 Algorithm 2 on the exported index, "
                             f"nprobe {chosen}, k {k}",
                   "oracle_pass_rates": {"stage1": round(tot["pass1"] / max(tot["scanned"], 1), 5),
                                         "stage2_exact": round(tot["pass2"] / max(tot["scanned"], 1), 6),
                                         "scanned_per_query": round(tot["scanned"] / max(n, 1), 1)}}
            log(f"cpu oracle: {cpu['value']} QPS over {n} queries")

    res = {
        "metric": "QPS at recall@10=0.95 (1 GPU, batched vs per-query); scan HBM GB/s vs peak",
        "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={N} D={D} nq={nq} nlist={args.nlist} d_r={args.d} "
                               f"bits={args.bits} k={k}",
                   "N": N, "D": D, "nq": nq, "nlist": args.nlist, "d_r": args.d, "bits": args.bits, "k": k,
                   "nprobe": chosen, "recall_at_10": None if rec_at is None else round(rec_at, 4),
                   "query_group": group, "phase_growth": growth,
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "build_s": round(build_s, 2),
        "kernel_ms_per_step": {n: round(v[0] / args.steps, 4) for n, v in kt.items()},
        "ms_per_step_instrumented": round(ms_instr, 4),
        "pass_rates": {"stage1": round(p1 / max(scanned, 1), 5), "ext": round(pext / max(scanned, 1), 5),
                       "stage2_exact": round(p2 / max(scanned, 1), 6),
                       "seed_scanned_per_query": round(float(cnt[4]) / nq, 1),
                       "seed_exact_per_query": round(float(cnt[7]) / nq, 1),
                       "exact_per_query": round(p2 / nq, 1),
                       "scanned_per_query": round(scanned / nq, 1)},
        "nprobe_sweep": sweep,
    }
    res.update(out_extra)
    print(json.dumps(res), flush=True)
    ix.close()


def sweep_d_main(args, np, torch, mrq, synth, dev):
    """Exp-4 (Section 6, the choice of d): for each projection dimension d_r of --sweep-d, build the index
    of --workload, find the smallest nprobe whose recall@k reaches --target-recall and time the batched
    search there (query group from the tuner); Eq 8's own choice of d_r for the same data is reported
    beside the grid."""
    X, Q, _ = synth.workload(args.workload, N=args.N, nq=args.nq)
    N, D = X.shape
    nq, k = Q.shape[0], args.k
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    gt = ground_truth(torch, Xd, Qd, k)
    ix = mrq.Index.build(Xd, d_r=0, bits=args.bits, nlist=args.nlist)
    eq8 = ix.d
    ix.close()
    log(f"Eq 8 chooses d_r = {eq8}")
    ids_buf = torch.empty((nq, k), dtype=torch.int64, device=dev)
    d_buf = torch.empty((nq, k), dtype=torch.float32, device=dev)
    rows = []
    for d in [int(v) for v in args.sweep_d.split(",") if v]:
        if d < 2 or d > D:
            continue
        t1 = time.time()
        ix = mrq.Index.build(Xd, d_r=d, bits=args.bits, nlist=args.nlist)
        build_s = time.time() - t1
        chosen, rec = None, None
        for npb in [8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]:
            if npb > args.nlist:
                break
            ix.search(Qd, k, npb, ids=ids_buf, dists=d_buf)
            torch.cuda.synchronize()
            chosen, rec = npb, recall(ids_buf.cpu().numpy(), gt, k)
            if rec >= args.target_recall:
                break
        group, growth = ix.tune(Qd, k, chosen)
        for _ in range(args.warmup):
            ix.search(Qd, k, chosen, ids=ids_buf, dists=d_buf)
        torch.cuda.synchronize()
        ts = time.perf_counter()  # plain searches for the throughput, then an instrumented pass
        for _ in range(args.steps):
            ix.search(Qd, k, chosen, ids=ids_buf, dists=d_buf)
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        ix.timing_enable(True, reset=True)
        for _ in range(args.steps):
            ix.search(Qd, k, chosen, ids=ids_buf, dists=d_buf)
        torch.cuda.synchronize()
        ix.timing_enable(False, reset=False)
        kt = ix.timing()
        row = {"d_r": d, "nprobe": chosen, "recall_at_k": round(rec, 4), "qps": round(nq * args.steps / el, 1),
               "query_group": group, "phase_growth": growth, "build_s": round(build_s, 2),
               "index_gib": round(ix.device_bytes / 2**30, 3),
               "kernel_ms_per_step": {n: round(v[0] / args.steps, 4) for n, v in kt.items()}}
        log(f"d_r {d}: nprobe {chosen} recall {rec:.4f} {row['qps']:,.0f} QPS")
        rows.append(row)
        ix.close()
    print(json.dumps({"metric": f"QPS at recall@{k}={args.target_recall} vs d_r (1 GPU)", "unit": "queries/s",
                      "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"{args.workload}: N={N} D={D} nq={nq} nlist={args.nlist} "
                                             f"bits={args.bits} k={k}", "steps": args.steps},
                      "eq8_d_r": eq8, "grid": rows}), flush=True)


def mrsq_main(args, np, torch, mrq, synth, dev):
    """Exp-5 (Appendix A.2): MR-SQ, the projection and split of MRQ applied to 8-bit scalar quantisation,
    against plain SQ (d_r = D).  For each d_r of --mrsq: build the index with its MR-SQ codes, find the
    smallest nprobe whose recall@k reaches --target-recall with --rerank candidates re-ranked per query,
    and time the batched search there.  Also reports the MRQ search of the same index at its own
    smallest nprobe for comparison."""
    X, Q, _ = synth.workload(args.workload, N=args.N, nq=args.nq)
    N, D = X.shape
    nq, k, R = Q.shape[0], args.k, args.rerank
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    gt = ground_truth(torch, Xd, Qd, k)
    ids_buf = torch.empty((nq, k), dtype=torch.int64, device=dev)
    d_buf = torch.empty((nq, k), dtype=torch.float32, device=dev)
    cnt = torch.zeros(8, dtype=torch.int64, device=dev)

    def measure(ix, opts_kw):
        chosen, rec = None, None
        for npb in [8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]:
            if npb > args.nlist:
                break
            ix.search(Qd, k, npb, ids=ids_buf, dists=d_buf, **opts_kw)
            torch.cuda.synchronize()
            chosen, rec = npb, recall(ids_buf.cpu().numpy(), gt, k)
            if rec >= args.target_recall:
                break
        cnt.zero_()
        ix.search(Qd, k, chosen, ids=ids_buf, dists=d_buf, counters=cnt, **opts_kw)
        for _ in range(args.warmup):
            ix.search(Qd, k, chosen, ids=ids_buf, dists=d_buf, **opts_kw)
        torch.cuda.synchronize()
        ts = time.perf_counter()  # plain searches for the throughput, then an instrumented pass
        for _ in range(args.steps):
            ix.search(Qd, k, chosen, ids=ids_buf, dists=d_buf, **opts_kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        ix.timing_enable(True, reset=True)
        for _ in range(args.steps):
            ix.search(Qd, k, chosen, ids=ids_buf, dists=d_buf, **opts_kw)
        torch.cuda.synchronize()
        ix.timing_enable(False, reset=False)
        c = cnt.cpu().numpy()
        return {"nprobe": chosen, "recall_at_k": round(rec, 4), "qps": round(nq * args.steps / el, 1),
                "ms_per_step": round(1e3 * el / args.steps, 4),
                "scanned_per_query": round(float(c[0]) / nq, 1), "exact_per_query": round(float(c[3]) / nq, 1),
                "kernel_ms_per_step": {n: round(v[0] / args.steps, 4) for n, v in ix.timing().items()}}

    rows = []
    for d in [int(v) for v in args.mrsq.split(",") if v]:
        if d < 2 or d > D:
            continue
        ix = mrq.Index.build(Xd, d_r=d, bits=args.bits, nlist=args.nlist, sq8=True)
        r = {"d_r": d, "method": "SQ" if d == D else "MR-SQ", "rerank": R}
        r.update(measure(ix, dict(method=mrq.MRQ_METHOD_MRSQ, rerank=R)))
        kt = r["kernel_ms_per_step"]
        if kt.get("sq_scan"):
            # estimate scan: per candidate the d_r code bytes + A_x, one FP32 estimate written
            dq = (d + 15) // 16 * 16
            r["sq_scan_GBps"] = round(r["scanned_per_query"] * nq * (dq + 4 + 4) / (kt["sq_scan"] * 1e-3) / 1e9, 1)
        log(f"{r['method']} d_r {d}: nprobe {r['nprobe']} recall {r['recall_at_k']:.4f} {r['qps']:,.0f} QPS")
        rows.append(r)
        if d < D:
            m = {"d_r": d, "method": "MRQ"}
            m.update(measure(ix, dict(method=mrq.MRQ_METHOD_MRQ)))
            log(f"MRQ d_r {d}: nprobe {m['nprobe']} recall {m['recall_at_k']:.4f} {m['qps']:,.0f} QPS")
            rows.append(m)
        ix.close()
    print(json.dumps({"metric": f"QPS at recall@{k}={args.target_recall}: MR-SQ vs SQ (1 GPU)", "unit": "queries/s",
                      "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"{args.workload}: N={N} D={D} nq={nq} nlist={args.nlist} k={k}",
                                 "steps": args.steps, "rerank": R},
                      "rows": rows}), flush=True)


def serve_main(args, np, torch, mrq, synth, dev):
    """Continuous batching under Poisson arrivals: the embedding-shaped index (N = 2,000,000, D = 1,536,
    d_r = 256, 4-bit codes, nlist = 4,096), requests drawn from its 20,000 queries with k in {10, 50, 100}
    and nprobe in {16, 32, 64}; per rate: achieved QPS, p50 / p99 latency (arrival to completion, as the
    server measures it) and recall@10 of the answers against exact brute force."""
    import ctypes as C
    t0 = time.time()
    X, Q, _ = synth.workload("openai2m")
    log(f"data {X.shape[0]}x{X.shape[1]}, {Q.shape[0]} queries in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    t1 = time.time()
    ix = mrq.Index.build(Xd, d_r=256, bits=4, nlist=4096)
    log(f"build {time.time() - t1:.1f}s, index {ix.device_bytes / 2**30:.2f} GiB")
    gt = ground_truth(torch, Xd, torch.from_numpy(Q).to(dev), 10)
    del Xd
    torch.cuda.empty_cache()
    L = mrq.lib()
    rng = np.random.default_rng(5005)
    out = []
    for rate in [float(r) for r in args.rates.split(",")]:
        R = args.requests
        qi = rng.integers(0, Q.shape[0], R)
        ks = rng.choice(np.array([10, 50, 100], np.int32), R)
        nps = rng.choice(np.array([16, 32, 64], np.int32), R)
        arrive = np.cumsum(rng.exponential(1.0 / rate, R))
        srv = C.c_void_p()
        budget = int(args.mem_budget * (1 << 30))
        if L.mrq_server_create(ix._h, C.c_size_t(budget), args.max_slots, None, C.byref(srv)) != mrq.MRQ_OK:
            raise mrq.MRQError(L.mrq_last_error().decode())
        cap = 4096
        rid = np.zeros(cap, np.uint64)
        kk = np.zeros(cap, np.int32)
        ids = np.zeros((cap, 100), np.int64)
        dd = np.zeros((cap, 100), np.float32)
        lat = np.zeros(cap, np.float64)
        lat_all = np.zeros(R)
        hit = np.zeros(R)
        Qc = np.ascontiguousarray(Q)
        late = 0.0
        i, done = 0, 0
        ts = time.perf_counter()
        while done < R:
            now = time.perf_counter() - ts
            while i < R and arrive[i] <= now:
                late = max(late, now - arrive[i])
                if L.mrq_server_submit(srv, C.c_uint64(i), Qc[qi[i]].ctypes.data, int(ks[i]), int(nps[i])) != 0:
                    raise mrq.MRQError(L.mrq_last_error().decode())
                i += 1
            got = L.mrq_server_poll(srv, rid.ctypes.data, kk.ctypes.data, ids.ctypes.data, dd.ctypes.data, 100, cap,
                                    lat.ctypes.data)
            for j in range(got):
                r = int(rid[j])
                lat_all[r] = lat[j]
                hit[r] = len(set(ids[j, :10].tolist()) & set(gt[qi[r], :10].tolist())) / 10.0
            done += got
        span = time.perf_counter() - ts
        L.mrq_server_destroy(srv)
        row = {"rate": rate, "requests": R, "qps": round(R / span, 1),
               "p50_ms": round(float(np.percentile(lat_all, 50)), 3),
               "p99_ms": round(float(np.percentile(lat_all, 99)), 3),
               "recall_at_10": round(float(hit.mean()), 4), "max_submit_lag_ms": round(float(1e3 * late), 3)}
        log(f"rate {rate:,.0f}: {row}")
        out.append(row)
    print(json.dumps({"metric": "serving latency under Poisson arrivals (continuous batching)",
                      "unit": "ms", "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
                      "config": {"workload": "openai2m: N=2000000 D=1536 d_r=256 bits=4 nlist=4096, "
                                             "k in {10,50,100}, nprobe in {16,32,64}",
                                 "max_slots": args.max_slots, "mem_budget_gib": args.mem_budget},
                      "rates": out}), flush=True)
    ix.close()


if __name__ == "__main__":
    main()
