#!/usr/bin/env python3
"""Benchmark of the batched MRQ search on one MI355X.

Metric: queries per second of the batched search at the smallest nprobe whose recall@10 against
exact brute-force ground truth is >= 0.95.  Headline: the DEEP-shaped synthetic workload, the largest
that fits one GPU (N = 10,000,000, D = 128, 10,000 queries, nlist = 16,384, d_r = 64, 1-bit codes,
k = 10); the GIST-shaped one (N = 1,000,000, D = 960, nlist = 4,096, d_r = 128) follows as a nested block.
A step is one batched search of all queries (projection, probe, query codes, seed pass, phased scans,
top-k) with the index and the queries resident in HBM.  Prints one JSON line.
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
MFMA_I8_PEAK = 5.0e15      # dense int8 matrix-core ops/s
MFMA_F32_PEAK = 157.3e12   # FP32 matrix-core FLOP/s
VALU_OPS_PEAK = 256 * 64 * 2.4e9   # vector lane-operations/s (256 CUs x 64 lanes x 2.4 GHz, one op per lane per
                                   # clock; the 157.3 TFLOP/s FP32 figure counts an FMA as two and packed FP32)
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


# Index and search configuration per workload (the stand-ins of the paper's data sets): nlist, d_r, bits.
WORKLOADS = {
    "small": dict(nlist=64, d=32, bits=1),         # the plain-method case: 20k x 128
    "gist1m": dict(nlist=4096, d=128, bits=1),     # GIST-shaped: 1M x 960
    "deep10m": dict(nlist=16384, d=64, bits=1),    # DEEP-shaped: 10M x 128 (the largest single-GPU case)
    "openai2m": dict(nlist=4096, d=256, bits=4),   # embedding-shaped: 2M x 1536
}


def cpu_description():
    """Host CPU model and clock (lscpu), for the oracle baseline."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k in ("Model name", "CPU max MHz", "CPU MHz", "CPU(s)"):
                info[k] = v
    except Exception:
        pass
    # lscpu may give neither clock inside a container: the kernel's per-core figures then
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and len(v) > len(info.get("Model name", "")):
                    info["Model name"] = v
                if k == "cpu MHz" and "CPU MHz" not in info:
                    info["CPU MHz"] = v
    except OSError:
        pass
    return info


def copy_bandwidth(torch, mrq, dev, gib=4, reps=10):
    """Achievable HBM bandwidth: the library's streaming copy over `gib` GiB (2 x bytes moved per copy)."""
    n = (gib << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    for _ in range(2):
        mrq.stream_copy(dst, src, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        mrq.stream_copy(dst, src, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(dst[:1024], src[:1024]))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9, ok


def measure(args, name, np, torch, mrq, synth, dev, headline, copy_gbs):
    """Build the index of workload `name`, find the smallest nprobe reaching the target recall, time K plain
    batched searches (the throughput) and K instrumented ones (per-kernel times, stage and work counters:
    the roofline).  The headline workload also times the per-query path, the CPU oracle and the per-result
    error report."""
    cfg = dict(WORKLOADS.get(name, WORKLOADS["gist1m"]))
    if headline:
        for key in ("nlist", "d", "bits"):
            if getattr(args, key):
                cfg[key] = getattr(args, key)
    t0 = time.time()
    X, Q, spec = synth.workload(name, N=args.N if headline else None, nq=args.nq if headline else None)
    N, D = X.shape
    nq = Q.shape[0]
    log(f"{name}: data {N}x{D}, {nq} queries in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    torch.cuda.synchronize()
    t1 = time.time()
    ix = mrq.Index.build(Xd, d_r=cfg["d"], bits=cfg["bits"], nlist=cfg["nlist"])
    build_s = time.time() - t1
    log(f"{name}: build {build_s:.1f}s, index {ix.device_bytes / 2**30:.2f} GiB")

    k = args.k
    ids_buf = torch.empty((nq, k), dtype=torch.int64, device=dev)
    d_buf = torch.empty((nq, k), dtype=torch.float32, device=dev)

    def run(nprobe, counters=None, mode=mrq.MRQ_BATCHED, Qs=None, ib=None, db=None):
        o = mrq.search_opts(mode=mode, counters=counters, group=args.group, phase_growth=args.phase_growth)
        Qs = Qd if Qs is None else Qs
        return ix.search(Qs, k, nprobe, ids=ids_buf if ib is None else ib, dists=d_buf if db is None else db,
                         opts=o)

    chosen, rec_at = (args.nprobe if headline else 0), None
    sweep = []
    gt = None
    if not args.profile_only:
        t2 = time.time()
        gt = ground_truth(torch, Xd, Qd, k)
        log(f"{name}: ground truth {time.time() - t2:.1f}s")
        # the smallest nprobe reaching the target: a coarse grid, the autotuner at its first value reaching
        # the target, then (with the tuned schedule) every value between the last one below the target and
        # that one
        cands = [chosen] if chosen else [8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]

        def try_np(npb):
            run(npb)
            torch.cuda.synchronize()
            r = recall(ids_buf.cpu().numpy(), gt, k)
            sweep.append((npb, r))
            log(f"{name}: nprobe {npb}: recall@{k} {r:.4f}")
            return r

        prev = 0
        fixed = bool(chosen)
        for npb in cands:
            if npb > cfg["nlist"]:
                break
            chosen, rec_at = npb, try_np(npb)
            if rec_at >= args.target_recall:
                break
            prev = npb
    else:
        fixed = bool(chosen)
    if not chosen:
        chosen = 64

    if args.calib_copy and headline:  # a copy kernel of known size: 1 GiB read + 1 GiB written
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
        log(f"{name}: query group {group}, phase growth {growth}")
    else:
        group, growth = ix.tune(Qd, k, chosen)
        log(f"{name}: autotuned query group {group}, phase growth {growth}")
    if not args.profile_only and not fixed and rec_at is not None and rec_at >= args.target_recall:
        for fine in list(range(prev + 1, chosen)) + [chosen]:
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
    cnt = torch.zeros(16, dtype=torch.int64, device=dev)
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
    log(f"{name}: batched {qps:,.0f} QPS, {ms_step:.2f} ms/step at nprobe {chosen} "
        f"({ms_instr:.2f} ms/step with per-step events and device counters)")
    log(f"{name}: kernel ms/step: " + ", ".join(f"{n}={v[0] / args.steps:.3f}" for n, v in kt.items()))

    # ---- roofline of the scan (and the exact stage) -------------------------------------------------------
    # per (query, candidate) pair: the bytes a candidate's tests read as if each pair streamed its list
    # (sign code + A, F, E per candidate; record + query levels per pair; the B-bit code and factors per
    # stage-1 survivor; x_d row + a_x per stage-2 entrant; 8 B per exact-stage candidate written)
    d, B = cfg["d"], cfg["bits"]
    d4 = (d + 3) // 4 * 4
    WP = next(w for w in (1, 2, 4, 8, 16, 32, 48) if 32 * w >= d)
    KI = (d + 63) // 64
    KP = 64 * (4 if KI == 3 else KI)
    scanned, p1, pext, p2 = (float(x) for x in cnt[:4])
    items, tiles2 = float(cnt[8]), float(cnt[9])
    pairs_scan = nq * (chosen - 1)
    pair_bytes = (scanned * (d / 8 + 12) + pairs_scan * (48 + KP)
                  + (p1 * ((B - 1) * d / 8 + 12) if B > 1 else 0) + pext * (4 * d4 + 4) + p2 * 8)
    # unique fetch: what the work items must read at least: each item's 64-row code block, factors and
    # descriptor once, the x_d rows (and a_x) of each row tile that entered stage 2 once, each pair's record
    # and levels once, the B-bit planes and factors of each item's block once (B > 1), the exact-stage
    # entries written
    split = D - d <= d   # the split exact stage: each bin entry carries dis_o' beside its row
    unique_bytes = (items * (64 * (4 * WP + 12) + 16) + tiles2 * 16 * (4 * d4 + 4) + pairs_scan * (48 + KP)
                    + (items * 64 * ((B - 1) * 4 * WP + 12) if B > 1 else 0) + p2 * (8 if split else 4))
    G = group if group else 16
    i8_ops = items * 2 * 64 * G * KP                  # stage-1 int8 products (64 rows x G queries x KP)
    f32_ops = tiles2 * 2 * 16 * G * d4                # stage-2 FP32 products
    valu_ops = items * 64 * G * 12                    # the Eq 4-6 epilogue per (row, query) entry
    # exact stage per candidate: its bin entry and its row of D floats, or (the split form: tail no wider than
    # the leading block, stage 2 on) the bin entry, dis_o' and the D - d tail floats; the id is read only for
    # candidates that can enter the result queue and is not counted
    rx = (D - d + 3) // 4 * 4 if split else (D + 3) // 4 * 4
    ex_b = 4 + 4 * rx + (4 if split else 0)
    kern = {"scan": dict(bytes=pair_bytes, unique=unique_bytes, ops=scanned * 2 * d + pext * 2 * d),
            "exact": dict(bytes=p2 * ex_b, unique=p2 * ex_b, ops=p2 * (2 if split else 3) * rx)}
    rows = {}
    for kn, kb in kern.items():
        ms_tot, launches = kt.get(kn, (0.0, 0))
        if launches == 0 or ms_tot <= 0:
            continue
        per_ms = ms_tot / launches
        lps = launches / args.steps
        rows[kn] = dict(ms_per_step=ms_tot / args.steps, launch_ms=per_ms, launches=lps,
                        gbs=kb["bytes"] / lps / (per_ms * 1e-3) / 1e9,
                        ugbs=kb["unique"] / lps / (per_ms * 1e-3) / 1e9,
                        tops=kb["ops"] / lps / (per_ms * 1e-3) / 1e12,
                        bytes_per_launch=kb["bytes"] / lps, unique_per_launch=kb["unique"] / lps)
    roof = None
    if "scan" in rows:
        r = rows["scan"]
        t = r["launch_ms"] * 1e-3
        lps = r["launches"]
        t_hbm = r["unique_per_launch"] / (HBM_PEAK_GBS * 1e9)
        t_cmp = (i8_ops / lps) / MFMA_I8_PEAK + (f32_ops / lps) / MFMA_F32_PEAK + (valu_ops / lps) / VALU_OPS_PEAK
        tag = f"{name}_d{d}_b{B}_np{chosen}_k{k}"
        traffic = counter_traffic(tag, "k_scan")
        roof = {"bound": "hbm", "achieved": round(r["ugbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(r["ugbs"] / HBM_PEAK_GBS, 4), "traffic": None if traffic is None else round(traffic),
                "kernel": "k_scan",
                "achieved_basis": "algorithmic bytes of the batched scan: each work item's 64-row code block, "
                                  "factors and descriptor once, the x_d rows of each row tile entering stage 2 "
                                  "once, each pair's record and query levels once, the exact-stage entries written",
                "algorithmic_bytes_per_launch": round(r["unique_per_launch"]), "launch_ms": round(r["launch_ms"], 4),
                "frac_of_copy": None if not copy_gbs else round(r["ugbs"] / copy_gbs, 4),
                "per_pair": {"bytes_per_launch": round(r["bytes_per_launch"]), "GB/s": round(r["gbs"], 1),
                             "frac": round(r["gbs"] / HBM_PEAK_GBS, 4),
                             "basis": "bytes per (query, candidate) pair: each candidate's code and factors once "
                                      "per pair, as if every (query, list) pair streamed its list (an effective "
                                      "rate: a work item reads a list block once for up to 16 queries)"},
                "roofline_frac": round(max(t_hbm, t_cmp) / t, 4),
                "roofline_bound": "hbm (unique bytes)" if t_hbm >= t_cmp else "compute (i8 + f32 MFMA, VALU)",
                "counter_GB/s": None if traffic is None else round(traffic / t / 1e9, 1),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                "work_per_launch": {"items": round(items / lps), "stage2_row_tiles": round(tiles2 / lps),
                                    "pairs": round(pairs_scan / lps), "candidates": round(scanned / lps)},
                "per_kernel": {n: {"ms_per_step": round(v["ms_per_step"], 4), "GB/s": round(v["gbs"], 1),
                                   "unique_GB/s": round(v["ugbs"], 1), "TOP/s": round(v["tops"], 3)}
                               for n, v in rows.items()}}

    # ---- per-result distance error against FP64 (every returned row) ----------------------------------------
    run(chosen)
    torch.cuda.synchronize()
    ids_h = ids_buf.cpu().numpy()
    ok = ids_h >= 0
    rel = []
    for s0 in range(0, nq, 1024):
        ii = ids_buf[s0:s0 + 1024].clamp(min=0)
        d64 = ((Xd[ii].double() - Qd[s0:s0 + 1024, None, :].double()) ** 2).sum(-1)
        e = (d_buf[s0:s0 + 1024].double() - d64).abs() / d64.clamp(min=1e-30)
        rel.append(e[ids_buf[s0:s0 + 1024] >= 0].cpu())
    rel = torch.cat(rel).numpy()
    dist_err = {"results": int(ok.sum()), "max_rel": float(rel.max()), "p99_rel": float(np.percentile(rel, 99)),
                "mean_rel": float(rel.mean())}

    out = {
        "value": round(qps, 1), "ms_per_step": round(ms_step, 4),
        "config": {"workload": f"{name}: N={N} D={D} nq={nq} nlist={cfg['nlist']} d_r={d} bits={B} k={k}",
                   "N": N, "D": D, "nq": nq, "nlist": cfg["nlist"], "d_r": d, "bits": B, "k": k,
                   "nprobe": chosen, "recall_at_10": None if rec_at is None else round(rec_at, 4),
                   "query_group": group, "phase_growth": growth, "parallelism": "single-gpu"},
        "roofline": roof,
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
        "distance_error_vs_fp64": dist_err,
    }
    if headline and not args.profile_only and args.per_query > 0:
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
        log(f"{name}: per-query path {pq_qps:,.0f} QPS (ids identical to batched: {same})")
        out.update({"per_query_qps": round(pq_qps, 1), "speedup_vs_per_query": round(qps / pq_qps, 1),
                    "per_query_matches_batched": same})
    if headline and not args.profile_only and not args.no_cpu_baseline:
        out.update(cpu_baseline_leg(args, ix, X, Q, k, chosen, np, mrq))
    del Xd, Qd, ids_buf, d_buf
    ix.close()
    torch.cuda.empty_cache()
    return out


def cpu_baseline_leg(args, ix, X, Q, k, nprobe, np, mrq):
    """The CPU oracle (test infrastructure) on the exported index: its single-threaded Algorithm 2 timed on
    one pinned host core over a bounded sample of the workload's queries, and, for the first queries, the
    per-result error of the device's Eq 7 projected distance (FP32 projection) and eps_r (BF16 tail
    coordinates) against the oracle's FP64 values."""
    import oracle
    res = {}
    tmp = "/dev/shm" if os.path.isdir("/dev/shm") else None
    with tempfile.TemporaryDirectory(dir=tmp) as td:
        path = os.path.join(td, "bench.mrqx")
        ix.export(path)
        orc = oracle.Index.load_export(path).attach(X)
    prm = oracle.params()
    cpu_info = cpu_description()
    core = sorted(os.sched_getaffinity(0))[-1]
    old_aff = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {core})  # this thread only, as `taskset -c core`
    try:
        n, tc = 0, time.perf_counter()
        tot = {}
        while n < Q.shape[0] and time.perf_counter() - tc < args.cpu_seconds:
            _, _, c = orc.search(Q[n], k, nprobe, mode=oracle.ALG2, prm=prm, counters=True)
            for key_, v in c.items():
                tot[key_] = tot.get(key_, 0) + v
            n += 1
        el = time.perf_counter() - tc
    finally:
        os.sched_setaffinity(0, old_aff)
    res["cpu_baseline"] = {
        "value": round(n / el, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
        "sample": f"first {n} queries, single-threaded FP64 Algorithm 2 on the exported index, nprobe {nprobe}, "
                  f"k {k}",
        "cpu_model": cpu_info.get("Model name"), "cpu_mhz": cpu_info.get("CPU max MHz") or cpu_info.get("CPU MHz"),
        "host_cpus": cpu_info.get("CPU(s)"), "pinning": f"sched_setaffinity of the oracle thread to core {core}",
        "oracle_pass_rates": {"stage1": round(tot["pass1"] / max(tot["scanned"], 1), 5),
                              "stage2_exact": round(tot["pass2"] / max(tot["scanned"], 1), 6),
                              "scanned_per_query": round(tot["scanned"] / max(n, 1), 1)}}
    log(f"cpu oracle: {res['cpu_baseline']['value']} QPS over {n} queries on core {core} "
        f"({cpu_info.get('Model name')})")
    # per-result projection error: the Eq 7 projected distance of every returned result that went through
    # stage 2, device (FP32 q_d from the projection product) vs the oracle (FP64), relative to its exact
    # distance; and eps_r per query (BF16 tail product) vs FP64
    nt = min(args.proj_queries, Q.shape[0])
    sub = np.ascontiguousarray(Q[:nt])
    ids, dists, pairs, _, _, cands = ix.search_trace(sub, k, nprobe, list(range(nt)), max_pairs=nt * (nprobe + 1),
                                                     max_cands=4 << 20)
    diso = {(int(c["q"]), int(c["id"])): (float(c["v0"]), int(c["list"])) for c in cands
            if c["kind"] == mrq.TRACE_STAGE2}
    errs, er_err = [], []
    cache = {}
    for q in range(nt):
        for i in ids[q][ids[q] >= 0].tolist():
            hit = diso.get((q, i))
            if hit is None:
                continue
            v, lst = hit
            if (q, lst) not in cache:
                cache[(q, lst)] = orc.pair_trace(sub[q], lst, prm)
            qs, _, _, lid, cand = cache[(q, lst)]
            r = int(np.nonzero(lid == i)[0][0])
            errs.append(abs(v - cand["diso"][r]) / max(cand["dis"][r], 1e-30))
        rec = pairs[pairs["q"] == q]
        if len(rec):
            qs0 = orc.pair_trace(sub[q], int(rec[0]["list"]), prm)[0]
            er_err.append(abs(float(rec[0]["er"]) - qs0["er"]) / max(qs0["er"], 1e-30))
    errs = np.array(errs) if errs else np.zeros(1)
    res["projection_error_vs_fp64_oracle"] = {
        "queries": nt, "results_with_stage2": int(len(errs)),
        "dis_o_rel_to_exact_max": float(errs.max()), "dis_o_rel_to_exact_p99": float(np.percentile(errs, 99)),
        "eps_r_rel_max": float(max(er_err) if er_err else 0.0),
        "note": "q_d from the FP32 matrix-core projection; the tail coordinates (sigma, eps_r of Eq 6) from the "
                "BF16 product with FP32 accumulation"}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="deep10m", help="headline workload (deep10m, gist1m, openai2m, small)")
    ap.add_argument("--nested", default="gist1m", help="workloads measured after the headline ('none' for none)")
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--nlist", type=int, default=0, help="headline override of the workload's nlist")
    ap.add_argument("--d", type=int, default=0, help="headline override of the workload's d_r")
    ap.add_argument("--bits", type=int, default=0, help="headline override of the workload's code bits")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--nprobe", type=int, default=0, help="fixed nprobe (0 = smallest reaching the recall)")
    ap.add_argument("--target-recall", type=float, default=0.95)
    ap.add_argument("--per-query", type=int, default=200, help="queries timed on the per-query path")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle CPU-baseline time budget")
    ap.add_argument("--proj-queries", type=int, default=32, help="queries of the per-result projection report")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true", help="skip GT/sweep/baselines (profiler runs)")
    ap.add_argument("--group", type=int, default=0,
                    help="queries per scan work item (16, 32 or 64); with --phase-growth skips the autotuner")
    ap.add_argument("--phase-growth", type=int, default=0,
                    help="probe-rank phase growth (2, 4 or 8); with --group skips the autotuner")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--c4", action="store_true",
                    help="one hipGraph-captured launch of a 20k-query mixed k / nprobe batch (embedding-shaped index)")
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
    if args.c4:
        c4_main(args, np, torch, mrq, synth, dev)
        return
    if args.sweep_d:
        if not args.nlist:
            args.nlist = WORKLOADS.get(args.workload, WORKLOADS["gist1m"])["nlist"]
        args.bits = args.bits or 1
        sweep_d_main(args, np, torch, mrq, synth, dev)
        return
    if args.mrsq:
        if not args.nlist:
            args.nlist = WORKLOADS.get(args.workload, WORKLOADS["gist1m"])["nlist"]
        args.bits = args.bits or 1
        mrsq_main(args, np, torch, mrq, synth, dev)
        return
    copy_gbs, copy_ok = copy_bandwidth(torch, mrq, dev)
    log(f"streaming copy: {copy_gbs:,.0f} GB/s (2 x 4 GiB per copy; correct: {copy_ok})")
    head = measure(args, args.workload, np, torch, mrq, synth, dev, True, copy_gbs)
    nested = {}
    if not args.profile_only:
        for nm in [w for w in args.nested.split(",") if w in WORKLOADS and w != args.workload]:
            nested[nm] = measure(args, nm, np, torch, mrq, synth, dev, False, copy_gbs)
    res = {
        "metric": "QPS at recall@10=0.95 (1 GPU, batched vs per-query); scan HBM GB/s vs peak",
        "value": head.pop("value"), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": head.pop("config"),
        "roofline": head.pop("roofline"),
        "cpu_baseline": head.pop("cpu_baseline", None),
        "achievable_copy_GBps": round(copy_gbs, 1),
    }
    res.update(head)
    for nm, r in nested.items():
        res[nm] = r
    print(json.dumps(res), flush=True)


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


def c4_main(args, np, torch, mrq, synth, dev):
    """One hipGraph-captured launch of a mixed batch: the embedding-shaped index (N = 2,000,000, D = 1,536,
    d_r = 256, 4-bit codes, nlist = 4,096) and its 20,000 queries, each with its own k ~ U{10..100} and
    nprobe ~ U{8..64} (seeded), searched by mrq_search_mixed_dev (per-query k / nprobe on the device).  Times
    K graph replays (and K eager calls) between synchronisations; reports queries/s, the replays' agreement
    with the eager rows, and recall@10 of each query's first 10 results against exact brute force."""
    t0 = time.time()
    X, Q, _ = synth.workload("openai2m")
    nq = Q.shape[0]
    log(f"c4: data {X.shape[0]}x{X.shape[1]}, {nq} queries in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    t1 = time.time()
    ix = mrq.Index.build(Xd, d_r=256, bits=4, nlist=4096)
    log(f"c4: build {time.time() - t1:.1f}s, index {ix.device_bytes / 2**30:.2f} GiB")
    gt = ground_truth(torch, Xd, Qd, 10)
    del Xd
    torch.cuda.empty_cache()
    rng = np.random.default_rng(4004)
    ks = rng.integers(10, 101, nq).astype(np.int32)
    nps = rng.integers(8, 65, nq).astype(np.int32)
    off = np.zeros(nq, np.int64)
    off[1:] = np.cumsum(ks[:-1].astype(np.int64))
    tot = int(ks.sum())
    kd, npd = torch.from_numpy(ks).to(dev), torch.from_numpy(nps).to(dev)
    ib = torch.empty(tot, dtype=torch.int64, device=dev)
    db = torch.empty(tot, dtype=torch.float32, device=dev)
    group, growth = ix.tune(Qd, 50, 32)
    log(f"c4: autotuned query group {group}, phase growth {growth} (k 50, nprobe 32)")
    opts = mrq.search_opts(group=group, phase_growth=growth)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ix.search_mixed_dev(Qd, kd, npd, 100, 64, ib, db, opts=opts, stream=s)  # sizes the workspace
    torch.cuda.synchronize()
    ref_i, ref_d = ib.clone(), db.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        ix.search_mixed_dev(Qd, kd, npd, 100, 64, ib, db, opts=opts, stream=s)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    el_graph = time.perf_counter() - ts
    same = bool(torch.equal(ib, ref_i)) and bool(torch.equal(db.view(torch.int32), ref_d.view(torch.int32)))
    ts = time.perf_counter()
    for _ in range(args.steps):
        ix.search_mixed_dev(Qd, kd, npd, 100, 64, ib, db, opts=opts, stream=s)
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - ts
    ih = ib.cpu().numpy()
    hit = sum(len(set(ih[off[i]:off[i] + 10].tolist()) & set(gt[i, :10].tolist())) for i in range(nq))
    rec = hit / (10.0 * nq)
    qps = nq * args.steps / el_graph
    log(f"c4: graph replay {qps:,.0f} QPS ({1e3 * el_graph / args.steps:.2f} ms), eager "
        f"{nq * args.steps / el_eager:,.0f} QPS, replay rows equal eager: {same}, recall@10 {rec:.4f}")
    print(json.dumps({"metric": "QPS of one hipGraph-captured mixed-k/nprobe launch (1 GPU)", "value": round(qps, 1),
                      "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(1e3 * el_graph / args.steps, 4), "higher_is_better": True,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "openai2m: N=2000000 D=1536 nq=20000 nlist=4096 d_r=256 bits=4, "
                                             "k ~ U{10..100}, nprobe ~ U{8..64} per query",
                                 "query_group": group, "phase_growth": growth},
                      "eager_qps": round(nq * args.steps / el_eager, 1), "replay_equals_eager": same,
                      "recall_at_10": round(rec, 4), "mean_k": round(float(ks.mean()), 2),
                      "mean_nprobe": round(float(nps.mean()), 2)}), flush=True)
    ix.close()


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
