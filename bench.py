"""Benchmark: exact reverse k-MIPS queries/sec on one MI355X.

Workload (default, the largest single-index workload): 1,000,000 users x
100,000 items, d = 100, log-normal norms (sigma 0.5), k_max = 25; 1,000 query
items drawn from P, each evaluated at k = 1, 10 and 25 (3,000 queries), float32
bulk products, exact result sets.  The index is built once (offline, reported
as build_ms, not part of the timed region).  A step is one pass of the whole
online path over all 3,000 queries, with queries, k values and outputs
resident on the device, results in CSR form in device memory.

Prints one JSON line.  Also reports: the batch latency (p50/p99 of single
steps), the one-query host API latency, the same workload with bf16 bulk
products and with the paper's short lower-bound prefix, the dominant
kernel's roofline fraction from per-kernel HIP events in the same run, and
the CPU oracle (the exact top-k_max table form) timed on the host cores.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="precision")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--lb-items", type=int, default=0,
                    help="|P'| of the lower-bound arrays; 0 = all items (exact table)")
    ap.add_argument("--latency-queries", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU seconds of each oracle table build (all cores, then one core)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the bf16 and short-prefix runs of the same workload")
    ap.add_argument("--form-steps", type=int, default=5)
    ap.add_argument("--handoff-tiles", type=int, default=0,
                    help="index option handoff_tiles (bounded table; 0 = the library default)")
    ap.add_argument("--block-size", type=int, default=0,
                    help="users per Lemma 3 block (16, 32 or 64; 0 = 64)")
    ap.add_argument("--no-blocks", action="store_true",
                    help="no Lemma 3 filter (the paper's Simpfer without blocks)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run 3 plain device copies of this many MiB (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark over the three serving catalogs (separate JSON line)")
    ap.add_argument("--serve-requests", type=int, default=10_000)
    ap.add_argument("--serve-warmup", type=int, default=1_000)
    ap.add_argument("--serve-batch", type=int, default=1024)
    ap.add_argument("--serve-slots", type=int, default=1,
                    help="launches in flight per catalog (continuous batching)")
    ap.add_argument("--serve-hw-queues", type=int, default=0,
                    help="GPU_MAX_HW_QUEUES for the serving run (0: the environment's, HIP's "
                         "default 4 if unset; at most 32)")
    return ap.parse_args()


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}
KERNEL_NAMES = {"filter": "k_filter", "batch_filter": "k_bfilter", "batch_pairs": "k_brecheck_exact/k_bscan",
                "batch_assemble": "k_boffsets+k_bassemble", "batch_prep": "k_bnorms+k_bsort+k_btile",
                "recheck": "k_recheck", "finalize": "k_finalize", "verify": "k_verify"}


def dominant_roofline(cls: str, times, st: dict, d: int, precision: str, passes: int = 1) -> dict:
    """Roofline entry of the dominant kernel class from its event-timed
    launches over `passes` steps and the counters of one step.

    batch_filter (MFMA): algorithmic flops = 2*d (unpadded) per evaluated
    (user, query) pair, i.e. pairs in blocks Lemma 3 did not prune.
    filter (one query, HBM): bytes = 8 per visited block + 64 users x (row +
    norm + bound) per evaluated block."""
    ms, launches_all = times
    avg_s = ms / 1e3 / max(launches_all, 1)
    launches = launches_all // max(passes, 1)  # per step
    if cls == "batch_pairs" and st["scan_items"] > 0:
        # bounded table: the grouped scan's float32 MFMA products, 2*d flops
        # per (user, item) product of the scanned prefixes
        flops = 2.0 * d * st["scan_items"] / max(launches, 1)
        ach = flops / avg_s / 1e12
        peak = MFMA_PEAK_TFLOPS["fp32"]
        return {"bound": "mfma", "kernel": "k_bscan", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "avg_launch_us": avg_s * 1e6,
                "launches_per_step": launches, "algorithmic_flops_per_launch": flops,
                "traffic": None}
    if cls == "batch_filter":
        flops = 2.0 * d * st["users_evaluated"] / max(launches, 1)
        ach = flops / avg_s / 1e12
        peak = MFMA_PEAK_TFLOPS[precision]
        return {"bound": "mfma", "kernel": KERNEL_NAMES[cls], "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "avg_launch_us": avg_s * 1e6,
                "launches_per_step": launches, "algorithmic_flops_per_launch": flops,
                "traffic": None}
    elem = 2 if precision == "bf16" else 4
    evaluated_blocks = st["blocks_visited"] - st["blocks_pruned"]
    nbytes = (8.0 * st["blocks_visited"] + evaluated_blocks * 64.0 * (d * elem + 8)) / max(launches, 1)
    ach = nbytes / avg_s / 1e9
    return {"bound": "hbm", "kernel": KERNEL_NAMES.get(cls, cls), "achieved": ach,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "avg_launch_us": avg_s * 1e6, "launches_per_step": launches,
            "algorithmic_bytes_per_launch": nbytes, "traffic": None}


def measured_traffic(kernel: str, key: str):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    from paper_2110_07131_amd.profiling import source_hash
    with open(path) as fh:
        e = json.load(fh).get(f"{kernel}:{key}")
    if not e or e.get("source_hash") != source_hash(kernel):
        return None
    return e["traffic_bytes_per_launch"]


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def theta_oracle_timing(w, ks, kmax: int, threads: int, budget_s: float, seed: int) -> dict:
    """The table form of the oracle (exact top-k_max values of every user over
    all of P in float64, then one order-statistic test per user and query)
    with `threads` OpenMP threads.  Both phases are linear in the number of
    users, so each is timed on a part of them and scaled by n / part:
      * table build: a uniform user sample sized from a probe so that the
        build takes about budget_s;
      * query phase: the first (q, k) queries over a larger block of users
        (the sampled table rows repeated: its cost does not depend on the
        values), so that the per-call overhead stays small against the work."""
    import oracle
    oracle.set_threads(threads)
    used = oracle.num_threads()
    n = w.Q.shape[0]
    rng = np.random.default_rng(seed)
    qs = w.queries
    probe = int(min(n, max(64 * used, 64)))
    Qp = np.ascontiguousarray(w.Q[rng.choice(n, probe, replace=False)])
    oracle.theta(Qp[:used], w.P, kmax)  # thread start-up outside the probe
    t0 = time.perf_counter()
    oracle.theta(Qp, w.P, kmax)
    per_user = (time.perf_counter() - t0) / probe
    S = int(min(n, max(probe, budget_s / max(per_user, 1e-9))))
    Qs = np.ascontiguousarray(w.Q[np.sort(rng.choice(n, S, replace=False))])
    t0 = time.perf_counter()
    th = oracle.theta(Qs, w.P, kmax)
    tb = time.perf_counter() - t0
    Sq = int(min(n, 100_000 if used > 1 else 20_000))
    nq_t = int(min(len(ks), 300))
    Qq = np.ascontiguousarray(w.Q[:Sq])
    thq = np.ascontiguousarray(th[np.arange(Sq) % S])
    t0 = time.perf_counter()
    for i in range(nq_t):
        oracle.theta_query(thq, Qq, qs[i], int(ks[i]))
    tq = time.perf_counter() - t0
    return {"threads": used, "sample_users": S, "table_build_s_sample": tb,
            "query_users": Sq, "query_count": nq_t, "query_phase_s_sample": tq,
            "build_s_full": tb * n / S, "query_ms_full": 1e3 * tq / nq_t * n / Sq,
            "queries_per_s_full": nq_t / (tq * n / Sq)}


def cpu_baseline(w, ks, kmax: int, budget_s: float) -> dict:
    import oracle
    info = cpu_info()
    allc = theta_oracle_timing(w, ks, kmax, oracle.num_threads(), budget_s, seed=7)
    one = theta_oracle_timing(w, ks, kmax, 1, budget_s, seed=8)
    oracle.set_threads(allc["threads"])
    return {"value": allc["queries_per_s_full"], "unit": "queries/s", "cores": allc["threads"],
            "kind": "oracle",
            "sample": (f"table form of the float64 oracle, {allc['threads']} threads: table build "
                       f"over {allc['sample_users']} sampled users ({allc['table_build_s_sample']:.1f} s), "
                       f"query phase of the first {allc['query_count']} (q,k) over "
                       f"{allc['query_users']} users ({allc['query_phase_s_sample']:.2f} s); one core: "
                       f"{one['sample_users']} and {one['query_users']} users; each scaled by n / users "
                       f"to the full workload.  value = query phase only (the table is built offline, "
                       f"like the index); build_s_full = the table build"),
            "build_s_full": allc["build_s_full"], "query_ms_full": allc["query_ms_full"],
            "one_core": {"value": one["queries_per_s_full"], "build_s_full": one["build_s_full"],
                         "query_ms_full": one["query_ms_full"], "sample_users": one["sample_users"]},
            **info}


def cpu_simpfer_baseline(w, ks, kmax: int, items_all: int = 8, items_one: int = 2) -> dict:
    """The paper's own design on the host: Simpfer (Algorithms 1-3, OpenMP
    over blocks, P' = 2 k_max items, blocks of ceil(log2 n) users), built once
    with all threads; the first (q, k) queries timed with all threads and with
    one."""
    import cpu_simpfer
    t_all = cpu_simpfer.threads()
    t0 = time.perf_counter()
    s = cpu_simpfer.CpuSimpfer(w.Q, w.P, kmax)
    build_s = time.perf_counter() - t0
    qs = w.queries
    per_item = len(ks) // max(len(np.unique(w.qidx)), 1)
    out = {}
    for label, t, items in (("all", t_all, items_all), ("one", 1, items_one)):
        cpu_simpfer.set_threads(t)
        nq = min(len(ks), items * max(per_item, 1))
        ip = 0
        t0 = time.perf_counter()
        for i in range(nq):
            s.query(qs[i], int(ks[i]))
            ip += s.last_stats["users"] + s.last_stats["scan_items"]
        dt = time.perf_counter() - t0
        out[label] = {"queries_per_s": nq / dt, "queries": nq, "seconds": dt,
                      "ip_per_query": ip / max(nq, 1)}
    cpu_simpfer.set_threads(t_all)
    s.free()
    return {"value": out["all"]["queries_per_s"], "unit": "queries/s", "cores": t_all,
            "kind": "paper's CPU design (Simpfer, Algorithms 1-3, OpenMP over blocks)",
            "build_s": build_s, "one_core": out["one"], "all_cores": out["all"],
            "sample": f"the first {out['all']['queries']} (q,k) queries of the workload "
                      f"({t_all} threads) and the first {out['one']['queries']} on one core; "
                      f"P' = {2 * kmax} items, blocks of ceil(log2 n) users, float64 inner products"}


def serve_main(args):
    """Serving form: three resident catalogs, one server with continuous
    batching.  Requests: catalog uniform, query item drawn from that
    catalog's P, k ~ U{1..k_max} (seeded).  First the closed-loop saturation
    rate (every request queued at once), then open-loop Poisson arrivals at
    fixed fractions of it; latency runs from a request's scheduled arrival
    to its ids on the host."""
    # hardware queues the slots' streams are spread over (streams that share
    # one run in order); read by HIP at the first HIP call
    hwq = args.serve_hw_queues or int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4)
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, hwq))
    import torch

    from paper_2110_07131_amd import datagen
    from paper_2110_07131_amd.rkmips import Index, Server

    assert torch.cuda.is_available(), "no HIP device"
    names = ["serve_small", "serve_mid", "serve_large"]
    cats, build = [], {}
    for i, nm in enumerate(names):
        c = datagen.CONFIGS[nm]
        w = datagen.workload(c["n"], c["m"], c["d"], c["sigma"], 0, seed=i)
        t0 = time.perf_counter()
        idx = Index.build(w.Q, w.P, c["k_max"], precision=args.precision, lb_items=args.lb_items)
        build[nm] = {"build_s": time.perf_counter() - t0, "index_bytes": idx.stats()["footprint_bytes"],
                     "n": c["n"], "m": c["m"], "d": c["d"]}
        cats.append((w, c["k_max"], idx))
        print(f"[serve] catalog {nm}: n={c['n']} m={c['m']} d={c['d']} built in "
              f"{build[nm]['build_s']:.2f} s", file=sys.stderr, flush=True)
    srv = Server(max_batch=args.serve_batch, slots=args.serve_slots)
    ids = [srv.add(idx) for _, _, idx in cats]
    rng = np.random.default_rng(12345)

    def draw(n):
        cat = rng.integers(0, len(cats), n).astype(np.int32)
        qs, ks = [], np.empty(n, np.int32)
        for i in range(n):
            w, kmax, _ = cats[cat[i]]
            qs.append(w.P[int(rng.integers(len(w.P)))])
            ks[i] = int(rng.integers(1, kmax + 1))
        return cat, qs, ks

    tag_base = [0]

    def run(cat, qs, ks, arrivals=None):
        """Submit (all at once, or at the scheduled arrivals) and wait for
        every result; returns per-request (catalog, latency ms) and the span."""
        n = len(ks)
        tags = np.arange(tag_base[0], tag_base[0] + n, dtype=np.int64)
        tag_base[0] += n
        lat = np.empty(n)
        first, last = None, 0.0
        got = 0
        if arrivals is None:
            srv.submit_many(cat, qs, ks, tags)
            first = srv.now_ms()
        else:
            i = 0
            first = arrivals[0]
            while i < n:
                now = srv.now_ms()
                j = int(np.searchsorted(arrivals, now, side="right"))
                if j > i:
                    srv.submit_many(cat[i:j], qs[i:j], ks[i:j], tags[i:j], arrivals[i:j])
                    i = j
                for tag, c, st, r, t_sub, t_done in srv.poll():
                    assert st == 0
                    lat[tag - tags[0]] = t_done - t_sub
                    last = max(last, t_done)
                    got += 1
                if j == i and i < n:
                    time.sleep(max(0.0, min(arrivals[i] - srv.now_ms(), 1.0)) / 1e3)
        while got < n:
            for tag, c, st, r, t_sub, t_done in srv.poll(wait_us=2000):
                assert st == 0
                lat[tag - tags[0]] = t_done - t_sub
                last = max(last, t_done)
                got += 1
        return lat, last - first

    cat, qs, ks = draw(args.serve_warmup)
    run(cat, qs, ks)
    n_sat = max(args.serve_requests, 2 * args.serve_batch * len(cats))
    cat, qs, ks = draw(n_sat)
    lat, span = run(cat, qs, ks)
    sat_qps = n_sat / (span / 1e3)
    print(f"[serve] closed loop: {n_sat} requests in {span:.1f} ms, {sat_qps:.0f} queries/s",
          file=sys.stderr, flush=True)
    loads = []
    for frac in (0.02, 0.25, 0.5, 0.75, 0.9):
        lam = frac * sat_qps
        ntot = args.serve_warmup + args.serve_requests
        cat, qs, ks = draw(ntot)
        gaps = rng.exponential(1e3 / lam, ntot)
        # the load generator must not pause (its lateness counts as latency)
        gc.collect()
        gc.disable()
        arrivals = srv.now_ms() + 1.0 + np.cumsum(gaps)
        lat, span = run(cat, qs, ks, arrivals)
        gc.enable()
        m = slice(args.serve_warmup, ntot)
        L, C = lat[m], cat[m]
        per = {names[c]: {"p50_ms": float(np.percentile(L[C == c], 50)),
                          "p99_ms": float(np.percentile(L[C == c], 99)), "requests": int((C == c).sum())}
               for c in range(len(cats))}
        loads.append({"load": frac, "offered_qps": lam,
                      "achieved_qps": ntot / (span / 1e3),
                      "p50_ms": float(np.percentile(L, 50)), "p99_ms": float(np.percentile(L, 99)),
                      "per_catalog": per,
                      "p99_ms_by_tenth": [float(np.percentile(x, 99)) for x in np.array_split(L, 10)]})
        print(f"[serve] load {frac}: offered {lam:.0f}/s, p50 {loads[-1]['p50_ms']:.3f} ms, "
              f"p99 {loads[-1]['p99_ms']:.3f} ms", file=sys.stderr, flush=True)
    line = {
        "metric": "reverse k-MIPS serving latency (exact sets), p50/p99 from arrival to ids on host",
        "unit": "ms", "n_gpus": 1, "dtype": args.precision.replace("fp", "f"), "data": "synthetic",
        "config": {"workload": "serving: catalogs (50k,10k,d50), (500k,50k,d100), (2M,100k,d200), "
                               "sigma 0.5, k_max 25; catalog uniform, query item from its P, "
                               "k ~ U{1..25}; Poisson arrivals",
                   "max_batch": args.serve_batch, "slots_per_catalog": args.serve_slots,
                   "hw_queues": hwq,
                   "lb_items": args.lb_items or "m",
                   "requests_per_load": args.serve_requests, "warmup": args.serve_warmup},
        "saturation_qps": sat_qps, "loads": loads, "catalogs": build,
        "server_device_bytes": srv.used_bytes(),
    }
    print(json.dumps(line))
    srv.close()


def main():
    args = parse()
    if args.serve:
        if args.gpus != 1:
            print("the serving benchmark runs on one GPU", file=sys.stderr)
            sys.exit(2)
        return serve_main(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has "
              f"no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2110_07131_amd import datagen
    from paper_2110_07131_amd.rkmips import Index

    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)
    if args.calib_copy_mb > 0:  # plain copies of a known size (counter calibration)
        n = (args.calib_copy_mb << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = datagen.CONFIGS[args.config]
    w = datagen.config_workload(args.config)
    n, m, d, kmax = cfg["n"], cfg["m"], cfg["d"], cfg["k_max"]
    qs_np, ks = w.queries, w.ks.astype(np.int32)
    nq = len(ks)
    print(f"[bench] workload {args.config}: n={n} m={m} d={d} k_max={kmax} queries={nq}",
          file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    idx = Index.build(w.Q, w.P, kmax, precision=args.precision, lb_items=args.lb_items,
                      handoff_tiles=args.handoff_tiles, block_size=args.block_size,
                      no_blocks=args.no_blocks)
    build_s = time.perf_counter() - t0
    st0 = idx.stats()
    print(f"[bench] index built in {build_s:.2f} s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    qs = torch.from_numpy(qs_np).to(dev)
    cap = max(1, nq * 256)
    offsets = torch.empty(nq + 1, dtype=torch.int64, device=dev)
    ids = torch.empty(cap, dtype=torch.int32, device=dev)
    torch_stream = torch.cuda.Stream()  # default priority
    torch.cuda.set_stream(torch_stream)
    stream = torch_stream.cuda_stream

    def step():
        idx.reverse_kmips_batch_dev(qs, ks, offsets, ids, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    qps = nq * args.steps / elapsed
    total = int(offsets[-1].item())
    print(f"[bench] {args.steps} steps, {ms_per_step:.3f} ms/step, {qps:.0f} queries/s, "
          f"{total} result ids per step", file=sys.stderr, flush=True)
    if total > cap:
        raise RuntimeError("result capacity exceeded")

    # Sampled exactness check of the timed output against the host API.
    off_h = offsets.cpu().numpy()
    ids_h = ids[:total].cpu().numpy()
    for i in np.linspace(0, nq - 1, 8).astype(int):
        ref = idx.reverse_kmips(qs_np[i], int(ks[i]))
        assert np.array_equal(ids_h[off_h[i]:off_h[i + 1]], ref), f"batch/single mismatch at {i}"

    # Dominant kernel: per-kernel HIP events over one more pass, and the
    # algorithmic work from the counters of one counted pass.
    idx.set_counting(True)
    idx.reset_counters()
    step()
    torch.cuda.synchronize()
    st = idx.stats()
    idx.set_counting(False)
    passes = max(3, min(args.steps, 10))
    idx.set_timing(passes * (8 * nq + 64))
    for _ in range(passes):
        step()
    torch.cuda.synchronize()
    kt = idx.kernel_times()
    idx.set_timing(0)
    dom = max(kt, key=lambda c: kt[c][0])
    roofline = dominant_roofline(dom, kt[dom], st, d, args.precision, passes)
    table = "exact" if (args.lb_items == 0 or args.lb_items >= m) else f"lb{args.lb_items}"
    roofline["traffic"] = measured_traffic(roofline["kernel"], f"{args.config}/{args.precision}/{table}")
    kernel_share = {c: {"ms_per_step": v[0] / passes, "launches": v[1] // passes} for c, v in kt.items()}

    # Batch latency: every query of a step completes when its step does; the
    # steps again, one at a time, each bracketed by device synchronisations.
    bt = []
    for _ in range(max(args.steps, 1)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        bt.append(time.perf_counter() - t)
    bt = np.array(bt) * 1e3
    batch_lat = {"p50_ms": float(np.percentile(bt, 50)), "p99_ms": float(np.percentile(bt, 99)),
                 "steps": len(bt),
                 "what": f"one device-resident step of {nq} queries (launch to completion); "
                         f"every query of the step completes with it"}

    lat = None
    if not args.no_latency:
        nl = min(args.latency_queries, nq)
        times = []
        gc.collect()
        gc.disable()  # the interpreter's collector must not pause inside the timed calls
        for i in range(nl):
            t = time.perf_counter()
            idx.reverse_kmips(qs_np[i], int(ks[i]))
            times.append(time.perf_counter() - t)
        gc.enable()
        times = np.array(times) * 1e3
        lat = {"p50_ms": float(np.percentile(times, 50)), "p99_ms": float(np.percentile(times, 99)),
               "qps": nl / (times.sum() / 1e3), "queries": nl,
               "what": "one query at a time through the host API (H2D of q, ids on host)"}
    idx.free()
    del ids, offsets

    # The same workload in the other forms: bf16 bulk products with float64
    # rechecks, and the paper's index (P' = 2 k_max items in the lower-bound
    # arrays, linear scans), each timed over a few steps and checked on a
    # sample against the host API.
    forms = {}
    if not args.no_forms:
        for name, prec, lb in (("bf16_exact_table", "bf16", 0),
                               ("fp32_paper_index", "fp32", 2 * kmax)):
            if prec == args.precision and lb == args.lb_items:
                continue
            fi = Index.build(w.Q, w.P, kmax, precision=prec, lb_items=lb)
            foff = torch.empty(nq + 1, dtype=torch.int64, device=dev)
            fids = torch.empty(cap, dtype=torch.int32, device=dev)
            fi.reverse_kmips_batch_dev(qs, ks, foff, fids, stream)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.form_steps):
                fi.reverse_kmips_batch_dev(qs, ks, foff, fids, stream)
            torch.cuda.synchronize()
            fel = time.perf_counter() - t
            fo = foff.cpu().numpy()
            fh = fids[:int(fo[-1])].cpu().numpy()
            for i in np.linspace(0, nq - 1, 4).astype(int):
                ref = fi.reverse_kmips(qs_np[i], int(ks[i]))
                assert np.array_equal(fh[fo[i]:fo[i + 1]], ref), f"{name}: batch/single mismatch at {i}"
            # one counted step: how many (user, query) pairs the bulk
            # precision left to float64 (the rest were certified)
            fi.reset_counters()
            fi.set_counting(True)
            fi.reverse_kmips_batch_dev(qs, ks, foff, fids, stream)
            torch.cuda.synchronize()
            fst = fi.stats()
            fi.set_counting(False)
            forms[name] = {"value": nq * args.form_steps / fel, "unit": "queries/s",
                           "ms_per_step": 1e3 * fel / args.form_steps, "steps": args.form_steps,
                           "precision": prec, "lb_items": lb or m,
                           "counters_per_step": {k: int(fst[k]) for k in (
                               "users_evaluated", "lemma1_no", "table_yes", "rechecks", "survivors",
                               "scan_items", "results")},
                           "float64_share_of_evaluated": fst["rechecks"] / max(fst["users_evaluated"], 1)}
            print(f"[bench] form {name}: {forms[name]['ms_per_step']:.3f} ms/step, "
                  f"{forms[name]['value']:.0f} queries/s", file=sys.stderr, flush=True)
            fi.free()
            del foff, fids

    cpu = None if args.no_cpu else cpu_baseline(w, ks, kmax, args.cpu_seconds)
    simpfer_cpu = None if args.no_cpu else cpu_simpfer_baseline(w, ks, kmax)

    line = {
        "metric": "reverse k-MIPS queries/sec (exact sets) and p50/p99 latency at 1 MI355X",
        "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision.replace("fp", "f"),
        "data": "synthetic",
        "config": {"workload": f"{args.config}: |Q|={n} |P|={m} d={d} k_max={kmax} "
                               f"lognormal-norm (sigma {cfg['sigma']}) Gaussian vectors, seed 0, "
                               f"{len(np.unique(w.qidx))} query items from P x k in "
                               f"{sorted(set(ks.tolist())) if len(set(ks.tolist())) < 8 else '1..' + str(kmax)}; "
                               f"{args.precision} bulk products, "
                               f"{'exact' if args.lb_items in (0, m) else 'P=' + str(args.lb_items)} lower-bound table",
                   "queries_per_step": nq, "lb_items": args.lb_items or m,
                   "block_size": args.block_size or 64, "lemma3_blocks": not args.no_blocks,
                   "precision": args.precision, "form": "device-resident batch, CSR output"},
        "p50_ms": batch_lat["p50_ms"], "p99_ms": batch_lat["p99_ms"],
        "latency": batch_lat, "single_query_latency": lat,
        "other_forms": forms,
        "roofline": roofline,
        "dominant_kernel_class": dom,
        "kernel_time_per_step": kernel_share,
        "counters_per_step": {k: st[k] for k in ("blocks_visited", "blocks_pruned", "users_evaluated",
                                                 "lemma1_no", "lemma2_yes", "table_yes", "survivors",
                                                 "scan_items", "rechecks", "results", "scan_long",
                                                 "scan_full_f64", "scan_handoff", "scan_quarters",
                                                 "scan_valu_tiles")},
        "build_ms": st0["build_ms"], "index_bytes": st0["footprint_bytes"],
        "cpu_baseline": cpu,
        "cpu_simpfer": simpfer_cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
