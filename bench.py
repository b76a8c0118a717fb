#!/usr/bin/env python3
"""Throughput benchmark of the greedy adaptive TT-cross hot path on one MI355X.

Workload: 6D Hilbert tensor 1/(i_1+..+i_6-5), n = 64 per mode (about 6.9e10
entries, never formed), split into a 2x2x2x2x2x2 grid of subtensor blocks,
eps = 1e-8, FP64 throughout; seeds 0..4 in turn.  A step is one complete
tt_cross_run: samples and first pivot, every search sweep until the stop test
holds, and the FP64 cores.  The metric is (entries evaluated + entries
pivoted) per second of wall time over the timed steps; time-to-eps per solve
comes from HIP events inside the library.

The roofline figure is for the search-tile kernel (the residual sweep): its
algorithmic residual traffic per launch over its average launch time, both
from HIP events on the library's stream, against the 8 TB/s HBM peak.  The
CPU baseline is the FP64 oracle timed on this host, single-threaded, over
complete solves of the same workload.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tensor entries evaluated+pivoted/s and time-to-eps; p50/p99 latency for served solves"
N, EPS, GRID, SEEDS = [64] * 6, 1e-8, [2] * 6, [0, 1, 2, 3, 4]
HBM_PEAK_GBS = 8000.0


PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_sweep_hilbert6d_n64_fp64.md")
EVAL_PROFILE = os.path.join(ROOT, "profiles", "k_fn_eval_maxwell6d_n128.md")
VALU_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}


def kernel_sources_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2407_11290_amd", "csrc", "*"))):
        if os.path.basename(p) in ("tt_kernels.h", "tt_device.h"):
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def counted_traffic():
    """Scaled FETCH_SIZE + WRITE_SIZE bytes per search launch from the committed
    rocprofv3 summary, or None when the kernel sources changed since."""
    try:
        with open(PROFILE_SUMMARY) as f:
            kv = dict(line.split(": ", 1) for line in f.read().splitlines()
                      if line.startswith(("traffic_per_launch_bytes:", "kernel_sources_sha256_16:")))
    except OSError:
        return None
    if kv.get("kernel_sources_sha256_16", "").strip() != kernel_sources_hash():
        return None
    return float(kv["traffic_per_launch_bytes"])


def eval_valu_flops():
    """VALU flops per evaluated entry of the bulk evaluation kernel, by
    precision, from the committed rocprofv3 counter summary; None when the
    kernel sources changed since."""
    try:
        with open(EVAL_PROFILE) as f:
            kv = dict(line.split(": ", 1) for line in f.read().splitlines()
                      if line.startswith(("valu_flops_per_entry_", "kernel_sources_sha256_16:")))
    except OSError:
        return None
    if kv.get("kernel_sources_sha256_16", "").strip() != kernel_sources_hash():
        return None
    return {k.split("_")[-1]: float(v) for k, v in kv.items() if k.startswith("valu_flops_per_entry_")}


def bench_eval(args):
    """Entry evaluation alone: the 6D Maxwellian of the phase-space workload
    (n = 128 per mode) at m seeded multi-indices resident on the GPU, in FP32
    (the arithmetic of FP32 sweeps) and in FP64.  A step is one bulk
    evaluation of all m entries."""
    import torch
    from paper_2407_11290_amd import FN_MAXWELL
    from paper_2407_11290_amd.api import fn_eval, fn_eval_last_kernel_ms
    n, m = [128] * 6, args.eval_m
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    idx = torch.randint(0, 128, (m, 6), dtype=torch.int32, device="cuda", generator=gen)
    flops = eval_valu_flops()
    lines = {}
    for prec in ("fp32", "fp64"):
        fp32 = prec == "fp32"
        for _ in range(args.warmup):
            fn_eval(FN_MAXWELL, n, idx, fp32=fp32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms = []
        for _ in range(args.steps):
            fn_eval(FN_MAXWELL, n, idx, fp32=fp32)
            # the kernel's own duration: events attached to its dispatch
            kms.append(fn_eval_last_kernel_ms())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern = statistics.median(kms) * 1e-3
        w = 4 if fp32 else 8
        bytes_per_entry = 4 * 6 + w
        hbm = {"bound": "hbm", "achieved": m * bytes_per_entry / kern / 1e9, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "traffic": None, "bytes_per_entry": bytes_per_entry}
        hbm["frac"] = hbm["achieved"] / hbm["peak"]
        valu = None
        if flops and prec in flops:
            valu = {"bound": "alu", "achieved": flops[prec] * m / kern / 1e12, "peak": VALU_PEAK_TFLOPS[prec],
                    "unit": "TFLOP/s", "flops_per_entry": flops[prec]}
            valu["frac"] = valu["achieved"] / valu["peak"]
        dom = hbm if (valu is None or hbm["frac"] >= valu["frac"]) else valu
        lines[prec] = {"entries_per_s": m * args.steps / wall, "kernel_s": kern, "roofline": dom,
                       "hbm": hbm, "valu": valu}
        print(f"bench: eval {prec}: {args.steps} steps, kernel {kern * 1e6:.1f} us", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import fn_eval as orc_fn_eval
        from oracle.oracle import FN_MAXWELL as O_MAXWELL
        sample = idx[: 1 << 18].cpu().numpy()
        t0, reps = time.perf_counter(), 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
            orc_fn_eval(O_MAXWELL, n, sample)
            reps += 1
        el = time.perf_counter() - t0
        cpu = {"value": reps * sample.shape[0] / el, "unit": "entries/s", "cores": 1, "kind": "oracle",
               "sample": f"the FP64 oracle's generating function at the first {sample.shape[0]} of the same "
                         f"indices, {reps} passes, {el:.1f} s, one host thread"}
    f32 = lines["fp32"]
    out = {
        "metric": METRIC, "value": f32["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f32["kernel_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fn_eval_maxwell6d_n128", "m": m, "fn": "3d3v Maxwellian, x1..x3 periodic, v in [-8,8]"},
        "roofline": f32["roofline"], "fp32": f32, "fp64": lines["fp64"], "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_rook(args):
    """Rook pivoting (Alg. 1 inside every subtensor block) on residual factors:
    the 3D Hilbert tensor with n = 100000 per mode on a 2x2x2 block grid,
    eps = 1e-8, FP64, rank cap 48.  Its superblocks reach 3.4e6 x 3.4e6
    entries (about 9e13 bytes in FP64), far beyond what stored residuals
    could hold; the factors take (rows + columns) x rank.  A step is one
    complete solve.  The rate counts the residuals the searches looked at;
    the roofline figure is the search launches' algorithmic bytes (8 r_k per
    residual: one factor vector streamed) over their HIP-event time."""
    import torch
    from paper_2407_11290_amd import FN_HILBERT, PIVOT_ROOK, PREC_FP64
    from paper_2407_11290_amd.api import TTCross
    n, grid, eps, rmax = [100000] * 3, [2, 2, 2], 1e-8, 48
    h = TTCross(n, eps, FN_HILBERT, seed=0, grid=grid, precision=PREC_FP64, pivot=PIVOT_ROOK, r_max=rmax)
    prof = TTCross(n, eps, FN_HILBERT, seed=0, grid=grid, precision=PREC_FP64, pivot=PIVOT_ROOK, r_max=rmax,
                   profile=1)
    h.run()
    prof.run()
    for _ in range(args.warmup):
        h.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    looked, tte = 0, []
    for _ in range(args.steps):
        if h.run() != 0:
            raise RuntimeError("rook solve did not converge")
        st = h.stats()
        looked += st["pivoted"]
        tte.append(st["time_to_eps_s"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ps = prof.stats()
    achieved = ps["sweep_alg_bytes"] / ps["sweep_kernel_s"] / 1e9
    err = h.sampled_error(1_000_000)
    print(f"bench: rook {args.steps} solves in {elapsed:.3f} s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle
        from oracle.oracle import FN_HILBERT as O_HILBERT
        on = [300] * 3
        t1 = time.perf_counter()
        o = Oracle(on, eps, O_HILBERT, seed=0, pivot="rook", grid=grid)
        o.run()
        el = time.perf_counter() - t1
        cpu = {"value": o.stats()["pivoted"] / el, "unit": "residuals looked at/s", "cores": 1, "kind": "oracle",
               "sample": f"one FP64 oracle rook solve of the 3D Hilbert tensor at n = 300 (the oracle forms whole "
                         f"superblocks and cannot hold n = 100000), {el:.1f} s, one host thread"}
    out = {
        "metric": METRIC, "value": looked / elapsed, "unit": "residuals looked at/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "rook_hilbert3d_n100000_grid2x2x2_eps1e-8_fp64", "rank_cap": rmax,
                   "ranks": [int(x) for x in h.ranks()], "sweeps": h.stats()["sweeps"]},
        "time_to_eps_ms": {"median": statistics.median(tte) * 1e3, "min": min(tte) * 1e3},
        "sampled_rel_error": err,
        "roofline": {"kernel": "rook search launches (sample, column/row steps, finish)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_sweep": ps["sweep_alg_bytes"] / max(1, ps["sweep_launches"]),
                     "search_s_per_solve": ps["sweep_kernel_s"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# The paper's experiments (Sec. 5) at its shapes and prescribed core ranks:
# (name, modes, generating function, ranks of unfoldings 1..d-1, its printed
# time in s, its printed sampled error or None, what the time covers).
PAPER_CASES = [
    ("hilbert3d_n250", [250] * 3, "hilbert", [25, 25], 1.71, 1.27e-6, "Table 6, full approximation, 64 ranks"),
    ("hilbert3d_n500", [500] * 3, "hilbert", [25, 25], 5.06, 9.99e-7, "Table 6, full approximation, 64 ranks"),
    ("hilbert3d_n1000", [1000] * 3, "hilbert", [25, 25], 16.07, 9.07e-7, "Table 6, full approximation, 64 ranks"),
    ("hilbert3d_n2000", [2000] * 3, "hilbert", [25, 25], 60.54, 8.64e-7, "Table 6, full approximation, 64 ranks"),
    ("hilbert6d_n300", [300] * 6, "hilbert", [15, 17, 18, 17, 15], 260.72, None, "Table 5, pivot selection, 64 ranks"),
    ("maxwell2d2v", [2000, 1000, 2000, 1000], "maxwell2d2v", [10, 5, 20], 147.34, None,
     "Table 5, pivot selection, 64 ranks"),
    ("maxwell3d3v", [800, 400, 800, 400, 800, 400], "maxwell3d3v", [10, 5, 30, 5, 20], 184.16, None,
     "Table 5, pivot selection, 64 ranks"),
]


def bench_paper(args):
    """The paper's own workloads at its shapes and prescribed ranks (eps = 0,
    every unfolding runs to its rank), FP64, 2 blocks per mode, greedy
    search.  Per case: time to the prescribed ranks (HIP events inside the
    library) with the default tile shape and with the shape tt_autotune picks
    for the case, and the sampled relative error over 1e6 entries of an
    independent stream, beside the paper's printed time and error, which are
    context (other hardware, 64 CPU processes), not a target.  The line's
    value uses the default-shape times."""
    import torch
    from paper_2407_11290_amd import FN_HILBERT, FN_MAXWELL_2D2V, FN_MAXWELL_3D3V, PREC_FP64
    from paper_2407_11290_amd.api import TTCross
    fns = {"hilbert": FN_HILBERT, "maxwell2d2v": FN_MAXWELL_2D2V, "maxwell3d3v": FN_MAXWELL_3D3V}
    rows = []
    for name, n, fn, caps, t_paper, e_paper, what in PAPER_CASES:
        h = TTCross(n, 0.0, fns[fn], seed=0, grid=[2] * len(n), precision=PREC_FP64)
        h.set_rank_caps(caps)
        h.run()                                   # allocates
        tt = []
        for _ in range(max(1, args.steps)):
            h.run()
            tt.append(h.stats()["time_to_eps_s"])
        st = h.stats()
        err = h.sampled_error(1_000_000)
        # the tile autotuner on the same problem (its table then serves the
        # tuned run; results do not depend on the tile shape)
        t_tune = time.perf_counter()
        tr, tc, _ = h.autotune(reps=2)
        t_tune = time.perf_counter() - t_tune
        h.run()
        tu = []
        for _ in range(max(1, args.steps)):
            h.run()
            tu.append(h.stats()["time_to_eps_s"])
        rows.append({"case": name, "n": n, "ranks": [int(x) for x in h.ranks()], "time_s": statistics.median(tt),
                     "tuned_time_s": statistics.median(tu), "tuned_tiles": [tr, tc], "tune_s": t_tune,
                     "sampled_rel_error": err, "sweeps": st["sweeps"], "evaluated": st["evaluated"],
                     "pivoted": st["pivoted"], "paper_time_s": t_paper, "paper_error": e_paper, "paper_time_is": what})
        print(f"bench: paper {name}: {statistics.median(tt) * 1e3:.1f} ms (tuned {tr}x{tc}: "
              f"{statistics.median(tu) * 1e3:.1f} ms), error {err:.2e}", file=sys.stderr, flush=True)
        h.close()
        torch.cuda.empty_cache()
    total = sum(r["time_s"] for r in rows)
    work = sum(r["evaluated"] + r["pivoted"] for r in rows)
    # roofline: the search kernel of the largest case, timed per launch with
    # dispatch-attached HIP events (a profiled solve)
    big = next(c for c in PAPER_CASES if c[0] == "hilbert3d_n2000")
    ph = TTCross(big[1], 0.0, fns[big[2]], seed=0, grid=[2] * len(big[1]), precision=PREC_FP64, profile=1)
    ph.set_rank_caps(big[3])
    ph.run()
    ph.run()
    ps = ph.stats()
    achieved = ps["sweep_alg_bytes"] / ps["sweep_kernel_s"] / 1e9
    roof = {"kernel": f"k_sweep<double, Hilbert> ({big[0]})", "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": ps["sweep_alg_bytes"] / max(1, ps["sweep_launches"]),
            "avg_launch_us": ps["sweep_kernel_s"] / max(1, ps["sweep_launches"]) * 1e6,
            "launches": ps["sweep_launches"]}
    ph.close()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle
        from oracle.oracle import FN_HILBERT as O_HILBERT
        c0 = PAPER_CASES[0]
        t1 = time.perf_counter()
        o = Oracle(c0[1], 0.0, O_HILBERT, seed=0, rank_caps=c0[3])
        o.run()
        el = time.perf_counter() - t1
        ost = o.stats()
        cpu = {"value": (ost["evaluated"] + ost["pivoted"]) / el, "unit": "entries/s", "cores": 1, "kind": "oracle",
               "sample": f"one FP64 oracle solve of {c0[0]} at ranks {c0[3]}, {el:.1f} s, one host thread"}
    out = {
        "metric": METRIC, "value": work / total, "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": total * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "paper_sec5_workloads_prescribed_ranks_fp64", "cases": [r["case"] for r in rows]},
        "cases": rows, "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(seconds):
    from oracle import Oracle
    from oracle.oracle import FN_HILBERT
    done, work, seeds = 0.0, 0, []
    t0 = time.perf_counter()
    i = 0
    while True:
        seed = SEEDS[i % len(SEEDS)]
        o = Oracle(N, EPS, FN_HILBERT, seed=seed)
        o.run()
        st = o.stats()
        work += st["evaluated"] + st["pivoted"]
        seeds.append(seed)
        i += 1
        done = time.perf_counter() - t0
        if done >= seconds:
            break
    return {"value": work / done, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(seeds)} complete FP64 oracle solves of the same workload, seeds {seeds}, "
                      f"{done:.1f} s, one host thread"}


def bench_batch(args):
    """Mixed batch of 512 problems (d 3..6, n 16..128, Hilbert / bi-Maxwellian,
    eps 1e-6, FP32 sweeps by the precision policy): one batched solve per step
    against the same problems solved one at a time."""
    import torch
    from paper_2407_11290_amd.api import TTCross, batch_run
    from paper_2407_11290_amd.workloads import batch_mix
    specs = batch_mix()
    hs = [TTCross(p.n, p.eps, p.fn_id, p.params, seed=p.seed, grid=p.grid) for p in specs]
    t0 = time.perf_counter()
    batch_run(hs)                                   # allocates every problem's buffers
    print(f"bench: first batch (with allocation) {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        batch_run(hs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch_run(hs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # every timed batch solves the same problems the same way (escalations
    # stick to their handles from the first batch on), so the work of one
    # batch, read after the timed region, counts for each
    work = args.steps * sum(st["evaluated"] + st["pivoted"] for st in (h.stats() for h in hs))
    print(f"bench: {args.steps} batched steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    # the same problems one after another on one stream
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    work1 = 0
    for h in hs:
        h.run()
        st = h.stats()
        work1 += st["evaluated"] + st["pivoted"]
    torch.cuda.synchronize()
    single = time.perf_counter() - t1
    statuses = [h.stats()["status"] for h in hs]
    escal = [i for i, h in enumerate(hs) if h.stats()["escalated"]]
    errs = [h.stats()["sampled_err"] for h in hs]
    out = {
        "metric": METRIC, "value": work / elapsed, "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch512_mixed_d3-6_n16-128_eps1e-6", "problems": len(hs)},
        "solves_per_s": len(hs) / (elapsed / args.steps),
        "one_at_a_time": {"s": single, "entries_per_s": work1 / single, "solves_per_s": len(hs) / single},
        "batched_over_one_at_a_time": single / (elapsed / args.steps),
        "statuses": {str(k): statuses.count(k) for k in sorted(set(statuses))},
        "escalated_to_fp64": escal,
        "sampled_err_max": max(errs),
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Served trace: requests d in {4,5,6}, n in {32,64,128,256}, eps in
    {1e-4, 1e-8} (FP32 / FP64 sweeps by the precision policy), half Hilbert,
    half bi-Maxwellian, rank cap 32, two subtensor blocks per mode.  First the
    whole trace at once (capacity), then Poisson arrivals at rate_frac of that
    capacity (latency = completion - arrival, queueing included), then the
    first requests one at a time through the single-solve path."""
    from paper_2407_11290_amd.api import Server, TTCross
    from paper_2407_11290_amd.workloads import served_trace
    N = args.requests
    specs = served_trace(count=N)
    srv = Server(int(args.budget_gib * (1 << 30)), max_slots=args.slots, r_max=32, grid=2)

    def run_all(arrivals):
        t0 = time.perf_counter()
        tickets = []
        for p, a in zip(specs, arrivals):
            while True:
                dt = t0 + a - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.001))
            tickets.append(srv.submit(p.n, p.eps, p.fn_id, p.params, seed=p.seed))
        lat, work, st = [], 0, {}
        for t in tickets:
            code, l = srv.wait(t)
            s, _ = srv.result(t)
            srv.release(t)
            lat.append(l)
            work += s["evaluated"] + s["pivoted"]
            st[code] = st.get(code, 0) + 1
        return time.perf_counter() - t0, lat, work, st

    # warm-up: one request of every shape, so that the pool holds its buffers
    seen, warm = set(), []
    for p in specs:
        key = (tuple(p.n), p.eps >= 1e-6)
        if key not in seen:
            seen.add(key)
            warm.append(srv.submit(p.n, p.eps, p.fn_id, p.params, seed=p.seed))
    for t in warm:
        srv.wait(t)
        srv.release(t)
    print(f"bench: warm-up {len(warm)} shapes, pool {srv.stats()['pool_bytes'] / 2**30:.1f} GiB",
          file=sys.stderr, flush=True)
    cap_s, cap_lat, cap_work, cap_st = run_all([0.0] * N)
    capacity = N / cap_s
    print(f"bench: closed loop {N} requests in {cap_s:.2f} s ({capacity:.0f} solves/s)", file=sys.stderr, flush=True)
    def pct(v, q):
        v = sorted(v)
        return v[min(len(v) - 1, int(q * len(v)))] * 1e3

    sweep = []
    for frac in (0.25, 0.5, 1.0, 1.25):
        r = frac * capacity
        s_, l_, _w, _st = run_all([p.arrival_s for p in served_trace(count=N, rate_hz=r)])
        sweep.append({"rate_frac": frac, "rate_per_s": r, "solves_per_s": N / s_, "p50_ms": pct(l_, 0.5),
                      "p99_ms": pct(l_, 0.99)})
        print(f"bench: open loop at {frac:.2f} x capacity: p50 {pct(l_, 0.5):.2f} ms p99 {pct(l_, 0.99):.2f} ms",
              file=sys.stderr, flush=True)
    rate = args.rate_frac * capacity
    arrivals = [p.arrival_s for p in served_trace(count=N, rate_hz=rate)]
    open_s, lat, work, st = run_all(arrivals)
    lat_ms = sorted(x * 1e3 for x in lat)
    print(f"bench: open loop at {rate:.0f}/s done in {open_s:.2f} s", file=sys.stderr, flush=True)
    srv_stats = srv.stats()
    srv.close()
    # one at a time: the first requests through the single-solve path, each on
    # a handle whose buffers already exist (allocation is not timed)
    M = min(args.alone, N)
    hs = [TTCross(p.n, p.eps, p.fn_id, p.params, seed=p.seed, r_max=32, grid=p.grid) for p in specs[:M]]
    for h in hs:
        h.run()
    t1 = time.perf_counter()
    for h in hs:
        h.run()
    alone_s = time.perf_counter() - t1
    for h in hs:
        h.close()
    out = {
        "metric": METRIC, "value": work / open_s, "unit": "entries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": open_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"serve_poisson_{N}req_d4-6_n32-256_eps1e-4or1e-8", "requests": N,
                   "rate_per_s": rate, "rate_frac_of_capacity": args.rate_frac, "budget_gib": args.budget_gib},
        "latency_ms": {"p50": lat_ms[len(lat_ms) // 2], "p99": lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))],
                       "max": lat_ms[-1]},
        "solves_per_s": N / open_s, "capacity_solves_per_s": capacity,
        "closed_loop_entries_per_s": cap_work / cap_s,
        "lambda_sweep": sweep,
        "one_at_a_time": {"requests": M, "s": alone_s, "solves_per_s": M / alone_s},
        "statuses": {str(k): v for k, v in sorted(st.items())},
        "server": srv_stats,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="hilbert6d", choices=["hilbert6d", "batch512", "serve", "eval", "rook", "paper"],
                    help="hilbert6d: the single-solve benchmark line; batch512: the mixed 512-problem "
                         "batch, solved together and one at a time; serve: a Poisson-arrival trace "
                         "through the continuous-batching server; eval: bulk entry evaluation of the 6D "
                         "Maxwellian in FP32 and FP64; rook: rook pivoting on the 3D Hilbert tensor with "
                         "n = 100000 per mode; paper: the paper's Sec. 5 workloads at its shapes and "
                         "prescribed ranks")
    ap.add_argument("--eval-m", type=int, default=1 << 24, help="eval: multi-indices per step")
    ap.add_argument("--requests", type=int, default=2000, help="serve: trace length")
    ap.add_argument("--rate-frac", type=float, default=0.8, help="serve: arrival rate / measured capacity")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serve: HBM budget of the server")
    ap.add_argument("--alone", type=int, default=200, help="serve: requests timed one at a time")
    ap.add_argument("--slots", type=int, default=64, help="serve: solves in flight at most")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain copy kernel (out = -in, FP64) over this many MiB, five times; "
                         "its FETCH_SIZE/WRITE_SIZE counters scale the search kernel's")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; a solve is not sharded across GPUs "
              "(see DESIGN.md for how it would shard). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.init()
    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy": {"bytes_read": nbytes, "bytes_written": nbytes, "launches": 5}}), flush=True)
        return
    from paper_2407_11290_amd import FN_HILBERT, PREC_FP64
    from paper_2407_11290_amd.api import TTCross
    if args.workload == "batch512":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "eval":
        return bench_eval(args)
    if args.workload == "rook":
        return bench_rook(args)
    if args.workload == "paper":
        return bench_paper(args)

    handles = [TTCross(N, EPS, FN_HILBERT, seed=s, precision=PREC_FP64, grid=GRID) for s in SEEDS]
    probes = [TTCross(N, EPS, FN_HILBERT, seed=s, precision=PREC_FP64, grid=GRID, profile=1) for s in SEEDS]
    for h in handles + probes:               # allocates device state; inputs resident from here on
        h.run()
    for i in range(args.warmup):
        handles[i % len(handles)].run()
    print(f"bench: warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # timed region: K complete solves, nothing else on the stream
    work, tte = 0, []
    ranks = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        h = handles[i % len(handles)]
        st_code = h.run()
        st = h.stats()
        work += st["evaluated"] + st["pivoted"]
        tte.append(st["time_to_eps_s"])
        if st_code != 0:
            raise RuntimeError(f"solve returned status {st_code}")
        ranks = st["ranks"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"bench: timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # kernel timing: the same solves again with HIP events around every
    # search-tile launch on the library's stream (events add ~4 us per launch,
    # so they stay out of the throughput pass above)
    kern_s, kern_bytes, launches, phase_s = 0.0, 0.0, 0, 0.0
    for i in range(args.steps):
        h = probes[i % len(probes)]
        h.run()
        st = h.stats()
        kern_s += st["sweep_kernel_s"]
        kern_bytes += st["sweep_alg_bytes"]
        launches += st["sweep_launches"]
        phase_s += st["sweep_phase_s"]

    avg_launch = kern_s / max(launches, 1)
    bytes_per_launch = kern_bytes / max(launches, 1)
    achieved = bytes_per_launch / avg_launch / 1e9 if avg_launch > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": work / elapsed,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hilbert6d_n64_grid2x2x2x2x2x2_eps1e-8_fp64", "d": 6, "n": 64,
                   "grid": GRID, "eps": EPS, "seeds": SEEDS, "ranks_last": ranks},
        "time_to_eps_ms": {"median": statistics.median(tte) * 1e3, "min": min(tte) * 1e3},
        "roofline": {"kernel": "k_sweep<double, Hilbert>", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": counted_traffic(),
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_launch * 1e6,
                     "launches": launches,
                     "sweep_phase_us_per_solve": phase_s / args.steps * 1e6,
                     "sweep_kernels_us_per_solve": kern_s / args.steps * 1e6},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
