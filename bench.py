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
CPU baseline is the FP64 oracle timed on this host over complete solves of
the same workload, in host threads on every usable core (at most 16), with
the CPU model, the CPU count and a single-thread figure beside it.

The same line carries measured summaries of the other configurations: the 6D
Maxwellian with FP32 sweeps (time-to-eps, error against FP64 entries), the
mixed 512-problem batch (batched against one at a time) and a served trace
(p50/p99 latency over three Poisson runs, capacity against the same request
list one at a time).  --workload selects one of them alone, with its own
roofline figure.
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

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


# The accuracy panels of Sec. 5.2/5.3: the four workloads of Table 5 with every
# core rank raised step by step to its prescribed value (rank m uses
# min(m, r_k) for unfolding k, from m = 2), the sampled error of Sec. 5 at
# each step, and the share of the tensor's entries that the run evaluated.
ERROR_CURVE_CASES = ["hilbert3d_n2000", "hilbert6d_n300", "maxwell2d2v", "maxwell3d3v"]


def paper_error_curves(fns, samples=1_000_000):
    """Per case: [(ranks, sampled error, evaluated / prod(n), device ms)]."""
    import torch
    from paper_2407_11290_amd import PREC_FP64
    from paper_2407_11290_amd.api import TTCross
    out = {}
    for name, n, fn, caps, *_ in PAPER_CASES:
        if name not in ERROR_CURVE_CASES:
            continue
        total = float(np.prod([float(x) for x in n]))
        h = TTCross(n, 0.0, fns[fn], seed=0, grid=[2] * len(n), precision=PREC_FP64, r_max=max(caps))
        rows = []
        for m in range(2, max(caps) + 1):
            step = [min(m, c) for c in caps]
            if rows and step == rows[-1]["ranks"][1:-1]:
                continue
            h.set_rank_caps(step)
            h.run()
            st = h.stats()
            rows.append({"ranks": [int(x) for x in h.ranks()], "sampled_rel_error": h.sampled_error(samples),
                         "evaluated_fraction": st["evaluated"] / total, "time_ms": st["time_to_eps_s"] * 1e3})
        out[name] = rows
        print(f"bench: error curve {name}: {len(rows)} points, last error {rows[-1]['sampled_rel_error']:.2e}",
              file=sys.stderr, flush=True)
        h.close()
        torch.cuda.empty_cache()
    return out


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
        "error_curves": paper_error_curves(fns),
    }
    print(json.dumps(out), flush=True)


MAXWELL_N, MAXWELL_EPS, MAXWELL_SEEDS = [128] * 6, 1e-6, [0, 1, 2, 3, 4]


def measure_maxwell6d(steps, profile=False):
    """The 6D Maxwellian phase-space tensor (x1,x2,x3 periodic on [0,1),
    v in [-8,8]^3 cell centres, n = 128 per mode, 2^6 subtensor blocks),
    eps = 1e-6, the precision policy's FP32 entry evaluation and sweeps with
    the FP64 candidate check, stop test, pivot block and cores, and the
    policy's 4096-sample check; seeds 0..4 in turn.  Per solve: device
    time-to-eps, and the sampled relative error of the result over 1e6
    indices against the tensor's FP64 entries."""
    import torch
    from paper_2407_11290_amd import FN_MAXWELL
    from paper_2407_11290_amd.api import TTCross
    hs = [TTCross(MAXWELL_N, MAXWELL_EPS, FN_MAXWELL, seed=s, grid=[2] * 6, profile=1 if profile else 0)
          for s in MAXWELL_SEEDS]
    for h in hs:
        h.run()                                    # allocates
    tte, work, errs, prec, esc = [], 0, [], set(), 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        h = hs[i % len(hs)]
        if h.run() != 0:
            raise RuntimeError("maxwellian solve did not meet eps")
        st = h.stats()
        tte.append(st["time_to_eps_s"])
        work += st["evaluated"] + st["pivoted"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for h in hs:
        st = h.stats()
        prec.add("fp32" if st["precision_used"] == 2 else "fp64")
        esc += st["escalated"]
        errs.append(h.sampled_error(1_000_000, seed=12345))
    out = {"workload": "maxwell6d_n128_grid2x2x2x2x2x2_eps1e-6_fp32sweeps", "solves": steps,
           "time_to_eps_ms": {"median": statistics.median(tte) * 1e3, "min": min(tte) * 1e3},
           "entries_per_s": work / wall, "ms_per_solve_wall": wall / steps * 1e3,
           "ranks": [int(x) for x in hs[0].ranks()], "sweep_precision": sorted(prec), "escalated": esc,
           "sampled_rel_error_vs_fp64_entries": {"max": max(errs), "per_seed": errs, "R": 1_000_000},
           "policy_check_error_max": max(h.stats()["sampled_err"] for h in hs)}
    if profile:
        ks = kb = kl = 0.0
        for h in hs:
            h.run()
            st = h.stats()
            ks += st["sweep_kernel_s"]
            kb += st["sweep_alg_bytes"]
            kl += st["sweep_launches"]
        out["search_kernel"] = {"avg_launch_us": ks / max(kl, 1) * 1e6, "bytes_per_launch": kb / max(kl, 1),
                                "launches": int(kl)}
    for h in hs:
        h.close()
    return out


def measure_batch(steps, warmup=1):
    """The mixed 512-problem batch solved together (tt_batch_run) against the
    same problems one at a time on their own handles (buffers allocated
    before timing in both)."""
    import torch
    from paper_2407_11290_amd.api import TTCross, batch_run
    from paper_2407_11290_amd.workloads import batch_mix
    specs = batch_mix()
    hs = [TTCross(p.n, p.eps, p.fn_id, p.params, seed=p.seed, grid=p.grid) for p in specs]
    t0 = time.perf_counter()
    batch_run(hs)                                   # allocates every problem's buffers
    first = time.perf_counter() - t0
    for _ in range(warmup):
        batch_run(hs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch_run(hs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # every timed batch solves the same problems the same way (escalations
    # stick to their handles from the first batch on)
    work = steps * sum(st["evaluated"] + st["pivoted"] for st in (h.stats() for h in hs))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for h in hs:
        h.run()
    torch.cuda.synchronize()
    single = time.perf_counter() - t1
    stats = [h.stats() for h in hs]
    statuses = [s["status"] for s in stats]
    for h in hs:
        h.close()
    return {"workload": "batch512_mixed_d3-6_n16-128_eps1e-6", "problems": len(hs), "batches": steps,
            "ms_per_batch": elapsed / steps * 1e3, "solves_per_s": len(hs) * steps / elapsed,
            "entries_per_s": work / elapsed, "first_batch_with_allocation_s": first,
            "one_at_a_time": {"s": single, "solves_per_s": len(hs) / single},
            "batched_over_one_at_a_time": single / (elapsed / steps),
            "statuses": {str(k): statuses.count(k) for k in sorted(set(statuses))},
            "escalated_to_fp64": [i for i, s in enumerate(stats) if s["escalated"]],
            "sampled_err_max": max(s["sampled_err"] for s in stats)}


def measure_escalation():
    """The precision policy's escalation decision (FP32 sweeps missed eps?)
    taken on the 4096-sample check against the same decision on 1e6
    samples: every problem solved with FP32 sweeps and no check, then the
    sampled error of its FP32 result over the first 4096 and the first 1e6
    indices of the check stream (seed + 1; the small set is the large one's
    prefix).  Problems: the 512-problem batch mix and the 6D Maxwellian
    (n = 128, 2^6 blocks, eps = 1e-6) over seeds 0..9."""
    import numpy as np
    from paper_2407_11290_amd import FN_MAXWELL, PREC_FP32
    from paper_2407_11290_amd.api import TTCross, batch_run
    from paper_2407_11290_amd.workloads import batch_mix
    specs = batch_mix()
    rows = []
    hs = [TTCross(p.n, p.eps, p.fn_id, p.params, seed=p.seed, grid=p.grid, precision=PREC_FP32, verify=0)
          for p in specs]
    batch_run(hs)
    for p, h in zip(specs, hs):
        rows.append(("batch", p.eps, h.sampled_error(4096, seed=p.seed + 1),
                     h.sampled_error(1_000_000, seed=p.seed + 1)))
        h.close()
    for s in range(10):
        h = TTCross(MAXWELL_N, MAXWELL_EPS, FN_MAXWELL, seed=s, grid=[2] * 6, precision=PREC_FP32, verify=0)
        h.run()
        rows.append(("maxwell6d", MAXWELL_EPS, h.sampled_error(4096, seed=s + 1),
                     h.sampled_error(1_000_000, seed=s + 1)))
        h.close()
    out = {}
    for name in ("batch", "maxwell6d"):
        r = [x for x in rows if x[0] == name]
        eps = np.array([x[1] for x in r])
        e4 = np.array([x[2] for x in r])
        e6 = np.array([x[3] for x in r])
        ratio = e4 / np.maximum(e6, 1e-300)
        near = (e6 > 0.3 * eps) & (e6 < 3 * eps)
        out[name] = {"problems": len(r),
                     "ratio_4096_over_1e6": {"median": float(np.median(ratio)), "min": float(ratio.min()),
                                             "max": float(ratio.max())},
                     "err_1e6_over_eps": {"median": float(np.median(e6 / eps)), "max": float((e6 / eps).max())},
                     "escalate_on_4096": int((e4 > eps).sum()), "escalate_on_1e6": int((e6 > eps).sum()),
                     "missed_by_4096": int(((e6 > eps) & (e4 <= eps)).sum()),
                     "extra_by_4096": int(((e4 > eps) & (e6 <= eps)).sum()),
                     "near_eps": int(near.sum()),
                     "near_eps_ratio": ({"min": float(ratio[near].min()), "max": float(ratio[near].max())}
                                        if near.any() else None)}
    return out


def bench_escalation(args):
    out = measure_escalation()
    print(json.dumps({"metric": METRIC, "value": None, "unit": "problems", "n_gpus": 1, "steps": 1, "warmup": 0,
                      "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "escalation_check_4096_vs_1e6_samples"}, "escalation": out}),
          flush=True)


def _pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(q * len(v)))] * 1e3


def measure_serve(requests, repeats=3, rate_frac=0.8, budget_gib=64.0, slots=64, sweep=False):
    """A served trace through the continuous-batching server: requests d in
    {4,5,6}, n in {32,64,128,256}, eps in {1e-4,1e-8} (FP32 / FP64 sweeps by
    the precision policy), half Hilbert, half bi-Maxwellian, rank cap 32, two
    subtensor blocks per mode.  Capacity: the whole list submitted at once
    (the median of three passes, after one pass that lets the pool allocate).
    Latency (completion - arrival, queueing included): Poisson arrivals at
    rate_frac of the capacity, repeated.  One at a time: the same list
    through the single-solve path, each request on a handle whose buffers
    exist before its solve is timed."""
    import torch
    from paper_2407_11290_amd.api import Server, TTCross
    from paper_2407_11290_amd.workloads import served_trace
    N = requests
    specs = served_trace(count=N)
    srv = Server(int(budget_gib * (1 << 30)), max_slots=slots, r_max=32, grid=2)

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
    # capacity: the whole list at once, after one such pass that lets the
    # pool reach the objects a full pass needs (the median of three passes)
    run_all([0.0] * N)
    caps = [run_all([0.0] * N) for _ in range(3)]
    cap_s, _l, cap_work, cap_st = sorted(caps, key=lambda c: c[0])[1]
    capacity = N / cap_s
    runs = []
    for r in range(repeats):
        arrivals = [p.arrival_s for p in served_trace(count=N, rate_hz=rate_frac * capacity)]
        s_, l_, w_, st_ = run_all(arrivals)
        runs.append({"s": s_, "p50_ms": _pct(l_, 0.5), "p99_ms": _pct(l_, 0.99), "solves_per_s": N / s_,
                     "entries_per_s": w_ / s_, "statuses": {str(k): v for k, v in sorted(st_.items())}})
    lam = []
    if sweep:
        for frac in (0.25, 0.5, 1.0, 1.25):
            s_, l_, _w, _st = run_all([p.arrival_s for p in served_trace(count=N, rate_hz=frac * capacity)])
            lam.append({"rate_frac": frac, "solves_per_s": N / s_, "p50_ms": _pct(l_, 0.5), "p99_ms": _pct(l_, 0.99)})
    srv_stats = srv.stats()
    srv.close()
    torch.cuda.empty_cache()
    # one at a time, the same list
    alone, alone_work = 0.0, 0
    for p in specs:
        h = TTCross(p.n, p.eps, p.fn_id, p.params, seed=p.seed, r_max=32, grid=p.grid)
        h.run()                                        # allocates
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h.run()
        alone += time.perf_counter() - t1
        st = h.stats()
        alone_work += st["evaluated"] + st["pivoted"]
        h.close()
    p50s = [r["p50_ms"] for r in runs]
    p99s = [r["p99_ms"] for r in runs]
    return {"workload": f"serve_poisson_{N}req_d4-6_n32-256_eps1e-4or1e-8", "requests": N,
            "rate_frac_of_capacity": rate_frac, "budget_gib": budget_gib, "slots": slots,
            "capacity_solves_per_s": capacity, "capacity_entries_per_s": cap_work / cap_s,
            "latency_ms": {"p50_median": statistics.median(p50s), "p99_median": statistics.median(p99s),
                           "p50_runs": p50s, "p99_runs": p99s},
            "open_loop_runs": runs, "lambda_sweep": lam,
            "one_at_a_time": {"s": alone, "solves_per_s": N / alone, "entries_per_s": alone_work / alone},
            "served_capacity_over_one_at_a_time": capacity / (N / alone),
            "server": srv_stats}


def host_cpu():
    """CPU model and logical CPU count of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline_all_cores(seconds):
    """The FP64 oracle on the bench workload, complete solves of seeds 0..4 in
    turn, run side by side in host threads on every usable core (at most 16,
    the host share of one GPU), then single-threaded for comparison."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import Oracle
    from oracle.oracle import FN_HILBERT
    model, nproc, usable = host_cpu()
    threads = max(1, min(16, usable))

    def worker(w):
        done, work, solves = 0.0, 0, 0
        t0 = time.perf_counter()
        i = w
        while done < seconds:
            o = Oracle(N, EPS, FN_HILBERT, seed=SEEDS[i % len(SEEDS)])
            o.run()
            st = o.stats()
            work += st["evaluated"] + st["pivoted"]
            solves += 1
            i += threads
            done = time.perf_counter() - t0
        return work, solves, done

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(worker, range(threads)))
    wall = time.perf_counter() - t0
    work = sum(r[0] for r in res)
    solves = sum(r[1] for r in res)
    single = cpu_baseline(min(4.0, seconds))
    return {"value": work / wall, "unit": "entries/s", "cores": threads, "kind": "oracle",
            "sample": f"{solves} complete FP64 oracle solves of the same workload (seeds 0..4 in turn) in "
                      f"{threads} host threads side by side, {wall:.1f} s",
            "cpu_model": model, "nproc": nproc, "usable_cpus": usable,
            "single_thread": {"value": single["value"], "sample": single["sample"]}}


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
    m = measure_batch(args.steps, args.warmup)
    print(f"bench: {args.steps} batched steps, {m['ms_per_batch']:.2f} ms per batch", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": m["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_batch"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": m["workload"], "problems": m["problems"]},
    }
    out.update({k: v for k, v in m.items() if k not in ("workload", "problems")})
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Served trace through the continuous-batching server (see
    measure_serve): capacity, Poisson-arrival latency at rate_frac of the
    capacity (three runs) and a rate sweep, and the same request list one at
    a time through the single-solve path."""
    m = measure_serve(args.requests, repeats=3, rate_frac=args.rate_frac, budget_gib=args.budget_gib,
                      slots=args.slots, sweep=True)
    print(f"bench: serve capacity {m['capacity_solves_per_s']:.0f} solves/s, p50/p99 "
          f"{m['latency_ms']['p50_median']:.2f}/{m['latency_ms']['p99_median']:.2f} ms", file=sys.stderr, flush=True)
    run = m["open_loop_runs"][0]
    out = {
        "metric": METRIC, "value": run["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": run["s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": m["workload"], "requests": m["requests"], "rate_frac_of_capacity": args.rate_frac,
                   "budget_gib": args.budget_gib},
    }
    out.update({k: v for k, v in m.items() if k not in ("workload", "requests")})
    print(json.dumps(out), flush=True)


MAXWELL_PROFILE = os.path.join(ROOT, "profiles", "k_sweep_maxwell6d_n128_fp32.md")


def sweep_valu_flops(path):
    """FP32 VALU flops per search launch from a committed rocprofv3 counter
    summary; None when the kernel sources changed since."""
    try:
        with open(path) as f:
            kv = dict(line.split(": ", 1) for line in f.read().splitlines()
                      if line.startswith(("valu_flops_per_launch:", "kernel_sources_sha256_16:",
                                          "traffic_per_launch_bytes:")))
    except OSError:
        return None
    if kv.get("kernel_sources_sha256_16", "").strip() != kernel_sources_hash():
        return None
    return {k: float(v) for k, v in kv.items() if k != "kernel_sources_sha256_16"}


def bench_maxwell(args):
    """The 6D Maxwellian phase-space configuration alone (see
    measure_maxwell6d): FP32 entry evaluation and sweeps, FP64 check, stop
    test, pivot block and cores.  The roofline figure is for its search
    kernel k_sweep<float, generic>, where the in-solve entry evaluation runs:
    HBM (algorithmic bytes over the dispatch-attached event time) and, from
    the committed counter summary, FP32 VALU flops per launch."""
    m = measure_maxwell6d(args.steps, profile=True)
    sk = m["search_kernel"]
    us = sk["avg_launch_us"]
    hbm = {"bound": "hbm", "achieved": sk["bytes_per_launch"] / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS,
           "unit": "GB/s"}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    prof = sweep_valu_flops(MAXWELL_PROFILE)
    hbm["traffic"] = prof.get("traffic_per_launch_bytes") if prof else None
    valu = None
    if prof and "valu_flops_per_launch" in prof:
        valu = {"bound": "alu", "achieved": prof["valu_flops_per_launch"] / (us * 1e-6) / 1e12,
                "peak": VALU_PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                "flops_per_launch": prof["valu_flops_per_launch"]}
        valu["frac"] = valu["achieved"] / valu["peak"]
    roof = dict(hbm if (valu is None or hbm["frac"] >= valu["frac"]) else valu)
    roof.update({"kernel": "k_sweep<float, generic>", "avg_launch_us": us, "launches": sk["launches"],
                 "bytes_per_launch": sk["bytes_per_launch"], "hbm": hbm, "valu": valu})
    out = {
        "metric": METRIC, "value": m["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": m["ms_per_solve_wall"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": m["workload"], "seeds": MAXWELL_SEEDS},
        "time_to_eps_ms": m["time_to_eps_ms"], "roofline": roof,
        "sampled_rel_error_vs_fp64_entries": m["sampled_rel_error_vs_fp64_entries"], "ranks": m["ranks"],
        "sweep_precision": m["sweep_precision"], "escalated": m["escalated"],
    }
    print(json.dumps(out), flush=True)


def bench_phases(args):
    """Where a sweep's time goes: the bench workload solved with the
    instrumented library (libttcross_stamps.so), whose search and commit
    kernels record the device's 100 MHz clock at phase boundaries
    (tt_cross_get_stamps).  Per sweep: the search launch's span (first
    workgroup entry to last workgroup end), each workgroup's phases, the
    commit's phases and the gaps between the launches; averaged over the
    sweeps of args.steps solves.  The instrumentation adds a few stores per
    workgroup, so absolute times are slightly above the normal build's."""
    import ctypes as C
    import numpy as np
    from paper_2407_11290_amd import FN_HILBERT, PREC_FP64, _lib
    from paper_2407_11290_amd.api import TTCross
    assert _lib.LIB_PATH.endswith("libttcross_stamps.so"), _lib.LIB_PATH
    L = _lib.load()
    hs = [TTCross(N, EPS, FN_HILBERT, seed=s, precision=PREC_FP64, grid=GRID) for s in SEEDS]
    for h in hs:
        h.run()
    tick_us = 0.01                                          # 100 MHz clock
    acc = {}

    def add(key, vals):
        vals = [float(v) * tick_us for v in vals]
        if vals:
            acc.setdefault(key, []).extend(vals)

    sweeps_total, solves = 0, 0
    for i in range(args.steps):
        h = hs[i % len(hs)]
        h.run()
        lay = (C.c_int32 * 4)()
        m = L.tt_cross_get_stamps(h.h, None, 0, lay)
        buf = np.zeros(m, dtype=np.uint64)
        _lib.check(L.tt_cross_get_stamps(h.h, buf.ctypes.data_as(C.c_void_p), m, lay))
        W16, W, S, nsw = lay[0], lay[1], lay[2], lay[3]
        search = buf[: S * W * W16].reshape(S, W, W16).astype(np.int64)
        commit = buf[S * W * W16:].reshape(S, W16).astype(np.int64)
        prev_commit_end = None
        for s in range(min(nsw, S)):
            r = search[s]
            act = (r[:, 0] != 0) & (r[:, 9] != 0)
            if not act.any():
                continue
            r = r[act]
            t0, t1 = r[:, 0].min(), r[:, 9].max()
            add("search_span", [t1 - t0])
            add("search_entry_spread", [r[:, 0].max() - t0])
            add("wg_state_load", r[:, 1] - r[:, 0])
            add("wg_total", r[:, 9] - r[:, 0])
            nt = r[r[:, 10] > 0]
            add("new_tile_geometry", nt[:, 2] - nt[:, 1])
            add("new_tile_staging", nt[:, 3] - nt[:, 2])
            add("new_tile_raw_factors", nt[:, 4] - nt[:, 3])
            add("new_tile_factor_solves", nt[:, 5] - nt[:, 4])
            add("new_tile_entries", nt[:, 6] - nt[:, 5])
            add("new_tile_entries_loop", nt[:, 12] - nt[:, 5])
            add("new_tile_reduce", nt[:, 6] - nt[:, 12])
            for kind, name in ((3, "new_rows"), (2, "new_cols"), (1, "new_both")):
                kt = nt[nt[:, 13] == kind]
                add(f"raw_factors_{name}", kt[:, 4] - kt[:, 3])
                add(f"factor_solves_{name}", kt[:, 5] - kt[:, 4])
            st = r[(r[:, 7] > 0) & (r[:, 10] == 0)]
            add("stored_tile_geometry", st[:, 7] - st[:, 1])
            add("stored_tile_data", st[:, 8] - st[:, 7])
            add("new_tiles_per_launch", [int((r[:, 10]).sum()) / tick_us])
            add("workgroups_per_launch", [int(act.sum()) / tick_us])
            c = commit[s]
            if c[0] and c[4]:
                add("gap_search_to_commit", [c[0] - t1])
                add("commit_span", [c[4] - c[0]])
                add("commit_state_load", [c[1] - c[0]])
                add("commit_candidate_scan", [c[2] - c[1]])
                add("commit_decide_append", [c[3] - c[2]])
                add("commit_shapes_publish", [c[4] - c[3]])
                if prev_commit_end is not None:
                    add("gap_commit_to_search", [t0 - prev_commit_end])
                prev_commit_end = c[4]
            sweeps_total += 1
        solves += 1
    out = {"metric": METRIC, "value": None, "unit": "us", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "hilbert6d_n64_grid2x2x2x2x2x2_eps1e-8_fp64_phase_stamps", "solves": solves,
                      "sweeps": sweeps_total},
           "phases_us": {k: {"mean": float(np.mean(v)), "median": float(np.median(v)), "p90": float(np.percentile(v, 90)),
                             "n": len(v)} for k, v in acc.items()}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="hilbert6d",
                    choices=["hilbert6d", "maxwell6d", "batch512", "serve", "eval", "rook", "paper", "phases",
                             "escalation"],
                    help="hilbert6d: the single-solve benchmark line (with summaries of the other "
                         "configurations); maxwell6d: the 6D Maxwellian with FP32 sweeps; batch512: the mixed 512-problem "
                         "batch, solved together and one at a time; serve: a Poisson-arrival trace "
                         "through the continuous-batching server; eval: bulk entry evaluation of the 6D "
                         "Maxwellian in FP32 and FP64; rook: rook pivoting on the 3D Hilbert tensor with "
                         "n = 100000 per mode; paper: the paper's Sec. 5 workloads at its shapes and "
                         "prescribed ranks; escalation: the policy's 4096-sample check against 1e6 samples")
    ap.add_argument("--eval-m", type=int, default=1 << 24, help="eval: multi-indices per step")
    ap.add_argument("--requests", type=int, default=2000, help="serve: trace length")
    ap.add_argument("--no-extras", action="store_true",
                    help="hilbert6d: leave out the summaries of the Maxwellian, batch and serving configurations")
    ap.add_argument("--extra-requests", type=int, default=400, help="hilbert6d: served requests in the summary")
    ap.add_argument("--rate-frac", type=float, default=0.8, help="serve: arrival rate / measured capacity")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serve: HBM budget of the server")
    ap.add_argument("--slots", type=int, default=64, help="serve: solves in flight at most")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain copy kernel (out = -in, FP64) over this many MiB, five times; "
                         "its FETCH_SIZE/WRITE_SIZE counters scale the search kernel's")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; a solve is not sharded across GPUs "
              "(see DESIGN.md for how it would shard). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "phases":
        os.environ["TT_CROSS_LIB"] = "stamps"           # the instrumented library
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
    if args.workload == "maxwell6d":
        return bench_maxwell(args)
    if args.workload == "phases":
        return bench_phases(args)
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
    if args.workload == "escalation":
        return bench_escalation(args)

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
    if not args.no_extras:
        # the other configurations of the workload list, measured in the same
        # run: the 6D Maxwellian with FP32 sweeps, the 512-problem batch and
        # the served trace (their own workloads give the full lines)
        out["maxwell6d_fp32"] = measure_maxwell6d(10)
        print("bench: maxwellian summary done", file=sys.stderr, flush=True)
        out["batch512"] = measure_batch(5)
        print("bench: batch summary done", file=sys.stderr, flush=True)
        out["serve"] = measure_serve(args.extra_requests, repeats=3)
        print("bench: serving summary done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_all_cores(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
