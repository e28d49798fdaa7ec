#!/usr/bin/env python
"""Throughput of the spectral ETD2RK-DS step on one MI355X.

A step is one full time step of the Pade-based dimension-split scheme (the
z, y and fused x stages with both reaction evaluations) over the 3-D
Fisher-KPP workload: 255^3 interior points, kappa = 0.005, q = 0.5,
f = u(1-u), tau = 0.005, seeded sine-plus-Gaussian-bumps initial data.  The
headline value is grid-point updates per second (n^3 * steps / wall seconds)
in FP64; the reduced-precision variant is timed beside it and its relative L2
distance to the FP64 result is reported.

Prints one JSON line.  Options: --steps K (timed steps), --warmup W,
--precision fp64|fp32|bf16x6, --reduced fp32,bf16x6|none, --cpu-steps S and
--cpu-seconds T (oracle sample: chunks of S steps until T seconds),
--no-cpu-baseline, --n (grid size per direction), --adjoint-steps N (the
adjoint leg: one gradient of 1/2||u(T) - u_target||^2 through N steps of the
3-D FitzHugh-Nagumo workload, 127^3, FP32; 0 skips it), --batched-steps N
(256 uneven 2-D Fisher-KPP instances, n in {127, 255, 511, 1023}, FP32, in one
batch: default tiles, autotuned tiles and a captured HIP graph; 0 skips it),
--latency-steps N (the 63^2 Fisher-KPP case, eager calls vs a graph),
--exact-steps N (the headline workload with the exact-exponential factors
e^{-z}, phi_1, phi_2 in place of the Pade ones, FP64), --fhn2d-steps N (the
2-D coupled FitzHugh-Nagumo workload, 511^2 x 2 components, FP64 and FP32
from the same u0; 0 skips it).
"""
import argparse
import hashlib
import json
import math
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/sec (m^d x steps) at 3D m=255, FP64 vs reduced at <=1e-6"
# dense matrix-core peaks (MI355X datasheet); split-BF16 products are priced
# at the BF16 rate, six MFMA terms per product
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x6": 2500.0 / 6, "fp64_fp32": 157.3, "fp64_bf16x6": 2500.0 / 6}
PRECISIONS = ["fp64", "fp32", "bf16x6", "fp64_fp32", "fp64_bf16x6"]
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x6": "bf16x6->f32", "fp64_fp32": "f64 state, f32 products",
         "fp64_bf16x6": "f64 state, bf16x6->f32 products"}
STAGE_NAMES = ("z_stage", "y_stage", "x_stage")
# mode products per launch of each stage kind (3-D): z and y apply Q1 to two
# fields (forward + back each), the fused x stage does five products
PRODUCTS = (4, 4, 5)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=PRECISIONS)
    ap.add_argument("--repeats", type=int, default=5, help="timed repetitions of --steps steps (median reported)")
    ap.add_argument("--settle-blocks", type=int, default=10,
                    help="at most this many 20-step warm-up blocks until the step time settles (0: none)")
    ap.add_argument("--reduced", default="fp32,bf16x6,fp64_fp32,fp64_bf16x6",
                    help="comma-separated reduced-precision variants timed beside fp64, or 'none'")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=255)
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--batched-steps", type=int, default=100)
    ap.add_argument("--latency-steps", type=int, default=100)
    ap.add_argument("--exact-steps", type=int, default=50)
    ap.add_argument("--fhn2d-steps", type=int, default=200)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration)")
    return ap.parse_args()


SETTLE_BLOCKS = 10


def timed_run(etd, torch, wl, precision, steps, warmup, repeats=5):
    """Warm up, then time `steps` steps from the workload's u0, `repeats` times
    without per-stage events (the value is the median), then once more with
    per-stage HIP events (the roofline's per-kernel launch times).  Warm-up:
    `warmup` steps, then further 20-step blocks until two consecutive blocks
    agree within 1% (clocks settled; at most --settle-blocks blocks).  Returns the final
    field of the first repetition, the median wall seconds, all repetition
    times and the event timings."""
    p = wl.problem.replace(precision=precision)
    st = etd.Stepper(p)
    u0 = wl.u0()
    u = st.field(u0)
    if warmup:
        st.advance(u, warmup)
    prev = None
    for _ in range(SETTLE_BLOCKS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.advance(u, 20)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if prev is not None and abs(dt - prev) <= 0.01 * prev:
            break
        prev = dt
    times = []
    first = None
    for r in range(repeats):
        u = st.field(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.advance(u, steps)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if first is None:
            first = u
    u = st.field(u0)
    etd.etd_timing_enable(st.plan, True)
    torch.cuda.synchronize()
    st.advance(u, steps)
    torch.cuda.synchronize()
    ms, counts = etd.etd_timing_read(st.plan)
    etd.etd_timing_enable(st.plan, False)
    st.close()
    return first, sorted(times)[len(times) // 2], times, ms, counts


CSRC = os.path.join(ROOT, "paper_2601_06849_amd", "csrc")


def source_fingerprint():
    """SHA-256 over every source of the library (csrc/, sorted by name)."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None when there is none or the
    kernel sources changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    fp = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    tb = re.search(rf"traffic_bytes_per_launch {kernel}: (\d+)", text)
    if not fp or not tb or fp.group(1) != source_fingerprint():
        return None
    return int(tb.group(1))


def roofline(wl, precision, ms, counts):
    n = wl.problem.n[0]
    per_product = 2.0 * n * n ** 3          # one dense mode product, true (unpadded) n
    stages = {}
    for k, name in enumerate(STAGE_NAMES):
        if counts[k] == 0:
            continue
        avg_ms = ms[k] / counts[k]
        flops = PRODUCTS[k] * per_product
        stages[name] = {"launches": counts[k], "avg_ms": avg_ms, "tflops": flops / (avg_ms * 1e-3) / 1e12}
    dom = max(stages, key=lambda s: stages[s]["avg_ms"] * stages[s]["launches"])
    a = stages[dom]["tflops"]
    peak = PEAK_TFLOPS[precision]
    return {"bound": "mfma", "kernel": dom, "achieved": round(a, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(a / peak, 4), "traffic": measured_traffic(wl.name, precision, dom)}, stages


def adjoint_leg(etd, torch, W, nsteps):
    """Time one forward run and the adjoint (gradient w.r.t. u0, kappa, q) over
    nsteps steps of the 3-D FitzHugh-Nagumo workload, with the shortest
    checkpoint segment (ceil(sqrt(N)) steps: forward work about 2N steps) and
    with one segment of N steps (every step's stage fields kept: one forward
    pass); the loss target is u(T) of a run at 1.1 kappa_u."""
    wl = W.fhn3d(nsteps=nsteps)
    p = wl.problem
    st = etd.Stepper(p)
    u0 = st.field(wl.u0())
    tp = etd.Stepper(p.replace(kappa=(p.kappa[0] * 1.1, p.kappa[1])))
    target = tp.advance(u0.clone(), nsteps)
    tp.close()
    u = st.advance(u0.clone(), 2)                      # warm the forward kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = st.advance(u0.clone(), nsteps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    ubar = u - target
    st.adjoint(u0, ubar, 2)                            # warm the adjoint kernels
    torch.cuda.synchronize()
    out = {"workload": wl.name, "steps": nsteps, "precision": p.precision,
           "forward_ms_per_step": 1e3 * fwd / nsteps}
    grads = {}
    for name, seg in (("sqrt_segments", math.ceil(math.sqrt(nsteps))), ("one_segment", nsteps)):
        aws = st.adjoint_workspace(nsteps, seg)          # allocated outside the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, grad = st.adjoint(u0, ubar, nsteps, workspace=aws)
        torch.cuda.synchronize()
        adj = time.perf_counter() - t0
        del aws
        grads[name] = grad
        out[name] = {"checkpoint_every": seg,
                     "adjoint_workspace_gb": etd.etd_adjoint_workspace_bytes_segment(st.plan, nsteps, seg) / 1e9,
                     "adjoint_ms_per_step": 1e3 * adj / nsteps, "adjoint_over_forward": adj / fwd,
                     "adjoint_updates_per_s": p.npoints * nsteps / adj,
                     "grad_kappa": grad[:p.ncomp], "grad_q": grad[p.ncomp]}
        torch.cuda.empty_cache()
    st.close()
    a, b = grads["sqrt_segments"], grads["one_segment"]
    out["grad_rel_diff_between_segmentings"] = max(abs(x - y) / abs(y) for x, y in zip(a, b))
    return out


def batched_leg(etd, torch, W, nsteps):
    """Grouped persistent launches over the 256-instance uneven 2-D workload:
    grid-point updates/s and useful FP32 TFLOP/s (18 n^3 per instance-step),
    with the default tile shapes, with autotuned ones, and as a graph."""
    problems, u0s, _ = W.batched2d(nsteps=nsteps)
    b = etd.Batch(problems)
    fields = b.fields(u0s)
    updates = sum(p.npoints for p in problems) * nsteps
    flops = sum(18.0 * p.n[0] ** 3 for p in problems) * nsteps
    peak = PEAK_TFLOPS["fp32"]

    def timed(run):
        run(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(nsteps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        return {"ms_per_step": 1e3 * sec / nsteps, "updates_per_s": updates / sec,
                "useful_tflops": flops / sec / 1e12, "frac_of_fp32_peak": flops / sec / 1e12 / peak}

    out = {"workload": "fisher2d_batched256", "instances": len(problems), "groups": b.groups(),
           "extents": {str(n): sum(1 for p in problems if p.n[0] == n) for n in (127, 255, 511, 1023)},
           "steps": nsteps, "precision": "fp32"}
    out["default_tiles"] = timed(lambda k: b.advance(fields, k))
    b.autotune()
    out["autotuned_tiles"] = timed(lambda k: b.advance(fields, k))
    out["autotuned_tiles"]["tiles"] = {str(p.n[0]): b.tiles(i)[:2] for i, p in
                                       reversed(list(enumerate(problems)))}
    s = torch.cuda.Stream()
    graphs = {}

    def graph_run(k):
        if k not in graphs:
            graphs[k] = b.capture(fields, k, s)
        graphs[k].launch(s)
        s.synchronize()
    out["graph"] = timed(graph_run)
    for g in graphs.values():
        g.close()
    b.close()
    return out


def latency_leg(etd, torch, W, nsteps, repeats=5):
    """The 63^2 Fisher-KPP case, where a step is 4.5 MFLOP: per-stage launches
    as eager one-step calls and as one captured graph of the run, and the
    resident schedule (every step of a call in one cooperative launch) as
    one-step calls and as one call of the whole run (median of `repeats`)."""
    wl = W.fisher2d_small()
    st = etd.Stepper(wl.problem)
    st.set_schedule("stages")
    u = st.field(wl.u0())
    st.advance(u, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        st.advance(u, 1)
    torch.cuda.synchronize()
    eager = time.perf_counter() - t0
    s = torch.cuda.Stream()
    g = st.capture(u, nsteps, s)
    g.launch(s)
    s.synchronize()
    t0 = time.perf_counter()
    g.launch(s)
    s.synchronize()
    graph = time.perf_counter() - t0
    g.close()
    st.set_schedule("resident")
    st.advance(u, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        st.advance(u, 1)
    torch.cuda.synchronize()
    res_calls = time.perf_counter() - t0
    runs = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.advance(u, nsteps)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    st.close()
    return {"workload": wl.name, "steps": nsteps, "eager_us_per_step": 1e6 * eager / nsteps,
            "graph_us_per_step": 1e6 * graph / nsteps,
            "resident_one_step_calls_us_per_step": 1e6 * res_calls / nsteps,
            "resident_us_per_step": 1e6 * statistics.median(runs) / nsteps,
            "resident_us_per_step_runs": [1e6 * r / nsteps for r in runs]}


def fhn2d_leg(etd, torch, W, nsteps, repeats=5):
    """2-D coupled FitzHugh-Nagumo, 511^2 x 2 components (the product-parallel
    2-D path): FP64 and the reduced-product precisions over the same steps
    from the same u0, timed without per-stage events (a step is only about
    0.1-0.2 ms; median of `repeats`), then the same steps replayed from a
    captured HIP graph.  Useful work is 18 n^3 flops per component and step
    (nine mode products)."""
    out = {"workload": "fhn2d_n511", "steps": nsteps}
    final = {}
    for prec in ("fp64", "fp32", "fp64_fp32", "fp64_bf16x6"):
        wl = W.fhn2d(precision=prec)
        n = wl.problem.n[0]
        st = etd.Stepper(wl.problem)
        u0 = wl.u0()
        st.advance(st.field(u0), 20)
        times = []
        for _ in range(repeats):
            u = st.field(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.advance(u, nsteps)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            final.setdefault(prec, u.clone())
        sec = sorted(times)[len(times) // 2]
        # the same steps captured once in a HIP graph and replayed
        s = torch.cuda.Stream()
        g = st.capture(u, nsteps, s)
        g.launch(s)
        s.synchronize()
        t0 = time.perf_counter()
        g.launch(s)
        s.synchronize()
        gsec = time.perf_counter() - t0
        g.close()
        st.close()
        useful = 18.0 * n ** 3 * wl.problem.ncomp * nsteps
        out[prec] = {"ms_per_step": 1e3 * sec / nsteps, "value": n * n * nsteps / sec,
                     "useful_tflops": useful / sec / 1e12, "frac_of_peak": useful / sec / 1e12 / PEAK_TFLOPS[prec],
                     "graph_ms_per_step": 1e3 * gsec / nsteps}
    for prec in ("fp32", "fp64_fp32", "fp64_bf16x6"):
        d = final[prec].double() - final["fp64"]
        out[prec]["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out[prec]["ms_per_step"]
        out[prec]["rel_l2_vs_fp64"] = float(d.norm() / final["fp64"].norm())
        out[prec]["rel_max_vs_fp64"] = float(d.abs().max() / final["fp64"].abs().max())
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, args):
    """The oracle as it stands, on a bounded sample of the same workload: with
    all host threads, chunks of --cpu-steps steps from u0 until about
    --cpu-seconds of host time (three chunks at least; the value is the median
    chunk rate), then one chunk on one thread."""
    import oracle
    p = wl.problem.replace(precision="fp64")
    npts = wl.problem.npoints
    cores = oracle.threads(0)
    u = wl.u0()
    done, spent, rates = 0, 0.0, []
    while (spent < args.cpu_seconds or len(rates) < 3) and done < 400:
        t0 = time.perf_counter()
        u = oracle.advance(p, u, args.cpu_steps, t0=done * p.tau, nthreads=0)
        dt = time.perf_counter() - t0
        spent += dt
        done += args.cpu_steps
        rates.append(npts * args.cpu_steps / dt)
    t0 = time.perf_counter()
    oracle.advance(p, wl.u0(), 1, nthreads=1)
    one = time.perf_counter() - t0
    return {"value": sorted(rates)[len(rates) // 2], "unit": "grid-point updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "chunk_rate_range": [min(rates), max(rates)],
            "statistic": f"median of {len(rates)} chunks of {args.cpu_steps} steps",
            "one_thread": {"value": npts / one, "sample": f"1 step of {wl.name} on 1 thread in {one:.1f} s"},
            "sample": f"first {done} steps of {wl.name} from the same u0 in {spent:.1f} s on {cores} threads "
                      f"(FP64 complex Thomas line solves, OpenMP over lines)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the stepper is a single-device path "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8, "repeats": 3}), flush=True)
        return

    import paper_2601_06849_amd as etd
    import workloads as W

    global SETTLE_BLOCKS
    SETTLE_BLOCKS = args.settle_blocks

    wl = W.fisher3d(precision=args.precision, n=args.n, nsteps=args.steps)
    npts = wl.problem.npoints
    u_main, sec, times, ms, counts = timed_run(etd, torch, wl, args.precision, args.steps, args.warmup, args.repeats)
    value = npts * args.steps / sec
    roof, stages = roofline(wl, args.precision, ms, counts)
    useful = 26.0 * args.n ** 4 * args.steps  # 13 mode products per 3-D step

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [args.n] * 3, "kappa": wl.problem.kappa[0], "q": wl.problem.q,
                   "tau": wl.problem.tau, "reaction": "u(1-u)", "precision": args.precision,
                   "init": "sine product + 8 Gaussian bumps (sigma 0.05), seed %d" % wl.seed},
        "timing": {"repeats": args.repeats, "statistic": "median of the repeats, each exactly --steps steps "
                   "from u0, no per-stage events; the roofline comes from one further repeat with per-stage "
                   "HIP events", "ms_per_step_repeats": [1e3 * t / args.steps for t in times]},
        "roofline": roof,
        "stages": stages,
        "useful_tflops": useful / sec / 1e12,
    }

    if args.reduced != "none" and args.precision == "fp64":
        # reduced-precision variants over the same steps from the same u0; the
        # FP64 result they are compared with matches the FP64 oracle to 1e-12
        out["reduced"] = {}
        for prec in args.reduced.split(","):
            u_red, sec_r, _, ms_r, counts_r = timed_run(etd, torch, wl, prec, args.steps, args.warmup,
                                                        args.repeats)
            d = u_red.double() - u_main
            roof_r, _ = roofline(wl, prec, ms_r, counts_r)
            out["reduced"][prec] = {"value": npts * args.steps / sec_r, "ms_per_step": 1e3 * sec_r / args.steps,
                                    "speedup_vs_fp64": sec / sec_r,
                                    "rel_l2_vs_fp64": float(d.norm() / u_main.norm()),
                                    "rel_max_vs_fp64": float(d.abs().max() / u_main.abs().max()),
                                    "dtype": DTYPE[prec], "roofline": roof_r}

    if args.adjoint_steps > 0:
        out["adjoint"] = adjoint_leg(etd, torch, W, args.adjoint_steps)
    if args.batched_steps > 0:
        out["batched"] = batched_leg(etd, torch, W, args.batched_steps)
    if args.latency_steps > 0:
        out["latency"] = latency_leg(etd, torch, W, args.latency_steps)
    if args.exact_steps > 0 and args.precision == "fp64":
        # same kernels, exact-exponential diagonals; compared with the Pade
        # result after the same steps from the same u0
        wl_e = W.fisher3d(precision="fp64", n=args.n, nsteps=args.exact_steps)
        u_e, sec_e, _, _, _ = timed_run(etd, torch, W.Workload(wl_e.name, wl_e.problem.replace(pade=0), wl_e.nsteps,
                                                               wl_e.init, wl_e.seed), "fp64", args.exact_steps, 2, 3)
        u_p, _, _, _, _ = timed_run(etd, torch, wl_e, "fp64", args.exact_steps, 0, 1)
        out["exact_exponential"] = {"ms_per_step": 1e3 * sec_e / args.exact_steps,
                                    "value": npts * args.exact_steps / sec_e, "steps": args.exact_steps,
                                    "rel_l2_vs_pade02": float((u_e - u_p).norm() / u_p.norm())}

    if args.fhn2d_steps > 0:
        out["fhn2d"] = fhn2d_leg(etd, torch, W, args.fhn2d_steps)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
