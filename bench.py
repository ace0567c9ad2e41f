#!/usr/bin/env python3
"""Benchmark of the hybrid micro-macro parareal solver on one MI355X.

Workload (default): the hybrid parareal problem of 512 cells x 64 velocities,
N = 64 time slices, T = 1, eps(x) the periodic tanh profile (fluid on the left
half, kinetic on the right), rho_in = 1 + 0.3 cos(2 pi x) + 0.05 noise,
thresholds 1e-3, FP64, slice starts carried from the previous fine sweep.

One bench "step" is one parareal iteration: the fine sweep of every
unconverged slice (the hot path, one batched persistent launch) plus the
sequential coarse correction.  The timed region is --steps iterations after
the coarse guess; --warmup iterations of the same kind run first on a
separate problem with short slices.

Reported value: kinetic phase-space cell-updates per second (one cell-update
= one kinetic (interface, velocity) pair advanced one fine step), counted by
the kernels themselves.  The fine-sweep launches are timed with HIP events on
the stream they run on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-step phase-space cell-updates/s FP32 vs FP64; parareal wall-clock; p50/p99"
HBM_PEAK_GBS = 8000.0
MACRO_BYTES_PER_IFACE_STEP = 64  # rho, E, J, Phi, e, a, eps, status per interface per step
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
# floating-point operations of one kinetic cell-update of the micro-macro
# step: transport 7 (upwind difference and scaling, two-sided G flux and its
# difference), projection 3, relaxation with source 5, flux moment 2, norm 2
FLOPS_PER_CELL_UPDATE = 19
KERNEL_SOURCES = ("paper_2511_13386_amd/csrc/sth_kernels.hip", "paper_2511_13386_amd/csrc/sth_internal.h")


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_key):
    """HBM bytes per fine-sweep launch from the committed counter summary of
    this workload, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"k_fine_{workload_key}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != sources_sha256():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_batch_traffic():
    """Counted HBM bytes of the first batched sweep of the 256-instance FP32
    batch and its algorithmic bytes, from the committed counter summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "k_fine_batch256_fp32_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != sources_sha256():
        return None
    try:
        return (float(kv["first_sweep_fetch_bytes"]) + float(kv["first_sweep_write_bytes"]),
                float(kv["first_sweep_algorithmic_bytes"]))
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--flip-steps", type=int, default=50000,
                    help="default workload: fine steps of slice 1 over which FP32-bulk and FP64 "
                         "threshold decisions are compared (0: skip)")
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--nv", type=int, default=64)
    ap.add_argument("--slices", type=int, default=64)
    ap.add_argument("--T", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unit-steps", type=int, default=2000, help="unit: fine steps of the one slice")
    ap.add_argument("--unit-hybrid", action="store_true", help="unit: domain adaptation on")
    ap.add_argument("--no-other-precision", action="store_true",
                    help="config2: skip the same solve in the other precision")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", choices=["config2", "batch", "serve", "convergence", "linf", "1d3v", "unit"],
                    default="config2",
                    help="config2: the hybrid parareal problem the metric is quoted on; "
                         "batch: many independent instances in one batched sweep per iteration")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-T", type=float, default=0.01)
    ap.add_argument("--batch-slices", type=int, default=32)
    ap.add_argument("--no-autotune", action="store_true", help="batch: keep the default launch configurations")
    ap.add_argument("--tune-steps", type=int, default=100, help="batch: steps per slice of the tuning sweeps")
    ap.add_argument("--baseline-every", type=int, default=20,
                    help="batch: every n-th instance also runs alone in FP64 (the baseline form)")
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--serve-baseline-every", type=int, default=20,
                    help="serve: every n-th request also runs alone in FP64 (the one-at-a-time baseline)")
    ap.add_argument("--serve-compare-ticks", action="store_true",
                    help="serve: also serve the same arrivals with one parareal iteration per tick")
    ap.add_argument("--serve-T-scale", type=float, default=1e-2,
                    help="serve: request horizons T ~ U[0.1, 1] times this factor")
    ap.add_argument("--load", type=float, default=0.5,
                    help="serve: arrival rate as a fraction of the measured saturated throughput")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="serve: device arena for admission")
    ap.add_argument("--serve-chunk", type=int, default=256,
                    help="serve: fine steps per slice per tick (0: one parareal iteration per tick)")
    ap.add_argument("--paper-steps-per-slice", type=int, default=50,
                    help="1d3v/convergence: fine steps per slice of the paper setting (fine dt = 1/(200 S))")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB elementwise copy kernel (HBM counter calibration)")
    ap.add_argument("--other-iterations", type=int, default=8,
                    help="config2: parareal iterations of the same solve in the other precision")
    ap.add_argument("--lift-iterations", type=int, default=8,
                    help="config2: parareal iterations with lifted slice starts (Algorithm 1); 0 skips")
    ap.add_argument("--no-batch", action="store_true",
                    help="config2: skip the batched FP32-bulk block (the 256-instance workload)")
    ap.add_argument("--batch-iterations", type=int, default=8,
                    help="config2: parareal iterations of the batched FP32-bulk block")
    return ap.parse_args()


def short_horizon(sth, d, steps):
    """The description with its horizon cut so that a slice takes about
    `steps` stable fine steps (warm-ups run the same kernels briefly without
    forcing an unstable step)."""
    import copy
    probe = sth.Problem(d)
    ns = probe.info().steps_per_slice
    probe.close()
    w = copy.copy(d)
    w.T = d.T * min(1.0, steps / ns)
    return w


def cpu_baseline(inst, target_s):
    """The CPU oracle (plain FP64 C, OpenMP over slices as in the paper's
    implementation) on a bounded sample of the same work: the first slices of
    iteration 0, each from its coarse-guess density and lifted start, for a
    step count sized to about target_s seconds."""
    from oracle import oracle as orc
    orc.lib()
    flags = orc.FIELD | orc.HYBRID
    p, ns, dtG = orc.setup(inst.nx, inst.nv, inst.eps_iface, inst.rho_in, T=inst.T, N=inst.N,
                           theta=inst.theta, eta0=inst.eta0, delta0=inst.delta0, flags=flags,
                           lift_order=1, start_mode=orc.START_CARRY)
    threads = orc.num_threads()
    nun = max(threads, 1)
    rhos = [inst.rho_in]
    for _ in range(nun):
        rhos.append(orc.coarse_step(p, dtG, rhos[-1]))
    starts = np.array(rhos[:nun])
    gs = np.array([np.zeros((inst.nx, inst.nv))] +
                  [orc.lift(p, inst.eps_iface, r) for r in starts[1:]])
    # calibrate on one unit, then one unit alone for about a second (one thread)
    t0 = time.perf_counter()
    _, kin1 = orc.fine_batch(p, inst.eps_iface, inst.eps_cell, starts[:1], 200, gs[:1])
    dt1 = time.perf_counter() - t0
    per_step_unit = dt1 / 200.0
    n1 = int(max(200, min(ns, 1.0 / per_step_unit)))
    t0 = time.perf_counter()
    _, kin1 = orc.fine_batch(p, inst.eps_iface, inst.eps_cell, starts[:1], n1, gs[:1])
    single = kin1 * inst.nv / (time.perf_counter() - t0)
    steps = int(max(200, min(ns, target_s / per_step_unit * threads / nun)))
    t0 = time.perf_counter()
    _, kin = orc.fine_batch(p, inst.eps_iface, inst.eps_cell, starts, steps, gs)
    el = time.perf_counter() - t0
    # one parareal iteration of the oracle (iteration 0: all N slices, one
    # per thread at a time with dynamic scheduling, as in the paper's
    # implementation), extrapolated from the sample: ceil(N / threads) rounds
    # of one slice each at the sampled per-step time
    rounds = -(-inst.N // threads)
    return {
        "value": kin * inst.nv / el,
        "unit": "cell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{nun} slices x {steps} fine steps of iteration 0 (of {ns} per slice), "
                   f"{el:.1f} s wall, OpenMP over slices"),
    }, {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "threads": threads,
        "parareal_iteration_wall_s_extrapolated": rounds * ns * el / steps,
        "parareal_iteration_extrapolation": (f"iteration 0 = {inst.N} slices of {ns} steps on {threads} "
                                             f"threads: {rounds} rounds x {ns} steps at the sampled "
                                             f"{el / steps * 1e6:.1f} us per step and slice"),
        "single_thread_value": single,
        "single_thread_sample": f"slice 1 alone, {n1} fine steps, one thread",
        "config1_single_thread": _config1_oracle(orc)}


def _config1_oracle(orc):
    """The oracle's one-thread rate on the plain serial micro-macro run
    (64 x 32, eps = 1e-2, full kinetic, the whole T = 0.1)."""
    from paper_2511_13386_amd import workloads as wl
    c1 = wl.config1()
    p, ns, _ = orc.setup(c1.nx, c1.nv, c1.eps_iface, c1.rho_in, T=c1.T, N=1, theta=c1.theta,
                         flags=orc.FIELD)
    t0 = time.perf_counter()
    _, _, _, st = orc.fine_propagate(p, c1.eps_iface, c1.eps_cell, c1.rho_in, None, ns)
    el = time.perf_counter() - t0
    return {"value": st["kinetic_iface_steps"] * c1.nv / el, "unit": "cell-updates/s",
            "steps": ns, "seconds": el}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_batch(args, torch, sth, wl):
    """Config 4 as its own bench line (--workload batch)."""
    prec = sth.FP64 if args.precision == "fp64" else sth.FP32_BULK
    out = batch_block(args, torch, sth, wl, prec, max(1, min(args.steps, args.batch_slices)),
                      with_graph=True)
    print(json.dumps(out), flush=True)


def batch_block(args, torch, sth, wl, prec, K, with_graph):
    """Config 4: independent instances of mixed size and eps, all slices of all
    instances in one batched fine sweep per parareal iteration, against the
    plain FP64 single-instance form on a subset."""
    insts = wl.batch_config(count=args.batch_count, T=args.batch_T, N=args.batch_slices)
    precision_label = "fp64" if prec == sth.FP64 else "fp32"

    def desc(inst, precision, steps_override=0):
        return sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                        rho0=inst.rho_in, T=inst.T, n_slices=inst.N, k_max=K, tol=0.0,
                        eta0=inst.eta0, delta0=inst.delta0, lift_order=1, start_mode=sth.START_CARRY,
                        cfl_theta=inst.theta, flags=sth.FIELD | sth.HYBRID, precision=precision,
                        steps_override=steps_override)

    stream = torch.cuda.Stream()
    tune_info = None
    if not args.no_autotune:
        from paper_2511_13386_amd import autotune
        t0 = time.perf_counter()
        tuned = autotune.autotune([desc(i, prec) for i in insts], steps=args.tune_steps, repeats=2,
                                  stream=stream)
        sp = [r.speedup_over_default for r in tuned.values()]
        tune_info = {"classes": len(tuned), "seconds": time.perf_counter() - t0,
                     "changed": sum(r.best != r.default for r in tuned.values()),
                     "class_speedup_min": min(sp), "class_speedup_max": max(sp),
                     "class_speedup_geomean": float(np.exp(np.mean(np.log(sp))))}
        print(f"# autotuned {len(tuned)} classes in {tune_info['seconds']:.1f} s, "
              f"{tune_info['changed']} changed, speedup {tune_info['class_speedup_geomean']:.3f} geomean",
              file=sys.stderr, flush=True)
    if args.warmup > 0:  # every kernel class once, short slices
        ws = [sth.Problem(short_horizon(sth, desc(i, prec), 20)) for i in insts]
        for w in ws:
            sth.sth_coarse_sweep(w, stream)
        sth.sth_fine_sweep_batched(ws, stream)
        torch.cuda.synchronize()
        for w in ws:
            w.close()
        print("# warmup done", file=sys.stderr, flush=True)

    def solve(problems, precision_label):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sth.sth_coarse_sweep_batched(problems, stream)
        for k in range(K):
            with torch.cuda.stream(stream):
                ev[k][0].record(stream)
            sth.sth_fine_sweep_batched(problems, stream)
            with torch.cuda.stream(stream):
                ev[k][1].record(stream)
            sth.sth_parareal_correct_batched(problems, want_err=False, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = [a.elapsed_time(b) for a, b in ev]
        kin = sum(p.info().kinetic_iface_steps * p.nv for p in problems)
        # algorithmic bytes: read and write of g' per kinetic cell-update,
        # plus the macroscopic data of each kinetic interface-step
        realsz = 8 if precision_label == "fp64" else 4
        alg = sum(p.info().kinetic_iface_steps * (p.nv * 2 * realsz + MACRO_BYTES_PER_IFACE_STEP)
                  for p in problems)
        solve.alg_bytes = alg
        return kin, ms, wall

    problems = [sth.Problem(desc(i, prec)) for i in insts]
    footprint = sum(p.info().footprint_bytes for p in problems)
    kin, ms, wall = solve(problems, precision_label)
    rate = kin / (sum(ms) * 1e-3)
    alg_gbs = solve.alg_bytes / (sum(ms) * 1e-3) / 1e9
    print(f"# batched {len(problems)} instances: {kin:.3e} kinetic cell-updates in {sum(ms):.0f} ms of sweeps",
          file=sys.stderr, flush=True)
    U_all = [sth.sth_get_rho(p) for p in problems]
    U_batch = {i: U_all[i] for i in range(0, len(insts), args.baseline_every)}
    mass = max(float(np.max(np.abs(U.sum(axis=1) - inst.rho_in.sum())) / abs(inst.rho_in.sum()))
               for U, inst in zip(U_all, insts))
    graph_wall = t_rec = graph_same = None
    if with_graph:
        # the same solves recorded once as a HIP graph and replayed by one launch
        t0 = time.perf_counter()
        graph = sth.Graph(problems)
        t_rec = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.launch(stream)
        graph.wait(stream)
        graph_wall = time.perf_counter() - t0
        graph_same = all(np.array_equal(sth.sth_get_rho(p), U) for p, U in zip(problems, U_all))
        graph.close()
        print(f"# eager solve {wall:.3f} s, graph replay {graph_wall:.3f} s (recorded in {t_rec:.2f} s), "
              f"identical: {graph_same}", file=sys.stderr, flush=True)
    del U_all
    for p in problems:
        p.close()

    # baseline: the same solves one instance at a time in FP64, on a subset
    kin1 = ms1 = 0.0
    errs = []
    for i in sorted(U_batch):
        p1 = sth.Problem(desc(insts[i], sth.FP64))
        k1, m1, _ = solve([p1], "fp64")
        kin1 += k1
        ms1 += sum(m1)
        U1 = sth.sth_get_rho(p1)
        errs.append(float(np.max(np.abs(U_batch[i] - U1)) / np.max(np.abs(U1))))
        p1.close()
    rate1 = kin1 / (ms1 * 1e-3)
    # the counter summary covers the FP32 batch workload of the defaults
    bt = (measured_batch_traffic() if prec == sth.FP32_BULK and args.batch_count == 256
          and args.batch_slices == 32 and args.batch_T == 0.01 else None)
    return {
        "metric": "batched fine-sweep kinetic cell-updates/s (independent instances, mixed sizes)",
        "value": rate, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": float(np.mean(ms)), "sweep_ms_per_iteration": [round(m, 1) for m in ms],
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == sth.FP64 else "f32-bulk/f64-macro",
        "data": "synthetic",
        "config": {"workload": (f"{len(insts)} instances seed 1000+i, Nx in {{128..2048}}, Nv in {{32,64,128}}, "
                                f"log10 eps ~ U[-4,0], 1-3 cosine modes, N={args.batch_slices}, T={args.batch_T}, "
                                f"{K} parareal iterations, carried slice starts"),
                   "instances": len(insts), "device_bytes": footprint},
        "single_instance_fp64": {"value": rate1, "unit": "cell-updates/s",
                                 "instances": len(U_batch),
                                 "sample": f"every {args.baseline_every}-th instance, alone, FP64"},
        "roofline": {"bound": "hbm", "achieved": alg_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg_gbs / HBM_PEAK_GBS, "traffic": bt[0] if bt else None,
                     "achieved_kind": ("algorithmic bytes: read and write of g' per kinetic cell-update "
                                       "plus 64 B per kinetic interface-step, over the sweep time"),
                     "traffic_kind": ("counted HBM bytes (FETCH_SIZE + WRITE_SIZE) of the first iteration's "
                                      "sweep, all kernel classes"),
                     "traffic_over_algorithmic_same_sweep": (bt[0] / bt[1]) if bt else None},
        "speedup_vs_single_fp64": rate / rate1,
        "max_rel_rho_diff_vs_single_fp64": max(errs) if errs else None,
        "mass_drift_rel_max": mass,
        "parareal_wall_s": wall,
        "parareal_wall_s_graph": graph_wall,
        "graph_record_s": t_rec,
        "graph_equals_eager": graph_same,
        "autotune": tune_info,
    }


def run_serve(args, torch, sth, wl):
    """Config 5: a Poisson stream of solve requests (sizes and eps as config 4,
    horizons scaled), served with continuous batching in FP32-bulk; p50/p99
    latency and throughput against the plain FP64 one-at-a-time form."""
    from paper_2511_13386_amd import serving
    R, K = args.requests, 2
    u = (wl.uniform_pm1(4242, R) + 1.0) * 0.5
    insts = []
    for r in range(R):
        T = (0.1 + 0.9 * u[r]) * args.serve_T_scale
        insts.append(wl.random_instance(5000 + r, N=32, T=T))

    def desc(inst, precision):
        return sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                        rho0=inst.rho_in, T=inst.T, n_slices=inst.N, k_max=K, tol=0.0,
                        eta0=inst.eta0, delta0=inst.delta0, lift_order=1, start_mode=sth.START_CARRY,
                        cfl_theta=inst.theta, flags=sth.FIELD | sth.HYBRID, precision=precision)

    budget = int(args.budget_gib * (1 << 30))
    chunk = args.serve_chunk if args.serve_chunk > 0 else None
    last = [0]

    def progress(n):
        if n // 250 > last[0] // 250 or n == R:
            print(f"# served {n}/{R}", file=sys.stderr, flush=True)
        last[0] = n

    srv = serving.Server(budget, chunk_steps=chunk)
    # warmup: every kernel class once
    warm = [serving.Request(r, desc(i, sth.FP32_BULK), 0.0, 1) for r, i in enumerate(insts[:48])]
    for w in warm:
        w.desc = short_horizon(sth, w.desc, 20)
    srv.run(warm)
    torch.cuda.synchronize()

    # saturated throughput: everything arrives at once
    reqs = [serving.Request(r, desc(i, sth.FP32_BULK), 0.0, K) for r, i in enumerate(insts)]
    t0 = time.perf_counter()
    last[0] = 0
    sat = srv.run(reqs, on_done=progress)
    sat_wall = time.perf_counter() - t0
    sat_rate = R / sat_wall
    print(f"# saturated: {R} requests in {sat_wall:.2f} s", file=sys.stderr, flush=True)

    # Poisson arrivals at a fraction of the saturated rate
    lam = args.load * sat_rate
    arr = wl.poisson_arrivals(R, lam, seed=99)
    reqs = [serving.Request(r, desc(i, sth.FP32_BULK), float(arr[r]), K) for r, i in enumerate(insts)]
    t0 = time.perf_counter()
    ticks0 = srv.ticks
    last[0] = 0
    res = srv.run(reqs, on_done=progress)
    wall = time.perf_counter() - t0
    ticks = srv.ticks - ticks0
    pct = serving.latency_percentiles(res)
    cells = sum(r.cell_updates for r in res)
    print(f"# Poisson arrivals: {R / wall:.2f} requests/s, p50 {pct['p50']:.3f} s, p99 {pct['p99']:.3f} s",
          file=sys.stderr, flush=True)
    other = None
    if chunk is not None and args.serve_compare_ticks:
        # the same arrivals with one parareal iteration per tick
        srv2 = serving.Server(budget, stream=srv.stream)
        t0 = time.perf_counter()
        res2 = srv2.run(reqs)
        wall2 = time.perf_counter() - t0
        other = {"requests_per_s": R / wall2, "latency_s": serving.latency_percentiles(res2),
                 "same_results": all(np.array_equal(a.rho, b.rho, equal_nan=True) for a, b in zip(res, res2))}
        del srv2

    # baseline: the plain FP64 form one request at a time, measured on every
    # n-th request; the service time of the others is extrapolated from the
    # measured time per kinetic cell-update of the subset (the cell-updates
    # of each request are those its served solve counted), and the FIFO
    # queue in arrival order is simulated with them
    service, diffs, cells_sub = {}, [], 0.0
    stream = torch.cuda.Stream()
    subset = list(range(0, R, max(1, args.serve_baseline_every)))
    for r in subset:
        p = sth.Problem(desc(insts[r], sth.FP64))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sth.parareal_solve(p, K=K, fixed_iterations=True, stream=stream)
        torch.cuda.synchronize()
        service[r] = time.perf_counter() - t1
        cells_sub += res[r].cell_updates
        U = sth.sth_get_rho(p)
        diffs.append(float(np.max(np.abs(res[r].rho - U)) / np.max(np.abs(U))))
        p.close()
    per_cell = sum(service.values()) / max(cells_sub, 1.0)
    est = [service.get(r, res[r].cell_updates * per_cell) for r in range(R)]
    fin, lat1 = 0.0, []
    for a, sv in zip(arr, est):
        fin = max(fin, a) + sv
        lat1.append(fin - a)
    out = {
        "metric": "serving: p50/p99 latency and throughput of hybrid parareal solve requests",
        "value": R / wall, "unit": "requests/s", "n_gpus": 1, "steps": K, "warmup": 1,
        "ms_per_step": wall * 1e3 / max(ticks, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-bulk/f64-macro", "data": "synthetic",
        "config": {"workload": (f"{R} requests seed 5000+r, sizes/eps as config 4, T ~ U[0.1,1] x "
                                f"{args.serve_T_scale}, N=32, {K} parareal iterations, Poisson arrivals at "
                                f"{args.load} x saturated rate, arena {args.budget_gib} GiB, "
                                f"ticks of {args.serve_chunk or 'one iteration'} fine steps"),
                   "arrival_rate_per_s": lam, "chunk_steps": chunk, "ticks": ticks},
        "latency_s": pct, "cell_updates_per_s": cells / wall,
        "saturated_requests_per_s": sat_rate,
        "fp64_one_at_a_time": {"requests_per_s": R / sum(est),
                               "latency_s": {"p50": float(np.percentile(lat1, 50)),
                                             "p99": float(np.percentile(lat1, 99))},
                               "measured_requests": len(subset),
                               "sample": (f"every {max(1, args.serve_baseline_every)}-th request solved alone in "
                                          f"FP64 ({len(subset)} of {R}); the others' service times extrapolated "
                                          f"from the subset's time per kinetic cell-update "
                                          f"({per_cell * 1e9:.3f} ns); FIFO queue simulated in arrival order")},
        "max_rel_rho_diff_fp32_served_vs_fp64_alone": float(np.nanmax(diffs)),
        "requests_with_nonfinite_result": int(sum(not np.all(np.isfinite(r.rho)) for r in res)),
        "iteration_ticks": other,
    }
    print(json.dumps(out), flush=True)


def run_convergence(args, torch, sth, wl):
    """Parareal iterations to a successive error of 1e-10 against eps, with
    and without domain adaptation, in the paper's Section 5 setting (1D1V):
    the convergence study of the paper's Section 5.1, from the paper's
    initial distribution with its micro part, with lifted (first and third
    order) or carried slice starts, and with the implicit drift-diffusion
    coarse propagator or the paper's explicit limit scheme S^0."""
    eps_list = [1e-7, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1, 0.5, 1.0]
    S = args.paper_steps_per_slice
    rows = []
    t0 = time.perf_counter()
    for mode, mode_name, L in ((sth.START_LIFT, "lift", 3), (sth.START_LIFT, "lift", 1),
                               (sth.START_CARRY, "carry", 1)):
        for coarse, cflag in (("implicit", 0), ("explicit_S0", sth.COARSE_EXPLICIT)):
            for adapt in (False, True):
                for eps in eps_list:
                    inst = wl.paper_setting(eps, adaptation=adapt, lift_order=L, micro=True)
                    d = sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                                 rho0=inst.rho_in, g0=inst.g_in, T=inst.T, n_slices=inst.N, k_max=inst.N,
                                 tol=inst.tol, eta0=inst.eta0, delta0=inst.delta0, lift_order=inst.lift_order,
                                 start_mode=mode, cfl_theta=inst.theta,
                                 flags=sth.FIELD | cflag | (sth.HYBRID if adapt else 0), Lx=inst.Lx,
                                 vstar=inst.vstar, steps_override=S)
                    p = sth.Problem(d)
                    try:
                        errs = sth.parareal_solve(p, K=inst.N, tol=inst.tol)
                        diverged = False
                    except sth.StHError as e:
                        # a correction reported a non-finite density (the L = 3
                        # lifting at eps ~ 1): the run is recorded as diverged
                        if e.code != sth.STH_ENONFINITE:
                            raise
                        errs = sth.sth_get_errors(p) or [float("nan")]
                        diverged = True
                    info = p.info()
                    rows.append({"start": mode_name, "lift_order": L, "coarse": coarse, "adaptation": adapt,
                                 "eps": eps, "iterations": len(errs), "diverged": diverged,
                                 "final_err": errs[-1] if np.isfinite(errs[-1]) else None,
                                 "steps_per_slice": info.steps_per_slice, "fine_dt": info.dt,
                                 "kinetic_fraction": info.kinetic_iface_steps / max(
                                     1.0, inst.nx * info.steps_per_slice * sum(inst.N - k for k in range(len(errs))))})
                    p.close()
            print(f"# convergence: {mode_name} L={L} {coarse} done", file=sys.stderr, flush=True)
    out = {"metric": "parareal iterations to successive error 1e-10 (convergence study)",
           "value": None, "unit": "iterations", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": ("paper Section 5 setting in 1D1V: Nx=Nv=32, x*=2pi, v*=8, N_g=200, T_f=1, "
                                   "eta0=delta0=1e-5, initial distribution M(v) v^4 (1+0.9cos x) with its micro "
                                   f"part, {S} fine steps per slice (fine dt {1.0 / (200 * S):.1e}); slice starts "
                                   "lifted (L=3, L=1) or carried; coarse propagator implicit drift-diffusion or "
                                   "the explicit limit scheme S^0")},
           "runs": rows, "wall_s": time.perf_counter() - t0}
    print(json.dumps(out), flush=True)


def run_linf(args, torch, sth, wl):
    """Distance over time of the multiscale solutions from the classical
    one (Section 5.1, the L-infinity comparison): the classical scheme is the
    fine scheme without parareal or domain adaptation, run from t = 0 to
    every sampled slice end; against it, the sequential hybrid run (domain
    adaptation, no parareal) and the converged parareal solutions (successive
    error 1e-10) with lifted slice starts of order L = 1, 2, 3 and with
    carried starts, with and without adaptation, for eps = 0.5 and 1e-4 in
    the paper's Section 5 setting (1D1V, the paper's initial distribution
    with its micro part, 50 fine steps per slice, implicit coarse G)."""
    S = args.paper_steps_per_slice
    every = 5
    rows = []
    t0 = time.perf_counter()
    for eps in (0.5, 1e-4):
        inst = wl.paper_setting(eps, adaptation=False, lift_order=1, micro=True)
        N = inst.N
        samples = list(range(every, N + 1, every))

        def desc(flags, lift_order=1, start_mode=sth.START_LIFT, n_slices=N, K=N, tol=inst.tol):
            return sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                            rho0=inst.rho_in, g0=inst.g_in, T=inst.T, n_slices=n_slices, k_max=K, tol=tol,
                            eta0=inst.eta0, delta0=inst.delta0, lift_order=lift_order, start_mode=start_mode,
                            cfl_theta=inst.theta, flags=flags, Lx=inst.Lx, vstar=inst.vstar, steps_override=S)

        def serial(flags):
            # from t = 0 to every sampled slice end, one fine run each
            p = sth.Problem(desc(flags))
            out = {}
            for n in samples:
                out[n] = sth.sth_fine_run(p, inst.rho_in, inst.g_in, n * S)[0]
            p.close()
            return out

        classical = serial(sth.FIELD)
        scale = max(float(np.max(np.abs(c))) for c in classical.values())

        def dist(U):
            return max(float(np.max(np.abs(U[n] - classical[n]))) for n in samples)

        hybrid = serial(sth.FIELD | sth.HYBRID)
        row = {"eps": eps, "density_scale": scale, "sequential_hybrid": dist(hybrid), "parareal": []}
        for start, L in (("lift", 1), ("lift", 2), ("lift", 3), ("carry", 1)):
            for adapt in (False, True):
                mode = sth.START_LIFT if start == "lift" else sth.START_CARRY
                p = sth.Problem(desc(sth.FIELD | (sth.HYBRID if adapt else 0), lift_order=L, start_mode=mode))
                try:
                    errs = sth.parareal_solve(p, K=N, tol=inst.tol)
                    bad = False
                except sth.StHError as e:
                    if e.code != sth.STH_ENONFINITE:
                        raise
                    errs, bad = sth.sth_get_errors(p) or [float("nan")], True
                U = sth.sth_get_rho(p)
                p.close()
                conv = (not bad) and errs[-1] < inst.tol
                row["parareal"].append({
                    "start": start, "lift_order": L, "adaptation": adapt, "iterations": len(errs),
                    "converged": conv, "final_err": errs[-1] if np.isfinite(errs[-1]) else None,
                    "linf_vs_classical": dist(U) if not bad else None})
        rows.append(row)
        print(f"# linf eps={eps:g} done", file=sys.stderr, flush=True)
    # the printed variants of the hybrid scheme, sequential runs to T_f:
    # the cell-wise density update (not conservative, Section 3.3 remark)
    # and the criterion on |R| without eps^2, against the defaults
    variants = []
    for eps in (0.5, 1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        inst = wl.paper_setting(eps, adaptation=True, lift_order=1, micro=True)
        m0 = float(np.sum(inst.rho_in))
        ns = inst.N * S
        res = {}
        for name, flags in (("classical", sth.FIELD), ("hybrid", sth.FIELD | sth.HYBRID),
                            ("hybrid_cellwise_update", sth.FIELD | sth.HYBRID | sth.LITERAL_FLUX),
                            ("hybrid_criterion_abs_R", sth.FIELD | sth.HYBRID | sth.LITERAL_R)):
            d = sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                         rho0=inst.rho_in, g0=inst.g_in, T=inst.T, n_slices=inst.N, k_max=1, tol=0.0,
                         eta0=inst.eta0, delta0=inst.delta0, lift_order=1, start_mode=sth.START_LIFT,
                         cfl_theta=inst.theta, flags=flags, Lx=inst.Lx, vstar=inst.vstar, steps_override=S)
            p = sth.Problem(d)
            r, _, _, kin = sth.sth_fine_run(p, inst.rho_in, inst.g_in, ns)
            p.close()
            res[name] = (r, kin / (inst.nx * ns))
        c = res["classical"][0]
        v = {"eps": eps}
        for name in ("hybrid", "hybrid_cellwise_update", "hybrid_criterion_abs_R"):
            r, kf = res[name]
            v[name] = {"linf_vs_classical_at_T": float(np.max(np.abs(r - c))),
                       "mass_drift_rel": float(abs(np.sum(r) - m0) / abs(m0)), "kinetic_fraction": kf}
        variants.append(v)
    print("# linf variants done", file=sys.stderr, flush=True)
    out = {"metric": "L-infinity distance over time from the classical scheme (Section 5.1)",
           "value": None, "unit": "density", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": ("paper Section 5 setting in 1D1V: Nx=Nv=32, x*=2pi, v*=8, N_g=200, T_f=1, "
                                   "eta0=delta0=1e-5, initial distribution M(v) v^4 (1+0.9cos x) with its micro "
                                   f"part, {S} fine steps per slice, implicit coarse G, parareal to successive "
                                   f"error 1e-10; distances over every {every}-th slice end, FP64")},
           "runs": rows, "hybrid_variants_at_T": variants, "wall_s": time.perf_counter() - t0}
    print(json.dumps(out), flush=True)


# The paper's Table 3 (1D3V, 2 x 24-core Xeon Platinum 8268, OpenMP, 48
# threads): wall-clock seconds per eps for parareal off/on x adaptation
# off/on, and the fluid solver; context for the shape of the study only.
TABLE3_S = {1.0: (96.1, 104.6, 42.38, 44.5), 1e-1: (96.1, 104.2, 35.2, 37.5), 1e-2: (96.1, 99.5, 31.1, 32.5),
            1e-3: (96.1, 20.6, 17.0, 4.0), 1e-4: (96.1, 0.19, 13.0, 1.32)}
TABLE3_FLUID_S = 0.25


def run_1d3v(args, torch, sth, wl):
    """The paper's 1D3V study shape (Section 5, Table 3): Nx = 32, Nv = 32 x
    16 x 16, N_g = 200, T_f = 1, tol 1e-10, eta0 = delta0 = 1e-5, the paper's
    initial distribution with its micro part, for eps = 1 .. 1e-4: the serial
    fine solver with and without domain adaptation, the parareal solve with
    and without it (lifted slice starts, first order), with the implicit
    drift-diffusion coarse propagator and with the paper's explicit limit
    scheme S^0, and the coarse solver alone.  The fine step is the same for
    every eps (as the equal serial times of Table 3 imply): T_f / (N_g S)."""
    eps_list = [1.0, 1e-1, 1e-2, 1e-3, 1e-4]
    S = args.paper_steps_per_slice
    rows = []
    t0 = time.perf_counter()
    st = torch.cuda.Stream()

    def desc(inst, N, steps, flags, K=1, tol=0.0):
        return sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                        rho0=inst.rho_in, g0=inst.g_in, T=inst.T, n_slices=N, k_max=K, tol=tol,
                        eta0=inst.eta0, delta0=inst.delta0, lift_order=1, start_mode=sth.START_LIFT,
                        cfl_theta=inst.theta, flags=flags, Lx=inst.Lx, vstar=inst.vstar, nv_y=16, nv_z=16,
                        steps_override=steps)

    for eps in eps_list:
        inst = wl.paper_setting(eps, adaptation=True, lift_order=1, micro=True)
        row = {"eps": eps}
        # serial fine solver over T_f (one slice of N_g S steps)
        for adapt in (False, True):
            p = sth.Problem(desc(inst, 1, inst.N * S, sth.FIELD | (sth.HYBRID if adapt else 0)))
            sth.sth_fine_run(p, inst.rho_in, inst.g_in, 10)  # warm
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, _, _, kin = sth.sth_fine_run(p, inst.rho_in, inst.g_in, inst.N * S)
            torch.cuda.synchronize()
            row[f"serial_{'hybrid' if adapt else 'kinetic'}_s"] = time.perf_counter() - t1
            row[f"serial_{'hybrid' if adapt else 'kinetic'}_kinetic_fraction"] = kin / (inst.nx * inst.N * S)
            if not adapt:
                row["fine_dt"] = p.info().dt
            p.close()
        for coarse, cflag in (("implicit", 0), ("explicit_S0", sth.COARSE_EXPLICIT)):
            # the coarse solver alone over the N_g slices
            p = sth.Problem(desc(inst, inst.N, S, sth.FIELD | cflag))
            sth.sth_coarse_sweep(p, st)
            torch.cuda.synchronize()
            p.close()
            p = sth.Problem(desc(inst, inst.N, S, sth.FIELD | cflag))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sth.sth_coarse_sweep(p, st)
            torch.cuda.synchronize()
            row[f"fluid_{coarse}_s"] = time.perf_counter() - t1
            p.close()
            for adapt in (False, True):
                p = sth.Problem(desc(inst, inst.N, S, sth.FIELD | cflag | (sth.HYBRID if adapt else 0),
                                     K=inst.N, tol=inst.tol))
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                try:
                    errs = sth.parareal_solve(p, K=inst.N, tol=inst.tol, stream=st)
                    div = False
                except sth.StHError as e:
                    if e.code != sth.STH_ENONFINITE:
                        raise
                    errs, div = sth.sth_get_errors(p) or [float("nan")], True
                torch.cuda.synchronize()
                key = f"parareal_{coarse}_{'hybrid' if adapt else 'kinetic'}"
                row[key + "_s"] = time.perf_counter() - t1
                row[key + "_iterations"] = len(errs)
                row[key + "_diverged"] = div
                p.close()
        base = row["serial_kinetic_s"]
        for k in list(row):
            if k.endswith("_s"):
                row[k[:-2] + "_speedup"] = base / row[k]
        t3 = TABLE3_S[eps]
        row["paper_table3_s"] = {"para_off_adapt_off": t3[0], "para_off_adapt_on": t3[1],
                                 "para_on_adapt_off": t3[2], "para_on_adapt_on": t3[3],
                                 "fluid": TABLE3_FLUID_S}
        row["paper_table3_speedup"] = {k: t3[0] / v for k, v in row["paper_table3_s"].items()}
        rows.append(row)
        print(f"# 1d3v eps={eps:g}: serial {base:.3f} s, parareal (implicit G, hybrid) "
              f"{row['parareal_implicit_hybrid_s']:.3f} s in {row['parareal_implicit_hybrid_iterations']} "
              f"iterations", file=sys.stderr, flush=True)
    out = {"metric": "1D3V Table-3 shape: wall clock and speedups against the serial full-kinetic fine solver",
           "value": None, "unit": "s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": ("Nx=32, Nv=32x16x16 (states g(x,vx)M(vy)M(vz), advanced through their vx "
                                   "factor), x*=2pi, v*=8, N_g=200, T_f=1, tol 1e-10, eta0=delta0=1e-5, "
                                   "initial distribution M(v) vx^4 (1+0.9cos x) with its micro part, lifted "
                                   f"slice starts (L=1), FP64, {S} fine steps per slice (fine dt "
                                   f"{1.0 / (200 * S):.1e}, the same for every eps)"),
                      "paper_hardware": "2x Xeon Platinum 8268, 48 OpenMP threads (context only)"},
           "runs": rows, "wall_s": time.perf_counter() - t0}
    print(json.dumps(out), flush=True)


def run_unit(args, torch, sth, wl):
    """Step latency of one slice (one workgroup) of --nx x --nv in the chosen
    precision, all kinetic unless --unit-hybrid: the per-step cost that
    bounds a long slice, and a single fine-kernel launch for counters."""
    prec = sth.FP64 if args.precision == "fp64" else sth.FP32_BULK
    inst = wl.config2(seed=args.seed, nx=args.nx, nv=args.nv, N=4, T=1e-3)
    d = sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell, rho0=inst.rho_in,
                 T=inst.T, n_slices=4, flags=sth.FIELD | (sth.HYBRID if args.unit_hybrid else 0),
                 precision=prec, cfl_theta=inst.theta)
    p = sth.Problem(d)
    info = p.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, kin = sth.sth_fine_run(p, inst.rho_in, None, args.unit_steps)
    el = time.perf_counter() - t0
    p.close()
    us = el * 1e6 / args.unit_steps
    realsz = 8 if prec == sth.FP64 else 4
    out = {"metric": "fine step latency of one slice", "value": us, "unit": "us/step", "n_gpus": 1,
           "steps": args.unit_steps, "warmup": 0, "higher_is_better": False, "data": "synthetic",
           "dtype": "f64" if prec == sth.FP64 else "f32-bulk/f64-macro",
           "config": {"workload": f"one slice {inst.nx}x{inst.nv}, {'hybrid' if args.unit_hybrid else 'all kinetic'}",
                      "fine_block": info.fine_block, "fine_form": "resident rows" if info.fine_resident
                      else "streamed rows"},
           "kinetic_cell_updates_per_s": kin * inst.nv / el,
           "slot_gb_per_s": kin * inst.nv * 2 * realsz / el / 1e9}
    print(json.dumps(out), flush=True)


def run_parareal(torch, sth, d, K, stream, keep_iterates=False, label=""):
    """One parareal solve of the description d: the coarse guess, then K
    iterations (fine sweep of every unconverged slice, timed with HIP events
    on the stream it runs on, then the sequential correction).  Returns the
    timings, successive errors, kinetic work, final iterate and, on request,
    the iterate after every iteration.  A correction that reports a
    non-finite density ends the solve (recorded as diverged)."""
    p = sth.Problem(d)
    info0 = p.info()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    sth.sth_coarse_sweep(p, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    errs, kin_iter, units_iter, t_iter, iterates = [], [], [], [], []
    kin_prev, diverged, done = 0.0, False, 0
    first_slice = None
    for k in range(K):
        with torch.cuda.stream(stream):
            ev[k][0].record(stream)
        sth.sth_fine_sweep_batched([p], stream)
        with torch.cuda.stream(stream):
            ev[k][1].record(stream)
        try:
            e, _ = sth.sth_parareal_correct(p, want_err=True, stream=stream)
        except sth.StHError as exc:
            if exc.code != sth.STH_ENONFINITE:
                raise
            e, diverged = float("nan"), True
        done = k + 1
        errs.append(e)
        t_iter.append(time.perf_counter() - t_start)
        if k == 0:  # slice 1 after one iteration: one fine propagation from rho_in
            first_slice = sth.sth_get_rho(p)[1]
        if keep_iterates:
            iterates.append(sth.sth_get_rho(p))
        kin_now = p.info().kinetic_iface_steps
        kin_iter.append(kin_now - kin_prev)
        units_iter.append(d.n_slices - k)
        kin_prev = kin_now
        print(f"# {label} iteration {k + 1}/{K}: err {e:.3e}, sweep {ev[k][0].elapsed_time(ev[k][1]):.1f} ms",
              file=sys.stderr, flush=True)
        if diverged:
            break
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = p.info()
    U = sth.sth_get_rho(p)
    p.close()
    return {"sweep_ms": [a.elapsed_time(b) for a, b in ev[:done]], "errs": errs, "kin_iter": kin_iter,
            "units_iter": units_iter, "elapsed": t1 - t0, "wall": t1 - t_start, "t_iter": t_iter,
            "info": info, "info0": info0, "U": U, "iterates": iterates, "first_slice": first_slice,
            "diverged": diverged, "iterations": done}


def accuracy_to_cost(r, N, tols=(1e-1, 1e-2, 1e-3)):
    """Parareal accuracy against cost (Algorithm 1).  After k iterations the
    first k slice ends equal the serial fine solution bit for bit (the
    identity U^k_k = F(U^{k-1}_{k-1}) the correction keeps), so after K
    iterations slices 0..K hold the serial fine solution: the distance of
    each earlier iterate from it is measured on those slices with no extra
    run.  The serial fine wall clock is estimated as N one-slice fine
    propagations at the measured time of the first sweep, which runs all
    slices concurrently, one per compute unit."""
    K = r["iterations"]
    its = r["iterates"]
    out = {"successive_errors": r["errs"], "iterations": K, "diverged": r["diverged"]}
    if its and not r["diverged"]:
        S = its[-1][:K + 1]
        scale = float(np.max(np.abs(S)))
        out["distance_from_serial_fine"] = [float(np.max(np.abs(U[:K + 1] - S))) / scale for U in its]
        out["serial_fine_slices_known"] = K
    reach = {}
    for tol in tols:
        k = next((i for i, e in enumerate(r["errs"]) if np.isfinite(e) and e < tol), None)
        reach[f"{tol:g}"] = None if k is None else {"iterations": k + 1, "wall_s": r["t_iter"][k]}
    out["to_successive_error_below"] = reach
    if r["sweep_ms"]:
        out["serial_fine_wall_s_estimate"] = N * r["sweep_ms"][0] * 1e-3
        out["parareal_wall_s"] = r["wall"]
        out["serial_fine_over_parareal_wall_estimate"] = out["serial_fine_wall_s_estimate"] / r["wall"]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                          "(the slice-parallel multi-GPU path is design only)"}))
        sys.exit(2)

    import torch
    from paper_2511_13386_amd import sth
    from paper_2511_13386_amd import workloads as wl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.workload == "batch":
        run_batch(args, torch, sth, wl)
        return
    if args.workload == "serve":
        run_serve(args, torch, sth, wl)
        return
    if args.workload == "convergence":
        run_convergence(args, torch, sth, wl)
        return
    if args.workload == "1d3v":
        run_1d3v(args, torch, sth, wl)
        return
    if args.workload == "linf":
        run_linf(args, torch, sth, wl)
        return
    if args.workload == "unit":
        run_unit(args, torch, sth, wl)
        return
    prec = sth.FP64 if args.precision == "fp64" else sth.FP32_BULK
    inst = wl.config2(seed=args.seed, nx=args.nx, nv=args.nv, N=args.slices, T=args.T,
                      K=args.steps)

    def desc(steps_override=0, precision=prec, start_mode=sth.START_CARRY, K=args.steps):
        return sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                        rho0=inst.rho_in, T=inst.T, n_slices=inst.N, k_max=max(K, 1),
                        tol=0.0, eta0=inst.eta0, delta0=inst.delta0, lift_order=1,
                        start_mode=start_mode, cfl_theta=inst.theta,
                        flags=sth.FIELD | sth.HYBRID, precision=precision,
                        steps_override=steps_override)

    stream = torch.cuda.Stream()
    # warmup: same kernels on a separate problem with short slices
    if args.warmup > 0:
        w = sth.Problem(short_horizon(sth, desc(), 2000))
        sth.sth_coarse_sweep(w, stream)
        for _ in range(min(args.warmup, inst.N)):
            sth.sth_fine_sweep_batched([w], stream)
            sth.sth_parareal_correct(w, want_err=True, stream=stream)
        w.close()
        print(f"# warmup done ({args.warmup} short iterations)", file=sys.stderr, flush=True)

    K = min(args.steps, inst.N)
    r = run_parareal(torch, sth, desc(), K, stream, keep_iterates=True, label=args.precision)
    info = r["info"]
    sweep_ms = r["sweep_ms"]
    elapsed = r["elapsed"]
    kin_total = info.kinetic_iface_steps
    cell_updates = kin_total * inst.nv
    value = cell_updates / elapsed
    realsz = 8 if prec == sth.FP64 else 4
    # algorithmic bytes of one fine-sweep launch: read + write of g per
    # kinetic cell-update plus the macroscopic per-interface data
    iface_steps = [u * inst.nx * info.steps_per_slice for u in r["units_iter"]]
    alg_bytes = [kin * inst.nv * 2 * realsz + it * MACRO_BYTES_PER_IFACE_STEP
                 for kin, it in zip(r["kin_iter"], iface_steps)]
    avg_ms = float(np.mean(sweep_ms))
    achieved_gbs = float(np.mean([b / (ms * 1e-3) for b, ms in zip(alg_bytes, sweep_ms)])) / 1e9
    alg_tflops = float(np.mean([kin * inst.nv * FLOPS_PER_CELL_UPDATE / (ms * 1e-3)
                                for kin, ms in zip(r["kin_iter"], sweep_ms)])) / 1e12
    vec_peak = FP64_VECTOR_PEAK_TFLOPS if prec == sth.FP64 else FP32_VECTOR_PEAK_TFLOPS
    workload_key = f"{inst.nx}x{inst.nv}_{args.precision}"
    traffic = measured_traffic(workload_key)
    m0 = float(np.sum(inst.rho_in))
    U = r["U"]
    mass_drift = float(np.max(np.abs(U.sum(axis=1) - m0)) / m0)
    cus_busy = min(inst.N, 256)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == sth.FP64 else "f32-bulk/f64-macro",
        "data": "synthetic",
        "config": {
            "workload": (f"hybrid parareal {inst.nx}x{inst.nv}, N={inst.N} slices, T={inst.T}, "
                         f"periodic tanh eps profile, rho_in=1+0.3cos+0.05 noise (seed {args.seed}), "
                         f"thresholds 1e-3, {args.precision}, carried slice starts"),
            "nx": inst.nx, "nv": inst.nv, "n_slices": inst.N, "T": inst.T,
            "fine_steps_per_slice": info.steps_per_slice, "fine_dt": info.dt,
            "parareal_iterations_timed": K, "parallelism": "single GPU, one workgroup per slice",
            "fine_form": "resident rows" if info.fine_resident else "streamed rows",
            "fine_block": info.fine_block,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "achieved_kind": ("algorithmic (equivalent) bytes: 2 x 8 B per kinetic cell-update (read and "
                              "write of g') plus 64 B per interface-step, over the sweep time; the resident "
                              "form keeps the rows on chip, so this is not counted HBM traffic"),
            "counted_hbm_gbs": (traffic / (avg_ms * 1e-3) / 1e9) if traffic else None,
            "binding": (f"vector-ALU issue and the per-step macroscopic latency on the {cus_busy} compute "
                        f"units that hold a slice (one workgroup per slice); see vector_alu"),
        },
        "vector_alu": {
            "bound": "alu", "achieved": alg_tflops, "peak": vec_peak, "unit": "TFLOP/s",
            "frac": alg_tflops / vec_peak, "flops_per_cell_update": FLOPS_PER_CELL_UPDATE,
            "cus_busy": cus_busy, "cus": 256, "frac_of_busy_cus": alg_tflops / (vec_peak * cus_busy / 256),
        },
        "fine_step_us": avg_ms * 1e3 / info.steps_per_slice,
        "fine_sweep_ms_avg": avg_ms,
        "fine_sweep_ms": sweep_ms,
        "kinetic_fraction": kin_total / max(sum(iface_steps), 1),
        "parareal_wall_s": r["wall"],
        "successive_errors": r["errs"],
        "mass_drift_rel": mass_drift,
        "parareal_accuracy": dict(start="carried (each slice starts from the fine end state of the "
                                        "previous slice of the latest sweep; lifting only for the coarse guess)",
                                  **accuracy_to_cost(r, inst.N)),
    }
    del r["iterates"]
    if args.copy_calibration:
        # one elementwise kernel that reads 1 GiB and writes 1 GiB, for
        # scaling the HBM byte counters
        x = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"kernel": "torch.neg float32", "read_bytes": 1 << 30, "write_bytes": 1 << 30}
    K2 = min(K, args.other_iterations)
    if not args.no_other_precision:
        # the same solve in the other precision (FP32 bulk against FP64),
        # over the first K2 iterations
        prec2 = sth.FP32_BULK if prec == sth.FP64 else sth.FP64
        q = run_parareal(torch, sth, desc(precision=prec2, K=K2), K2, stream, label="other precision")
        ms2 = q["sweep_ms"]
        v2 = q["info"].kinetic_iface_steps * inst.nv / (sum(ms2) * 1e-3)
        v1 = sum(r["kin_iter"][:K2]) * inst.nv / (sum(sweep_ms[:K2]) * 1e-3)
        key = "fp32_bulk" if prec2 == sth.FP32_BULK else "fp64"
        realsz2 = 4 if prec2 == sth.FP32_BULK else 8
        iface2 = [u * inst.nx * q["info"].steps_per_slice for u in q["units_iter"]]
        alg2 = [kin * inst.nv * 2 * realsz2 + it * MACRO_BYTES_PER_IFACE_STEP
                for kin, it in zip(q["kin_iter"], iface2)]
        gbs2 = float(np.mean([b / (ms * 1e-3) for b, ms in zip(alg2, ms2)])) / 1e9
        traffic2 = measured_traffic(f"{inst.nx}x{inst.nv}_{'fp32' if prec2 == sth.FP32_BULK else 'fp64'}")
        out[key] = {
            "value": v2, "unit": "cell-updates/s (over the fine sweeps)",
            "iterations": K2,
            "value_this_precision_same_measure": v1,
            "speedup_fp32_over_fp64": v2 / v1 if prec2 == sth.FP32_BULK else v1 / v2,
            "fine_step_us": float(np.mean(ms2)) * 1e3 / q["info"].steps_per_slice,
            "parareal_wall_s": q["wall"],
            "roofline": {"bound": "hbm", "achieved": gbs2, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs2 / HBM_PEAK_GBS, "traffic": traffic2,
                         "achieved_kind": "algorithmic (equivalent) bytes, as the main roofline",
                         "counted_hbm_gbs": (traffic2 / (float(np.mean(ms2)) * 1e-3) / 1e9) if traffic2 else None},
            "first_slice_max_rel_rho_diff": float(np.max(np.abs(q["first_slice"] - r["first_slice"]))
                                                  / np.max(np.abs(r["first_slice"]))),
            "first_slice_note": ("slice 1 after one iteration is one fine propagation of 369,148 steps from "
                                 "rho_in; the FP64 kernel equals the FP64 oracle there to 4e-14 with no "
                                 "threshold decision taken differently (tests/test_config_parity.py)"),
            "mass_drift_rel": float(np.max(np.abs(q["U"].sum(axis=1) - m0)) / m0),
            "fine_form": "resident rows" if q["info"].fine_resident else "streamed rows",
        }
        print(f"# other precision: {v2:.3e} cell-updates/s", file=sys.stderr, flush=True)
        if args.flip_steps > 0:
            # threshold decisions against rounding on slice 1 (from rho_in,
            # g' = 0) over a bounded horizon: the (step, cell) states whose
            # status differs between FP32 bulk and FP64, and the density
            # difference once the FP64 status history is imposed on FP32
            nflip = min(args.flip_steps, info.steps_per_slice)
            p64 = sth.Problem(desc(precision=sth.FP64))
            p32 = sth.Problem(desc(precision=sth.FP32_BULK))
            r64, _, _, _, h64 = sth.sth_fine_run_masks(p64, inst.rho_in, None, nflip)
            r32, _, _, _, h32 = sth.sth_fine_run_masks(p32, inst.rho_in, None, nflip)
            r32i, _, _, _, _ = sth.sth_fine_run_masks(p32, inst.rho_in, None, nflip, replay=h64)
            p64.close()
            p32.close()
            scale = float(np.max(np.abs(r64)))
            out[key]["decisions_slice1"] = {
                "steps": nflip, "cells": inst.nx,
                "states_differing": int(np.sum(h32 != h64)),
                "max_rel_rho_diff": float(np.max(np.abs(r32 - r64))) / scale,
                "max_rel_rho_diff_fp64_history_imposed": float(np.max(np.abs(r32i - r64))) / scale,
            }
            del h64, h32
    if args.lift_iterations > 0:
        # Algorithm 1 as written: every slice starts from the lifting of its
        # start density (first order), in the precision of the main run
        KL = min(K, args.lift_iterations)
        rl = run_parareal(torch, sth, desc(start_mode=sth.START_LIFT, K=KL), KL, stream, keep_iterates=True,
                          label="lifted starts")
        out["parareal_accuracy_lifted_starts"] = dict(
            start="lifted (Algorithm 1: every slice starts from the first-order lifting of its start density)",
            fine_sweep_ms_avg=float(np.mean(rl["sweep_ms"])) if rl["sweep_ms"] else None,
            **accuracy_to_cost(rl, inst.N))
    if not args.no_batch:
        out["batch_fp32_bulk"] = batch_block(args, torch, sth, wl, sth.FP32_BULK,
                                             max(1, min(args.batch_iterations, args.batch_slices)),
                                             with_graph=False)
        print("# batched workload done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["cpu_oracle_host"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
