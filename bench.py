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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--nv", type=int, default=64)
    ap.add_argument("--slices", type=int, default=64)
    ap.add_argument("--T", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB elementwise copy kernel (HBM counter calibration)")
    return ap.parse_args()


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
    # calibrate on one unit
    t0 = time.perf_counter()
    _, kin1 = orc.fine_batch(p, inst.eps_iface, inst.eps_cell, starts[:1], 200, gs[:1])
    dt1 = time.perf_counter() - t0
    per_step_unit = dt1 / 200.0
    steps = int(max(200, min(ns, target_s / per_step_unit * threads / nun)))
    t0 = time.perf_counter()
    _, kin = orc.fine_batch(p, inst.eps_iface, inst.eps_cell, starts, steps, gs)
    el = time.perf_counter() - t0
    return {
        "value": kin * inst.nv / el,
        "unit": "cell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{nun} slices x {steps} fine steps of iteration 0 (of {ns} per slice), "
                   f"{el:.1f} s wall, OpenMP over slices"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(the slice-parallel multi-GPU path is design only)"}))
        sys.exit(2)

    import torch
    from paper_2511_13386_amd import sth
    from paper_2511_13386_amd import workloads as wl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    prec = sth.FP64 if args.precision == "fp64" else sth.FP32_BULK
    inst = wl.config2(seed=args.seed, nx=args.nx, nv=args.nv, N=args.slices, T=args.T,
                      K=args.steps)

    def desc(steps_override=0):
        return sth.Desc(nx=inst.nx, nv=inst.nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                        rho0=inst.rho_in, T=inst.T, n_slices=inst.N, k_max=max(args.steps, 1),
                        tol=0.0, eta0=inst.eta0, delta0=inst.delta0, lift_order=1,
                        start_mode=sth.START_CARRY, cfl_theta=inst.theta,
                        flags=sth.FIELD | sth.HYBRID, precision=prec,
                        steps_override=steps_override)

    stream = torch.cuda.Stream()
    # warmup: same kernels on a separate problem with short slices
    if args.warmup > 0:
        w = sth.Problem(desc(steps_override=2000))
        sth.sth_coarse_sweep(w, stream)
        for _ in range(min(args.warmup, inst.N)):
            sth.sth_fine_sweep_batched([w], stream)
            sth.sth_parareal_correct(w, want_err=True, stream=stream)
        w.close()
        print(f"# warmup done ({args.warmup} short iterations)", file=sys.stderr, flush=True)

    p = sth.Problem(desc())
    info0 = p.info()
    K = min(args.steps, inst.N)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    sth.sth_coarse_sweep(p, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    errs, kin_per_iter, units_per_iter = [], [], []
    kin_prev = 0.0
    for k in range(K):
        with torch.cuda.stream(stream):
            ev[k][0].record(stream)
        sth.sth_fine_sweep_batched([p], stream)
        with torch.cuda.stream(stream):
            ev[k][1].record(stream)
        e, _ = sth.sth_parareal_correct(p, want_err=True, stream=stream)
        errs.append(e)
        kin_now = p.info().kinetic_iface_steps
        kin_per_iter.append(kin_now - kin_prev)
        units_per_iter.append(inst.N - k)
        kin_prev = kin_now
        print(f"# iteration {k + 1}/{K}: err {e:.3e}, sweep {ev[k][0].elapsed_time(ev[k][1]):.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    wall = t1 - t_start
    info = p.info()
    U = sth.sth_get_rho(p)
    p.close()

    sweep_ms = [a.elapsed_time(b) for a, b in ev]
    kin_total = info.kinetic_iface_steps
    cell_updates = kin_total * inst.nv
    value = cell_updates / elapsed
    realsz = 8 if prec == sth.FP64 else 4
    # algorithmic bytes of one fine-sweep launch: read + write of g per
    # kinetic cell-update plus the macroscopic per-interface data
    iface_steps = [u * inst.nx * info.steps_per_slice for u in units_per_iter]
    alg_bytes = [kin * inst.nv * 2 * realsz + it * MACRO_BYTES_PER_IFACE_STEP
                 for kin, it in zip(kin_per_iter, iface_steps)]
    avg_ms = float(np.mean(sweep_ms))
    achieved_gbs = float(np.mean([b / (ms * 1e-3) for b, ms in zip(alg_bytes, sweep_ms)])) / 1e9
    alg_tflops = float(np.mean([kin * inst.nv * FLOPS_PER_CELL_UPDATE / (ms * 1e-3)
                                for kin, ms in zip(kin_per_iter, sweep_ms)])) / 1e12
    vec_peak = FP64_VECTOR_PEAK_TFLOPS if prec == sth.FP64 else FP32_VECTOR_PEAK_TFLOPS
    workload_key = f"{inst.nx}x{inst.nv}_{args.precision}"
    traffic = measured_traffic(workload_key)
    m0 = float(np.sum(inst.rho_in))
    mass_drift = float(np.max(np.abs(U.sum(axis=1) - m0)) / m0)

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
        },
        "vector_alu": {
            "achieved": alg_tflops, "peak": vec_peak, "unit": "TFLOP/s",
            "frac": alg_tflops / vec_peak, "flops_per_cell_update": FLOPS_PER_CELL_UPDATE,
            "cus_busy": min(inst.N, 256), "cus": 256,
        },
        "fine_step_us": avg_ms * 1e3 / info.steps_per_slice,
        "fine_sweep_ms_avg": avg_ms,
        "fine_sweep_ms": sweep_ms,
        "kinetic_fraction": kin_total / max(sum(iface_steps), 1),
        "parareal_wall_s": wall,
        "successive_errors": errs,
        "mass_drift_rel": mass_drift,
    }
    if args.copy_calibration:
        # one elementwise kernel that reads 1 GiB and writes 1 GiB, for
        # scaling the HBM byte counters
        x = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"kernel": "torch.neg float32", "read_bytes": 1 << 30, "write_bytes": 1 << 30}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
