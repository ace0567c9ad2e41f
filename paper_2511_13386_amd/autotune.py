"""Autotuner of the fine kernel's launch configuration, per kernel class.

A kernel class is (precision, nv, nx rounded up to 64).  Its knobs are the
workgroup size, i.e. how many interfaces each thread carries (1 to 4), and
the row form (rows resident in registers for the whole slice, or streamed
from device memory every step); one workgroup always runs one slice, so the
workgroup size also sets how many slices share a compute unit.  For every
class of a workload the tuner builds a synthetic problem of that class with
as many slices as the workload has units of it (so that occupancy is that
of the real sweep), times a short batched sweep under every supported
configuration (`sth_fine_config_candidates`) and keeps the fastest
(`sth_set_fine_config`).  Results can be saved to and loaded from JSON.
A sweep of one class runs the chosen configuration as it is; a batch that
mixes classes runs grouped launches, where a class keeps its row form and
its choice between the 1024-thread streamed form and the others, and takes
the group's workgroup size.

Host-side orchestration only: the timed work is the library's own sweep.
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np

from . import sth
from . import workloads as wl

ClassKey = Tuple[int, int, int]  # (precision, nx rounded up to 64, nv)


def class_of(desc: sth.Desc) -> ClassKey:
    return (int(desc.precision), (int(desc.nx) + 63) // 64 * 64, int(desc.nv))


@dataclass
class ClassResult:
    key: ClassKey
    units: int
    timings_ms: Dict[Tuple[int, int], float] = field(default_factory=dict)
    best: Optional[Tuple[int, int]] = None
    default: Optional[Tuple[int, int]] = None

    @property
    def speedup_over_default(self) -> float:
        return self.timings_ms[self.default] / self.timings_ms[self.best]


def _probe_desc(key: ClassKey, units: int, steps: int) -> sth.Desc:
    """A hybrid problem of the class (the tanh eps profile of the hybrid
    workload) with `units` slices of about `steps` stable steps each."""
    prec, nx, nv = key
    inst = wl.config2(seed=0, nx=nx, nv=nv, N=int(units), T=1e-3, K=1)
    d = sth.Desc(nx=nx, nv=nv, eps_iface=inst.eps_iface, eps_cell=inst.eps_cell,
                 rho0=inst.rho_in, T=inst.T, n_slices=int(units), k_max=1,
                 eta0=inst.eta0, delta0=inst.delta0, flags=sth.FIELD | sth.HYBRID,
                 precision=prec, start_mode=sth.START_CARRY, cfl_theta=inst.theta)
    probe = sth.Problem(d)
    ns = probe.info().steps_per_slice
    probe.close()
    d.T = d.T * steps / ns
    return d


def tune_class(key: ClassKey, units: int, steps: int = 200, repeats: int = 3,
               max_units: int = 1024, stream=None) -> ClassResult:
    """Time every supported configuration of one class on `units` slices of
    `steps` steps; set and return the fastest."""
    import torch
    prec, nx, nv = key
    units = int(max(1, min(units, max_units)))
    res = ClassResult(key, units)
    sth.sth_set_fine_config(prec, nx, nv, None)
    res.default = sth.sth_get_fine_config(prec, nx, nv)
    s = stream if stream is not None else torch.cuda.Stream()
    p = sth.Problem(_probe_desc(key, units, steps))
    try:
        sth.sth_coarse_sweep(p, s)
        for cfg in sth.sth_fine_config_candidates(prec, nx, nv):
            sth.sth_set_fine_config(prec, nx, nv, cfg)
            sth.sth_fine_sweep_batched([p], s)  # warm-up of this kernel
            times = []
            for _ in range(repeats):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(s)
                sth.sth_fine_sweep_batched([p], s)
                b.record(s)
                b.synchronize()
                times.append(a.elapsed_time(b))
            res.timings_ms[tuple(cfg)] = float(np.median(times))
    finally:
        p.close()
    res.best = min(res.timings_ms, key=res.timings_ms.get)
    sth.sth_set_fine_config(prec, nx, nv, res.best)
    return res


def autotune(descs: Iterable[sth.Desc], steps: int = 200, repeats: int = 3,
             stream=None) -> Dict[ClassKey, ClassResult]:
    """Tune every class of a workload (units per class = the slices of its
    problems) and set the winners."""
    units: Dict[ClassKey, int] = {}
    for d in descs:
        k = class_of(d)
        units[k] = units.get(k, 0) + int(d.n_slices)
    return {k: tune_class(k, u, steps=steps, repeats=repeats, stream=stream)
            for k, u in sorted(units.items())}


def reset(results: Dict[ClassKey, ClassResult]) -> None:
    for (prec, nx, nv) in results:
        sth.sth_set_fine_config(prec, nx, nv, None)


def save(results: Dict[ClassKey, ClassResult], path: str) -> None:
    out = [{"precision": k[0], "nx": k[1], "nv": k[2], "units": r.units,
            "block": r.best[0], "resident": r.best[1],
            "timings_ms": {f"{b}x{m}": t for (b, m), t in r.timings_ms.items()}}
           for k, r in results.items()]
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


def load(path: str) -> List[ClassKey]:
    """Apply saved winners; returns the classes set."""
    with open(path) as f:
        rows = json.load(f)
    keys = []
    for r in rows:
        sth.sth_set_fine_config(int(r["precision"]), int(r["nx"]), int(r["nv"]),
                                (int(r["block"]), int(r["resident"])))
        keys.append((int(r["precision"]), int(r["nx"]), int(r["nv"])))
    return keys
