"""Continuous-batching solve server on one GPU.

Requests are hybrid parareal solves (one `Desc` each) arriving over time.
The server

* admits a waiting request as soon as its device footprint
  (`sth_footprint_bytes`) fits in the free part of a preallocated device arena
  and an active slot is free (no device allocation per request: blocks are
  carved first-fit from one torch tensor);
* keeps every admitted solve's state resident on the device;
* advances all active solves together, one tick at a time.  With
  `chunk_steps` unset a tick is one parareal iteration of each of them: one
  batched fine sweep over every unconverged slice of every active solve
  (`sth_fine_sweep_batched`, all kernel classes concurrent) followed by their
  corrections in one launch (`sth_parareal_correct_batched`, one read-back of
  all errors).  With `chunk_steps = S` a tick advances every active sweep by
  at most S fine steps per slice (`sth_fine_sweep_chunk`), and only the
  solves whose sweep ended get their correction: a tick then lasts about S
  steps of the slowest active class instead of a whole slice, so short solves
  are not held behind long ones and arrivals join sooner;
* retires a solve when it reaches its tolerance or its iteration limit, or
  as failed (`Result.ok` False) when a slice density turns non-finite,
  returns the slice-end densities and frees its block, which admits the next
  waiting requests at the next tick.

Requests that arrive while others run join at the next tick; each result is
the same as the solve alone (the batched sweep is batch-invariant bit for
bit).  Host-side orchestration only: every step of a solve runs in libsth.so.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import sth

_ALIGN = 256


class FreeList:
    """First-fit bookkeeping of 256-byte aligned blocks in [0, nbytes)."""

    def __init__(self, nbytes: int):
        self.nbytes = int(nbytes) // _ALIGN * _ALIGN
        self.free: List[List[int]] = [[0, self.nbytes]] if self.nbytes > 0 else []  # sorted [offset, size]

    @staticmethod
    def rounded(size: int) -> int:
        return (int(size) + _ALIGN - 1) // _ALIGN * _ALIGN

    def alloc(self, size: int) -> Optional[int]:
        size = self.rounded(size)
        for k, (off, sz) in enumerate(self.free):
            if sz >= size:
                if sz == size:
                    self.free.pop(k)
                else:
                    self.free[k] = [off + size, sz - size]
                return off
        return None

    def release(self, off: int, size: int) -> None:
        size = self.rounded(size)
        self.free.append([off, size])
        self.free.sort()
        merged: List[List[int]] = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] > o:
                raise ValueError("released block overlaps a free block")
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1][1] += s
            else:
                merged.append([o, s])
        self.free = merged

    @property
    def free_bytes(self) -> int:
        return sum(s for _, s in self.free)


class ArenaAllocator(FreeList):
    """FreeList over one device tensor (no device allocation per request)."""

    def __init__(self, nbytes: int, device: str = "cuda"):
        import torch
        super().__init__(nbytes)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.base = int(self.buf.data_ptr())
        if self.base % _ALIGN:
            raise RuntimeError("device arena is not 256-byte aligned")

    def view(self, off: int, size: int):
        return self.buf[off:off + size]


@dataclass
class Request:
    rid: int
    desc: sth.Desc
    arrival: float                  # seconds from the start of the run
    max_iters: int = 2
    tol: float = 0.0


@dataclass
class Result:
    rid: int
    rho: np.ndarray                 # (N+1, nx) slice-end densities
    errors: List[float]
    arrival: float
    admitted: float
    finished: float
    cell_updates: float
    ok: bool = True                 # False: a slice density went non-finite

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Active:
    req: Request
    prob: sth.Problem
    off: int
    size: int
    admitted: float
    errors: List[float] = field(default_factory=list)


class Server:
    def __init__(self, budget_bytes: int, max_active: int = 512, stream=None,
                 chunk_steps: Optional[int] = None):
        import torch
        self.arena = ArenaAllocator(budget_bytes)
        self.max_active = max_active
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.chunk_steps = chunk_steps
        self.ticks = 0

    def _admit(self, req: Request, now: float) -> Optional[_Active]:
        size = sth.sth_footprint_bytes(req.desc)
        if size > self.arena.nbytes:
            raise ValueError(f"request {req.rid} needs {size} bytes, more than the whole arena")
        off = self.arena.alloc(size)
        if off is None:
            return None
        prob = sth.Problem(req.desc, arena=self.arena.view(off, size))
        sth.sth_coarse_sweep(prob, self.stream)
        return _Active(req, prob, off, size, now)

    def run(self, requests: List[Request], clock=time.perf_counter,
            on_done: Optional[Callable[[int], None]] = None) -> List[Result]:
        """Serve the requests (sorted by arrival) in real time; returns one
        result per request.  on_done(n) is called with the number of finished
        requests after each tick that finished some."""
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: List[Request] = []
        active: List[_Active] = []
        results: Dict[int, Result] = {}
        t0 = clock()
        k = 0
        while k < len(pending) or waiting or active:
            now = clock() - t0
            while k < len(pending) and pending[k].arrival <= now:
                waiting.append(pending[k])
                k += 1
            # admission: FIFO while a slot and memory are free
            while waiting and len(active) < self.max_active:
                a = self._admit(waiting[0], now)
                if a is None:
                    break
                active.append(a)
                waiting.pop(0)
            if not active:
                if k < len(pending):  # idle until the next arrival
                    time.sleep(max(0.0, pending[k].arrival - (clock() - t0)))
                continue
            # one tick: a parareal iteration of every active solve, or a
            # chunk of fine steps of every active sweep
            if self.chunk_steps is None:
                ready = list(active)
                sth.sth_fine_sweep_batched([a.prob for a in active], self.stream)
            else:
                done = sth.sth_fine_sweep_chunk([a.prob for a in active], self.chunk_steps, self.stream)
                ready = [a for a, d in zip(active, done) if d]
            if ready:
                errs = sth.sth_parareal_correct_batched([a.prob for a in ready], want_err=True,
                                                        stream=self.stream, nonfinite_ok=True)
                for a, e in zip(ready, errs):
                    a.errors.append(e)
            self.ticks += 1
            done_t = clock() - t0
            still: List[_Active] = []
            for a in active:
                it = len(a.errors)
                bad = bool(it) and not np.isfinite(a.errors[-1])
                if it and (bad or it >= a.req.max_iters or it >= a.prob.N or a.errors[-1] < a.req.tol):
                    info = a.prob.info()
                    results[a.req.rid] = Result(a.req.rid, sth.sth_get_rho(a.prob), list(a.errors),
                                                a.req.arrival, a.admitted, done_t,
                                                info.kinetic_iface_steps * a.prob.nv, ok=not bad)
                    a.prob.close()
                    self.arena.release(a.off, a.size)
                else:
                    still.append(a)
            if on_done is not None and len(still) < len(active):
                on_done(len(results))
            active = still
        return [results[r.rid] for r in requests]


def latency_percentiles(results: List[Result], qs=(50, 99)) -> Dict[str, float]:
    lat = np.array([r.latency for r in results])
    return {f"p{q}": float(np.percentile(lat, q)) for q in qs}
