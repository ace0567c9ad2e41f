"""Seeded synthetic inputs for the hybrid parareal solver.

This module only draws input data (initial densities, Knudsen-number profiles,
instance sizes, arrival times).  It holds none of the method's arithmetic and
is shared by the GPU path, the oracle-based tests and the benchmark so that
both sides see bit-identical inputs.

The paper uses no public dataset: its experiments are initial-value problems
(Section 5).  The workloads below are synthetic problems of the same kind on
the unit torus, 1D1V.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, n: int) -> np.ndarray:
    """n outputs of the SplitMix64 generator (Steele, Lea, Flood 2014) as uint64."""
    out = np.empty(n, dtype=np.uint64)
    x = seed & _MASK64
    for k in range(n):
        x = (x + 0x9E3779B97F4A7C15) & _MASK64
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out[k] = z ^ (z >> 31)
    return out


def uniform_pm1(seed: int, n: int) -> np.ndarray:
    """i.i.d. U[-1, 1) doubles from the top 53 bits of SplitMix64."""
    u = (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def cell_centres(nx: int, Lx: float = 1.0) -> np.ndarray:
    return (np.arange(nx) + 0.5) * (Lx / nx)


def interfaces(nx: int, Lx: float = 1.0) -> np.ndarray:
    return (np.arange(nx) + 1.0) * (Lx / nx)


def eps_tanh_literal(x: np.ndarray) -> np.ndarray:
    """Knudsen profile 1e-4 + 0.5 (1 + tanh((x - 0.5)/0.05)) as written: on the
    unit torus it jumps from ~1 to 1e-4 across x = 0 == 1."""
    return 1e-4 + 0.5 * (1.0 + np.tanh((x - 0.5) / 0.05))


def eps_tanh(x: np.ndarray, w: float = 0.05) -> np.ndarray:
    """Periodic continuation of 1e-4 + 0.5 (1 + tanh((x - 0.5)/w)) on the unit
    torus: the sum over periodic images of the smoothed box [0.5, 1).  It equals
    the written profile to within 1e-4 on [0.25, 0.75] and replaces its jump
    at x = 0 == 1 by the mirror transition of the same width.  Fluid on the left
    half (eps ~ 1e-4), kinetic on the right half (eps ~ 1)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.zeros_like(x)
    for m in (-2, -1, 0, 1, 2):
        s += np.tanh((x - 0.5 - m) / w) - np.tanh((x - 1.0 - m) / w)
    return 1e-4 + 0.5 * s


@dataclass
class Instance:
    """One initial-value problem of the hybrid parareal solver."""
    nx: int
    nv: int
    rho_in: np.ndarray
    eps_iface: np.ndarray
    eps_cell: np.ndarray
    T: float
    N: int
    K: int = 8
    tol: float = 0.0
    theta: float = 1.0
    vstar: float = 8.0
    Lx: float = 1.0
    eta0: float = 1e-3
    delta0: float = 1e-3
    hybrid: bool = True
    field_on: bool = True
    lift_order: int = 3
    g_in: Optional[np.ndarray] = None
    name: str = ""


def config1() -> Instance:
    """Plain serial micro-macro solver, FP64: Nx=64, Nv=32, eps=1e-2,
    rho_in = 1 + 0.5 cos(2 pi x), T=0.1, dt = 0.5 x stable step, full kinetic,
    one slice (no parareal)."""
    nx, nv = 64, 32
    xc = cell_centres(nx)
    return Instance(nx=nx, nv=nv, rho_in=1.0 + 0.5 * np.cos(2 * math.pi * xc),
                    eps_iface=np.full(nx, 1e-2), eps_cell=np.full(nx, 1e-2),
                    T=0.1, N=1, K=1, theta=0.5, hybrid=False, name="serial-64x32-eps1e-2")


def config2(seed: int = 0, nx: int = 512, nv: int = 64, N: int = 64, T: float = 1.0,
            K: int = 8) -> Instance:
    """Hybrid parareal: eps(x) tanh profile, rho_in = 1 + 0.3 cos(2 pi x) + 0.05 xi,
    xi ~ U[-1,1) i.i.d. from SplitMix64(seed); thresholds 1e-3; lifting order 3."""
    xc, xp = cell_centres(nx), interfaces(nx)
    rho = 1.0 + 0.3 * np.cos(2 * math.pi * xc) + 0.05 * uniform_pm1(seed, nx)
    return Instance(nx=nx, nv=nv, rho_in=rho, eps_iface=eps_tanh(xp), eps_cell=eps_tanh(xc),
                    T=T, N=N, K=K, theta=1.0, hybrid=True,
                    name=f"hybrid-parareal-{nx}x{nv}-N{N}-seed{seed}")


def config3(seed: int = 0, T: float = 1.0) -> Instance:
    """Same hybrid parareal at Nx=2048, Nv=128, N=128 slices."""
    inst = config2(seed=seed, nx=2048, nv=128, N=128, T=T)
    inst.name = f"hybrid-parareal-2048x128-N128-seed{seed}"
    return inst


def random_instance(seed: int, *, N: int = 32, T: float = 0.01,
                    nx_choices=(128, 256, 512, 1024, 2048), nv_choices=(32, 64, 128),
                    log_eps=(-4.0, 0.0)) -> Instance:
    """Batching/serving instance: Nx and Nv uniform over the choices, constant
    eps with log10 eps ~ U[log_eps], rho_in = 1 + sum_m A_m cos(2 pi k_m x + phi_m)
    with 1-3 modes, A_m ~ U[0, 0.5], distinct k_m in 1..8, phi_m ~ U[0, 2 pi).
    All draws come from one SplitMix64 stream of the seed."""
    u = (uniform_pm1(seed, 64) + 1.0) * 0.5  # U[0,1)
    it = iter(u)
    nx = int(nx_choices[min(int(next(it) * len(nx_choices)), len(nx_choices) - 1)])
    nv = int(nv_choices[min(int(next(it) * len(nv_choices)), len(nv_choices) - 1)])
    eps = 10.0 ** (log_eps[0] + (log_eps[1] - log_eps[0]) * next(it))
    nmodes = 1 + min(int(next(it) * 3), 2)
    ks: List[int] = []
    while len(ks) < nmodes:
        k = 1 + min(int(next(it) * 8), 7)
        if k not in ks:
            ks.append(k)
    xc = cell_centres(nx)
    rho = np.ones(nx)
    for k in ks:
        A = 0.5 * next(it)
        phi = 2 * math.pi * next(it)
        rho = rho + A * np.cos(2 * math.pi * k * xc + phi)
    return Instance(nx=nx, nv=nv, rho_in=rho, eps_iface=np.full(nx, eps),
                    eps_cell=np.full(nx, eps), T=T, N=N, K=8, theta=1.0, hybrid=True,
                    name=f"random-{seed}-{nx}x{nv}-eps{eps:.2e}")


def batch_config(count: int = 256, base_seed: int = 1000, **kw) -> List[Instance]:
    return [random_instance(base_seed + i, **kw) for i in range(count)]


def poisson_arrivals(n: int, rate: float, seed: int = 99) -> np.ndarray:
    """Arrival times of a Poisson process: cumulative exponential gaps."""
    u = (uniform_pm1(seed, n) + 1.0) * 0.5
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


def paper_setting(eps: float, adaptation: bool = True, nx: int = 32, nv: int = 32, N: int = 200,
                  T: float = 1.0, lift_order: int = 3, micro: bool = False) -> Instance:
    """The numerical setting of the paper's Section 5 in 1D1V: torus length
    2 pi, v* = 8, Nx = Nvx = 32, N_g = 200 slices, T_f = 1, thresholds
    eta0 = delta0 = 1e-5, lifting order 3, constant eps.  micro=False: the
    density 3 (1 + 0.9 cos(x)) of the paper's initial condition (<v^4 M> = 3)
    at local equilibrium (g' = 0).  micro=True: the paper's initial
    distribution itself (see paper_initial_distribution), with its density
    and its micro part g' = (f - rho M)/eps."""
    Lx = 2 * math.pi
    xc = cell_centres(nx, Lx)
    rho = 3.0 * (1.0 + 0.9 * np.cos(2 * math.pi * xc / Lx))
    g_in = None
    if micro:
        rho, g_in = paper_initial_distribution(nx, nv, eps, Lx=Lx, vstar=8.0)
    return Instance(nx=nx, nv=nv, rho_in=rho, g_in=g_in,
                    eps_iface=np.full(nx, eps), eps_cell=np.full(nx, eps), T=T, N=N, K=N,
                    tol=1e-10, theta=1.0, vstar=8.0, Lx=Lx, eta0=1e-5, delta0=1e-5,
                    hybrid=adaptation, lift_order=lift_order,
                    name=f"paper-setting-eps{eps:.0e}-{'adapt' if adaptation else 'noadapt'}"
                         f"{'-micro' if micro else ''}")


def paper_initial_distribution(nx: int, nv: int, eps: float, Lx: float = 2 * math.pi, vstar: float = 8.0):
    """The initial distribution of the paper's Section 5 on the grid nodes,
    f(x, v) = M(v) v^4 (1 + 0.9 cos(2 pi x / Lx)) with M(v) = exp(-v^2/2)/sqrt(2 pi)
    (for the 1D3V statement this is the vx factor of f; the transverse
    factors are M(vy) M(vz)), at cell centres and midpoint velocity nodes.
    Returns the density rho_i = sum_j f_ij dv and the scaled perturbation
    g'_ij = (f_ij - rho_i M_j)/eps, x-major."""
    xc = cell_centres(nx, Lx)
    dv = 2.0 * vstar / nv
    v = -vstar + (np.arange(nv) + 0.5) * dv
    M = np.exp(-0.5 * v * v) / math.sqrt(2.0 * math.pi)
    f = (1.0 + 0.9 * np.cos(2 * math.pi * xc / Lx))[:, None] * (M * v ** 4)[None, :]
    rho = f.sum(axis=1) * dv
    g = (f - rho[:, None] * M[None, :]) / eps
    return rho, g


def small_hybrid(seed: int = 0, nx: int = 96, nv: int = 32, N: int = 4, T: float = 2e-3,
                 K: int = 4) -> Instance:
    """A small hybrid instance with the tanh eps profile: oracle-sized (seconds)
    but with several tiles and a ragged tail."""
    inst = config2(seed=seed, nx=nx, nv=nv, N=N, T=T, K=K)
    inst.name = f"small-hybrid-{nx}x{nv}-N{N}-seed{seed}"
    return inst
