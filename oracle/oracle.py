"""ctypes wrapper of the plain FP64 CPU oracle (``sth_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  Every array crossing the boundary is float64 (int32 for masks), C order;
phase-space arrays are x-major ``g[p, j]``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sth_oracle.c")
_LIB = os.path.join(_HERE, "libsth_oracle.so")

HYBRID = 1
FIELD = 2
LITERAL_R = 4
LITERAL_FLUX = 8
COARSE_EXPLICIT = 16
STORE_F32 = 32  # g' stored in binary32 after every step (precision floor of FP32 storage)
START_LIFT = 0
START_CARRY = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over independent slices)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
             "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("nv", ctypes.c_int),
        ("Lx", ctypes.c_double), ("vstar", ctypes.c_double),
        ("rhobar", ctypes.c_double), ("dt", ctypes.c_double),
        ("eta0", ctypes.c_double), ("delta0", ctypes.c_double),
        ("flags", ctypes.c_int), ("lift_order", ctypes.c_int),
        ("start_mode", ctypes.c_int),
        ("coarse_steps", ctypes.c_long),
        ("norm_scale", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [("kinetic_iface_steps", ctypes.c_double),
                ("mask_flips", ctypes.c_double),
                ("final_kinetic", ctypes.c_double)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_P = ctypes.POINTER(Params)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_velocity_grid.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, _D]
        L.orc_maxwellian_raw.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        L.orc_fd_coef.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_fd_coef.restype = ctypes.c_double
        L.orc_poisson.argtypes = [ctypes.c_int, ctypes.c_double, _D, ctypes.c_double, _D]
        L.orc_flux_J.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, _D]
        L.orc_remainder.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, ctypes.c_double,
                                    ctypes.c_int, _D]
        L.orc_dt_max.argtypes = [_P, _D, ctypes.c_double, ctypes.c_double]
        L.orc_dt_max.restype = ctypes.c_double
        L.orc_steps_per_slice.argtypes = [ctypes.c_double, ctypes.c_double, _D]
        L.orc_steps_per_slice.restype = ctypes.c_long
        L.orc_lift.argtypes = [_P, _D, _D, _D]
        L.orc_transport.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    _D, _D, _D]
        L.orc_diagnostics.argtypes = [_P, _D, _D, _D, _D, _D, _D, _D, _D, _D, _I]
        L.orc_fine_propagate.argtypes = [_P, _D, _D, _D, _D, ctypes.c_long, _D, _D, _I,
                                         ctypes.POINTER(Stats)]
        _U8 = ctypes.POINTER(ctypes.c_uint8)
        L.orc_fine_propagate_masks.argtypes = [_P, _D, _D, _D, _D, ctypes.c_long, _U8, _U8, _D, _D, _I,
                                               ctypes.POINTER(Stats)]
        L.orc_coarse_step.argtypes = [_P, ctypes.c_double, _D, _D]
        L.orc_cyclic_tridiag.argtypes = [ctypes.c_int, _D, _D, _D, _D, _D]
        L.orc_cyclic_tridiag.restype = ctypes.c_int
        L.orc_parareal.argtypes = [_P, _D, _D, ctypes.c_int, ctypes.c_long, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_double, _D, _D, _D, _D, _D]
        L.orc_parareal.restype = ctypes.c_int
        L.orc_serial_fine.argtypes = [_P, _D, _D, ctypes.c_int, ctypes.c_long, _D, _D, _D]
        L.orc_fine_batch.argtypes = [_P, _D, _D, ctypes.c_int, ctypes.c_long, _D, _D, _D, _D]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(nx, nv, *, Lx=1.0, vstar=8.0, rhobar=1.0, dt=0.0, eta0=1e-3, delta0=1e-3,
           flags=FIELD, lift_order=3, start_mode=START_LIFT) -> Params:
    return Params(int(nx), int(nv), float(Lx), float(vstar), float(rhobar), float(dt),
                  float(eta0), float(delta0), int(flags), int(lift_order), int(start_mode))


# ----------------------------------------------------------------------------- pieces
def velocity_grid(nv, vstar=8.0):
    v = np.zeros(nv)
    M = np.zeros(nv)
    m2 = ctypes.c_double()
    lib().orc_velocity_grid(nv, vstar, _d(v), _d(M), ctypes.byref(m2))
    return v, M, m2.value


def maxwellian_raw(nv, vstar=8.0):
    M = np.zeros(nv)
    lib().orc_maxwellian_raw(nv, vstar, _d(M))
    return M


def fd_coef(d, k):
    return lib().orc_fd_coef(d, k)


def poisson(rho, rhobar, dx):
    rho = _f64(rho)
    E = np.zeros_like(rho)
    lib().orc_poisson(rho.size, dx, _d(rho), rhobar, _d(E))
    return E


def flux_J(rho, E, dx):
    rho, E = _f64(rho), _f64(E)
    J = np.zeros_like(rho)
    lib().orc_flux_J(rho.size, dx, _d(rho), _d(E), _d(J))
    return J


def remainder(rho, E, rhobar, dx, field=True):
    rho, E = _f64(rho), _f64(E)
    R = np.zeros_like(rho)
    lib().orc_remainder(rho.size, dx, _d(rho), _d(E), rhobar, int(field), _d(R))
    return R


def dt_max(p: Params, eps_iface, Emax, theta):
    eps_iface = _f64(eps_iface)
    return lib().orc_dt_max(ctypes.byref(p), _d(eps_iface), float(Emax), float(theta))


def steps_per_slice(slice_len, dtmax):
    dt = ctypes.c_double()
    n = lib().orc_steps_per_slice(float(slice_len), float(dtmax), ctypes.byref(dt))
    return int(n), dt.value


def transport(g, E, Lx=1.0, vstar=8.0):
    """Upwind (v d_x + E d_v) g' at every interface, before the projection."""
    g, E = _f64(g), _f64(E)
    A = np.zeros_like(g)
    lib().orc_transport(g.shape[0], g.shape[1], float(Lx), float(vstar), _d(g), _d(E), _d(A))
    return A


def lift(p: Params, eps_iface, rho):
    eps_iface, rho = _f64(eps_iface), _f64(rho)
    g = np.zeros((p.nx, p.nv))
    lib().orc_lift(ctypes.byref(p), _d(eps_iface), _d(rho), _d(g))
    return g


def diagnostics(p: Params, eps_iface, eps_cell, rho, g):
    eps_iface, eps_cell, rho, g = map(_f64, (eps_iface, eps_cell, rho, g))
    out = {k: np.zeros(p.nx) for k in ("E", "J", "Phi", "N", "R")}
    mask = np.zeros(p.nx, dtype=np.int32)
    lib().orc_diagnostics(ctypes.byref(p), _d(eps_iface), _d(eps_cell), _d(rho), _d(g),
                          _d(out["E"]), _d(out["J"]), _d(out["Phi"]), _d(out["N"]),
                          _d(out["R"]), mask.ctypes.data_as(_I))
    out["mask"] = mask
    return out


def fine_propagate(p: Params, eps_iface, eps_cell, rho_in, g_in, nsteps):
    eps_iface, eps_cell, rho_in = map(_f64, (eps_iface, eps_cell, rho_in))
    g_ptr = None
    if g_in is not None:
        g_in = _f64(g_in)
        g_ptr = _d(g_in)
    rho = np.zeros(p.nx)
    g = np.zeros((p.nx, p.nv))
    mask = np.zeros(p.nx, dtype=np.int32)
    st = Stats()
    lib().orc_fine_propagate(ctypes.byref(p), _d(eps_iface), _d(eps_cell), _d(rho_in), g_ptr,
                             int(nsteps), _d(rho), _d(g), mask.ctypes.data_as(_I),
                             ctypes.byref(st))
    return rho, g, mask, {"kinetic_iface_steps": st.kinetic_iface_steps,
                          "mask_flips": st.mask_flips, "final_kinetic": st.final_kinetic}


def fine_propagate_masks(p: Params, eps_iface, eps_cell, rho_in, g_in, nsteps, replay=None):
    """fine_propagate with the cell status of every step: returns (rho, g,
    cell_mask, stats, hist) with hist[n, i] = 1 if cell i is kinetic at step n
    (n = 0..nsteps).  replay ([nsteps+1, nx], nonzero = kinetic) imposes the
    statuses instead of the rule.  Hybrid runs only."""
    if not p.flags & HYBRID:
        raise ValueError("cell status history needs the hybrid flag")
    eps_iface, eps_cell, rho_in = map(_f64, (eps_iface, eps_cell, rho_in))
    g_ptr = None
    if g_in is not None:
        g_in = _f64(g_in)
        g_ptr = _d(g_in)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    rp = None
    if replay is not None:
        replay = np.ascontiguousarray(np.asarray(replay) != 0, dtype=np.uint8)
        if replay.shape != (int(nsteps) + 1, p.nx):
            raise ValueError("replay must have shape (nsteps + 1, nx)")
        rp = replay.ctypes.data_as(u8)
    hist = np.zeros((int(nsteps) + 1, p.nx), dtype=np.uint8)
    rho = np.zeros(p.nx)
    g = np.zeros((p.nx, p.nv))
    mask = np.zeros(p.nx, dtype=np.int32)
    st = Stats()
    lib().orc_fine_propagate_masks(ctypes.byref(p), _d(eps_iface), _d(eps_cell), _d(rho_in), g_ptr,
                                   int(nsteps), rp, hist.ctypes.data_as(u8), _d(rho), _d(g),
                                   mask.ctypes.data_as(_I), ctypes.byref(st))
    return rho, g, mask, {"kinetic_iface_steps": st.kinetic_iface_steps,
                          "mask_flips": st.mask_flips, "final_kinetic": st.final_kinetic}, hist


def coarse_step(p: Params, dtG, rho_in):
    rho_in = _f64(rho_in)
    out = np.zeros_like(rho_in)
    lib().orc_coarse_step(ctypes.byref(p), float(dtG), _d(rho_in), _d(out))
    return out


def cyclic_tridiag(a, b, c, d):
    a, b, c, d = map(_f64, (a, b, c, d))
    x = np.zeros_like(d)
    rc = lib().orc_cyclic_tridiag(d.size, _d(a), _d(b), _d(c), _d(d), _d(x))
    if rc != 0:
        raise ValueError("cyclic tridiagonal solve needs n >= 3")
    return x


def parareal(p: Params, eps_iface, eps_cell, N, steps, dtG, K, tol, rho_in, g_in=None):
    eps_iface, eps_cell, rho_in = map(_f64, (eps_iface, eps_cell, rho_in))
    g_ptr = None
    if g_in is not None:
        g_in = _f64(g_in)
        g_ptr = _d(g_in)
    U = np.zeros((N + 1, p.nx))
    err = np.zeros(max(K, 1))
    kin = np.zeros(1)
    it = lib().orc_parareal(ctypes.byref(p), _d(eps_iface), _d(eps_cell), int(N), int(steps),
                            float(dtG), int(K), float(tol), _d(rho_in), g_ptr, _d(U), _d(err),
                            _d(kin))
    return U, err[:it], it, float(kin[0])


def serial_fine(p: Params, eps_iface, eps_cell, N, steps, rho_in, g_in=None):
    eps_iface, eps_cell, rho_in = map(_f64, (eps_iface, eps_cell, rho_in))
    g_ptr = None
    if g_in is not None:
        g_in = _f64(g_in)
        g_ptr = _d(g_in)
    S = np.zeros((N + 1, p.nx))
    lib().orc_serial_fine(ctypes.byref(p), _d(eps_iface), _d(eps_cell), int(N), int(steps),
                          _d(rho_in), g_ptr, _d(S))
    return S


def fine_batch(p: Params, eps_iface, eps_cell, rho_in, nsteps, g_in=None):
    """Independent fine propagations of rho_in[u] (OpenMP over units)."""
    eps_iface, eps_cell, rho_in = map(_f64, (eps_iface, eps_cell, rho_in))
    g_ptr = None
    if g_in is not None:
        g_in = _f64(g_in)
        g_ptr = _d(g_in)
    out = np.zeros_like(rho_in)
    kin = np.zeros(1)
    lib().orc_fine_batch(ctypes.byref(p), _d(eps_iface), _d(eps_cell), rho_in.shape[0],
                         int(nsteps), _d(rho_in), g_ptr, _d(out), _d(kin))
    return out, float(kin[0])


def num_threads():
    return lib().orc_num_threads()


# ----------------------------------------------------------------------------- problem set-up
def axis_m2sum(n, vstar):
    """sum_j M_j^2 dv of the discrete normalised Maxwellian on n midpoint
    nodes of [-vstar, vstar] (a transverse velocity axis in 1D3V)."""
    dv = 2.0 * vstar / n
    v = -vstar + (np.arange(n) + 0.5) * dv
    M = np.exp(-0.5 * v * v)
    M = M / (np.sum(M) * dv)
    return float(np.sum(M * M) * dv)


def setup(nx, nv, eps_iface, rho_in, *, T, N, theta=1.0, Lx=1.0, vstar=8.0, eta0=1e-3,
          delta0=1e-3, flags=FIELD, lift_order=3, start_mode=START_LIFT, nv_y=0, nv_z=0):
    """Derive rhobar, the fine step and steps per slice the way the oracle
    defines them (mean initial density; stable step bound; equal steps per
    slice).  Returns (Params, steps_per_slice, dtG)."""
    rho_in = _f64(rho_in)
    dx = Lx / nx
    rhobar = _seq_mean(rho_in)
    p = params(nx, nv, Lx=Lx, vstar=vstar, rhobar=rhobar, eta0=eta0, delta0=delta0,
               flags=flags, lift_order=lift_order, start_mode=start_mode)
    if flags & FIELD:
        Emax = float(np.max(np.abs(poisson(rho_in, rhobar, dx))))
    else:
        Emax = 0.0
    dtm = dt_max(p, eps_iface, Emax, theta)
    ns, dt = steps_per_slice(T / N, dtm)
    p.dt = dt
    # explicit coarse scheme: its diffusive stable step with the same margin
    m2 = velocity_grid(nv, vstar)[2]
    p.coarse_steps = int(math.ceil((T / N) / (theta * 0.75 * dx * dx / (2.0 * m2))))
    if nv_y:
        p.norm_scale = math.sqrt(axis_m2sum(nv_y, vstar) * axis_m2sum(nv_z, vstar))
    return p, ns, T / N


def _seq_mean(a):
    s = 0.0
    for x in a:
        s += float(x)
    return s / len(a)
