"""Brute-force 1D3V fine propagator (numpy, FP64): TEST INFRASTRUCTURE ONLY.

The paper states the model and the schemes in 1D3V: x in a periodic interval,
v in R^3 (truncated to the box [-vstar, vstar]^3 as in Section 5), the field
along x.  This module runs the hybrid scheme S^HMM of Section 2.3 on a full
3D velocity grid, so that the 1D1V reduction used by the library for states
of the form g(x, vx) M(vy) M(vz) can be checked against the scheme itself on
small grids.  It is written from the paper's equations: every velocity
quantity is a 3D array, the projection integrates over all three velocity
axes, the norm of the perturbation is the 3D one.  Only the macroscopic
helpers (Gauss law, limit flux J, remainder R of eq. (RemainderBis) with the
Table 1 stencils), which do not involve the velocity variable, are taken
from the pinned 1D oracle.

Readings are the same as those of the 1D oracle (upwind r+ = max(r, 0),
r- = min(r, 0); zero velocity flux through the box faces in vx; g' = g/eps
stored at interfaces; e = exp(-dt/eps^2), a = -expm1(-dt/eps^2);
flux-matched density update; status rules of Section 2.2 evaluated on the
data of step n and applied at n + 1).

Parity unpinned beyond: mass conservation, the equilibrium, and agreement
with the 1D1V oracle on separable states (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np

from . import oracle as orc


def axis_grid(n, vstar):
    """Midpoint nodes of [-vstar, vstar] and the discrete normalised
    Maxwellian exp(-v^2/2)/sqrt(2 pi) on them (sum M dv = 1)."""
    dv = 2.0 * vstar / n
    v = -vstar + (np.arange(n) + 0.5) * dv
    M = np.exp(-0.5 * v * v) / np.sqrt(2.0 * np.pi)
    return v, M / (np.sum(M) * dv), dv


class Grid3:
    def __init__(self, nvx, nvy, nvz, vstar):
        self.vx, self.Mx, self.dvx = axis_grid(nvx, vstar)
        self.vy, self.My, self.dvy = axis_grid(nvy, vstar)
        self.vz, self.Mz, self.dvz = axis_grid(nvz, vstar)
        self.dv3 = self.dvx * self.dvy * self.dvz
        self.M = self.Mx[:, None, None] * self.My[None, :, None] * self.Mz[None, None, :]
        self.VX = np.broadcast_to(self.vx[:, None, None], self.M.shape)
        # <vx^2 M> over the box: the diffusion coefficient of the limit
        self.m2 = float(np.sum(self.VX ** 2 * self.M) * self.dv3)


def _transport(g, E, vx, dx, dvx):
    """(vx d_x + E d_vx) g' at every interface, upwind, before the projection.
    g: [nx, nvx, nvy, nvz]; E: [nx]."""
    vp = np.maximum(vx, 0.0)[None, :, None, None]
    vm = np.minimum(vx, 0.0)[None, :, None, None]
    gm = np.roll(g, 1, axis=0)    # interface p-1
    gp = np.roll(g, -1, axis=0)   # interface p+1
    ax = (vp * (g - gm) + vm * (gp - g)) / dx
    Ep = np.maximum(E, 0.0)[:, None, None, None]
    Em = np.minimum(E, 0.0)[:, None, None, None]
    # G_{j+1/2} = E+ g_j + E- g_{j+1} between vx nodes j and j+1; zero at the faces
    G = np.zeros((g.shape[0], g.shape[1] + 1) + g.shape[2:])
    G[:, 1:-1] = Ep * g[:, :-1] + Em * g[:, 1:]
    return ax + (G[:, 1:] - G[:, :-1]) / dvx


def _cell_rule(N, Rc, eps_c, eta0, delta0, literal_r, prev=None):
    """Kinetic-cell rule of Section 2.2: a cell is kinetic if its remainder
    criterion exceeds eta0, or (when it was kinetic, or at the first step)
    if the perturbation norm of an adjacent interface exceeds delta0."""
    c = np.abs(Rc) if literal_r else eps_c * eps_c * np.abs(Rc)
    nmax = np.maximum(np.roll(N, 1), N)      # interfaces i-1/2 and i+1/2
    by_norm = nmax > delta0
    if prev is not None:
        by_norm = by_norm & (prev == 1)
    return ((c > eta0) | by_norm).astype(int)


def fine_propagate_3d(p, eps_iface, eps_cell, rho_in, g_in, nsteps, nvy, nvz):
    """nsteps steps of S^HMM in 1D3V from (rho_in [nx], g_in [nx, nvx, nvy,
    nvz] or None).  p: the 1D oracle's Params (nx, nv = nvx, Lx, vstar,
    rhobar, dt, eta0, delta0, flags).  Returns (rho, g, cell_mask,
    kinetic_iface_steps)."""
    nx, nvx = p.nx, p.nv
    hybrid, field = bool(p.flags & orc.HYBRID), bool(p.flags & orc.FIELD)
    literal_r = bool(p.flags & orc.LITERAL_R)
    dx, dt = p.Lx / nx, p.dt
    G3 = Grid3(nvx, nvy, nvz, p.vstar)
    eps = np.asarray(eps_iface, dtype=np.float64)
    e = np.exp(-dt / eps ** 2)
    a = -np.expm1(-dt / eps ** 2)
    rho = np.array(rho_in, dtype=np.float64)
    g = np.zeros((nx, nvx, nvy, nvz)) if g_in is None else np.array(g_in, dtype=np.float64)
    VXM = (G3.VX * G3.M)[None]

    def norms(g):
        return eps * np.sqrt(np.sum(g * g, axis=(1, 2, 3)) * G3.dv3)

    def field_of(rho):
        return orc.poisson(rho, p.rhobar, dx) if field else np.zeros(nx)

    kin = 0.0
    if hybrid:
        E = field_of(rho)
        Rc = orc.remainder(rho, E, p.rhobar, dx, field=field)
        cell = _cell_rule(norms(g), Rc, eps_cell, p.eta0, p.delta0, literal_r)
        ifc = cell | np.roll(cell, -1)            # interface p between cells p, p+1
        g[ifc == 0] = 0.0
    else:
        cell = np.ones(nx, dtype=int)
        ifc = np.ones(nx, dtype=int)
    for _ in range(nsteps):
        E = field_of(rho)
        J = orc.flux_J(rho, E, dx)
        if hybrid:
            Rc = orc.remainder(rho, E, p.rhobar, dx, field=field)
            ncell = _cell_rule(norms(g), Rc, eps_cell, p.eta0, p.delta0, literal_r, prev=cell)
            nifc = ncell | np.roll(ncell, -1)
        kin += float(np.sum(ifc))
        A = _transport(g, E, G3.vx, dx, G3.dvx)
        sA = np.sum(A, axis=(1, 2, 3)) * G3.dv3                       # <A>
        T = A - G3.M[None] * sA[:, None, None, None]                  # (I - Pi) A
        gn = (e[:, None, None, None] * g
              - a[:, None, None, None] * (eps[:, None, None, None] * T + VXM * J[:, None, None, None]))
        Phi = -np.sum(G3.VX[None] * gn, axis=(1, 2, 3)) * G3.dv3
        k = ifc == 1
        gn[~k] = 0.0
        Phi = np.where(k, Phi, G3.m2 * J)
        rho = rho + dt / dx * (Phi - np.roll(Phi, 1))
        if hybrid:
            gn[nifc == 0] = 0.0
            cell, ifc = ncell, nifc
        g = gn
    return rho, g, cell, kin


def separable(a, nvy, nvz, vstar):
    """g(x, vx) M(vy) M(vz) from the vx profile a [nx, nvx]."""
    _, My, _ = axis_grid(nvy, vstar)
    _, Mz, _ = axis_grid(nvz, vstar)
    return a[:, :, None, None] * My[None, None, :, None] * Mz[None, None, None, :]
