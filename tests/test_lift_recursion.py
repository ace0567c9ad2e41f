"""Independent pin of the oracle's lifting L^L at orders 2 and 3.

The lifting of Definition 1 (Section 3.3) is g = sum_l eps^l h^(l) with the
h^(l) of the Chapman-Enskog identification (eq. Identification, Section
2.1): h1 = -T(rho M), h2 = -d_t(rho M) - T h1, h3 = -d_t h1 - T h2, where
T f = v d_x f + E d_v f.  Here sympy carries that recursion out on symbolic
fields rho(t, x), E(t, x) with the drift-diffusion closures the method rests
on (problem P^0: d_t rho = d_x J, J = d_x rho - E rho; the time derivative of
the Gauss law with the zero-mean gauge: d_t E = J - mean J), then evaluates
h1, h2, h3 for a smooth two-mode density with the field on.  The oracle's
hand-written terms are compared with it at the interfaces: h2 from the L = 2
and L = 1 liftings, h3 from L = 3 and L = 2.  The only differences left are
the second-order discretisation of the interface flux, the interface average
of rho and the Gauss-law field (O(dx^2)); the test checks that the
difference is small and shrinks fourfold when dx halves.  Each term of h3 is
large compared with the tolerance, so a dropped term or a wrong sign or
coefficient in any of them fails the comparison.
"""
import math

import numpy as np
import pytest
import sympy as sp

LX = 2.0 * math.pi          # the paper's x* = 2 pi
A1, A2 = 0.5, 0.3           # rho = 1 + A1 cos x + A2 sin 2x


def _recursion():
    """h1, h2, h3 (paper's f-units: f = rho M + sum eps^l h^(l)) as numpy
    functions of (x, v), from the identification recursion and closures."""
    t, x, v, mJ = sp.symbols("t x v mJ", real=True)
    rho = sp.Function("rho")(t, x)
    E = sp.Function("E")(t, x)
    M = sp.exp(-v ** 2 / 2) / sp.sqrt(2 * sp.pi)

    def T(f):
        return v * sp.diff(f, x) + E * sp.diff(f, v)

    h1 = -T(rho * M)
    h2 = -sp.diff(rho * M, t) - T(h1)
    h3 = -sp.diff(h1, t) - T(h2)

    # closures: d_t rho = d_x J, d_t E = J - mean J (and their x-derivatives)
    J = sp.diff(rho, x) - E * rho
    dt_of = {rho: sp.diff(J, x), E: J - mJ}

    def close(expr):
        reps = {}
        for d in expr.atoms(sp.Derivative):
            counts = dict(d.variable_count)
            if t not in counts:
                continue
            assert counts[t] == 1, d
            rep = dt_of[d.expr]
            if counts.get(x, 0):
                rep = sp.diff(rep, x, counts[x])
            reps[d] = rep
        return expr.xreplace(reps)

    h2c, h3c = close(sp.expand(h2)), close(sp.expand(h3))
    for h in (h2c, h3c):
        assert not any(t in dict(d.variable_count) for d in h.atoms(sp.Derivative))

    # the test density and its zero-mean Gauss-law field (d_x E = rho - mean rho)
    X = sp.Symbol("X", real=True)
    rho_c = 1 + sp.Rational(1, 2) * sp.cos(X) + sp.Rational(3, 10) * sp.sin(2 * X)
    E_c = sp.Rational(1, 2) * sp.sin(X) - sp.Rational(3, 20) * sp.cos(2 * X)
    assert sp.simplify(sp.diff(E_c, X) - (rho_c - 1)) == 0
    assert sp.integrate(E_c, (X, 0, 2 * sp.pi)) == 0
    J_c = sp.diff(rho_c, X) - E_c * rho_c
    mJ_c = sp.integrate(sp.expand(J_c), (X, 0, 2 * sp.pi)) / (2 * sp.pi)

    def concrete(expr):
        e = expr.subs({rho: rho_c.subs(X, x), E: E_c.subs(X, x)}).doit()
        return sp.lambdify((x, v), e.subs(mJ, mJ_c), "numpy")

    return concrete(h1), concrete(h2c), concrete(h3c)


@pytest.fixture(scope="module")
def recursion():
    return _recursion()


def _oracle_terms(orc, nx, nv):
    """h1, h2, h3 of the oracle's lifting at the interfaces x_p = (p+1) dx."""
    dx = LX / nx
    xc = (np.arange(nx) + 0.5) * dx
    rho = 1.0 + A1 * np.cos(xc) + A2 * np.sin(2.0 * xc)
    eps = np.ones(nx)
    g = {}
    for L in (1, 2, 3):
        p = orc.params(nx, nv, Lx=LX, rhobar=float(np.mean(rho)), flags=orc.FIELD, lift_order=L)
        g[L] = orc.lift(p, eps, rho)
    xp = (np.arange(nx) + 1.0) * dx
    return xp, g[1], g[2] - g[1], g[3] - g[2]


def test_lift_orders_follow_the_chapman_enskog_recursion(orc, recursion):
    f1, f2, f3 = recursion
    nv = 32
    v, _, _ = orc.velocity_grid(nv)
    errs = {1: [], 2: [], 3: []}
    for nx in (512, 1024, 2048):
        xp, o1, o2, o3 = _oracle_terms(orc, nx, nv)
        X, V = np.meshgrid(xp, v, indexing="ij")
        for L, o, f in ((1, o1, f1), (2, o2, f2), (3, o3, f3)):
            ref = f(X, V)
            errs[L].append(np.max(np.abs(o - ref)) / np.max(np.abs(ref)))
    for L in (1, 2, 3):
        e = errs[L]
        # second order in dx: the interface flux, density average and field
        assert e[-1] < 2e-5, (L, e)
        assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, (L, e)


def test_every_h3_term_is_visible(orc, recursion):
    """The terms of h3 (d_t J with its closure parts, the d_x K term and the
    field term) are each far larger than the comparison's tolerance, so the
    comparison above would see any one of them dropped or flipped."""
    nx, nv = 2048, 32
    dx = LX / nx
    v, M, m2 = orc.velocity_grid(nv)
    xc = (np.arange(nx) + 0.5) * dx
    xp = (np.arange(nx) + 1.0) * dx
    rho = 1.0 + A1 * np.cos(xc) + A2 * np.sin(2.0 * xc)
    E = 0.5 * np.sin(xp) - 0.15 * np.cos(2.0 * xp)
    J = (-0.5 * np.sin(xp) + 0.6 * np.cos(2.0 * xp)) - E * (1.0 + A1 * np.cos(xp) + A2 * np.sin(2.0 * xp))
    ref = np.max(np.abs(recursion[2](*np.meshgrid(xp, v, indexing="ij"))))
    vM = np.abs(v * M)
    w = v * v - m2
    # magnitudes of the pieces at their largest
    K = np.gradient(J, dx) - E * J
    pieces = {
        "d2J": np.max(np.abs(np.gradient(np.gradient(J, dx), dx))) * np.max(vM),
        "(J - mean J) rho~": np.max(np.abs((J - J.mean()) * rho)) * np.max(vM),
        "E d1J": np.max(np.abs(E * np.gradient(J, dx))) * np.max(vM),
        "(v^2 - m2) d1K": np.max(np.abs(np.gradient(K, dx))) * np.max(np.abs(w * v * M)),
        "(2 + m2 - v^2) E K": np.max(np.abs(E * K)) * np.max(np.abs((2 + m2 - v * v) * v * M)),
    }
    for name, mag in pieces.items():
        assert mag / ref > 0.05, (name, mag / ref)
