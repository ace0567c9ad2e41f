"""Edge cases of the fine propagator and the parareal loop on the GPU, each
against the FP64 oracle on the same inputs: the smallest grid (8 cells, one
partial wavefront, stencils wider than half the torus), the largest with a
ragged last wavefront (2047 cells), zero steps, the exact equilibrium,
eps = 1 (no stiffness) and eps = 1e-7 (the asymptotic limit), one slice,
and the smallest velocity grid."""
import numpy as np
import pytest

from paper_2511_13386_amd import sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of, oracle_of, rel_err

pytestmark = pytest.mark.gpu

RHO64, G64 = 1e-12, 1e-10
RHO32, G32 = 2e-6, 2e-4


def _pair(orc, inst, steps, precision=sth.FP64):
    p = sth.Problem(desc_of(inst, precision=precision))
    po, ns, _ = oracle_of(orc, inst)
    assert p.info().steps_per_slice == ns
    out = sth.sth_fine_run(p, inst.rho_in, inst.g_in, steps)
    p.close()
    ref = orc.fine_propagate(po, inst.eps_iface, inst.eps_cell, inst.rho_in, inst.g_in, steps)
    return out, ref


def _check(out, ref, precision=sth.FP64):
    (rg, gg, mg, kg), (ro, go, mo, st) = out, ref
    tr, tg = (RHO64, G64) if precision == sth.FP64 else (RHO32, G32)
    assert rel_err(rg, ro) < tr
    if np.any(go):
        assert rel_err(gg, go) < tg
    else:
        assert not np.any(gg)
    if precision == sth.FP64:
        assert np.array_equal(mg, mo) and kg == st["kinetic_iface_steps"]


@pytest.mark.parametrize("nx,nv", [(8, 16), (8, 128), (13, 32)])
@pytest.mark.parametrize("hybrid", [False, True])
def test_smallest_grids(orc, nx, nv, hybrid):
    inst = wl.small_hybrid(nx=nx, nv=nv)
    inst.hybrid = hybrid
    _check(*_pair(orc, inst, 400))


@pytest.mark.parametrize("nx,nv", [(2047, 128), (2048, 16), (2048, 32), (2040, 64)])
@pytest.mark.parametrize("precision", [sth.FP64, sth.FP32_BULK])
def test_largest_grids(orc, nx, nv, precision):
    """The largest grids in every velocity class (resident rows with four
    interfaces per thread at nv = 16, wide streamed workgroups, ragged last
    wavefronts)."""
    inst = wl.config2(nx=nx, nv=nv, N=4, T=1e-3)
    _check(*_pair(orc, inst, 60, precision), precision)


@pytest.mark.parametrize("hybrid", [False, True])
def test_zero_steps_return_the_start_after_the_status_rule(orc, hybrid):
    inst = wl.small_hybrid(nx=96, nv=32)
    inst.hybrid = hybrid
    rng = np.random.default_rng(3)
    inst.g_in = 1e-2 * rng.standard_normal((inst.nx, inst.nv))
    (rg, gg, mg, kg), (ro, go, mo, st) = _pair(orc, inst, 0)
    assert np.array_equal(rg, inst.rho_in) and np.array_equal(ro, inst.rho_in)
    assert np.array_equal(mg, mo) and kg == 0 == st["kinetic_iface_steps"]
    assert rel_err(gg, go) < 1e-15     # the start state, zeroed where fluid


@pytest.mark.parametrize("precision", [sth.FP64, sth.FP32_BULK])
@pytest.mark.parametrize("hybrid", [False, True])
def test_equilibrium_is_bitwise_stationary(orc, precision, hybrid):
    nx, nv = 200, 64
    inst = wl.small_hybrid(nx=nx, nv=nv)
    inst.rho_in = np.full(nx, 1.25)
    inst.hybrid = hybrid
    p = sth.Problem(desc_of(inst, precision=precision))
    rg, gg, mg, kg = sth.sth_fine_run(p, inst.rho_in, None, 500)
    p.close()
    assert np.array_equal(rg, inst.rho_in) and not np.any(gg)
    if hybrid:
        assert not np.any(mg) and kg == 0     # nothing to resolve kinetically


@pytest.mark.parametrize("eps,steps", [(1.0, 2000), (1e-7, 2000)])
def test_extreme_eps(orc, eps, steps):
    inst = wl.small_hybrid(nx=96, nv=32)
    inst.eps_iface = np.full(inst.nx, eps)
    inst.eps_cell = np.full(inst.nx, eps)
    _check(*_pair(orc, inst, steps))


def test_one_slice_parareal_is_the_fine_solve(orc):
    inst = wl.small_hybrid(nx=96, nv=32, N=1, T=1e-3, K=1)
    p = sth.Problem(desc_of(inst, lift_order=1))
    errs = sth.parareal_solve(p, K=1, fixed_iterations=True)
    U = sth.sth_get_rho(p)
    ns = p.info().steps_per_slice
    p.close()
    po, ns_o, _ = oracle_of(orc, inst, lift_order=1)
    assert ns == ns_o
    ro, _, _, _ = orc.fine_propagate(po, inst.eps_iface, inst.eps_cell, inst.rho_in, None, ns)
    assert len(errs) == 1
    assert rel_err(U[1], ro) < RHO64 and np.array_equal(U[0], inst.rho_in)
