"""The allocation-free single-slice run (sth_fine_run_noalloc, static
device workspace) against the allocating one (sth_fine_run) through the
C-ABI: the same kernel on the same inputs gives the same densities,
perturbation, cell status and kinetic count bit for bit, on calls in a
row that leave different contents in the shared workspace (the second
smaller than the first), and a run beyond the workspace is refused."""
import numpy as np
import pytest

from paper_2511_13386_amd import sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of

pytestmark = pytest.mark.gpu


def _same_as_fine_run(p, rho, g0, n, want_g=True):
    ra, ga, ma, ka = sth.sth_fine_run(p, rho, g0, n)
    rb, gb, mb, kb = sth.sth_fine_run_noalloc(p, rho, g0, n, want_g=want_g)
    assert np.array_equal(ra, rb)
    if want_g:
        assert np.array_equal(ga, gb)
    assert np.array_equal(ma, mb) and ka == kb
    return ra, ka


def test_noalloc_run_equals_fine_run_on_consecutive_calls():
    # first call: hybrid 512 x 64 FP64 (the resident form) from a start perturbation
    i1 = wl.small_hybrid(seed=5, nx=512, nv=64, N=2, T=2e-3)
    p1 = sth.Problem(desc_of(i1, precision=sth.FP64))
    rng = np.random.default_rng(11)
    g0 = 1e-3 * rng.standard_normal((i1.nx, i1.nv))
    r1, k1 = _same_as_fine_run(p1, i1.rho_in, g0, 1500)
    assert k1 > 0 and np.all(np.isfinite(r1))
    # second call, smaller: 96 x 32 FP32 bulk (a ragged wavefront segment), g' = 0
    i2 = wl.small_hybrid(seed=6, nx=96, nv=32, N=2, T=2e-3)
    p2 = sth.Problem(desc_of(i2, precision=sth.FP32_BULK))
    _same_as_fine_run(p2, i2.rho_in, None, 800)
    # third: the first problem again without its perturbation output, then zero steps
    _same_as_fine_run(p1, i1.rho_in, g0, 700, want_g=False)
    _same_as_fine_run(p1, i1.rho_in, None, 0)
    p1.close()
    p2.close()


def test_noalloc_refuses_runs_beyond_its_workspace():
    inst = wl.config2(nx=2048, nv=128, N=2, T=1e-4)
    p = sth.Problem(desc_of(inst, precision=sth.FP64))
    with pytest.raises(sth.StHError) as e:
        sth.sth_fine_run_noalloc(p, inst.rho_in, None, 1)
    assert e.value.code == sth.STH_EINVAL and "2 MiB" in str(e.value)
    p.close()
