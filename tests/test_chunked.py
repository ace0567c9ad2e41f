"""Chunked fine sweeps (sth_fine_sweep_chunk) against whole sweeps.

A slice run in chunks of steps, suspended and resumed through its
checkpoint and slot, must give the same end state as the slice run in one
launch, bit for bit: every kernel form (resident rows in registers, rows
streamed, wide workgroups), both precisions, adaptation on and off, the
cell-wise update flag, chunk lengths from one step up."""
import numpy as np
import pytest

from paper_2511_13386_amd import sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of

pytestmark = pytest.mark.gpu

CASES = [
    # nx, nv, precision, hybrid, extra flags, chunk
    (96, 32, sth.FP64, True, 0, 7),            # resident, ragged segment
    (130, 64, sth.FP32_BULK, True, 0, 1),      # resident, one step per chunk
    (200, 128, sth.FP64, True, 0, 64),         # streamed
    (1100, 64, sth.FP32_BULK, False, 0, 37),   # streamed, wide workgroup, two slabs
    (1100, 16, sth.FP64, True, 0, 50),         # resident, three slabs
    (96, 32, sth.FP64, True, sth.LITERAL_FLUX, 13),
    # many short chunks in a row: the unit tables of successive calls must
    # not share host staging memory
    (512, 128, sth.FP32_BULK, True, 0, 10),
    (1024, 32, sth.FP32_BULK, True, 0, 16),
]


@pytest.mark.parametrize("nx,nv,prec,hybrid,flags,chunk", CASES)
def test_chunked_sweep_equals_whole_sweep(nx, nv, prec, hybrid, flags, chunk):
    inst = wl.small_hybrid(seed=7, nx=nx, nv=nv, N=4, T=2e-3, K=3)
    inst.hybrid = hybrid
    d = desc_of(inst, precision=prec, start_mode=sth.START_CARRY)
    d.flags |= flags
    # about 300 stable fine steps per slice
    probe = sth.Problem(d)
    d.T *= 300.0 / probe.info().steps_per_slice
    probe.close()
    whole, chunked = sth.Problem(d), sth.Problem(d)
    ns = whole.info().steps_per_slice
    assert 250 < ns < 350
    for q in (whole, chunked):
        sth.sth_coarse_sweep(q)
    for it in range(2):
        sth.sth_fine_sweep_batched([whole])
        calls = 0
        while True:
            calls += 1
            (done,) = sth.sth_fine_sweep_chunk([chunked], chunk)
            if done:
                break
            with pytest.raises(sth.StHError):
                sth.sth_fine_sweep_batched([chunked])  # a chunked sweep is in progress
        assert calls == -(-ns // chunk)
        for n in range(it + 1, inst.N + 1):
            assert np.array_equal(sth.sth_get_g(whole, n), sth.sth_get_g(chunked, n)), (it, n)
        e1 = sth.sth_parareal_correct(whole)[0]
        e2 = sth.sth_parareal_correct(chunked)[0]
        assert np.isfinite(e1) and e1 == e2
        assert np.array_equal(sth.sth_get_rho(whole), sth.sth_get_rho(chunked))
    assert whole.info().kinetic_iface_steps == chunked.info().kinetic_iface_steps
    whole.close()
    chunked.close()


@pytest.mark.parametrize("r,chunk", [(7, 256), (47, 100), (61, 256)])
def test_chunked_mostly_fluid_solves(r, chunk):
    """Requests of the serving workload with small constant eps (most
    segments fluid, so the resident form's pass skips them and their
    other-parity halos and projections must survive a suspension) and
    thousands of steps per slice: a chunked solve equals the whole-sweep
    solve bit for bit."""
    u = (wl.uniform_pm1(4242, 200)[r] + 1.0) * 0.5
    inst = wl.random_instance(5000 + r, N=32, T=(0.1 + 0.9 * u) * 1e-2)
    d = desc_of(inst, precision=sth.FP32_BULK, start_mode=sth.START_CARRY, K=2)
    d.lift_order = 1
    whole, chunked = sth.Problem(d), sth.Problem(d)
    assert whole.info().fine_resident == 1 and whole.info().steps_per_slice > 4 * chunk
    sth.parareal_solve(whole, K=2, fixed_iterations=True)
    sth.sth_coarse_sweep(chunked)
    for it in range(2):
        while not sth.sth_fine_sweep_chunk([chunked], chunk)[0]:
            pass
        sth.sth_parareal_correct(chunked)
    U = sth.sth_get_rho(chunked)
    assert np.all(np.isfinite(U))
    assert np.array_equal(U, sth.sth_get_rho(whole))
    whole.close()
    chunked.close()


def test_chunks_of_several_problems_in_one_call():
    """Problems of different classes and step counts advance together; each
    reports its own end."""
    a = desc_of(wl.small_hybrid(seed=8, nx=96, nv=32, N=3))
    b = desc_of(wl.small_hybrid(seed=9, nx=300, nv=64, N=2), precision=sth.FP32_BULK)
    for d, target in ((a, 120), (b, 50)):   # 120 and 50 stable steps per slice
        probe = sth.Problem(d)
        ns0 = probe.info().steps_per_slice
        probe.close()
        d.T *= target / ns0
        for _ in range(20):
            probe = sth.Problem(d)
            ns = probe.info().steps_per_slice
            probe.close()
            if ns == target:
                break
            d.T *= (target - 0.5) / ns if ns > target else (target + 0.5) / ns
        assert ns == target
    ref = [sth.Problem(a), sth.Problem(b)]
    ch = [sth.Problem(a), sth.Problem(b)]
    for q in ref + ch:
        sth.sth_coarse_sweep(q)
    sth.sth_fine_sweep_batched(ref)
    ends = []
    for t in range(3):
        ends.append(sth.sth_fine_sweep_chunk(ch, 50))
    # a problem whose sweep has ended waits for its correction
    assert ends == [[False, True], [False, True], [True, True]]
    for r, c in zip(ref, ch):
        sth.sth_parareal_correct(r)
        sth.sth_parareal_correct(c)
        assert np.array_equal(sth.sth_get_rho(r), sth.sth_get_rho(c))
    for q in ref + ch:
        q.close()
