"""Batched corrections and the recorded (HIP graph) whole solve against the
ordinary call sequence.

Both paths run the same kernels on the same tables, so the comparisons are
bit for bit: slice values, per-iteration errors, iteration counts and
kinetic counters.  The graph is replayed several times with other device
work and synchronisations in between, and every replay is checked."""
import numpy as np
import pytest

from paper_2511_13386_amd import sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of

pytestmark = pytest.mark.gpu


def _descs(tol_third=0.0):
    """Four problems over several kernel classes and both coarse schemes."""
    out = []
    a = wl.small_hybrid(seed=3, nx=96, nv=32, N=5, T=5e-3, K=3)
    out.append(desc_of(a, start_mode=sth.START_CARRY))
    b = wl.small_hybrid(seed=4, nx=64, nv=16, N=4, T=0.02, K=4)
    x = wl.cell_centres(64)
    b.rho_in = 1.0 + 0.3 * np.cos(2 * np.pi * x)
    b.eps_iface = np.full(64, 0.1)
    b.eps_cell = np.full(64, 0.1)
    out.append(desc_of(b, precision=sth.FP32_BULK, start_mode=sth.START_LIFT, lift_order=1))
    c = wl.small_hybrid(seed=5, nx=200, nv=64, N=6, T=4e-3, K=5)
    x = wl.cell_centres(200)
    c.rho_in = 1.0 + 0.3 * np.cos(2 * np.pi * x) + 0.1 * np.sin(4 * np.pi * x)
    c.eps_iface = np.full(200, 1e-2)   # successive errors decrease monotonically here
    c.eps_cell = np.full(200, 1e-2)
    d = desc_of(c, start_mode=sth.START_CARRY)
    d.flags |= sth.COARSE_EXPLICIT
    d.tol = tol_third
    out.append(d)
    e = wl.small_hybrid(seed=6, nx=130, nv=128, N=3, T=2e-3, K=3)
    out.append(desc_of(e, precision=sth.FP32_BULK, start_mode=sth.START_CARRY))
    return out


def _eager(desc):
    p = sth.Problem(desc)
    errs = sth.parareal_solve(p, K=desc.k_max, tol=desc.tol)
    return p, errs


def test_batched_coarse_and_correction_equal_single():
    ds = _descs()
    single = [sth.Problem(d) for d in ds]
    batched = [sth.Problem(d) for d in ds]
    for q in single:
        sth.sth_coarse_sweep(q)
    sth.sth_coarse_sweep_batched(batched)
    for q1, q2 in zip(single, batched):
        assert np.array_equal(sth.sth_get_rho(q1), sth.sth_get_rho(q2))
    for it in range(2):
        sth.sth_fine_sweep_batched(single)
        e1 = [sth.sth_parareal_correct(q)[0] for q in single]
        sth.sth_fine_sweep_batched(batched)
        e2 = sth.sth_parareal_correct_batched(batched)
        assert e1 == e2, it
        for q1, q2 in zip(single, batched):
            assert np.array_equal(sth.sth_get_rho(q1), sth.sth_get_rho(q2))
            assert q1.info().k_done == q2.info().k_done == it + 1
    for q1, q2 in zip(single, batched):
        assert sth.sth_get_errors(q1) == sth.sth_get_errors(q2)
        q1.close()
        q2.close()


def test_batched_correction_rejects_bad_batches():
    ds = _descs()[:2]
    ps = [sth.Problem(d) for d in ds]
    for q in ps:
        sth.sth_coarse_sweep(q)
    with pytest.raises(sth.StHError):
        sth.sth_parareal_correct_batched(ps)  # no fine sweep yet
    sth.sth_fine_sweep_batched(ps)
    with pytest.raises(sth.StHError):
        sth.sth_parareal_correct_batched([ps[0], ps[0]])
    for q in ps:
        q.close()


def test_graph_replays_equal_eager_solves():
    import torch
    # a tolerance that stops the third problem after its third iteration
    probe, perr = _eager(_descs()[2])
    probe.close()
    assert perr[2] < perr[1]
    tol = float(np.sqrt(perr[1] * perr[2]))
    ds = _descs(tol_third=tol)
    ref = [_eager(d) for d in ds]
    ref_rho = [sth.sth_get_rho(p) for p, _ in ref]
    ref_kin = [p.info().kinetic_iface_steps for p, _ in ref]
    assert len(ref[2][1]) == 3 and len(ref[0][1]) == 3 and len(ref[1][1]) == 4

    probs = [sth.Problem(d) for d in ds]
    g = sth.Graph(probs)
    s = torch.cuda.Stream()
    other = sth.Problem(_descs()[0])
    for replay in range(3):
        g.launch(s)
        iters, last = g.wait(s)
        assert iters == [len(e) for _, e in ref], replay
        for q, (p, errs), r, kin, le in zip(probs, ref, ref_rho, ref_kin, last):
            assert np.array_equal(sth.sth_get_rho(q), r), replay
            assert sth.sth_get_errors(q) == errs, replay
            assert le == errs[-1]
            assert q.info().kinetic_iface_steps == kin, replay
        # other device work between replays
        sth.parareal_solve(other, K=1)
        z = torch.zeros(1 << 20, device="cuda")
        z += 1.0
        torch.cuda.synchronize()
    # after a replay the problems continue with ordinary calls
    q, (p, _) = probs[0], ref[0]
    for h in (q, p):
        sth.sth_fine_sweep_batched([h])
        sth.sth_parareal_correct(h)
    assert np.array_equal(sth.sth_get_rho(q), sth.sth_get_rho(p))
    g.close()
    other.close()
    for q in probs:
        q.close()
    for p, _ in ref:
        p.close()
