"""Serving loop: admission bookkeeping (CPU) and continuous batching on the
GPU, where every served result equals the same solve alone, bit for bit."""
import numpy as np
import pytest

from paper_2511_13386_amd import serving, sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of, oracle_of, rel_err


def test_free_list_first_fit_and_coalescing():
    fl = serving.FreeList(10_000)
    assert fl.nbytes == 9984  # whole 256-byte blocks
    a = fl.alloc(1000)
    b = fl.alloc(300)
    c = fl.alloc(256)
    assert (a, b, c) == (0, 1024, 1536)
    assert fl.alloc(9000) is None
    fl.release(b, 300)
    assert fl.alloc(200) == 1024        # first fit reuses the hole
    fl.release(1024, 200)
    fl.release(a, 1000)
    fl.release(c, 256)
    assert fl.free == [[0, 9984]]       # everything merged back
    with pytest.raises(ValueError):
        fl.release(0, 256)              # double release is caught


def test_free_list_admission_order_under_pressure():
    fl = serving.FreeList(4096)
    blocks = [fl.alloc(1024) for _ in range(4)]
    assert blocks == [0, 1024, 2048, 3072]
    assert fl.alloc(1) is None
    fl.release(1024, 1024)
    fl.release(2048, 1024)
    assert fl.alloc(2048) == 1024       # adjacent holes coalesce


@pytest.mark.gpu
@pytest.mark.parametrize("chunk", [None, 97])
def test_served_results_equal_solves_alone(orc, chunk):
    """Six requests of different sizes and precisions arrive staggered and
    overlap on the device (an arena small enough that some must wait for
    memory); each served result equals its solve alone, and the oracle's
    parareal (Algorithm 1, carried starts): FP64 requests to 1e-11, FP32-bulk
    requests to 1e-5 or four times the floor of binary32 storage (the
    oracle's own solve with g' stored in binary32)."""
    torch = pytest.importorskip("torch")
    insts = [
        (wl.small_hybrid(seed=1, nx=96, nv=32, N=3, T=2e-3, K=2), sth.FP64),
        (wl.random_instance(11, N=4, T=1e-3, nx_choices=(128,), nv_choices=(64,)), sth.FP32_BULK),
        (wl.random_instance(12, N=3, T=1e-3, nx_choices=(256,), nv_choices=(32,)), sth.FP64),
        (wl.random_instance(13, N=2, T=1e-3, nx_choices=(512,), nv_choices=(128,)), sth.FP32_BULK),
        (wl.random_instance(14, N=4, T=1e-3, nx_choices=(128,), nv_choices=(32,)), sth.FP64),
        (wl.random_instance(15, N=3, T=1e-3, nx_choices=(1024,), nv_choices=(64,)), sth.FP32_BULK),
    ]
    descs = [desc_of(i, precision=p, K=2) for i, p in insts]
    sizes = [sth.sth_footprint_bytes(d) for d in descs]
    budget = sum(sorted(sizes)[-3:]) + 4096  # not all fit at once
    srv = serving.Server(budget, chunk_steps=chunk)
    reqs = [serving.Request(r, d, 0.002 * r, max_iters=2) for r, d in enumerate(descs)]
    res = srv.run(reqs)
    assert srv.ticks >= 3
    assert srv.arena.free_bytes == srv.arena.nbytes
    for r, d in zip(res, descs):
        p = sth.Problem(d)
        sth.parareal_solve(p, K=2, fixed_iterations=True)
        assert np.array_equal(r.rho, sth.sth_get_rho(p))
        assert r.latency > 0 and r.finished >= r.admitted >= 0
        p.close()
    torch.cuda.synchronize()
    if chunk is None:
        for r, (inst, prec) in zip(res, insts):
            po, ns, dtG = oracle_of(orc, inst)
            Uo = orc.parareal(po, inst.eps_iface, inst.eps_cell, inst.N, ns, dtG, 2, 0.0, inst.rho_in)[0]
            err = rel_err(r.rho, Uo)
            if prec == sth.FP64:
                print(f"request {r.rid}: FP64 served vs oracle {err:.2e}", flush=True)
                assert err < 1e-11
            else:
                q = type(po).from_buffer_copy(po)
                q.flags |= orc.STORE_F32
                floor = rel_err(orc.parareal(q, inst.eps_iface, inst.eps_cell, inst.N, ns, dtG, 2, 0.0,
                                             inst.rho_in)[0], Uo)
                print(f"request {r.rid}: FP32 bulk served vs oracle {err:.2e}, binary32-storage floor "
                      f"{floor:.2e}", flush=True)
                assert err < max(1e-5, 4.0 * floor)


@pytest.mark.gpu
def test_a_nonfinite_request_fails_alone():
    """A request whose densities overflow is retired as failed after its
    first correction; the requests served with it are unaffected."""
    torch = pytest.importorskip("torch")
    good = [desc_of(wl.small_hybrid(seed=21 + i, nx=96, nv=32, N=3, T=2e-3, K=2), K=2) for i in range(2)]
    inst = wl.small_hybrid(seed=23, nx=64, nv=32, N=3, T=2e-3, K=2)
    # a start perturbation whose fluxes overflow
    inst.g_in = 1e300 * np.sign(np.sin(np.arange(64 * 32) * 0.7)).reshape(64, 32)
    bad = desc_of(inst, K=2)
    descs = [good[0], bad, good[1]]
    srv = serving.Server(sum(sth.sth_footprint_bytes(d) for d in descs) + 4096, chunk_steps=64)
    res = srv.run([serving.Request(r, d, 0.0, max_iters=2) for r, d in enumerate(descs)])
    assert [r.ok for r in res] == [True, False, True]
    assert len(res[1].errors) == 1 and not np.isfinite(res[1].errors[0])
    for r, d in ((res[0], good[0]), (res[2], good[1])):
        p = sth.Problem(d)
        sth.parareal_solve(p, K=2, fixed_iterations=True)
        assert np.array_equal(r.rho, sth.sth_get_rho(p))
        p.close()
    torch.cuda.synchronize()
