"""Config 3 at its parity horizon (2048 x 128, 128 slices, T = 1/64: 13,747
fine steps per slice) against the FP64 oracle (OpenMP over slices).  The
oracle needs a few minutes on 16 cores, so these tests run only when
STH_LONG_PARITY=1 (they print their progress).

At this size the two FP64 implementations take some 3.6e9 threshold
decisions per iteration; the oracle sums sequentially and the kernels in
trees and pairs, so a criterion value within rounding of its threshold can
go either way, and the hybrid scheme is not continuous in those decisions.
The whole parareal iteration is therefore compared and reported; parity is
asserted slice by slice, with the number of (step, cell) status differences
counted and the oracle's status history imposed where they differ."""
import os
import threading
import time

import numpy as np
import pytest

from paper_2511_13386_amd import sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of, oracle_of, rel_err

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("STH_LONG_PARITY") != "1",
                                 reason="minutes of oracle time; set STH_LONG_PARITY=1")]

RHO64, G64 = 1e-12, 1e-10
# FP32 bulk against the oracle run from the same start rounded to FP32 (the
# slice map amplifies high-frequency start differences about a thousandfold,
# so the rounding of a lifted start is an input difference, not the FP32
# arithmetic of the slice)
RHO32, G32 = 1e-5, 1e-3


def _wait(threads, t0, what):
    for th in threads:
        while th.is_alive():
            th.join(30.0)
            print(f"{what}: {time.time() - t0:.0f} s", flush=True)


def test_config3_one_iteration_reported(orc):
    """One parareal iteration of the whole problem: mass exact in both
    precisions, the kinetic work within 1e-6 (FP64) and 1e-5 (FP32 bulk) and
    the successive error within 1e-5 and 1e-4 of the oracle's.  The slice
    values are reported as a number, not asserted: from slice 2 on the starts
    are liftings of coarse values that differ from the oracle's by rounding,
    and the lifting (a third derivative at dx = 1/2048) and the slice map
    amplify that; slice parity from identical starts, with the oracle's
    status history imposed where decisions differ, is asserted in
    test_config3_slices_with_status_histories and, for three slices in the
    default run, in test_config_parity.py."""
    inst = wl.config3(T=1.0 / 64)
    K = 1
    po, ns, dtG = oracle_of(orc, inst, lift_order=1)
    assert ns == 13747
    res = {}
    th = threading.Thread(target=lambda: res.setdefault(
        "oracle", orc.parareal(po, inst.eps_iface, inst.eps_cell, inst.N, ns, dtG, K, 0.0, inst.rho_in)))
    t0 = time.time()
    th.start()
    gpu = {}
    for prec in (sth.FP64, sth.FP32_BULK):
        p = sth.Problem(desc_of(inst, precision=prec, K=K, lift_order=1))
        errs = sth.parareal_solve(p, K=K, fixed_iterations=True)
        gpu[prec] = (sth.sth_get_rho(p), errs, p.info().kinetic_iface_steps)
        p.close()
    _wait([th], t0, "oracle parareal")
    Uo, erro, it, kin = res["oracle"]
    m0 = np.sum(inst.rho_in)
    U64, e64, k64 = gpu[sth.FP64]
    U32, e32, k32 = gpu[sth.FP32_BULK]
    print(f"config 3, T = 1/64, one iteration: FP64 rho {rel_err(U64, Uo):.2e}, FP32 bulk rho "
          f"{rel_err(U32, Uo):.2e}; kinetic interface-steps oracle {kin:.0f}, FP64 {k64:.0f}, "
          f"FP32 {k32:.0f}; error oracle {erro[0]:.9e}, FP64 {e64[0]:.9e}, FP32 {e32[0]:.9e}", flush=True)
    per = np.max(np.abs(U64 - Uo), axis=1) / np.max(np.abs(Uo))
    first = int(np.argmax(per > 1e-10))
    print(f"FP64 slice values: {int(np.sum(per > 1e-10))} of {inst.N + 1} differ by more than 1e-10, "
          f"the first at slice {first} ({per[first]:.1e}), those before it by at most "
          f"{np.max(per[:first]) if first else 0.0:.1e}", flush=True)
    assert abs(k64 - kin) < 1e-6 * kin and abs(k32 - kin) < 1e-5 * kin
    assert abs(e64[0] - erro[0]) < 1e-5 * erro[0] and abs(e32[0] - erro[0]) < 1e-4 * erro[0]
    assert abs(np.max(np.abs(U64[1] - Uo[1]))) < RHO64 * np.max(np.abs(Uo[1]))
    for U in (U64, U32):
        assert np.max(np.abs(U.sum(axis=1) - m0)) < 1e-12 * m0


def test_config3_slices_with_status_histories(orc):
    """Nine slices of the first sweep (the coarse-guess densities with their
    lifted perturbations as starts, 13,747 steps each): the GPU's status
    history against the oracle's, and with the oracle's imposed the slice
    ends to the FP64 and FP32-bulk tolerances."""
    inst = wl.config3(T=1.0 / 64)
    po, ns, dtG = oracle_of(orc, inst, lift_order=1)
    starts = [np.array(inst.rho_in, dtype=np.float64)]
    for _ in range(inst.N - 1):
        starts.append(orc.coarse_step(po, dtG, starts[-1]))
    sample = [0, 1] + list(range(inst.N // 8, inst.N, inst.N // 8))
    res = {}

    def run(n):
        g0 = None if n == 0 else orc.lift(po, inst.eps_iface, starts[n])
        res[n] = (g0,) + tuple(orc.fine_propagate_masks(po, inst.eps_iface, inst.eps_cell, starts[n], g0, ns))
        if g0 is not None:
            g032 = g0.astype(np.float32).astype(np.float64)
            res[(n, 32)] = (g032,) + tuple(orc.fine_propagate_masks(po, inst.eps_iface, inst.eps_cell,
                                                                    starts[n], g032, ns))

    t0 = time.time()
    threads = [threading.Thread(target=run, args=(n,)) for n in sample]
    for th in threads:
        th.start()
    _wait(threads, t0, "oracle slices")
    p64 = sth.Problem(desc_of(inst, precision=sth.FP64, lift_order=1))
    p32 = sth.Problem(desc_of(inst, precision=sth.FP32_BULK, lift_order=1))
    # the coarse guess itself: implicit solves with alpha = m2 dtG/dx^2 ~ 500
    sth.sth_coarse_sweep(p64)
    coarse = sth.sth_get_rho(p64)[:inst.N]
    print(f"coarse guess against the oracle's: {rel_err(coarse, np.array(starts)):.1e}", flush=True)
    assert rel_err(coarse, np.array(starts)) < 1e-8
    total = 0
    for n in sample:
        g0, ro, go, mo, st, ho = res[n]
        r64, g64, _, k64, h64 = sth.sth_fine_run_masks(p64, starts[n], g0, ns)
        diff = int(np.sum(h64 != ho))
        total += diff
        g32s, ro32, go32, _, _, ho32 = res[(n, 32)] if n > 0 else res[n]
        r32, g32, _, _, h32 = sth.sth_fine_run_masks(p32, starts[n], g32s, ns)
        print(f"slice {n + 1}: FP64 {diff} and FP32 bulk {int(np.sum(h32 != ho32))} of {ho.size} (step, cell) "
              f"states differ from the oracle's; rho {rel_err(r64, ro):.1e} / {rel_err(r32, ro32):.1e}",
              flush=True)
        if diff == 0:
            assert k64 == st["kinetic_iface_steps"]
        else:
            r64, g64, _, k64, _ = sth.sth_fine_run_masks(p64, starts[n], g0, ns, replay=ho)
        assert rel_err(r64, ro) < RHO64 and rel_err(g64, go) < G64
        r32, g32, _, _, _ = sth.sth_fine_run_masks(p32, starts[n], g32s, ns, replay=ho32)
        print(f"slice {n + 1}, FP32 bulk with the oracle's history: rho {rel_err(r32, ro32):.1e}, "
              f"g' {rel_err(g32, go32):.1e}", flush=True)
        assert rel_err(r32, ro32) < RHO32 and rel_err(g32, go32) < G32
    p64.close()
    p32.close()
    print(f"FP64: {total} differing (step, cell) states over {len(sample)} slices", flush=True)
