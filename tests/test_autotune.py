"""Launch configurations of the fine kernel and the autotuner.

CPU: the candidate list, validation and the per-class table are host logic.
GPU: every configuration the tuner may pick is checked against the oracle
(and, within one row form, against the other workgroup sizes bit for bit),
and a tuning pass sets its winner."""
import numpy as np
import pytest

from paper_2511_13386_amd import autotune
from paper_2511_13386_amd import sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of, oracle_of, rel_err


@pytest.fixture
def clean_table():
    touched = []
    yield touched
    for prec, nx, nv in touched:
        sth.sth_set_fine_config(prec, nx, nv, None)


@pytest.mark.parametrize("prec", [sth.FP64, sth.FP32_BULK])
@pytest.mark.parametrize("nx", [8, 64, 96, 200, 300, 512, 1100, 2048])
@pytest.mark.parametrize("nv", [16, 32, 64, 128])
def test_candidates_are_supported_and_include_the_default(prec, nx, nv):
    cands = sth.sth_fine_config_candidates(prec, nx, nv)
    assert cands and len(set(cands)) == len(cands)
    assert sth.sth_get_fine_config(prec, nx, nv) in cands
    nxr = (nx + 63) // 64 * 64
    wide_ok = prec == sth.FP32_BULK or nv == 32
    for block, resident in cands:
        assert block % 64 == 0 and 64 <= block <= nxr
        assert block <= (1024 if (wide_ok and not resident) else 512)
        assert -(-nx // block) <= (2 if block > 512 else 4)
        assert resident in (0, 1)
    # the streamed form exists for every workgroup size
    blocks = {b for b, _ in cands}
    assert all((b, 0) in cands for b in blocks)


def test_set_get_reset_and_validation(clean_table):
    prec, nx, nv = sth.FP32_BULK, 512, 32
    clean_table.append((prec, nx, nv))
    default = sth.sth_get_fine_config(prec, nx, nv)
    assert default == (512, 1)
    sth.sth_set_fine_config(prec, nx, nv, (128, 0))
    assert sth.sth_get_fine_config(prec, nx, nv) == (128, 0)
    # the class is nx rounded up to 64: every member sees the setting
    assert sth.sth_get_fine_config(prec, 449, nv) == (128, 0)
    assert sth.sth_get_fine_config(prec, 448, nv) == (448, 1)   # another class
    sth.sth_set_fine_config(prec, nx, nv, None)
    assert sth.sth_get_fine_config(prec, nx, nv) == default
    with pytest.raises(sth.StHError):
        sth.sth_set_fine_config(sth.FP64, 2048, 32, (64, 0))     # 32 interfaces per thread
    with pytest.raises(sth.StHError):
        sth.sth_set_fine_config(sth.FP64, 512, 128, (512, 1))    # rows do not fit registers
    with pytest.raises(sth.StHError):
        sth.sth_set_fine_config(sth.FP64, 512, 32, (100, 0))     # not a wavefront multiple
    with pytest.raises(sth.StHError):
        sth.sth_set_fine_config(sth.FP64, 96, 32, (256, 0))      # larger than nx rounded up
    with pytest.raises(sth.StHError):
        sth.sth_set_fine_config(sth.FP64, 2048, 64, (1024, 0))   # no wide FP64 kernel for nv = 64
    with pytest.raises(sth.StHError):
        sth.sth_set_fine_config(sth.FP32_BULK, 2048, 64, (1024, 1))  # wide workgroups stream rows
    with pytest.raises(sth.StHError):
        sth.sth_set_fine_config(sth.FP32_BULK, 2048, 64, (704, 0))   # 3 interfaces per thread
    sth.sth_set_fine_config(sth.FP32_BULK, 2048, 64, (1024, 0))
    clean_table.append((sth.FP32_BULK, 2048, 64))
    assert sth.sth_get_fine_config(sth.FP32_BULK, 2048, 64) == (1024, 0)


def test_classes_and_saved_results_round_trip(tmp_path, clean_table):
    descs = [desc_of(wl.small_hybrid(nx=nx, nv=nv, N=n), precision=p)
             for nx, nv, n, p in [(96, 32, 4, sth.FP64), (100, 32, 3, sth.FP64),
                                  (96, 32, 2, sth.FP32_BULK), (1100, 128, 5, sth.FP32_BULK)]]
    keys = [autotune.class_of(d) for d in descs]
    assert keys[0] == keys[1] == (sth.FP64, 128, 32)
    assert keys[2] == (sth.FP32_BULK, 128, 32) and keys[3] == (sth.FP32_BULK, 1152, 128)
    res = {keys[0]: autotune.ClassResult(keys[0], 7, {(128, 1): 2.0, (64, 0): 1.0}, (64, 0), (128, 1))}
    path = str(tmp_path / "tuned.json")
    autotune.save(res, path)
    clean_table.append(keys[0])
    assert autotune.load(path) == [keys[0]]
    assert sth.sth_get_fine_config(sth.FP64, 100, 32) == (64, 0)
    assert res[keys[0]].speedup_over_default == 2.0
    autotune.reset(res)
    assert sth.sth_get_fine_config(sth.FP64, 100, 32) == (128, 1)


@pytest.mark.gpu
@pytest.mark.parametrize("nx,nv,prec,steps", [
    (200, 32, sth.FP64, 400),        # 1, 2 and 4 interfaces per thread, both forms
    (300, 64, sth.FP32_BULK, 400),   # workgroups of 3 and 5 wavefronts
    (1100, 16, sth.FP64, 150),       # 3 and 4 interfaces per thread, resident
    (512, 128, sth.FP32_BULK, 150),  # streamed with 1..4 interfaces per thread
    (1100, 64, sth.FP32_BULK, 150),  # wide workgroups (576 and 1024 threads)
    (1100, 32, sth.FP64, 150),       # wide FP64 workgroups
])
def test_every_candidate_matches_the_oracle(orc, clean_table, nx, nv, prec, steps):
    inst = wl.small_hybrid(nx=nx, nv=nv)
    po, ns, _ = oracle_of(orc, inst)
    ro, go, mo, st = orc.fine_propagate(po, inst.eps_iface, inst.eps_cell, inst.rho_in, None, steps)
    clean_table.append((prec, nx, nv))
    ref = {}
    tol_r, tol_g = (1e-12, 1e-10) if prec == sth.FP64 else (2e-6, 2e-4)
    for cfg in sth.sth_fine_config_candidates(prec, nx, nv):
        sth.sth_set_fine_config(prec, nx, nv, cfg)
        p = sth.Problem(desc_of(inst, precision=prec))
        info = p.info()
        assert (info.fine_block, info.fine_resident) == cfg
        out = sth.sth_fine_run(p, inst.rho_in, None, steps)
        p.close()
        rg, gg, mg, kg = out
        assert rel_err(rg, ro) < tol_r, cfg
        assert rel_err(gg, go) < tol_g, cfg
        if prec == sth.FP64:
            assert np.array_equal(mg, mo), cfg
            assert kg == st["kinetic_iface_steps"], cfg
        # within a row form the workgroup size changes neither the
        # arithmetic nor its order
        r0 = ref.setdefault(cfg[1], out)
        assert np.array_equal(rg, r0[0]) and np.array_equal(gg, r0[1]), cfg


@pytest.mark.gpu
def test_tuning_pass_sets_the_fastest(clean_table):
    d = desc_of(wl.small_hybrid(nx=200, nv=32, N=64), precision=sth.FP32_BULK)
    res = autotune.autotune([d], steps=50, repeats=2)
    (key, r), = res.items()
    clean_table.append(key)
    assert key == (sth.FP32_BULK, 256, 32) and r.units == 64
    assert set(r.timings_ms) == set(sth.sth_fine_config_candidates(*key))
    assert all(t > 0 for t in r.timings_ms.values())
    assert r.best == min(r.timings_ms, key=r.timings_ms.get)
    assert sth.sth_get_fine_config(sth.FP32_BULK, 200, 32) == r.best
