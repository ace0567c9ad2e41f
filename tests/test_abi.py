"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and its host-only logic (sizes, validation) works without a
GPU.  No compute call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2511_13386_amd import sth
from paper_2511_13386_amd import workloads as wl

from helpers import desc_of

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sth.h")).read()
    return sorted(set(re.findall(r"\b(sth_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared() == sorted(sth.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = sth.lib()
    for name in _declared():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def _slot_elems(nx, nv):
    # one slice's state: rows [nv][ld] plus two projection rows, ld = nx
    # padded to the wavefront, plus the halo rows [2][2][ld/64][nv/2]
    ld = (nx + 63) // 64 * 64
    return ld * (nv + 2) + 2 * (ld // 64) * nv


def test_footprint_of_the_configs():
    d2 = desc_of(wl.config2())
    b2 = sth.sth_footprint_bytes(d2)
    # two (N+1)-slice state buffers dominate, then the (N+1) checkpoints of
    # chunked sweeps (7 arrays of nx doubles each)
    s2 = 2 * 65 * _slot_elems(512, 64) * 8 + 65 * 7 * 512 * 8
    assert s2 < b2 < s2 + (2 << 20)
    d3 = desc_of(wl.config3(), precision=sth.FP32_BULK)
    b3 = sth.sth_footprint_bytes(d3)
    s3 = 2 * 129 * _slot_elems(2048, 128) * 4 + 129 * 7 * 2048 * 8
    assert s3 < b3 < s3 + (10 << 20)


@pytest.mark.parametrize("field,value,code", [
    ("nx", 4, sth.STH_EINVAL), ("nx", 4096, sth.STH_EINVAL), ("nv", 48, sth.STH_EINVAL),
    ("n_slices", 0, sth.STH_EINVAL), ("lift_order", 4, sth.STH_EINVAL),
    ("cfl_theta", 1.5, sth.STH_EINVAL), ("precision", 7, sth.STH_EINVAL),
    ("flags", 64, sth.STH_EINVAL), ("start_mode", 3, sth.STH_EINVAL),
])
def test_validation_errors(field, value, code):
    d = desc_of(wl.small_hybrid())
    setattr(d, field, value)
    with pytest.raises(sth.StHError) as e:
        sth.sth_footprint_bytes(d)
    assert e.value.code == code
    assert sth.sth_last_error()


@pytest.mark.parametrize("precision", [sth.FP64, sth.FP32_BULK])
@pytest.mark.parametrize("nv", [16, 32, 64, 128])
def test_every_supported_shape_fits_one_workgroup(nv, precision):
    # the largest unit of each velocity grid and precision is accepted
    # (its LDS layout fits one gfx950 workgroup)
    for nx in (8, 100, 2048):
        d = desc_of(wl.small_hybrid(nx=nx, nv=nv), precision=precision)
        assert sth.sth_footprint_bytes(d) > 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sth, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sth, "_lib", None)
    with pytest.raises(ImportError):
        sth.lib()


def test_workload_generators_are_deterministic():
    a, b = wl.config2(seed=3), wl.config2(seed=3)
    assert np.array_equal(a.rho_in, b.rho_in)
    assert not np.array_equal(a.rho_in, wl.config2(seed=4).rho_in)
    x = wl.interfaces(512)
    e = wl.eps_tanh(x)
    lit = wl.eps_tanh_literal(x)
    mid = (x > 0.25) & (x < 0.75)
    assert np.max(np.abs(e[mid] - lit[mid])) < 1e-4
    assert abs(e[-1] - e[0]) < 0.2  # periodic continuation, no seam jump
    s = wl.splitmix64(0, 3)
    # published first outputs of SplitMix64 with seed 0
    assert [int(v) for v in s] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_data_without_a_stable_step_is_refused():
    """A density whose field overflows the stable-step bound is refused at
    creation (no device work), so no slice runs an unbounded step count."""
    import ctypes
    inst = wl.small_hybrid(seed=26, nx=64, nv=32, N=3)
    for scale, code, word in ((1e300, sth.STH_EINVAL, "stable"), (1e308, sth.STH_ENONFINITE, "overflows")):
        inst.rho_in = scale * (1.0 + 0.5 * np.cos(2 * np.pi * wl.cell_centres(64)))
        c, keep = desc_of(inst).to_c()
        h = ctypes.c_void_p()
        rc = sth.lib().sth_create(ctypes.byref(c), None, 0, ctypes.byref(h))
        assert rc == code and not h.value
        assert word in sth.sth_last_error()
