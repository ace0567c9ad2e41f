"""Host-side parts of bench.py: the one-GPU guard, the CPU baseline block
and the reading of the committed HBM counter summary (no GPU needed)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2511_13386_amd import workloads as wl  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_cpu_baseline_block_has_the_contract_fields():
    inst = wl.config2(nx=64, nv=32, N=4, T=1e-3)
    base, host = bench.cpu_baseline(inst, 0.3)
    assert set(base) == {"value", "unit", "cores", "kind", "sample"}
    assert base["kind"] == "oracle" and base["unit"] == "cell-updates/s"
    assert base["value"] > 0 and base["cores"] >= 1 and "fine steps" in base["sample"]
    assert host["single_thread_value"] > 0 and host["threads"] == base["cores"]
    c1 = host["config1_single_thread"]
    assert c1["value"] > 0 and c1["steps"] > 10000
    assert host["parareal_iteration_wall_s_extrapolated"] > 0


def test_accuracy_to_cost_uses_the_exact_leading_slices():
    """After k iterations slices 0..k equal the serial fine solution, so the
    distance of iterate k from it is read on slices 0..K of the last iterate;
    tolerance crossings report the first iteration below each tolerance."""
    N, nx, K = 6, 4, 3
    S = np.arange(1.0, (N + 1) * nx + 1.0).reshape(N + 1, nx)
    its = []
    for k in range(1, K + 1):
        U = S.copy()
        U[k + 1:] += 0.5 ** k  # slices beyond k not yet exact
        its.append(U)
    r = {"iterates": its, "iterations": K, "diverged": False, "errs": [0.3, 0.05, 0.002],
         "t_iter": [1.0, 2.0, 3.0], "sweep_ms": [100.0, 90.0, 80.0], "wall": 3.5}
    a = bench.accuracy_to_cost(r, N)
    scale = np.max(np.abs(its[-1][:K + 1]))
    assert a["distance_from_serial_fine"] == pytest.approx([0.5 / scale, 0.25 / scale, 0.0])
    assert a["serial_fine_slices_known"] == K
    assert a["to_successive_error_below"]["0.1"] == {"iterations": 2, "wall_s": 2.0}
    assert a["to_successive_error_below"]["0.001"] is None
    assert a["serial_fine_wall_s_estimate"] == pytest.approx(N * 0.1)


def test_traffic_is_read_only_for_the_current_sources(tmp_path, monkeypatch):
    """The committed FETCH_SIZE/WRITE_SIZE summary is used only when its
    recorded source hash is that of the kernels being run."""
    path = os.path.join(ROOT, "profiles", "k_fine_512x64_fp64_hbm_traffic.txt")
    if not os.path.exists(path):
        pytest.skip("no committed counter summary")
    lines = open(path).read().splitlines()
    assert any(l.startswith("kernel_sources_sha256:") for l in lines)
    assert len(bench.sources_sha256()) == 64
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_sha256", lambda: "a" * 64)
    os.makedirs(tmp_path / "profiles")
    target = tmp_path / "profiles" / "k_fine_512x64_fp64_hbm_traffic.txt"

    def with_sha(h):
        return "\n".join(f"kernel_sources_sha256: {h}" if l.startswith("kernel_sources_sha256:") else l
                         for l in lines) + "\n"
    target.write_text(with_sha("0" * 64))
    assert bench.measured_traffic("512x64_fp64") is None
    target.write_text(with_sha("a" * 64))
    t = bench.measured_traffic("512x64_fp64")
    assert t is not None and t > 0
    assert bench.measured_traffic("no_such_workload") is None


def test_batch_traffic_is_read_only_for_the_current_sources(tmp_path, monkeypatch):
    """The batch counter summary gives (counted bytes, algorithmic bytes) of
    the first sweep, only when its source hash is that of the kernels run;
    the counted bytes are the sum of its fetch and write lines."""
    path = os.path.join(ROOT, "profiles", "k_fine_batch256_fp32_hbm_traffic.txt")
    if not os.path.exists(path):
        pytest.skip("no committed batch counter summary")
    lines = open(path).read().splitlines()
    kv = dict(l.split(":", 1) for l in lines if ":" in l and not l.startswith("#"))
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_sha256", lambda: "b" * 64)
    os.makedirs(tmp_path / "profiles")
    target = tmp_path / "profiles" / "k_fine_batch256_fp32_hbm_traffic.txt"

    def with_sha(h):
        return "\n".join(f"kernel_sources_sha256: {h}" if l.startswith("kernel_sources_sha256:") else l
                         for l in lines) + "\n"
    target.write_text(with_sha("0" * 64))
    assert bench.measured_batch_traffic() is None
    target.write_text(with_sha("b" * 64))
    counted, alg = bench.measured_batch_traffic()
    assert counted == float(kv["first_sweep_fetch_bytes"]) + float(kv["first_sweep_write_bytes"])
    assert alg == float(kv["first_sweep_algorithmic_bytes"])
    assert abs(counted / alg - float(kv["counted_over_algorithmic"])) < 1e-3
