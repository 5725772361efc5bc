"""CPU: the benchmark's contract (no GPU needed).

- `bench.py --gpus N` with N > 1 exits with a message and a non-zero status (one GPU only);
- the HBM traffic figure comes from the committed counter summary only while the kernel's
  source file is unchanged (its hash matches the summary), and is absent otherwise;
- the oracle's one-thread rate is measured over operator rows and restores the thread count.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_traffic_only_for_the_profiled_source():
    for kernel, src, workload in (("k_p2p_f32_sym", "sym_kernels.hpp", "globule5000"),
                                  ("k_p2p_f32", "pair_kernels.hpp", "globule500")):
        path = os.path.join(ROOT, "profiles", f"{kernel.replace('k_', '')}_{workload}_hbm.txt")
        kv = dict(line.split(" = ", 1) for line in open(path) if " = " in line and not line.startswith("#"))
        srcpath = os.path.join(ROOT, "paper_1709_08070_amd", "csrc", src)
        assert kv["source"].strip().endswith(src)
        assert bench.kernel_source_hash(srcpath) == kv["source_sha256_16"].split()[0]
        assert bench.measured_traffic(kernel, workload) == float(kv["traffic_bytes"].split()[0])
        # traffic = fetch·scale + write·scale, in bytes (KiB counters)
        t = (float(kv["fetch_size_kib"].split()[0]) * float(kv["fetch_scale"].split()[0])
             + float(kv["write_size_kib"].split()[0]) * float(kv["write_scale"].split()[0])) * 1024
        assert abs(t - float(kv["traffic_bytes"].split()[0])) <= 1e-6 * t + 1.0
    # no summary for this kernel at this workload: no traffic figure
    assert bench.measured_traffic("k_p2p_f32_sym", "globule500") is None


def test_executed_counts_from_the_profiled_source():
    """The executed VALU work of the dominant kernel comes from the committed counter summary,
    only while its source is unchanged."""
    n = 638391
    ex = bench.executed_counts("k_p2p_f32_sym", "globule5000", float(n) * n, 192.46e-3)
    assert ex is not None
    assert 22.5 < ex["valu_insts_per_pair"] < 23.5
    assert 0.3 < ex["frac_of_peak"] < 0.6
    # 1.46e11 wave instructions in 192.46 ms against the 7.9e11/s of an FP32 FMA stream
    assert 0.9 < ex["frac_of_fp32_fma_stream"] < 1.0
    assert bench.issue_rates()["fp32_fma_stream_wave_insts_per_s"] == pytest.approx(7.896e11)
    assert bench.executed_counts("k_p2p_f32_sym", "globule500", 1.0, 1.0) is None


def test_one_thread_rate():
    rng = np.random.default_rng(0)
    n = 300
    nodes = np.zeros((n, 8))
    nodes[:, :3] = rng.normal(size=(n, 3)) * 5
    v = rng.normal(size=(n, 3))
    nodes[:, 3:6] = v / np.linalg.norm(v, axis=1)[:, None]
    nodes[:, 7] = 1.0
    x = rng.normal(size=2 * n)
    r = bench.one_thread_rate(oracle, nodes, oracle.params(0.5), x, 8)
    assert r is not None and r["cores"] == 1 and r["value"] > 0
    assert isinstance(bench.cpu_model(), str)
