"""Host logic of the benchmark: the byte model behind its GB/s figures and
the roofline (the counts quoted for the 256x256x20 pressure operator), the
gate that reports counted HBM traffic only for the kernel and sources the
counters were taken with, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N, NNZ = 1387029, 20192829   # 256x256x20 basin: 257 * 257 * 21 nodes, 15-point Kuhn pattern


def test_operator_bytes():
    # symmetric diagonal storage reads the unique values, no indices
    assert bench.matrix_bytes("sdia", N, NNZ, 8) == 8 * (NNZ + N) // 2
    # the Jacobi-scaled operator has a unit diagonal that is not stored
    assert bench.matrix_bytes("sdia", N, NNZ, 8, unit=True) == 8 * (NNZ - N) // 2
    # CSR: value and column index per entry, row pointers
    assert bench.matrix_bytes("csr", N, NNZ, 8) == 12 * NNZ + 4 * (N + 1)
    assert bench.matrix_bytes("sell", N, NNZ, 4) == 8 * NNZ + 4 * (N + 1)


def test_spmv_and_iteration_bytes():
    assert bench.bytes_spmv("sdia", N, NNZ, 8) == 108511896
    assert bench.bytes_spmv("sdia", N, NNZ, 8, unit=True) == 97415664
    assert bench.bytes_spmv("csr", N, NNZ, 8) == 270054532
    # plain Jacobi-PCG iteration: operator + 12 vector passes
    assert bench.bytes_iter("sdia", N, NNZ, 8) == 8 * (NNZ + N) // 2 + 12 * 8 * N
    # scaled: operator without its diagonal + 10 passes + FP32 weights
    scaled = bench.bytes_iter_scaled(N, NNZ, 8)
    assert scaled == 8 * (NNZ - N) // 2 + 10 * 8 * N + 4 * N
    assert 0.86 < scaled / bench.bytes_iter("sdia", N, NNZ, 8) < 0.88


class _Info:
    def __init__(self, iterations, outer=1):
        self.iterations = iterations
        self.outer_iterations = outer


def test_solve_bytes():
    info = _Info(100)
    assert bench.solve_bytes(info, "sdia", N, NNZ, "fp64") == 100 * bench.bytes_iter("sdia", N, NNZ, 8)
    assert (bench.solve_bytes(info, "sdia", N, NNZ, "fp64", scaled=True)
            == 100 * bench.bytes_iter_scaled(N, NNZ, 8))
    mixed = bench.solve_bytes(_Info(100, 3), "sdia", N, NNZ, "mixed")
    assert mixed == (100 * bench.bytes_iter("sdia", N, NNZ, 4)
                     + 4 * (bench.bytes_residual("sdia", N, NNZ) + 24 * N))


class _Op:
    def __init__(self, fmt, ndiag, n):
        self.format, self.ndiag, self.n = fmt, ndiag, n


def test_jacobi_scaled_predicate():
    assert bench.jacobi_scaled(_Op("sdia", 7, N))
    assert bench.jacobi_scaled(_Op("sdia", 13, N))
    assert not bench.jacobi_scaled(_Op("sdia", 62, N))      # wide format keeps A
    assert not bench.jacobi_scaled(_Op("csr", 0, N))
    assert not bench.jacobi_scaled(_Op("sdia", 7, 1445))    # single-workgroup size


def test_counted_traffic_gate(monkeypatch):
    """Counted traffic is reported for the counted kernel while the kernel
    sources hash to the value recorded with the counters, and never else."""
    import re
    with open(bench.COUNTER_SUMMARY) as f:
        text = f.read()
    recorded = re.search(r"^- source_sha256: `([0-9a-f]+)`", text, flags=re.M).group(1)
    kernel = re.search(r"^- kernel: `([^`]+)`", text, flags=re.M).group(1)
    traffic = int(re.search(r"^- traffic_bytes_per_launch: `(\d+)`", text, flags=re.M).group(1))
    assert 1.0 < traffic / bench.bytes_spmv("sdia", N, NNZ, 8, unit="true>" in kernel) < 1.1
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: recorded)
    assert bench.counted_traffic(kernel) == traffic
    assert bench.counted_traffic("k_spmv_csr<double, double, true>") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.counted_traffic(kernel) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert "one GPU only" in (r.stdout + r.stderr)


@pytest.mark.parametrize("period", ["0", "64"])
def test_untimed_sampling_is_refused(period):
    """The roofline needs timed SpMV launches: a sampling period of 0, or one
    longer than a chunk (no iteration of a chunk reaches its middle), is
    refused before any GPU work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--profile-period", period,
                        "--check-every", "32"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--profile-period must be between 1 and --check-every" in r.stderr
