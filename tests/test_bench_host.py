"""Host-side checks of bench.py (no GPU): the one-GPU refusal, the product
step's byte model against sums written out by hand, and the guard that keeps
a stored HBM-traffic summary from being reported for other kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_step_bytes_by_hand():
    # 128^3 7-point workload, all slices in offset mode
    n, nnz, meta = 2097152, 14581760, 393512
    # FP16 z, p (three vectors of 2 B: z, p_old read, p written) and FP64 A, q (8 B)
    assert bench.step_bytes(n, nnz, meta, 16, 64) == nnz * 8 + meta + n * (2 + 2 + 2 + 8)
    # FP16 z, p and FP32 A, q
    assert bench.step_bytes(n, nnz, meta, 16, 32) == nnz * 4 + meta + n * (2 + 2 + 2 + 4)
    # FP64 PCG: 8 B everywhere
    assert bench.step_bytes(n, nnz, meta, 64, 64) == nnz * 8 + meta + n * 32
    # the amp16 solve's launch-weighted mean (666 FP64-product, 835 FP32-product iterations)
    mean = (666 * bench.step_bytes(n, nnz, meta, 16, 64) + 835 * bench.step_bytes(n, nnz, meta, 16, 32)) / 1501
    assert abs(mean - 109294085) < 1.0


def test_cheb_bytes_by_hand():
    # 256^3 Q1 workload, degree 4: three step launches per application
    n, nnz, meta = 16777216, 449455096, 2062568
    # FP16 z (FP32 work vectors), iterate form: B values 2 B per nonzero in
    # each of the three launches; vectors: step 0 gathers v and writes x_2
    # (2 x 4 B), step 1 gathers x_2, reads v, writes x_3 (3 x 4 B), the last
    # step gathers x_3, reads v, x_2 and D^-1/2 (4 x 4 B), r (4 or 8) and
    # writes z (2)
    assert bench.cheb_iteration_bytes(n, nnz, meta, 16, 32) == 3 * (2 * nnz + meta) + n * (8 + 12 + 16 + 4 + 2)
    assert bench.cheb_iteration_bytes(n, nnz, meta, 16, 64) == 3 * (2 * nnz + meta) + n * (8 + 12 + 16 + 8 + 2)
    # FP64 z: FP64 work vectors
    assert bench.cheb_iteration_bytes(n, nnz, meta, 64, 64) == 3 * (2 * nnz + meta) + n * (16 + 24 + 32 + 8 + 8)
    # degree 2: one step that is first and last (gathers v, reads D^-1/2, r; writes z)
    assert bench.cheb_iteration_bytes(n, nnz, meta, 32, 32, degree=2) == 2 * nnz + meta + n * (4 + 4 + 4 + 4)
    # degree 5: a second inner step reads x_{k-1} as well
    assert bench.cheb_iteration_bytes(n, nnz, meta, 16, 32, degree=5) == \
        4 * (2 * nnz + meta) + n * (8 + 12 + 16 + 16 + 4 + 2)


def test_stored_traffic_requires_matching_sources(monkeypatch, tmp_path):
    from paper_2505_04155_amd import build
    f = tmp_path / "counters.txt"
    f.write_text("# header\nsource_digest abc123\nkernel k_spmv\ntraffic_bytes_per_launch 112041016\n")
    monkeypatch.setattr(build, "source_digest", lambda: "abc123")
    assert bench.stored_traffic(str(f)) == 112041016
    monkeypatch.setattr(build, "source_digest", lambda: "other")
    assert bench.stored_traffic(str(f)) is None
    assert bench.stored_traffic(str(tmp_path / "missing.txt")) is None


def test_committed_summary_is_parseable():
    fields = {}
    with open(os.path.join(ROOT, "profiles", "k_spmv_fv3d128_hbm_counters.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, _, v = line.partition(" ")
                fields[k] = v.strip()
    assert fields["kernel"] == "k_spmv"
    assert len(fields["source_digest"]) == 16
    t = int(float(fields["traffic_bytes_per_launch"]))
    # within a few percent of the algorithmic bytes of the same launches
    assert 1.0 <= t / 109294085 <= 1.1


def test_jacobi_iteration_bytes_by_hand():
    # 128^3 7-point workload: preconditioning 4 + 2 + 2, product 4 nnz + meta
    # + 10 per row, update 12 + (16 + 2 x 2) / 2 per row
    n, nnz, meta = 2097152, 14581760, 393512
    assert bench.jacobi_iteration_bytes(n, nnz, meta, 16, 32) == n * 8 + nnz * 4 + meta + n * 10 + n * 22
    assert bench.jacobi_iteration_bytes(n, nnz, meta, 64, 64) == n * 24 + nnz * 8 + meta + n * 32 + n * 40


def test_phase_iterations_from_switch_points():
    info = {"iters": 10, "k_z32": 2, "k_z16": 5, "k_r32": 7}
    assert bench.phase_iterations(info, "amp64") == {(64, 64): 2, (32, 64): 3, (16, 64): 2, (16, 32): 3}
    assert bench.phase_iterations(info, "amp16") == {(16, 64): 7, (16, 32): 3}
    assert bench.phase_iterations({"iters": 4, "k_z32": -1, "k_z16": -1, "k_r32": -1}, "pcg64") == {(64, 64): 4}
