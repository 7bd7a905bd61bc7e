"""Host-side checks that need no GPU: the plane layout the library reports,
the benchmark's refusal of more than one GPU, and that the committed
rocprofv3 summaries were made from the current kernel sources (the benchmark
reports HBM traffic only from a matching summary)."""
import json
import os
import subprocess
import sys

import pytest

from paper_2609_18177_amd import arlbm as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _swe_cfg(nx, ny, precision=A.F32):
    c = A.Config()
    c.abi_version = A.ABI_VERSION
    c.system, c.dim, c.precision = A.SWE, 2, precision
    c.nx, c.ny, c.nz = nx, ny, 1
    c.x0, c.x1, c.y0, c.y1, c.z0, c.z1 = 0.0, 1.0, 0.0, ny / nx, 0.0, 1.0
    c.cfl, c.eps, c.gamma, c.g = 0.5, 1e-10, 1.4, 9.81
    c.h_dry, c.rho_floor, c.p_floor = 1e-6, 1e-12, 1e-12
    c.has_bed = 1
    return c


@pytest.mark.parametrize("nx,ny,precision", [
    (64, 64, A.F32),    # even nx: two columns per lane
    (65, 64, A.F32),    # odd nx: one column per lane
    (64, 64, A.F64),    # FP64 shallow water also runs two columns per lane
    (65, 65, A.F64),    # nx ny = 4225: rounded up to 4288 elements
])
def test_plane_stride_is_rounded_to_64(nx, ny, precision):
    """Every plane is nx ny elements rounded up to a multiple of 64, plus a
    pad of 1088 elements that staggers the planes of power-of-two lattices
    over the memory interleave, whatever the strip width (the bed plane is
    one plane stride, rounded up to 256 bytes)."""
    size = 8 if precision == A.F64 else 4
    s = A.query_sizes(_swe_cfg(nx, ny, precision))
    stride = (nx * ny + 63) // 64 * 64 + 1088
    assert s.bed_bytes == (stride * size + 255) // 256 * 256


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_profiles_match_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    for name in ("euler2d_2048_batched_f32", "euler2d_2048_f32", "euler2d_2048_f64", "swe2d_4096_batched_f32",
                 "swe2d_4096_f32", "euler3d_256_f32", "serving_fixed_f32"):
        with open(os.path.join(ROOT, "profiles", f"{name}_pmc.json")) as f:
            rec = json.load(f)
        assert rec["kernel_source_sha256_16"] == h, name
        assert rec["hbm_bytes_per_launch"] > 0 and rec["avg_kernel_ns"] > 0, name


def test_profiled_kernel_time_within_the_event_timed_step():
    """In each profile, the kernel time per step that rocprofv3 traced over
    the benchmark's timed launches is at most the step time the benchmark's
    own events measured in the same run (the events also hold the gaps
    between launches)."""
    for name in ("euler2d_2048_batched_f32", "euler2d_2048_f32", "euler2d_2048_f64", "swe2d_4096_batched_f32",
                 "swe2d_4096_f32", "euler3d_256_f32", "serving_fixed_f32"):
        with open(os.path.join(ROOT, "profiles", f"{name}_pmc.json")) as f:
            rec = json.load(f)
        assert rec["kernel_ns_per_step"] <= rec["event_ms_per_step_same_run"] * 1e6, name
