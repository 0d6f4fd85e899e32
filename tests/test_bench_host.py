"""Host logic of bench.py that needs no GPU: the one-GPU guard and the
algorithmic byte counts behind the roofline figure (K-apply 15 n w + n/8
bytes; one CG update 16 n w)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("shape", [(256, 256, 256), (512, 512, 512), (560, 560, 560), (64, 32, 16)])
@pytest.mark.parametrize("w", [4, 8])
def test_kapply_pass_bytes_sum_to_model(shape, w):
    """Five volume passes move the work array once each way (10 n w), the
    K epilogue reads T, p_beta, p_z, Sigma_1, Sigma_2 and writes q_beta, q_z
    instead of the work array (5 n w more), and the axis-3 pass reads the
    n-bit mask: 15 n w + n/8 in all."""
    n1, n2, n3 = shape
    n = n1 * n2 * n3
    by = bench.pass_bytes(shape, w)
    assert len(by) == len(bench.PASS_NAMES) == 5
    assert sum(by) == 15 * n * w + n // 8


def test_kernel_bytes_of_the_roofline_kernels():
    shape = (256, 256, 256)
    n = 256 ** 3
    # x, p, q, r, Sigma (2 each) in; x, r, z (2 each) out: 16 arrays
    assert bench.kernel_bytes("cg_update.f32", shape, False) == 16 * n * 4
    assert bench.kernel_bytes("cg_update.f64", shape, False) == 16 * n * 8
    # the learned correction adds one FP32 n-array to every P_c^{-1} apply
    assert bench.kernel_bytes("cg_update.f32", shape, True) == 16 * n * 4 + 4 * n
    assert bench.kernel_bytes("axis1_fwd_K.f64", shape, False) == 7 * n * 8
    assert bench.kernel_bytes("axis3.f32", shape, False) == 2 * n * 4 + n // 8
    # the finalize kernels carry no byte count
    assert bench.kernel_bytes("fin_alpha", shape, False) is None


def test_working_launch_threshold():
    """A working launch moves at least 2 n FP32 words; at 8 TB/s that is
    16.8 us at 256^3, taken with a 20 % margin; small grids keep 8 us."""
    assert bench.working_min_us((256, 256, 256)) == pytest.approx(0.8 * 2 * 256 ** 3 * 4 / 8e12 * 1e6)
    assert 13.0 < bench.working_min_us((256, 256, 256)) < 14.0
    assert bench.working_min_us((64, 64, 64)) == 8.0
