"""The Arrhenius factor's exponential (Section 5.4: R = K rho Y exp(-T_i/T))
as the kernels evaluate it, called on the host through the library, pinned
against the C library's exp: the FP64 kernels' within 4 units in the last
place over [-708, 700], the FP32 kernels' within 2 over the float range of
normal results, both against the correctly rounded value of exp at the same
argument; and the special values (NaN, overflow, underflow)."""
import math

import numpy as np

from paper_2609_18177_amd import arlbm as A


def _ulps64(a, b):
    return abs(int(np.float64(a).view(np.int64)) - int(np.float64(b).view(np.int64)))


def _ulps32(a, b):
    return abs(int(np.float32(a).view(np.int32)) - int(np.float32(b).view(np.int32)))


def test_fp64_exp_against_libm():
    rng = np.random.default_rng(0)
    xs = np.concatenate([np.linspace(-708.0, 700.0, 20001), rng.uniform(-60.0, 5.0, 20000),
                         [0.0, -0.0, 1e-300, -1e-300, 0.5, -0.5, math.log(2.0), -math.log(2.0)]])
    worst = max(_ulps64(A.kernel_exp(x), math.exp(x)) for x in xs)
    assert worst <= 4, worst
    assert A.kernel_exp(0.0) == 1.0
    assert math.isnan(A.kernel_exp(float("nan")))
    assert A.kernel_exp(800.0) == math.inf and A.kernel_exp(-800.0) == 0.0


def test_fp32_exp_against_libm():
    rng = np.random.default_rng(1)
    xs = np.concatenate([np.linspace(-87.3, 88.7, 20001), rng.uniform(-60.0, 5.0, 20000),
                         [0.0, 0.5, -0.5]]).astype(np.float32)
    worst = max(_ulps32(A.kernel_exp(float(x), A.F32), np.float32(math.exp(float(x)))) for x in xs)
    assert worst <= 2, worst
    assert A.kernel_exp(0.0, A.F32) == 1.0
    assert math.isnan(A.kernel_exp(float("nan"), A.F32))
    assert A.kernel_exp(100.0, A.F32) == math.inf and A.kernel_exp(-200.0, A.F32) == 0.0
