"""Helpers for GPU parity tests: run the HIP library and the CPU oracle on
the same seeded problem and compare."""
import sys

import numpy as np
import pytest

from paper_2609_18177_amd import arlbm as A
from helpers import ora_from


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU (torch.cuda.is_available() is False)")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_lattice(p, precision=A.F64, owner="torch", omega_fixed=None, bc=None, omega_export=False):
    over = {} if bc is None else {"bc": bc}
    cfg = A.config_from(p, precision=precision, omega_fixed=omega_fixed, **over)
    L = A.Lattice(cfg, owner=owner)
    if omega_export:
        L.set_omega_export(True)
    L.set_state(p.U0, p.bed)
    return L


def rel_l2_per_comp(a, b):
    out = []
    for c in range(a.shape[0]):
        den = np.sqrt(np.sum(b[c] ** 2))
        num = np.sqrt(np.sum((a[c] - b[c]) ** 2))
        out.append(float(num / den) if den > 0 else float(num))
    return out


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def oracle_run(p, steps, **kw):
    L = ora_from(p, **kw)
    L.run(steps)
    return L
