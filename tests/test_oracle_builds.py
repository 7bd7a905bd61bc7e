"""The oracle's two builds (single-threaded, and OpenMP over rows for the
all-core timing) give the same bits: every cell's arithmetic is the same in
both, and the one reduction, the wave-speed maximum, does not depend on the
order of its terms."""
import os

import numpy as np
import pytest

from paper_2609_18177_amd import workloads as W
from helpers import ora_from


@pytest.mark.parametrize("make,steps", [
    (lambda: W.euler_seeded_2d(1, n=64), 40),
    (lambda: W.swe_bed_2d(2, n=64), 40),
    (lambda: W.reactive_seeded_2d(0, n=48), 30),
    (lambda: W.euler_octants_3d(seed=0, n=12), 8),
    (lambda: W.euler_seeded_1d(2, n=300), 60),
])
def test_openmp_build_is_bitwise(make, steps):
    os.environ.setdefault("OMP_NUM_THREADS", "4")
    p = make()
    a = ora_from(p)
    b = ora_from(p, parallel=True)
    a.run(steps)
    b.run(steps)
    assert a.t == b.t
    assert np.array_equal(a.moments(), b.moments())
    assert np.array_equal(a.last_omega(), b.last_omega())
