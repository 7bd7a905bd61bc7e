"""The allocation-free entry point (arlbm_conservation_noalloc): the
library's device scratch array instead of a buffer the lattice allocates,
the same sums bit for bit as arlbm_conservation, on two calls in a row, the
second on a smaller lattice (the array keeps the first call's partial sums
beyond what the second one writes and reads)."""
import numpy as np
import pytest

from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W
from gpu_common import require_gpu, say, gpu_lattice

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [A.F32, A.F64])
def test_conservation_noalloc_equals_conservation(prec):
    require_gpu()
    # each lattice smaller than the one before (cells): 90000, 13824, 1600
    cases = [W.euler_seeded_2d(1, n=300, steps=30), W.reactive_sphere_3d(n=24), W.swe_bed_2d(2, n=40, steps=5)]
    for p in cases:
        G = gpu_lattice(p, prec)
        G.step(p.steps if p.dim == 2 else 3)
        a = G.conservation_noalloc()
        b = G.conservation()
        c = G.conservation_noalloc()
        say(f"[no-alloc {p.name} prec={prec}] m={len(a)} noalloc {a} allocating {b}")
        assert np.array_equal(a, b) and np.array_equal(c, b)
        G.close()
