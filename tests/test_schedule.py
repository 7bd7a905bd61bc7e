"""The batched launch's static schedule (host logic, no GPU): every cell of
every served 1D and 2D lattice is stepped by exactly one segment, the
schedule fits the waves it is given, a lattice alone gets the single-lattice
kernel's decomposition (one band of one strip per wave, bands of equal
height), and the work per wave is balanced."""
import numpy as np
import pytest

from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W

WAVES = 1024  # one wave per SIMD: 256 CUs of 4 SIMDs


def _strips(cfg):
    cpl = 2 if (cfg.nx % 2 == 0 and cfg.dim == 2 and
                ((cfg.precision == A.F32 and cfg.system in (A.ADVECTION, A.SWE)) or
                 (cfg.precision == A.F64 and cfg.system == A.SWE))) else 1
    width = 120 if cpl == 2 else 58
    return (cfg.nx + width - 1) // width, cpl


def _cost(cfg, seg):
    """The cost model the header describes: rows + 6 (2D) or strips + 2 (1D),
    times the values a wave moves per row or strip."""
    ncols, cpl = _strips(cfg)
    m = {A.ADVECTION: 1, A.EULER: cfg.dim + 2, A.SWE: cfg.dim + 1, A.REACTIVE: cfg.dim + 3}[cfg.system]
    if cfg.dim == 2:
        return (seg[3] - seg[2] + 6) * 64 * cpl * 5 * m
    return (seg[3] - seg[1] + 2) * (64 * 3 * m + 1280)


def _check_cover(cfgs, ws, segs):
    assert ws[0] == 0 and np.all(np.diff(ws) >= 1) and ws[-1] == len(segs)
    for i, cfg in enumerate(cfgs):
        if cfg.dim == 3:
            assert not np.any(segs[:, 0] == i)
            continue
        ncols, _ = _strips(cfg)
        mine = segs[segs[:, 0] == i]
        if cfg.dim == 2:
            hits = np.zeros((ncols, cfg.ny), dtype=np.int32)
            for _, c, y0, y1 in mine:
                assert 0 <= c < ncols and 0 <= y0 < y1 <= cfg.ny
                hits[c, y0:y1] += 1
        else:
            hits = np.zeros(ncols, dtype=np.int32)
            for _, c0, _, c1 in mine:
                assert 0 <= c0 < c1 <= ncols
                hits[c0:c1] += 1
        assert np.all(hits == 1), (i, cfg.nx, cfg.ny)


def test_lattice_alone_gets_the_single_kernel_bands():
    p = W.euler_seeded_2d(0, n=2048, steps=1)
    cfg = A.config_from(p, precision=A.F32)
    ws, segs = A.plan_schedule([cfg], WAVES)
    _check_cover([cfg], ws, segs)
    # 36 strips of 58 columns; 28 bands of 74 rows (the last one 50): one
    # segment per wave, consecutive waves on neighbouring strips of a band
    assert len(ws) - 1 == 28 * 36 and len(segs) == 28 * 36
    assert np.all(segs[:36, 2] == 0) and np.array_equal(segs[:36, 1], np.arange(36))
    heights = segs[:, 3] - segs[:, 2]
    assert heights.max() == 74 and set(heights.tolist()) <= {74, 2048 - 27 * 74}


@pytest.mark.parametrize("precision", [A.F32, A.F64])
def test_serving_mix_is_covered_and_balanced(precision):
    reqs = W.serving_requests(60, rate_hz=200.0, seed=3)
    cfgs = [A.config_from(r.problem(), precision=precision) for r in reqs]
    ws, segs = A.plan_schedule(cfgs, WAVES)
    nw = len(ws) - 1
    assert nw <= WAVES
    _check_cover(cfgs, ws, segs)
    cost = np.array([sum(_cost(cfgs[s[0]], s) for s in segs[ws[w]:ws[w + 1]]) for w in range(nw)])
    total = sum(_cost(c, s) for c, s in ((cfgs[s[0]], s) for s in segs))
    # a wave's work stays near the mean over all the waves the GPU has: the
    # launch takes about as long as its longest wave
    assert cost.max() <= 1.5 * total / WAVES, (cost.max(), total / WAVES)


def test_small_mix_spreads_and_3d_is_left_out():
    """Far less work than the GPU holds: every 1D strip gets a wave of its
    own and 2D bands are cut down to 8 rows, as the single-lattice kernel
    spreads a small lattice, so the step takes as little time as it can."""
    cfgs = [A.config_from(W.euler_seeded_1d(0, n=3000), precision=A.F32),
            A.config_from(W.swe_bed_2d(1, n=40), precision=A.F32),
            A.config_from(W.euler_octants_3d(seed=0, n=12), precision=A.F32)]
    ws, segs = A.plan_schedule(cfgs, WAVES)
    _check_cover(cfgs, ws, segs)
    one_d = segs[segs[:, 0] == 0]
    assert np.all(one_d[:, 3] - one_d[:, 1] == 1) and len(one_d) == (3000 + 57) // 58
    two_d = segs[segs[:, 0] == 1]
    assert np.all(two_d[:, 3] - two_d[:, 2] == 8)
    assert len(ws) - 1 == len(segs)


def test_plan_rejects_bad_input():
    cfg = A.config_from(W.euler_seeded_2d(0, n=64), precision=A.F32)
    cfg.cfl = 2.0
    with pytest.raises(A.ArlbmError):
        A.plan_schedule([cfg], WAVES)
