"""The batched launch's work list (host logic, no GPU): every cell of every
served 1D and 2D lattice is stepped by exactly one item; a lattice alone
gets the single-lattice kernel's bands (one band of one strip per wave);
the list fits one round of the launch's waves where the work allows; it holds each
lattice's bands in order with each band's strips left to right; each of its
eight per-XCD queues holds bands, then 1D runs; in one round every band is a
wave's first item, over several rounds the queues carry about equal work."""
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
    """The cost model the runtime describes: rows + 6 (2D) or strips + 2
    (1D), times the values a wave moves per row or strip."""
    ncols, cpl = _strips(cfg)
    seg = [int(v) for v in seg]
    m = {A.ADVECTION: 1, A.EULER: cfg.dim + 2, A.SWE: cfg.dim + 1, A.REACTIVE: cfg.dim + 3}[cfg.system]
    if cfg.dim == 2:
        return (seg[3] - seg[2] + 6) * 64 * cpl * 5 * m
    return (seg[3] - seg[1] + 2) * (64 * 3 * m + 1280)


def _check_cover(cfgs, qs, segs):
    assert qs[0] == 0 and qs[-1] == len(segs) and np.all(np.diff(qs) >= 0)
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
            # bands in order, each band's strips left to right, one height
            keys = [(y0, c) for _, c, y0, _ in mine]
            assert keys == sorted(keys)
            h = mine[0, 3] - mine[0, 2]
            assert np.all(mine[:, 3] - mine[:, 2] <= h)
        else:
            hits = np.zeros(ncols, dtype=np.int32)
            for _, c0, _, c1 in mine:
                assert 0 <= c0 < c1 <= ncols
                hits[c0:c1] += 1
        assert np.all(hits == 1), (i, cfg.nx, cfg.ny)


def test_lattice_alone_gets_the_single_kernel_bands():
    p = W.euler_seeded_2d(0, n=2048, steps=1)
    cfg = A.config_from(p, precision=A.F32)
    qs, segs, nw = A.plan_schedule([cfg], WAVES)
    _check_cover([cfg], qs, segs)
    # 36 strips of 58 columns; 28 bands of 74 rows (the last one 50): one
    # item per wave
    assert len(segs) == 28 * 36 and nw == len(segs)
    assert np.all(segs[:36, 2] == 0) and np.array_equal(segs[:36, 1], np.arange(36))
    heights = segs[:, 3] - segs[:, 2]
    assert heights.max() == 74 and set(heights.tolist()) <= {74, 2048 - 27 * 74}


def test_shallow_water_alone_gets_tall_bands():
    """4096^2 shallow water with two columns per lane: 35 strips of 120
    columns, 29 bands of 142 rows, one round."""
    p = W.swe_bed_2d(0, n=4096, steps=1)
    cfg = A.config_from(p, precision=A.F32)
    qs, segs, nw = A.plan_schedule([cfg], WAVES)
    _check_cover([cfg], qs, segs)
    assert len(segs) == 35 * 29 <= WAVES
    assert (segs[:, 3] - segs[:, 2]).max() == 142


def _queue_parts(cfgs, qs, segs):
    """Each queue: its 2D bands, then its 1D runs (the runs dealt round
    robin over the queues, largest first)."""
    runs = []
    for q in range(8):
        part = segs[qs[q]:qs[q + 1]]
        dims = np.array([cfgs[i].dim for i in part[:, 0]], dtype=int)
        if len(dims) and np.any(dims == 1):
            first = int(np.argmax(dims == 1))
            assert np.all(dims[first:] == 1), q
        runs.append(part[dims == 1] if len(dims) else part[:0])
    counts = [len(r) for r in runs]
    assert max(counts) - min(counts) <= 1, counts
    return [segs[qs[q]:qs[q + 1]][np.array([cfgs[i].dim == 2 for i in segs[qs[q]:qs[q + 1], 0]], dtype=bool)]
            for q in range(8)]


@pytest.mark.parametrize("n,precision", [(60, A.F32), (60, A.F64), (512, A.F32)])
def test_serving_mix_rounds_and_queues(n, precision):
    reqs = W.serving_requests(n, rate_hz=200.0, seed=0)
    cfgs = [A.config_from(r.problem(), precision=precision) for r in reqs]
    qs, segs, nw = A.plan_schedule(cfgs, WAVES)
    assert nw == min(WAVES, len(segs))
    _check_cover(cfgs, qs, segs)
    two_d = segs[np.array([cfgs[i].dim == 2 for i in segs[:, 0]])]
    rows = two_d[:, 3] - two_d[:, 2]
    # the 2D items: at most 256 rows, one round of the waves where the work
    # allows it, lattices with the tallest bands first
    assert rows.max() <= 256
    strip_rows = sum(_strips(c)[0] * c.ny for c in cfgs if c.dim == 2)
    rounds = -(-strip_rows // (WAVES * 256))
    parts = _queue_parts(cfgs, qs, segs)
    bands = np.concatenate(parts)
    heights = [max(s[3] - s[2] for s in bands[bands[:, 0] == i]) for i in dict.fromkeys(bands[:, 0])]
    assert heights == sorted(heights, reverse=True)
    if len(two_d) <= WAVES:
        # one round: every band is the first item of a wave of its XCD
        assert max(len(p) for p in parts) <= WAVES // 8
    else:
        assert rounds > 1 or rows.max() >= strip_rows // (2 * WAVES)
        work = [sum(_cost(cfgs[s[0]], s) for s in p) for p in parts]
        mean = sum(work) / 8
        assert max(work) <= 1.05 * mean and min(work) >= 0.95 * mean, [w / mean for w in work]


def test_small_mix_and_3d_left_out():
    """Far less work than the waves: every 1D strip an item of its own, 2D
    bands of 8 rows, as the single-lattice kernel spreads a small lattice."""
    cfgs = [A.config_from(W.euler_seeded_1d(0, n=3000), precision=A.F32),
            A.config_from(W.swe_bed_2d(1, n=40), precision=A.F32),
            A.config_from(W.euler_octants_3d(seed=0, n=12), precision=A.F32)]
    qs, segs, nw = A.plan_schedule(cfgs, WAVES)
    _check_cover(cfgs, qs, segs)
    assert nw == len(segs)
    one_d = segs[segs[:, 0] == 0]
    assert np.all(one_d[:, 3] - one_d[:, 1] == 1)
    assert np.all(segs[segs[:, 0] == 1][:, 3] - segs[segs[:, 0] == 1][:, 2] == 8)


def test_1d_lattices_alone_spread_over_the_waves():
    """Only 1D lattices (no 2D work to size items from): runs short enough
    that the strips fill the waves in one round."""
    cfgs = [A.config_from(W.euler_seeded_1d(s, n=65536), precision=A.F32) for s in range(3)]
    qs, segs, nw = A.plan_schedule(cfgs, WAVES)
    _check_cover(cfgs, qs, segs)
    strips = 3 * ((65536 + 57) // 58)
    assert len(segs) <= WAVES and np.max(segs[:, 3] - segs[:, 1]) <= -(-strips // WAVES)


def test_plan_rejects_bad_input():
    cfg = A.config_from(W.euler_seeded_2d(0, n=64), precision=A.F32)
    cfg.cfl = 2.0
    with pytest.raises(A.ArlbmError):
        A.plan_schedule([cfg], WAVES)


def test_heavy_round_with_1d_runs():
    """2D bands filling one round of the waves beside 1D lattices: every band
    is a wave's first item and the 1D strips go in runs of at least 8, dealt
    round robin to the ends of the queues."""
    cfgs = [A.config_from(W.euler_seeded_2d(s, n=n), precision=A.F32)
            for s, n in enumerate((1000, 984, 900, 882, 861, 742, 692, 602, 525, 507, 469, 431))]
    cfgs += [A.config_from(W.euler_seeded_1d(s, n=n), precision=A.F32) for s, n in enumerate((60603, 33971, 8438))]
    qs, segs, nw = A.plan_schedule(cfgs, WAVES)
    _check_cover(cfgs, qs, segs)
    parts = _queue_parts(cfgs, qs, segs)
    assert sum(len(p) for p in parts) <= WAVES
    assert max(len(p) for p in parts) <= WAVES // 8
    one_d = segs[np.array([cfgs[i].dim == 1 for i in segs[:, 0]])]
    lengths = one_d[:, 3] - one_d[:, 1]
    ends = {i: _strips(cfgs[i])[0] for i in set(one_d[:, 0])}
    inner = np.array([s[3] < ends[s[0]] for s in one_d])
    assert np.all(lengths[inner] >= 8)


@pytest.mark.parametrize("waves", [1, 2, 3, 4, 5, 7, 8, 9])
def test_few_waves(waves):
    """A launch of fewer waves than XCDs (a host plan asked for any count):
    with the 2D bands taking every wave, the 1D strips still go in runs and
    every cell is covered once."""
    cfgs = [A.config_from(W.euler_seeded_2d(0, n=200), precision=A.F32),
            A.config_from(W.euler_seeded_1d(1, n=5000), precision=A.F32)]
    qs, segs, nw = A.plan_schedule(cfgs, waves)
    _check_cover(cfgs, qs, segs)
    assert 1 <= nw <= waves


def _fixed_mix_cfgs(budget=4 * 2 ** 30):
    """The default serving mix's requests in arrival order, as many as a
    budget holds at once (FP32)."""
    cfgs, used = [], 0
    for r in W.serving_requests(512, rate_hz=200.0, seed=0):
        c = A.config_from(r.problem(), precision=A.F32)
        b = A.query_sizes(c).total_bytes * 1.25
        if used + b > budget:
            break
        cfgs.append(c)
        used += b
    return cfgs


def _two_d_items(cfgs, segs):
    return int(np.sum([cfgs[i].dim == 2 for i in segs[:, 0]])) if len(segs) else 0


def test_launch_groups_of_the_fixed_mix():
    """2D work beyond one round of the waves is split into launches that each
    fit one round: every lattice in exactly one group, and in each group's
    work list every band a wave's first item."""
    cfgs = _fixed_mix_cfgs()
    grp, ng = A.plan_groups(cfgs, WAVES)
    qs, segs, nw = A.plan_schedule(cfgs, WAVES)
    assert _two_d_items(cfgs, segs) > WAVES  # one launch would take two rounds
    assert ng >= 2 and set(grp.tolist()) == set(range(ng))
    for g in range(ng):
        sub = [c for c, k in zip(cfgs, grp) if k == g]
        # one cost class per launch here: Euler, with the 1D lattices;
        # shallow water of two columns per lane; of one column
        assert len(set(_strips(c)[1] * 10 + c.system for c in sub if c.dim == 2)) == 1
        qs, segs, nw = A.plan_schedule(sub, WAVES)
        _check_cover(sub, qs, segs)
        assert _two_d_items(sub, segs) <= WAVES
        parts = _queue_parts(sub, qs, segs)
        assert max(len(p) for p in parts) <= WAVES // 8


def test_launch_groups_one_round_and_3d():
    """Work that fits one round stays one launch; 3D lattices are in none."""
    cfgs = [A.config_from(W.euler_seeded_2d(s, n=n), precision=A.F32) for s, n in enumerate((600, 300, 130))]
    cfgs.append(A.config_from(W.euler_octants_3d(seed=0, n=16), precision=A.F32))
    cfgs.append(A.config_from(W.euler_seeded_1d(0, n=9000), precision=A.F32))
    grp, ng = A.plan_groups(cfgs, WAVES)
    assert ng == 1 and grp.tolist() == [0, 0, 0, -1, 0]
    grp, ng = A.plan_groups([cfgs[3]], WAVES)
    assert ng == 0 and grp.tolist() == [-1]


def test_launch_groups_with_a_lattice_beyond_one_round():
    """A 2D lattice that alone needs more than one round keeps a group of its
    own (no split shortens it); the others fit one round beside it."""
    big = A.config_from(W.euler_seeded_2d(0, n=8192), precision=A.F32)
    cfgs = [big] + [A.config_from(W.euler_seeded_2d(s, n=n), precision=A.F32) for s, n in enumerate((1000, 700, 500))]
    grp, ng = A.plan_groups(cfgs, WAVES)
    assert ng >= 2
    assert all(grp[i] != grp[0] for i in range(1, len(cfgs)))
    for g in range(ng):
        sub = [c for c, k in zip(cfgs, grp) if k == g]
        qs, segs, nw = A.plan_schedule(sub, WAVES)
        _check_cover(sub, qs, segs)
        if all(c is not big for c in sub):
            assert _two_d_items(sub, segs) <= WAVES


@pytest.mark.parametrize("waves", [1, 3, 8, 64])
def test_launch_groups_few_waves(waves):
    cfgs = _fixed_mix_cfgs(512 << 20)
    grp, ng = A.plan_groups(cfgs, waves)
    assert ng >= 1 and np.all((grp >= 0) & (grp < ng))
    for g in range(ng):
        sub = [c for c, k in zip(cfgs, grp) if k == g]
        qs, segs, nw = A.plan_schedule(sub, waves)
        _check_cover(sub, qs, segs)
