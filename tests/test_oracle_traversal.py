"""Pins of the oracle's exact grid traversal and LiDAR ranges (CPU only).

The traversal is checked against an exact rational slab test written here with
``fractions.Fraction`` (brute force over every cell of a tiny grid), and the
ranges against the closed form of an empty rectangular room.  Paper passage:
the LiDAR senses the occupancy grid by ray casting (arXiv 2603.25834, Sec.
IV-A sensor description; Sec. III-D grid).
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

Q16 = 1 << 16
ONE = 1 << 14


def cell_interval(i, j, ox, oy, a, b, den, tmax, open_cell=False):
    """Parameter interval where O + t*(a,b)/den lies in cell [i,i+1]x[j,j+1], t in [0,tmax].

    With ``open_cell`` a ray running along a cell edge does not count as inside it."""
    lo, hi = F(0), tmax
    for o, d, c in ((F(ox, Q16), F(a, den), i), (F(oy, Q16), F(b, den), j)):
        if d == 0:
            inside = (c < o < c + 1) if open_cell else (c <= o <= c + 1)
            if not inside:
                return None
            continue
        t0, t1 = (c - o) / d, (c + 1 - o) / d
        if t0 > t1:
            t0, t1 = t1, t0
        lo, hi = max(lo, t0), min(hi, t1)
    return (lo, hi) if lo <= hi else None


def check_walk(O, ox, oy, a, b, lim, s, scale=ONE):
    cells, E, axis, end = O.walk(ox, oy, a, b, scale, lim, s)
    # parameter units: t in cells for rays (direction (a,b)/2^14); in [0,1] for segments
    den = ONE if scale == ONE else Q16
    tmax = F(lim, Q16) if scale == ONE else F(lim)
    ocx, ocy = ox // Q16, oy // Q16
    if not (0 <= ocx < s and 0 <= ocy < s):
        assert end == 2 and len(cells) == 0
        return
    seen = {}
    prev_t = F(-1)
    for k, ((cx, cy), e, ax) in enumerate(zip(cells, E, axis)):
        cx, cy = int(cx), int(cy)
        assert (cx, cy) not in seen, "cell visited twice"
        iv = cell_interval(cx, cy, ox, oy, a, b, den, tmax)
        assert iv is not None, f"visited cell {(cx, cy)} does not touch the ray"
        if k == 0:
            assert (cx, cy) == (ocx, ocy) and ax == -1 and e == 0
            t_entry = F(0)
        else:
            comp = a if ax == 0 else b
            # E is a Q16 axis distance; parameter = (E/2^16) / (|comp|/den)
            t_entry = F(int(e), Q16) / F(abs(comp), den)
            assert t_entry == iv[0], "entry parameter is not where the ray enters the cell"
            px, py = cells[k - 1]
            assert abs(cx - int(px)) + abs(cy - int(py)) == 1
        assert t_entry >= prev_t
        prev_t = t_entry
        seen[(cx, cy)] = iv
    # every cell crossed over a positive length is visited
    for j in range(s):
        for i in range(s):
            iv = cell_interval(i, j, ox, oy, a, b, den, tmax, open_cell=True)
            if iv is not None and iv[1] > iv[0]:
                assert (i, j) in seen, f"cell {(i, j)} crossed with positive length but not visited"
    # cells visited with zero length are exact corner, origin-boundary or end-of-limit touches
    for (i, j), (lo, hi) in seen.items():
        if hi == lo:
            on_corner = any(
                (F(ox, Q16) + lo * F(a, den)) == X and (F(oy, Q16) + lo * F(b, den)) == Y
                for X in (i, i + 1) for Y in (j, j + 1))
            assert on_corner or lo == 0 or lo == tmax, f"zero-length visit of {(i, j)} not explained"
    # termination: the ray leaves the last cell beyond the limit (end 0) or,
    # within the limit, across the grid border (end 1)
    lx, ly = (int(v) for v in cells[-1])
    big = tmax + 4 * s
    lo, hi = cell_interval(lx, ly, ox, oy, a, b, den, big)
    if a == 0 and b == 0:
        assert end == 0 and len(cells) == 1
    elif end == 0:
        assert hi > tmax
    else:
        assert end == 1 and hi <= tmax
        xo = F(ox, Q16) + hi * F(a, den)
        yo = F(oy, Q16) + hi * F(b, den)
        assert xo in (0, s) or yo in (0, s), "walk stopped inside the grid"


@pytest.mark.parametrize("seed", range(6))
def test_walk_brute_force_random(oracle_mod, seed):
    O = oracle_mod
    cq, sq = O.trig_table()
    rng = np.random.default_rng(seed)
    s = 8
    for _ in range(60):
        ox = int(rng.integers(0, s * Q16))
        oy = int(rng.integers(0, s * Q16))
        k = int(rng.integers(0, O.NANG))
        lim = int(rng.integers(0, 12 * Q16))
        check_walk(O, ox, oy, int(cq[k]), int(sq[k]), lim, s)


def test_walk_special_directions_and_lattice_origins(oracle_mod):
    O = oracle_mod
    s = 8
    dirs = [(ONE, 0), (-ONE, 0), (0, ONE), (0, -ONE), (ONE, ONE), (-ONE, ONE), (ONE, -ONE),
            (-ONE, -ONE), (2 * 4096, 4096), (-4096, 3 * 4096)]
    origins = [(3 * Q16, 4 * Q16), (3 * Q16 + Q16 // 2, 4 * Q16), (3 * Q16, 4 * Q16 + 7),
               (5 * Q16 + 12345, 2 * Q16 + 4321), (0, 0), (s * Q16 - 1, s * Q16 - 1)]
    for (a, b) in dirs:
        for (ox, oy) in origins:
            for lim in (0, 3 * Q16, 3 * Q16 + Q16 // 2, 20 * Q16):
                check_walk(O, ox, oy, a, b, lim, s)


def test_walk_segments(oracle_mod):
    """Motion segments: parameter in [0, 1], direction = Q16 displacement."""
    O = oracle_mod
    rng = np.random.default_rng(11)
    s = 8
    for _ in range(200):
        ox = int(rng.integers(Q16, (s - 1) * Q16))
        oy = int(rng.integers(Q16, (s - 1) * Q16))
        dx = int(rng.integers(-2 * Q16, 2 * Q16))
        dy = int(rng.integers(-2 * Q16, 2 * Q16))
        if rng.random() < 0.2:
            dx = 0
        check_walk(O, ox, oy, dx, dy, 1, s, scale=1)


def test_origin_outside(oracle_mod):
    cells, E, axis, end = oracle_mod.walk(-5, 3 * Q16, ONE, 0, ONE, 5 * Q16, 8)
    assert end == 2 and len(cells) == 0


def test_trig_table_and_heading_index(oracle_mod):
    O = oracle_mod
    cq, sq = O.trig_table()
    k = np.arange(O.NANG)
    ang = 2 * np.pi * k / O.NANG
    assert np.max(np.abs(cq - np.cos(ang) * ONE)) <= 0.5 + 1e-9
    assert np.max(np.abs(sq - np.sin(ang) * ONE)) <= 0.5 + 1e-9
    assert cq[0] == ONE and sq[0] == 0 and cq[O.NANG // 4] == 0 and sq[O.NANG // 4] == ONE
    # heading index: nearest step, non-negative modulo
    for th in (0.0, 1e-5, -1e-5, 1.0, -1.0, 3.1415925, -3.1415925, 2.5, -0.7):
        i = O.heading_index(th)
        assert 0 <= i < O.NANG
        d = (th * O.NANG / (2 * math.pi) - i) % O.NANG
        d = min(d, O.NANG - d)
        assert d <= 0.5 + 1e-3


def _room_env(O, s, cell, R, rmax, pose):
    occ = np.zeros((s, s), bool)
    occ[0, :] = occ[-1, :] = occ[:, 0] = occ[:, -1] = True
    from paper_2603_25834_amd import synth
    p = dict(synth.ENV_DEFAULTS)
    p.update(n_rays=R, cell_m=cell, r_max_m=rmax, loop_closure=0, sigma_x=0.0, sigma_y=0.0, sigma_th=0.0)
    words = synth.pack_bits(occ)
    env = O.OracleEnv(p, np.array([s], np.int32), words, np.array([0], np.int64))
    env.reset(np.array([pose], np.float32))
    return env


@pytest.mark.parametrize("pose", [(3.21, 2.47, 0.3), (1.05, 5.9, -2.0), (4.0, 4.0, 0.0), (0.55, 0.55, 3.0)])
def test_ranges_closed_form_empty_room(oracle_mod, pose):
    """Range = distance along the table direction to the first inner wall face."""
    O = oracle_mod
    s, cell, R, rmax = 64, 0.1, 360, 20.0
    env = _room_env(O, s, cell, R, rmax, pose)
    out = env.step(np.zeros((1, 2), np.float32), np.zeros((1, 5), np.float32))
    cq, sq = O.trig_table()
    x, y, th = env.pose[0]
    ox = int(np.rint(np.float32(x) * np.float32(65536.0 / cell)))
    oy = int(np.rint(np.float32(y) * np.float32(65536.0 / cell)))
    ib = O.heading_index(th)
    for k in range(R):
        idx = (ib + k * (O.NANG // R)) % O.NANG
        a, b = int(cq[idx]), int(sq[idx])
        cands = []
        if a > 0:
            cands.append(F((s - 1) * Q16 - ox, Q16) / F(a, ONE))
        if a < 0:
            cands.append(F(ox - Q16, Q16) / F(-a, ONE))
        if b > 0:
            cands.append(F((s - 1) * Q16 - oy, Q16) / F(b, ONE))
        if b < 0:
            cands.append(F(oy - Q16, Q16) / F(-b, ONE))
        t = min(cands)
        want = float(t) * cell
        got = float(out.ranges[0, k])
        assert abs(got - want) <= 1e-5 * want + 1e-6 * cell, (k, got, want)
        assert out.hit_cell[0, k] >= 0


def test_no_return_gives_max_range(oracle_mod):
    O = oracle_mod
    env = _room_env(O, 256, 0.05, 36, 2.0, (6.4, 6.4, 0.1))
    out = env.step(np.zeros((1, 2), np.float32), np.zeros((1, 5), np.float32))
    assert np.all(out.hit_cell == -1)
    assert np.allclose(out.ranges, 2.0, rtol=1e-6)
    assert np.all(out.rho_q == round(2.0 / 0.05 * 65536))
