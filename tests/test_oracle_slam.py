"""Pins of the fixed-lag SLAM oracle (CPU only).

Paper passage: arXiv 2603.25834, Sec. III-D (correlative scan matching on the log-odds grid; a
fixed-lag pose graph solved by Gauss-Newton; the newest pose's covariance as the last block of the
inverse Hessian).  The matcher is pinned by geometry (its integer endpoints against FP64 trigonometry),
by a scene built around a known pose (the search must return it and the score bound), by the
equivariances of the lattice (a shifted grid shifts the best candidate; a heading step on the
candidate equals the same step on every ray) and by its tie and second-peak rules.  The graph solve is
pinned by closed forms (a prior alone, a prior plus a scan factor, a motionless chain), by convergence
to exact poses from consistent factors, and by finite differences of the residuals.  The weighted
map integration is pinned against the env oracle's own map update (unweighted case), by closed forms
along axis rays (cells, end rule, rounding of the weighted increments, saturation) and by its weight
extremes.
"""
import numpy as np
import pytest

from oracle import slam_ref as S

TRIG = None


def trig():
    global TRIG
    if TRIG is None:
        TRIG = S._trig()
    return TRIG


def _scene(seed, s=96, R=120, W=4, V=3, step_xy=65536, step_h=32, true=(2, -1, 3)):
    """Grid with occupied cells exactly at the scan's endpoints under the true candidate."""
    rng = np.random.default_rng(seed)
    px, py, ph = 48 * 65536 + 12345, 47 * 65536 + 40000, int(rng.integers(0, S.NANG))
    rho = (rng.uniform(3.0, 30.0, R) * 65536).astype(np.int32)
    rho[rng.random(R) < 0.1] = -1
    a = (np.arange(R) * (S.NANG // R)).astype(np.int32)
    cq, sq = trig()
    ti, tj, tk = true
    h = np.mod(ph + tk * step_h + a.astype(np.int64), S.NANG)
    ok = rho >= 0
    ex = (px + ti * step_xy + ((rho.astype(np.int64) * cq[h]) >> 14)) >> 16
    ey = (py + tj * step_xy + ((rho.astype(np.int64) * sq[h]) >> 14)) >> 16
    g = np.zeros((s, s), np.int16)
    g[ey[ok], ex[ok]] = 800
    # free-space evidence elsewhere, never on an endpoint cell
    free = rng.random((s, s)) < 0.3
    g[free & (g == 0)] = -100
    return g, px, py, ph, rho, a, W, V, step_xy, step_h


def test_integer_endpoints_match_fp64_geometry():
    """The Q14-table endpoint cell equals the FP64 one except within a hair of a cell boundary."""
    rng = np.random.default_rng(1)
    cq, sq = trig()
    n = 20000
    x = rng.uniform(10, 90, n)
    y = rng.uniform(10, 90, n)
    h = rng.integers(0, S.NANG, n)
    rho = rng.uniform(0.5, 40.0, n)
    xq = np.floor(x * 65536).astype(np.int64)
    yq = np.floor(y * 65536).astype(np.int64)
    rq = np.floor(rho * 65536).astype(np.int64)
    cx = (xq + ((rq * cq[h]) >> 14)) >> 16
    cy = (yq + ((rq * sq[h]) >> 14)) >> 16
    ang = 2 * np.pi * h / S.NANG
    fx = x + rho * np.cos(ang)
    fy = y + rho * np.sin(ang)
    mism = (cx != np.floor(fx)) | (cy != np.floor(fy))
    # the table rounds directions to 1/16384: at 40 cells the endpoint moves by at most ~0.0025 cells
    near = (np.abs(fx - np.rint(fx)) < 0.01) | (np.abs(fy - np.rint(fy)) < 0.01)
    assert mism.mean() < 0.02
    assert np.all(near[mism])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_match_finds_the_pose_the_scene_was_built_around(seed):
    g, px, py, ph, rho, a, W, V, sxy, sh = _scene(seed)
    bi, bj, bk, best, second, n_used = S.csm_match(g, px, py, ph, rho, a, W, V, sxy, sh, trig())
    assert (bi, bj, bk) == (2, -1, 3)
    assert n_used == int((rho >= 0).sum())
    assert best == 800 * n_used            # every ray on an occupied cell: the largest possible score
    assert second < best


def test_grid_shift_moves_the_best_candidate():
    """Shifting the grid by whole cells (and nothing else) shifts the best lattice offset with it."""
    g, px, py, ph, rho, a, W, V, sxy, sh = _scene(3, true=(0, 0, 0))
    g2 = np.zeros_like(g)
    g2[2:, :-1] = g[:-2, 1:]                  # content moves by (-1, +2) cells
    bi, bj, bk, best, _, _ = S.csm_match(g2, px, py, ph, rho, a, W, V, sxy, sh, trig())
    assert (bi, bj, bk) == (-1, 2, 0)


def test_heading_step_equals_rotating_every_ray():
    g, px, py, ph, rho, a, W, V, sxy, sh = _scene(4)
    sc = S.csm_scores(g, px, py, ph, rho, a, W, V, sxy, sh, trig())
    k = 2
    sc2 = S.csm_scores(g, px, py, ph, rho, a + k * sh, W, 0, sxy, sh, trig())
    assert np.array_equal(sc[V + k], sc2[0])


def test_tie_rule_and_second_peak():
    rng = np.random.default_rng(5)
    g = np.zeros((32, 32), np.int16)
    rho = (rng.uniform(1, 10, 30) * 65536).astype(np.int32)
    a = (np.arange(30) * 1536).astype(np.int32)
    bi, bj, bk, best, second, _ = S.csm_match(g, 16 << 16, 16 << 16, 0, rho, a, 2, 1, 65536, 16, trig())
    assert (bi, bj, bk, best, second) == (-2, -2, -1, 0, 0)     # all equal: smallest index; a far peak of 0
    # a lattice with no candidate two steps away from the best has no second peak
    _, _, _, _, second, _ = S.csm_match(g, 16 << 16, 16 << 16, 0, rho, a, 0, 0, 65536, 16, trig())
    assert second == S.INT32_MIN


def test_second_peak_skips_the_best_neighbours():
    g, px, py, ph, rho, a, W, V, sxy, sh = _scene(6, true=(0, 0, 0))
    sc = S.csm_scores(g, px, py, ph, rho, a, W, V, sxy, sh, trig())
    bi, bj, bk, best, second, _ = S.csm_match(g, px, py, ph, rho, a, W, V, sxy, sh, trig())
    near = sc[V - 1:V + 2, W - 1:W + 2, W - 1:W + 2].copy()
    masked = sc.copy()
    masked[V - 1:V + 2, W - 1:W + 2, W - 1:W + 2] = np.iinfo(np.int64).min
    assert second == masked.max()
    assert near.max() == best


def test_scan_factor_pose_and_weight():
    z, info = S.scan_factor(3, -2, 1, 4000, 1000, 10, 100 * 65536, 50 * 65536, 0, 65536, 64, 0.05, 800, 0.05,
                            0.02)
    assert np.allclose(z, [103 * 0.05, 48 * 0.05, 2 * np.pi * 64 / S.NANG], rtol=0, atol=1e-15)
    w = (4000 / 8000) * (3000 / 4000)
    assert np.allclose(info, [w / 0.05 ** 2, w / 0.05 ** 2, w / 0.02 ** 2], rtol=1e-15)
    _, info0 = S.scan_factor(0, 0, 0, -50, -60, 10, 0, 0, 0, 65536, 64, 0.05, 800, 0.05, 0.02)
    assert np.all(info0 == 0)


# ------------------------------------------------------------------ fixed-lag graph

def test_prior_alone_and_prior_plus_scan():
    prior = np.array([1.0, -2.0, 0.3, 50.0, 80.0, 400.0])
    x, Sig = S.fixedlag_solve(np.zeros((1, 3)), prior, np.zeros((0, 6)), np.zeros((1, 6)), 2)
    assert np.allclose(x[0], prior[:3], atol=1e-12)
    assert np.allclose(Sig, np.diag(1.0 / prior[3:]), rtol=1e-12, atol=1e-15)
    scan = np.array([[1.2, -1.9, 0.25, 150.0, 20.0, 100.0]])
    x, Sig = S.fixedlag_solve(np.zeros((1, 3)), prior, np.zeros((0, 6)), scan, 3)
    w = prior[3:] + scan[0, 3:]
    assert np.allclose(x[0], (prior[:3] * prior[3:] + scan[0, :3] * scan[0, 3:]) / w, atol=1e-12)
    assert np.allclose(Sig, np.diag(1.0 / w), rtol=1e-12, atol=1e-15)


def test_motionless_chain_covariance_adds_up():
    """No motion: the odometry Jacobians lose their rotation coupling, so the newest pose's
    covariance is the prior's plus one odometry covariance per link, the odometry's translation
    part rotated from the robot frame (heading th) into the world frame."""
    L = 6
    th = 0.7
    prior = np.array([0.5, 0.5, th, 100.0, 200.0, 1000.0])
    odo = np.tile([0.0, 0.0, 0.0, 400.0, 300.0, 2000.0], (L - 1, 1))
    x0 = np.tile(prior[:3], (L, 1))
    x, Sig = S.fixedlag_solve(x0, prior, odo, np.zeros((L, 6)), 2)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    want = np.diag(1.0 / prior[3:])
    want[:2, :2] += (L - 1) * R @ np.diag(1.0 / odo[0, 3:5]) @ R.T
    want[2, 2] += (L - 1) / odo[0, 5]
    assert np.allclose(x, x0, atol=1e-12)
    assert np.allclose(Sig, want, rtol=1e-12, atol=1e-16)


def _truth(L, seed):
    rng = np.random.default_rng(seed)
    t = np.zeros((L, 3))
    t[0] = [rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-3, 3)]
    for i in range(1, L):
        d, w = rng.uniform(0.05, 0.2), rng.uniform(-0.3, 0.3)
        th = t[i - 1, 2]
        t[i] = [t[i - 1, 0] + d * np.cos(th), t[i - 1, 1] + d * np.sin(th), S.wrap(th + w)]
    odo = np.zeros((L - 1, 6))
    for i in range(L - 1):
        c, s = np.cos(t[i, 2]), np.sin(t[i, 2])
        dt = t[i + 1, :2] - t[i, :2]
        odo[i, :3] = [c * dt[0] + s * dt[1], -s * dt[0] + c * dt[1], S.wrap(t[i + 1, 2] - t[i, 2])]
        odo[i, 3:] = [400.0, 400.0, 2500.0]
    return t, odo, rng


def test_consistent_factors_are_met_exactly():
    L = 8
    t, odo, rng = _truth(L, 7)
    prior = np.concatenate([t[0], [100.0, 100.0, 1000.0]])
    scan = np.zeros((L, 6))
    scan[::3, :3] = t[::3]
    scan[::3, 3:] = [50.0, 50.0, 200.0]
    x0 = t + rng.normal(0, [0.05, 0.05, 0.05], t.shape)
    x, Sig = S.fixedlag_solve(x0, prior, odo, scan, 6)
    d = x - t
    d[:, 2] = S.wrap(d[:, 2])
    assert np.abs(d).max() < 1e-10
    assert np.all(np.linalg.eigvalsh(Sig) > 0)


def test_jacobians_match_finite_differences():
    L = 5
    t, odo, rng = _truth(L, 8)
    prior = np.concatenate([t[0] + 0.01, [100.0, 120.0, 900.0]])
    scan = np.zeros((L, 6))
    scan[1, :3] = t[1] + [0.02, -0.01, 0.03]
    scan[1, 3:] = [30.0, 40.0, 300.0]
    odo[:, :3] += rng.normal(0, 0.01, (L - 1, 3))
    x = t + rng.normal(0, 0.02, t.shape)
    H, g = S.normal_equations(x, prior, odo, scan)

    def stacked(xv):
        res, info = S.residuals(xv.reshape(L, 3), prior, odo, scan)
        return np.concatenate(res), np.concatenate(info)

    r0, om = stacked(x.reshape(-1))
    J = np.zeros((r0.size, 3 * L))
    eps = 1e-6
    for c in range(3 * L):
        e = np.zeros(3 * L); e[c] = eps
        J[:, c] = (stacked(x.reshape(-1) + e)[0] - stacked(x.reshape(-1) - e)[0]) / (2 * eps)
    assert np.allclose(H, J.T @ (om[:, None] * J), rtol=1e-6, atol=1e-5)
    assert np.allclose(g, J.T @ (om * r0), rtol=1e-6, atol=1e-7)


# ------------------------------------------------------------------ weighted map integration

def test_unweighted_integration_equals_the_env_update():
    """With no match (w = 1) the integration reproduces the env oracle's map update of a step, taken from
    the step's estimated pose with its measured ranges (rays without a hit walk to the maximum range)."""
    from oracle import oracle as O
    from paper_2603_25834_amd import synth
    name = "small_16x64"
    w = synth.WORKLOADS[name]
    p = w.params()
    b = synth.make_batch(name, 5)
    env = O.OracleEnv(p, b.sides, b.world, b.world_off)
    env.reset(b.start)
    A = synth.actions(name, 5, 6)
    G = synth.noise(name, 5, 6)
    for t in range(5):
        env.step(A[t], G[t])
    before = [env.belief_of(i).copy() for i in range(env.n)]
    out = env.step(A[5], G[5])
    R = int(p["n_rays"])
    inv_c16 = np.float32(65536.0 / float(np.float32(p["cell_m"])))
    rmax_q = int(round(float(np.float32(p["r_max_m"])) / float(np.float32(p["cell_m"])) * 65536.0))
    a_off = (np.arange(R) * (S.NANG // R)).astype(np.int32)
    changed = 0
    for i in range(env.n):
        e = env.est[i]
        px = int(np.rint(np.float32(e[0]) * inv_c16))
        py = int(np.rint(np.float32(e[1]) * inv_c16))
        ph = O.heading_index(float(e[2]))
        rho = np.where(out.hit_cell[i] >= 0, out.rho_q[i], -1).astype(np.int32)
        got, n_coded = S.integrate(before[i], px, py, ph, rho, a_off, rmax_q, 218, -102, 896)
        assert np.array_equal(got, env.belief_of(i)), i
        assert n_coded == int(out.counters[i, 2])          # the env's count of distinct updated cells
        changed += n_coded
    assert changed > 0


def _axis_rays(s=64):
    """Origin at the centre of cell (20, 30); ray directions along +x (a_off 0) and -x (a_off NANG/2)."""
    return 20 * 65536 + 32768, 30 * 65536 + 32768, 0


def test_axis_ray_cells_end_rule_and_weighted_increments():
    s = 64
    px, py, ph = _axis_rays(s)
    g = np.zeros((s, s), np.int16)
    g[30, 23] = 880          # a MISS that stays below the clamp
    g[30, 30] = 850          # the HIT, saturating at +896
    g[30, 25] = -880         # a MISS saturating at -896
    rho = np.array([int(10.25 * 65536)], np.int32)           # ends inside cell 30
    a_off = np.zeros(1, np.int32)
    # w = q m = 1 * 0.5: best = n_used * l_max, second = best / 2  ->  w_q = 128
    match = (0, 0, 0, 896, 448, 1)
    got, n_coded = S.integrate(g, px, py, ph, rho, a_off, 40 * 65536, 218, -102, 896, match=match,
                               step_xy=65536, step_h=64, l_max=896.0)
    want = g.astype(np.int64)
    want[30, 20:30] += -51                                   # round(0.5 * -102) = -51
    want[30, 30] += 109                                      # round(0.5 * 218) = 109
    want = np.clip(want, -896, 896).astype(np.int16)
    assert n_coded == 11 and np.array_equal(got, want)
    # a range ending exactly on a cell boundary enters that cell (entry distance = range)
    got2, n2 = S.integrate(np.zeros((s, s), np.int16), px, py, ph, np.array([int(10.5 * 65536)], np.int32), a_off,
                           40 * 65536, 218, -102, 896)
    assert n2 == 12 and got2[30, 31] == 218 and np.all(got2[30, 20:31] == -102)


def test_hit_beats_miss_grid_exit_and_no_return():
    s = 64
    px, py, ph = _axis_rays(s)
    half = S.NANG // 2
    rho = np.array([int(10.25 * 65536), int(5.25 * 65536), int(40.0 * 65536), -1], np.int32)
    a_off = np.array([0, 0, half, S.NANG // 4], np.int32)   # +x, +x, -x (leaves the grid), +y (no return)
    got, n_coded = S.integrate(np.zeros((s, s), np.int16), px, py, ph, rho, a_off, int(12.5 * 65536), 218, -102, 896)
    want = np.zeros((s, s), np.int16)
    want[30, 0:31] = -102          # +x to cell 30 and -x out of the grid past cell 0 (no HIT there)
    want[30, 30] = 218             # HIT of the long +x ray
    want[30, 25] = 218             # HIT of the short +x ray beats the long ray's MISS
    want[31:44, 20] = -102         # +y without a return: free space up to 12.5 cells (cell 43 entered at 12.5)
    assert np.array_equal(got, want)
    assert n_coded == 31 + 13


def test_weight_extremes():
    """w = 0 leaves the grid as it was; w = 1 equals the unweighted update from the aligned pose."""
    rng = np.random.default_rng(9)
    s, R = 80, 90
    g = rng.integers(-400, 400, (s, s)).astype(np.int16)
    px, py, ph = 40 * 65536 + 1234, 38 * 65536 + 50000, 12345
    rho = (rng.uniform(2.0, 30.0, R) * 65536).astype(np.int32)
    rho[rng.random(R) < 0.2] = -1
    a_off = (np.arange(R) * (S.NANG // R)).astype(np.int32)
    n_used = int((rho >= 0).sum())
    zero, nz = S.integrate(g, px, py, ph, rho, a_off, 35 * 65536, 218, -102, 896, match=(1, -2, 3, 0, -5, n_used),
                           step_xy=32768, step_h=64, l_max=896.0)
    assert np.array_equal(zero, g) and nz > 0
    full, nf = S.integrate(g, px, py, ph, rho, a_off, 35 * 65536, 218, -102, 896,
                           match=(1, -2, 3, 896 * n_used, 0, n_used), step_xy=32768, step_h=64, l_max=896.0)
    ref, nr = S.integrate(g, px + 32768, py - 65536, ph + 192, rho, a_off, 35 * 65536, 218, -102, 896)
    assert np.array_equal(full, ref) and nf == nr
    # an aligned pose off the grid leaves it unchanged
    off, no = S.integrate(g, -3 * 65536, py, ph, rho, a_off, 35 * 65536, 218, -102, 896)
    assert np.array_equal(off, g) and no == 0
