"""Pins of the oracle env step with the fixed-lag SLAM backbone in the loop (CPU only).

The paper's SLAM of Sec. III-D matches each scan against the log-odds grid, integrates the aligned scan
with a weight that follows the match score, and keeps a fixed-lag graph of poses whose newest-pose
covariance is the uncertainty of the reward (Sec. III-E) and observation (Eq. 3).  The composed step
(oracle/fixedlag_env.py, readings F1-F7) is pinned by closed forms of special cases:
  * an empty map: the first scan goes in at the prediction with the floor weight, cell by cell along
    an axis ray (the increments floor((w_q l + 128) / 256) at w_q = 128);
  * a map that already holds the world: a prediction one cell off is pulled back onto the true pose;
  * a robot at rest with no returns: the window slides and the newest covariance is the prior plus one
    odometry covariance per step, diag(var0 + t Q), for any window length;
  * a straight drive with no returns inside the first window: the newest covariance equals the
    closed form of a linear chain with a lever arm, Sigma_t = [[(a + t q) I + (t^2 b + r S2) u u^T,
    (t b + r S1) u], [., b + t r]], S1 = t (t - 1) / 2, S2 = (t - 1) t (2 t - 1) / 6, u = d (-sin, cos);
  * the reward is Eq. (7) with U_{t-1}, U_t = cbrt(det Sigma) of those covariances.
"""
import math

import numpy as np
import pytest

from paper_2603_25834_amd import synth

CELL = 0.0625   # binary-exact cell size, so positions on cell centres are exact in FP32


def f32(v):
    return float(np.float32(v))


def scene(O, poses, block=True, s=64, **over):
    from oracle.fixedlag_env import FixedLagOracleEnv
    occ = np.zeros((s, s), bool)
    occ[0, :] = occ[-1, :] = occ[:, 0] = occ[:, -1] = True
    if block:
        occ[20:26, 30:41] = True
    p = dict(synth.ENV_DEFAULTS)
    p.update(synth.PAPER_MODE)
    p.update(n_rays=128, cell_m=CELL, r_max_m=3.0, loop_closure=0, range_sigma_m=0.0, range_quant_m=0.0,
             r_min_m=0.0, d_crash_m=0.0, episode_len=0, lag_len=10, slam_backend=1)
    p.update(over)
    words = synth.pack_bits(occ)
    n = len(poses)
    env = FixedLagOracleEnv(p, np.full(n, s, np.int32), np.tile(words, n), np.arange(n, dtype=np.int64) * len(words))
    env.reset(np.array(poses, np.float32))
    return env, occ, p


def step(env, a=(0.0, 0.0)):
    n = env.n
    act = np.tile(np.array(a, np.float32), (n, 1))
    return env.step(act, np.zeros((n, 5), np.float32))


def test_first_scan_enters_an_empty_map_at_the_floor_weight(oracle_mod):
    """Robot at the centre of cell (10, 20) facing +x; ray 64 (straight ahead) meets the block's face at
    x = 30.  Empty map: every candidate scores 0, so the scan goes in at the prediction with weight
    0.5: w_q = 128, MISS floor((128 (-102) + 128) / 256) = -51, HIT floor((128 * 218 + 128) / 256) = 109."""
    env, occ, p = scene(oracle_mod, [((10.5) * CELL, (20.5) * CELL, 0.0)])
    step(env)
    row = env.belief.reshape(64, 64)[20]
    assert np.all(row[10:30] == -51)
    assert row[30] == 109
    assert row[31] == 0 and row[9] == 0   # behind the robot: outside the 180-degree fan
    # no motion, no noise: the estimate is the prediction, the pose itself
    assert env.est[0].tolist() == [10.5 * CELL, 20.5 * CELL, 0.0]
    assert tuple(env.match[0][:3]) == (-4, -4, -5)   # all-zero scores: the first candidate (ignored, w = 0)


def test_a_known_map_pulls_the_estimate_back(oracle_mod):
    """The grid holds the world (occupied +896, free -896); the robot faces the right wall 0.8 m away (so
    x is observable, not only y) and the estimate starts one cell to the right of the true pose.  The
    match is the candidate one step back in x and the estimate lands on the true pose exactly."""
    env, occ, p = scene(oracle_mod, [((50.5) * CELL, (30.5) * CELL, 0.0)])
    env.belief[:] = np.where(occ, 896, -896).astype(np.int16).reshape(-1)
    env.est[0] = np.array([51.5 * CELL, 30.5 * CELL, 0.0], np.float32)
    step(env)
    bi, bj, bk, best, second, used = env.match[0]
    assert (bi, bj, bk) == (-1, 0, 0)
    # nearly every return's endpoint lies in an occupied cell (a diagonal endpoint on a cell corner may
    # round into its free neighbour)
    assert best >= 0.95 * 896 * used and best > second
    assert env.est[0].tolist() == [50.5 * CELL, 30.5 * CELL, 0.0]


@pytest.mark.parametrize("lag", [2, 3, 10])
def test_resting_robot_without_returns(oracle_mod, lag):
    """r_max 0.3 m in the open: no ray returns, so no scan factor carries information and every
    candidate ties; at rest the window is a motionless chain and its newest covariance is
    diag(var0 + t Q) whatever the window length (the prior of a sliding window is the oldest pose's
    covariance from when it was newest).  The reward is Eq. (7) with U = cbrt(det)."""
    O = oracle_mod
    env, occ, p = scene(O, [(32.5 * CELL, 40.5 * CELL, 0.3)], block=False, r_max_m=0.3, lag_len=lag)
    a, b = f32(p["var0_xy"]), f32(p["var0_th"])
    q, r_ = f32(p["sigma_x"]) ** 2, f32(p["sigma_th"]) ** 2
    u_prev = (a * a * b) ** (1.0 / 3.0)
    for t in range(1, 8):
        o = step(env)
        want = np.array([a + t * q, 0.0, 0.0, a + t * q, 0.0, b + t * r_])
        got = env.cov[0].astype(np.float64)
        assert np.allclose(got, want, rtol=1e-6, atol=1e-12), (t, got, want)
        u = ((a + t * q) ** 2 * (b + t * r_)) ** (1.0 / 3.0)
        assert env.u_prev[0] == pytest.approx(u, rel=1e-6)
        want_r = O.paper_reward(p, False, float(o.dcells[0]), u_prev, float(env.u_prev[0]), float(o.d_min[0]))
        assert o.reward[0] == want_r
        u_prev = float(env.u_prev[0])
        assert env.match[0][5] == 0            # no returns
        assert env.count[0] == min(t + 1, lag)
    # the estimate never moved
    assert env.est[0].tolist() == [f32(32.5 * CELL), f32(40.5 * CELL), f32(0.3)] or \
        np.allclose(env.est[0], [32.5 * CELL, 40.5 * CELL, 0.3], atol=2e-4)


def test_straight_drive_covariance_closed_form(oracle_mod):
    """Driving straight along +x without returns, within the first window (no sliding): the newest
    pose's covariance of the Gauss-Newton window equals the closed form of the linear chain (the
    heading error swings the position along u = d (-sin th, cos th) = (0, d))."""
    O = oracle_mod
    env, occ, p = scene(O, [(20.5 * CELL, 32.5 * CELL, 0.0)], block=False, r_max_m=0.3, lag_len=10)
    a, b = f32(p["var0_xy"]), f32(p["var0_th"])
    q, r_ = f32(p["sigma_x"]) ** 2, f32(p["sigma_th"]) ** 2
    d = f32(np.float32(0.25) * np.float32(p["dt"]))
    for t in range(1, 8):
        step(env, (0.25, 0.0))
        s1, s2 = t * (t - 1) / 2.0, (t - 1) * t * (2 * t - 1) / 6.0
        yy = (a + t * q) + (t * t * b + r_ * s2) * d * d
        yt = (t * b + r_ * s1) * d
        want = np.array([a + t * q, 0.0, 0.0, yy, yt, b + t * r_])
        got = env.cov[0].astype(np.float64)
        assert np.allclose(got, want, rtol=1e-6, atol=1e-12), (t, got, want)
    # the estimate advanced by d per step (the prediction, quantised to 1/65536 cell)
    assert env.est[0][0] == pytest.approx(20.5 * CELL + 7 * d, abs=7 * CELL / 65536.0)
