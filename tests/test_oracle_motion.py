"""Pins of the oracle's motion mean: the true pose and the filter's estimate (CPU only).

Paper passage: the robot moves under the continuous action (v, w) of Sec. III-C
(Eq. 4) and the pose estimate follows the motion model that the odometry
factors of Sec. III-D are derived from (no model is printed; the reading is
the Euler unicycle with the heading at the start of the step, additive
world-frame noise on the true pose, the commanded motion in the filter).

The inputs are chosen so that FP32 arithmetic is exact (steps of 2^-4 m,
noise scales that are powers of two, headings on table steps whose cosine and
sine are 0 or +-1), so the expected values are closed forms in exact
arithmetic.  A general heading is checked against FP64 trigonometry.  Each
case is built so that a swapped cosine and sine, the post-step heading, a
wrong noise column or a missing wrap changes the result.
"""
import math

import numpy as np
import pytest

from paper_2603_25834_amd import synth

TWO_PI_F32 = float(np.float32(6.28318530717959))


def open_room(O, poses, s=64, cell=0.1, **over):
    """An empty s x s room (one-cell border wall), one robot per pose."""
    occ = np.zeros((s, s), bool)
    occ[0, :] = occ[-1, :] = occ[:, 0] = occ[:, -1] = True
    p = dict(synth.ENV_DEFAULTS)
    p.update(n_rays=180, cell_m=cell, r_max_m=5.0, loop_closure=0, dt=0.125)
    p.update(over)
    words = synth.pack_bits(occ)
    n = len(poses)
    env = O.OracleEnv(p, np.full(n, s, np.int32), np.tile(words, n), np.arange(n, dtype=np.int64) * len(words))
    env.reset(np.array(poses, np.float32))
    return env


def quantised_heading(theta: float) -> float:
    """The table heading of theta: 2 pi k / 46080 with k = rint(theta * (float)(46080 / 2 pi)) mod 46080,
    the product taken in FP32 (the heading quantisation of the traversal's direction table)."""
    k_ang = np.float32(46080.0 / (2.0 * math.pi))
    k = int(np.rint(np.float32(theta) * k_ang)) % 46080
    return 2.0 * math.pi * k / 46080.0


@pytest.mark.parametrize("theta,axis,sign", [(0.0, 0, 1.0), (math.pi / 2, 1, 1.0), (-math.pi, 0, -1.0),
                                             (-math.pi / 2, 1, -1.0)])
def test_straight_line_along_axes_is_exact(oracle_mod, theta, axis, sign):
    """omega = 0, no noise, heading on an axis: after t steps the pose moved t d along that axis only,
    exactly (d = 0.5 m/s x 0.125 s = 2^-4 m), and the estimate equals it."""
    start = {0: (1.0, 3.05), 1: (1.55, 0.5)}[axis]
    if sign < 0:
        start = {0: (5.5, 3.05), 1: (1.55, 5.5)}[axis]
    env = open_room(oracle_mod, [(start[0], start[1], theta)], sigma_x=0.0, sigma_y=0.0, sigma_th=0.0)
    act = np.array([[0.5, 0.0]], np.float32)
    g = np.zeros((1, 5), np.float32)
    th32 = float(np.float32(theta))
    for t in range(1, 61):
        out = env.step(act, g)
        assert out.collided[0] == 0
        want = [np.float32(start[0]), np.float32(start[1])]
        want[axis] = np.float32(want[axis] + sign * 0.0625 * t)
        assert env.pose[0, 0] == want[0] and env.pose[0, 1] == want[1], (t, env.pose[0], want)
        assert env.pose[0, 2] == np.float32(th32)
        assert np.array_equal(env.est[0], env.pose[0])


def test_general_heading_matches_fp64_trigonometry(oracle_mod):
    """A heading off the axes: the displacement per step is d (cos, sin) of the quantised heading,
    checked against FP64 cos / sin to FP32 accumulation accuracy over 40 steps."""
    theta = 0.3
    x0, y0 = 1.0, 1.0
    env = open_room(oracle_mod, [(x0, y0, theta)], sigma_x=0.0, sigma_y=0.0, sigma_th=0.0)
    act = np.array([[0.5, 0.0]], np.float32)
    g = np.zeros((1, 5), np.float32)
    tq = quantised_heading(theta)
    assert abs(tq - theta) < 7e-5
    for t in range(1, 41):
        env.step(act, g)
        wx = x0 + t * 0.0625 * math.cos(tq)
        wy = y0 + t * 0.0625 * math.sin(tq)
        tol = t * (3e-7 + 0.0625 * 2.0 ** -14)
        assert abs(float(env.pose[0, 0]) - wx) < tol and abs(float(env.pose[0, 1]) - wy) < tol, t
        assert np.array_equal(env.est[0], env.pose[0])
    # a swap of cosine and sine would have moved x by 40 d sin(0.3) instead
    assert abs(float(env.pose[0, 0]) - (x0 + 40 * 0.0625 * math.sin(tq))) > 1.0


def test_turning_uses_the_heading_before_the_step(oracle_mod):
    """From heading 0 with omega = 1 rad/s: the first step moves along +x exactly and only then turns
    (phi = 0.125 rad); the second step moves along the turned heading."""
    env = open_room(oracle_mod, [(2.0, 3.0, 0.0)], sigma_x=0.0, sigma_y=0.0, sigma_th=0.0)
    act = np.array([[0.5, 1.0]], np.float32)
    g = np.zeros((1, 5), np.float32)
    env.step(act, g)
    assert env.pose[0, 0] == np.float32(2.0625) and env.pose[0, 1] == np.float32(3.0)
    assert env.pose[0, 2] == np.float32(0.125)
    assert np.array_equal(env.est[0], env.pose[0])
    env.step(act, g)
    tq = quantised_heading(0.125)
    tol = 3e-7 + 0.0625 * 2.0 ** -14  # FP32 rounding + the table's 1/16384 quantum
    assert abs(float(env.pose[0, 0]) - (2.0625 + 0.0625 * math.cos(tq))) < tol
    assert abs(float(env.pose[0, 1]) - (3.0 + 0.0625 * math.sin(tq))) < tol
    assert env.pose[0, 2] == np.float32(0.25)
    assert np.array_equal(env.est[0], env.pose[0])


def test_noise_columns_enter_the_true_pose_only(oracle_mod):
    """One step with distinct exact draws: x gets sigma_x g0, y gets sigma_y g1, theta gets
    sigma_th g2; the loop-closure columns g3, g4 are unused with loop closure off; the estimate
    integrates the commanded motion without noise."""
    env = open_room(oracle_mod, [(2.0, 3.0, 0.0)], sigma_x=0.25, sigma_y=0.125, sigma_th=0.0625)
    g = np.array([[0.5, -0.75, 0.25, 7.0, -9.0]], np.float32)
    env.step(np.array([[0.5, 0.0]], np.float32), g)
    assert env.pose[0, 0] == np.float32(2.0 + 0.0625 + 0.125)
    assert env.pose[0, 1] == np.float32(3.0 - 0.09375)
    assert env.pose[0, 2] == np.float32(0.015625)
    assert env.est[0, 0] == np.float32(2.0625) and env.est[0, 1] == np.float32(3.0)
    assert env.est[0, 2] == np.float32(0.0)
    # the noise-free estimate keeps integrating the commanded motion along its own heading
    for t in range(2, 21):
        env.step(np.array([[0.5, 0.0]], np.float32), g)
        assert env.est[0, 0] == np.float32(2.0 + 0.0625 * t) and env.est[0, 1] == np.float32(3.0)
        assert env.est[0, 2] == np.float32(0.0)
    # the true heading drifted by 20 x sigma_th g2 and its position followed that heading
    assert env.pose[0, 2] == np.float32(20 * 0.015625)


@pytest.mark.parametrize("theta,omega", [(3.1, 1.0), (-3.1, -1.0), (3.0, 1.0)])
def test_heading_wraps_into_minus_pi_pi(oracle_mod, theta, omega):
    """theta + phi past +-pi comes back by one turn (FP32 2 pi), for the true pose and the estimate."""
    env = open_room(oracle_mod, [(3.0, 3.0, theta)], sigma_x=0.0, sigma_y=0.0, sigma_th=0.0)
    env.step(np.array([[0.0, omega]], np.float32), np.zeros((1, 5), np.float32))
    raw = float(np.float32(np.float32(theta) + np.float32(omega * 0.125)))
    want = raw
    if raw >= math.pi:
        want = raw - TWO_PI_F32
    elif raw < -math.pi:
        want = raw + TWO_PI_F32
    got = float(env.pose[0, 2])
    assert -math.pi <= got < math.pi
    assert abs(got - want) < 1e-6
    assert abs(math.remainder(got - (theta + omega * 0.125), 2 * math.pi)) < 1e-6
    assert env.est[0, 2] == env.pose[0, 2]
    if abs(theta + omega * 0.125) > math.pi:
        assert abs(got - (theta + omega * 0.125)) > 6.0
