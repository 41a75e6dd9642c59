"""Seeded synthetic inputs for the batched Active-SLAM environment step.

This module holds input generation only -- worlds, start poses, actions and
the standard-normal draws the step consumes -- and none of the method's
arithmetic.  Both the GPU path and the CPU oracle take their inputs from here,
by value.

The worlds stand in for the paper's indoor Isaac Sim scenes (walls and turns,
arXiv 2603.25834 Sec. IV-A): square occupancy grids with a one-cell border
wall, axis-aligned rectangular obstacles and thin walls.  Each robot's world is
drawn from its own generator ``default_rng([seed, 0, i])``, so any subset of a
batch can be regenerated on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Environment parameters shared by every workload (units: m, rad, s, nats).
ENV_DEFAULTS = dict(
    dt=0.1, v_max=0.5, w_max=1.0,
    sigma_x=0.02, sigma_y=0.02, sigma_th=0.01,
    var0_xy=1e-4, var0_th=1e-4,
    lc_cell_m=0.5, lc_radius_m=0.5, lc_sigma_m=0.05, lc_gap=50,
    l_hit=0.85, l_miss=-0.4, l_clamp=3.5,
    w_entropy=1.0, w_dopt=1.0, lambda_col=10.0,
    episode_len=0,
    # sensor model and the paper's reward (zeros: full-circle fan, exact ranges, workload reward)
    fov_steps=0, reward_mode=0, r_min_m=0.0, range_sigma_m=0.0, range_quant_m=0.0,
    d_crash_m=0.0, d_full_m=0.0, lambda_explore=0.0, lambda_abs=0.0, lambda_delta=0.0, u_hi=0.0, kappa=0.0,
    # SLAM backend: 0 the EKF; 1 the fixed-lag graph of Sec. III-D (window, Gauss-Newton steps, scan-match
    # lattice of 9 x 9 x 11 candidates one cell and 0.5 degree apart, scan-factor sigmas, integration floor)
    slam_backend=0, lag_len=10, gn_iters=3, csm_W=4, csm_V=5, csm_step_xy_q=65536, csm_step_h=64,
    scan_sigma_xy_m=0.05, scan_sigma_th=0.02, int_weight_floor=0.5,
)

# The paper's sensor, collision rule and reward (Sec. IV-A, Sec. III-E): 128 rays over the 180-degree
# front field of view, 0.1 m minimum range, N(0, 0.01 m) range noise, 0.01 m quantisation, collision
# closer than 0.15 m, Eq. (7); v in [0, 0.4] m/s (Eq. 4), 2048-step episodes.  The reward weights are
# not printed in the paper; these values are readings.
PAPER_MODE = dict(
    n_rays=128, fov_steps=23040, reward_mode=1, r_min_m=0.1, range_sigma_m=0.01, range_quant_m=0.01,
    d_crash_m=0.15, d_full_m=0.5, lambda_explore=1.0, lambda_abs=0.1, lambda_delta=10.0, u_hi=0.05,
    kappa=0.005, v_max=0.4, episode_len=2048,
)


@dataclass
class Workload:
    name: str
    n_robots: int
    sides: tuple            # grid sides to draw from (uniformly)
    cell_m: float
    n_rays: int
    r_max_m: float
    steps: int
    loop_closure: int
    rects: tuple            # (min, max) rectangle count at side 256 (scaled by (s/256)^2)
    rect_side: tuple        # (min, max) rectangle side, cells
    thin_walls: tuple       # (min, max) thin wall count at side 256 (scaled)
    thin_len: tuple         # (min, max) thin wall length, cells
    scale_counts: bool = True
    extra: dict = field(default_factory=dict)

    def params(self) -> dict:
        p = dict(ENV_DEFAULTS)
        p.update(n_rays=self.n_rays, cell_m=self.cell_m, r_max_m=self.r_max_m,
                 loop_closure=self.loop_closure)
        p.update(self.extra)
        return p


WORKLOADS = {
    # 16 robots in 64x64 worlds at 0.1 m, 180 rays over 360 deg, 5 m, 100 steps.
    "small_16x64": Workload("small_16x64", 16, (64,), 0.1, 180, 5.0, 100, 0,
                            rects=(4, 8), rect_side=(3, 15), thin_walls=(0, 0), thin_len=(0, 0),
                            scale_counts=False),
    # 750 robots in 256x256 worlds at 0.05 m, 360 rays, 10 m, 1000 steps, loop closure.
    "paper_750x256": Workload("paper_750x256", 750, (256,), 0.05, 360, 10.0, 1000, 1,
                              rects=(20, 40), rect_side=(4, 24), thin_walls=(4, 8), thin_len=(16, 64)),
    # 4096 robots, grid side uniform in {128,...,512}, 360 rays, 10 m, 1000 steps.
    "ragged_4096": Workload("ragged_4096", 4096, (128, 192, 256, 384, 512), 0.05, 360, 10.0, 1000, 1,
                            rects=(20, 40), rect_side=(4, 24), thin_walls=(4, 8), thin_len=(16, 64)),
    # The 750-robot scene with the paper's sensor model, collision rule and reward.
    "paper_sensor_750x256": Workload("paper_sensor_750x256", 750, (256,), 0.05, 128, 10.0, 1000, 0,
                                     rects=(20, 40), rect_side=(4, 24), thin_walls=(4, 8), thin_len=(16, 64),
                                     extra=dict(PAPER_MODE)),
    # The paper's mode with the fixed-lag SLAM backbone in the loop instead of the EKF.
    "paper_fixedlag_750x256": Workload("paper_fixedlag_750x256", 750, (256,), 0.05, 128, 10.0, 1000, 0,
                                       rects=(20, 40), rect_side=(4, 24), thin_walls=(4, 8), thin_len=(16, 64),
                                       extra=dict(PAPER_MODE, slam_backend=1)),
    # 8192 robots in 512x512 worlds, 720 rays, 15 m.
    "full_8192x512": Workload("full_8192x512", 8192, (512,), 0.05, 720, 15.0, 1000, 1,
                              rects=(80, 160), rect_side=(4, 24), thin_walls=(16, 32), thin_len=(16, 64),
                              scale_counts=False),
}


def draw_sides(w: Workload, seed: int, n: int | None = None) -> np.ndarray:
    n = w.n_robots if n is None else n
    rng = np.random.default_rng([seed, 7])
    return np.asarray(w.sides, np.int32)[rng.integers(0, len(w.sides), size=n)]


def draw_world(w: Workload, side: int, seed: int, i: int) -> np.ndarray:
    """Occupancy (bool [s, s], indexed [j, i] = [row y, column x]) of robot i."""
    rng = np.random.default_rng([seed, 0, i])
    s = int(side)
    occ = np.zeros((s, s), bool)
    occ[0, :] = occ[-1, :] = True
    occ[:, 0] = occ[:, -1] = True
    f = (s / 256.0) ** 2 if w.scale_counts else 1.0
    k = int(round(rng.integers(w.rects[0], w.rects[1] + 1) * f))
    for _ in range(k):
        rw = int(rng.integers(w.rect_side[0], w.rect_side[1] + 1))
        rh = int(rng.integers(w.rect_side[0], w.rect_side[1] + 1))
        x0 = int(rng.integers(0, max(1, s - rw + 1)))
        y0 = int(rng.integers(0, max(1, s - rh + 1)))
        occ[y0:y0 + rh, x0:x0 + rw] = True
    if w.thin_walls[1] > 0:
        m = int(round(rng.integers(w.thin_walls[0], w.thin_walls[1] + 1) * f))
        for _ in range(m):
            ln = int(rng.integers(w.thin_len[0], w.thin_len[1] + 1))
            if rng.integers(0, 2):
                x0 = int(rng.integers(0, max(1, s - ln + 1)))
                y0 = int(rng.integers(0, s))
                occ[y0, x0:x0 + ln] = True
            else:
                x0 = int(rng.integers(0, s))
                y0 = int(rng.integers(0, max(1, s - ln + 1)))
                occ[y0:y0 + ln, x0] = True
    return occ


def pack_bits(occ: np.ndarray) -> np.ndarray:
    """Row-major bit packing: cell (i, j) -> bit j*s + i, little-endian 32-bit words."""
    b = np.packbits(occ.reshape(-1).astype(np.uint8), bitorder="little")
    return b.view("<u4").astype(np.uint32)


def draw_start(occ: np.ndarray, cell_m: float, seed: int, i: int) -> np.ndarray:
    """Uniform over free cells, uniform inside the inner 80% of the cell, heading U[-pi, pi)."""
    rng = np.random.default_rng([seed, 1, i])
    free = np.flatnonzero(~occ.reshape(-1))
    c = int(free[rng.integers(0, len(free))])
    s = occ.shape[0]
    ci, cj = c % s, c // s
    x = (ci + rng.uniform(0.1, 0.9)) * cell_m
    y = (cj + rng.uniform(0.1, 0.9)) * cell_m
    th = rng.uniform(-math.pi, math.pi)
    return np.array([x, y, th], np.float32)


@dataclass
class Batch:
    workload: Workload
    seed: int
    index: np.ndarray        # robot ids within the workload
    sides: np.ndarray        # int32 [n]
    world: np.ndarray        # uint32 ragged words
    world_off: np.ndarray    # int64 [n] word offsets
    start: np.ndarray        # float32 [n, 3]
    occ: list                # bool grids (kept for tests)


def make_batch(name: str, seed: int = 0, robots=None, keep_occ: bool = False) -> Batch:
    w = WORKLOADS[name]
    all_sides = draw_sides(w, seed)
    idx = np.arange(w.n_robots) if robots is None else np.asarray(robots, np.int64)
    sides = all_sides[idx].astype(np.int32)
    words, offs, starts, occs = [], [], np.zeros((len(idx), 3), np.float32), []
    off = 0
    for k, i in enumerate(idx):
        occ = draw_world(w, int(all_sides[i]), seed, int(i))
        pw = pack_bits(occ)
        words.append(pw)
        offs.append(off)
        off += len(pw)
        starts[k] = draw_start(occ, w.cell_m, seed, int(i))
        if keep_occ:
            occs.append(occ)
    return Batch(w, seed, idx, sides, np.concatenate(words).astype(np.uint32),
                 np.asarray(offs, np.int64), starts, occs)


def actions(name: str, seed: int, steps: int, robots=None) -> np.ndarray:
    """Actions [steps, n, 2]: v ~ U[0, 0.5] m/s, w ~ U[-1, 1] rad/s."""
    w = WORKLOADS[name]
    rng = np.random.default_rng([seed, 2])
    a = np.empty((steps, w.n_robots, 2), np.float32)
    a[..., 0] = rng.uniform(0.0, 0.5, size=(steps, w.n_robots))
    a[..., 1] = rng.uniform(-1.0, 1.0, size=(steps, w.n_robots))
    return a if robots is None else np.ascontiguousarray(a[:, np.asarray(robots)])


def noise_width(p: dict) -> int:
    """Normal draws per robot and step: odometry (x, y, theta), loop-closure fix (x, y), then one
    per ray when the range noise is on."""
    return 5 + (int(p["n_rays"]) if p.get("range_sigma_m", 0.0) > 0.0 else 0)


def noise(name: str, seed: int, steps: int, robots=None) -> np.ndarray:
    """Standard-normal draws [steps, n, noise_width]."""
    w = WORKLOADS[name]
    rng = np.random.default_rng([seed, 3])
    g = rng.standard_normal((steps, w.n_robots, noise_width(w.params())), dtype=np.float32)
    return g if robots is None else np.ascontiguousarray(g[:, np.asarray(robots)])


# ----------------------------------------------------------------- policy inputs

def policy_param_layout(n_scan: int = 360):
    """(name, shape) of the actor-critic's flat FP32 parameter vector, in order.

    Interface description shared by the library's binding and the tests: conv1
    [16,1,3,3]+[16], conv2 [32,16,3,3]+[32], fc1 [256, 8192+n_scan+12]+[256],
    fc2 [256,256]+[256], mean head [2,256]+[2], value head [1,256]+[1], log std [2]."""
    k1 = 32 * 16 * 16 + n_scan + 12
    return [("conv1.w", (16, 1, 3, 3)), ("conv1.b", (16,)), ("conv2.w", (32, 16, 3, 3)), ("conv2.b", (32,)),
            ("fc1.w", (256, k1)), ("fc1.b", (256,)), ("fc2.w", (256, 256)), ("fc2.b", (256,)),
            ("mu.w", (2, 256)), ("mu.b", (2,)), ("v.w", (1, 256)), ("v.b", (1,)), ("log_std", (2,))]


def init_policy_params(n_scan: int = 360, seed: int = 0) -> np.ndarray:
    """Seeded fan-in-scaled uniform initialisation, float32 flat vector; log std starts at -0.5."""
    rng = np.random.default_rng([seed, 10])
    parts = []
    for name, shp in policy_param_layout(n_scan):
        n = int(np.prod(shp))
        if name == "log_std":
            parts.append(np.full(n, -0.5, np.float32))
        elif name.endswith(".b"):
            parts.append(rng.uniform(-0.05, 0.05, n).astype(np.float32))
        else:
            bound = 1.0 / math.sqrt(int(np.prod(shp[1:])))
            parts.append(rng.uniform(-bound, bound, n).astype(np.float32))
    return np.concatenate(parts)


def recurrent_param_layout(n_scan: int = 128):
    """(name, shape) of the recurrent actor-critic's flat FP32 parameter vector: the feed-forward
    layout with FC2 replaced by a GRU of 256 units (input and hidden weights [768, 256], gate rows in
    the order reset / update / new, then their biases [768] each)."""
    out = []
    for name, shp in policy_param_layout(n_scan):
        if name == "fc2.w":
            out += [("gru.w_ih", (768, 256)), ("gru.w_hh", (768, 256)), ("gru.b_ih", (768,)), ("gru.b_hh", (768,))]
        elif name != "fc2.b":
            out.append((name, shp))
    return out


def init_recurrent_params(n_scan: int = 128, seed: int = 0) -> np.ndarray:
    """Seeded initialisation of the recurrent layout: as init_policy_params, GRU weights and biases
    uniform in +-1/sqrt(256)."""
    rng = np.random.default_rng([seed, 12])
    parts = []
    for name, shp in recurrent_param_layout(n_scan):
        n = int(np.prod(shp))
        if name == "log_std":
            parts.append(np.full(n, -0.5, np.float32))
        elif name.startswith("gru."):
            parts.append(rng.uniform(-1.0 / 16.0, 1.0 / 16.0, n).astype(np.float32))
        elif name.endswith(".b"):
            parts.append(rng.uniform(-0.05, 0.05, n).astype(np.float32))
        else:
            bound = 1.0 / math.sqrt(int(np.prod(shp[1:])))
            parts.append(rng.uniform(-bound, bound, n).astype(np.float32))
    return np.concatenate(parts)


def recurrent_batch(T: int, nb: int, n_scan: int = 128, seed: int = 0, reset_p: float = 0.05):
    """A synthetic rollout segment of T steps for nb robots (time-major [T, nb, ...]): the arrays of
    policy_batch, an entering hidden state h0 [nb, 256] in (-0.5, 0.5) and episode starts first [T, nb]
    (uint8, each step starts an episode with probability reset_p)."""
    d = policy_batch(T * nb, n_scan, seed)
    out = {k: v.reshape((T, nb) + v.shape[1:]) for k, v in d.items()}
    rng = np.random.default_rng([seed, 13])
    out["h0"] = rng.uniform(-0.5, 0.5, size=(nb, 256)).astype(np.float32)
    out["first"] = (rng.random((T, nb)) < reset_p).astype(np.uint8)
    return out


def policy_batch(n: int, n_scan: int = 360, seed: int = 0):
    """Synthetic PPO minibatch shaped like rollout data: belief crops (int16 log-odds made of
    hit/miss counts, clamped), normalised scans, pose/covariance states, actions, old log-probs,
    advantages and returns."""
    rng = np.random.default_rng([seed, 11])
    hits = rng.poisson(0.3, size=(n, 64, 64))
    misses = rng.poisson(1.5, size=(n, 64, 64)) * (rng.random((n, 64, 64)) < 0.6)
    crop = np.clip(218 * hits - 102 * misses, -896, 896).astype(np.int16)
    scan = rng.uniform(0.0, 1.0, size=(n, n_scan)).astype(np.float32)
    state = np.zeros((n, 12), np.float32)
    state[:, 0:2] = rng.uniform(0, 1, size=(n, 2))
    state[:, 2] = rng.uniform(-1, 1, size=n)
    var = rng.uniform(1e-4, 5e-2, size=(n, 3))
    cov = np.zeros((n, 3, 3))
    cov[:, [0, 1, 2], [0, 1, 2]] = var
    cxy = rng.uniform(-0.5, 0.5, size=n) * np.sqrt(var[:, 0] * var[:, 1])
    cov[:, 0, 1] = cov[:, 1, 0] = cxy
    state[:, 3:] = cov.reshape(n, 9)
    act = np.stack([rng.uniform(0, 0.5, n), rng.uniform(-1, 1, n)], 1).astype(np.float32)
    old_logp = rng.normal(-1.0, 0.3, size=n).astype(np.float32)
    adv = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    ret = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    return dict(crop=crop, scan=scan, state=state, act=act, old_logp=old_logp, adv=adv, ret=ret)
