"""Oracle of the env step with the fixed-lag SLAM backbone in the loop (arXiv 2603.25834, Sec. III-D).

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU-baseline leg, never by the
product path.  It composes two pinned oracles: the C oracle step (action, true motion and collision,
the predicted estimate, the visit bookkeeping of Eq. (9) and the LiDAR march with the sensor model of
Sec. IV-A; `slam_backend = 1` stops it there) and slam_ref (scan matching, the scan factor, the
weighted map integration and the Gauss-Newton window with the newest pose's covariance); the reward is
the oracle's Eq. (7) with U_t from the window's covariance.

The paper runs scan matching, integration and a fixed-lag graph (Sec. III-D) and gives no rules for
how they are wired together; the readings taken here (the library follows the same ones):

  F1  Front end.  The predicted pose is the previous estimate moved by the commanded motion (the env's
      unicycle prediction, FP32, table trigonometry).  Its Q16 position and heading index are the
      centre of the correlative search over the robot's log-odds grid; the scan is the reported ranges
      of the rays whose true march hit (Q16 cells), the others have no return.
  F2  Alignment.  With match weight w = q m > 0 (slam_ref S4) the aligned pose is the best candidate,
      else (an empty or featureless map, no returns) the prediction itself.  The estimate becomes the
      aligned pose: x = ax c / 65536, y likewise, theta = wrap(2 pi h / 46080), formed in FP64 and
      stored in FP32.  So the estimate, the matches and the map are integer-exact functions of the
      inputs; the graph below only yields the covariance.
  F3  Window.  The last L poses (L >= 2), FP64: a prior on the oldest, odometry factors between
      consecutive poses (the commanded motion (d, 0, phi) in the earlier pose's frame, zero when the
      move was blocked, information diag(1 / sigma_x^2, 1 / sigma_y^2, 1 / sigma_th^2) of the odometry
      noise), and a scan factor on each pose added by a step (the aligned pose, information
      w diag(1 / s_xy^2, 1 / s_xy^2, 1 / s_th^2)).  After a reset the window is the initial pose with the
      prior (initial pose, 1 / var0) and no scan factor.
  F4  Sliding.  When a step adds a pose to a full window the oldest pose leaves; the new oldest keeps
      its current estimate as the prior mean with the inverse diagonal of the covariance it had when
      it was the newest pose as the prior information (a diagonal stand-in for marginalisation).
  F5  Solve.  The new pose starts at the aligned pose, the others at their last estimates; K
      Gauss-Newton steps (slam_ref S6); Sigma_t = the newest pose's covariance; the env's covariance
      entries are its FP32 values and U_t = cbrt(det Sigma_t) of those (as in the EKF mode).
  F6  Integration.  The scan is cast into the grid from the aligned pose (slam_ref S8) with weight
      w_int = floor + (1 - floor) w, w_q = rint(256 w_int): the paper weights the aligned scan by the
      match score, and the floor lets an empty map receive its first scans.
  F7  Reward and observation: Eq. (7) with U_{t-1}, U_t as above (reward_mode 1 is required), the
      observation of Eq. (3).  The map entropy is not tracked (Eq. (7) does not use it).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O
from oracle import slam_ref as S

NANG = 46080


class FixedLagOracleEnv:
    """A batch of robots stepped with the fixed-lag backbone (F1-F7)."""

    def __init__(self, params: dict, sides, world, world_off):
        p = dict(params)
        p["slam_backend"] = 1
        if int(p.get("reward_mode", 0)) != 1 or int(p.get("loop_closure", 0)) != 0:
            raise ValueError("the fixed-lag backbone needs reward_mode 1 and no EKF loop closure")
        self.p = p
        self.env = O.OracleEnv(p, sides, world, world_off)
        self.n, self.R = self.env.n, self.env.R
        self.L = int(p["lag_len"])
        if self.L < 2:
            raise ValueError("lag_len must be >= 2")
        self.K = int(p["gn_iters"])
        self.W, self.V = int(p["csm_W"]), int(p["csm_V"])
        self.sxy, self.sh = int(p["csm_step_xy_q"]), int(p["csm_step_h"])
        f32 = lambda k: float(np.float32(p[k]))
        self.cell = f32("cell_m")
        self.l_hit = O.logodds_q(p["l_hit"])
        self.l_miss = O.logodds_q(p["l_miss"])
        self.l_clamp = O.logodds_q(p["l_clamp"])
        self.rmax_q = int(math.floor(f32("r_max_m") / self.cell * 65536.0 + 0.5))   # llround of the step
        fov = int(p.get("fov_steps", 0))
        fan = fov if 0 < fov < NANG else NANG
        step_ang = fan // self.R
        ray0 = 0 if fan == NANG else NANG - fan // 2
        self.a_off = ((ray0 + np.arange(self.R) * step_ang) % NANG).astype(np.int32)
        self.odo_info = np.array([1.0 / (f32(k) * f32(k)) for k in ("sigma_x", "sigma_y", "sigma_th")])
        sxy, sth = f32("scan_sigma_xy_m"), f32("scan_sigma_th")
        self.scan_info = np.array([1.0 / (sxy * sxy), 1.0 / (sxy * sxy), 1.0 / (sth * sth)])
        self.floor = f32("int_weight_floor")
        self.var0 = np.array([f32("var0_xy"), f32("var0_xy"), f32("var0_th")])
        n, L = self.n, self.L
        self.x = np.zeros((n, L, 3))
        self.prior = np.zeros((n, 6))
        self.odo = np.zeros((n, L - 1, 6))
        self.scan = np.zeros((n, L, 6))
        self.sig = np.zeros((n, L, 3))
        self.count = np.zeros(n, np.int64)
        self.match = np.zeros((n, 6), np.int64)
        self.trig = S._trig()

    # ---------------------------------------------------------------- state views
    def __getattr__(self, k):
        if k in ("pose", "est", "cov", "belief", "step_ct", "u_prev", "draws", "visit_last", "h_q", "sides",
                 "cell_off"):
            return getattr(self.env, k)
        raise AttributeError(k)

    def reset(self, init_pose, mask=None):
        self.env.reset(init_pose, mask)
        ip = np.asarray(init_pose, np.float32).reshape(self.n, 3)
        rows = range(self.n) if mask is None else np.flatnonzero(np.asarray(mask))
        for r in rows:
            self.count[r] = 1
            self.x[r] = 0.0
            self.x[r, 0] = ip[r].astype(np.float64)
            self.prior[r] = np.concatenate([ip[r].astype(np.float64), 1.0 / self.var0])
            self.odo[r] = 0.0
            self.scan[r] = 0.0
            self.sig[r] = 0.0
            self.sig[r, 0] = self.var0

    # ---------------------------------------------------------------- the step
    def _aligned_estimate(self, ax: int, ay: int, ah: int) -> np.ndarray:
        """F2: the aligned pose in metres / radians (FP64)."""
        th = 2.0 * np.pi * ah / NANG
        th = th - 2.0 * np.pi * np.rint(th / (2.0 * np.pi))
        return np.array([ax / 65536.0 * self.cell, ay / 65536.0 * self.cell, th])

    def step(self, actions, noise, threads: int = 0):
        o = self.env.step(actions, noise, threads)   # motion, prediction, visits, march (F1)
        e = self.env
        grids = e.belief
        for r in range(self.n):
            s = int(e.sides[r])
            co = int(e.cell_off[r])
            grid = grids[co:co + s * s].reshape(s, s)
            est = e.est[r]
            px, py = O.to_q16(float(est[0]), self.cell), O.to_q16(float(est[1]), self.cell)
            ph = int(O.heading_index(float(est[2])))
            rho = np.where(o.hit_cell[r] >= 0, o.rho_q[r], -1).astype(np.int64)
            m = S.csm_match(grid, px, py, ph, rho, self.a_off, self.W, self.V, self.sxy, self.sh, self.trig)
            self.match[r] = m
            bi, bj, bk, best, second, used = m
            w = S.match_weight(best, second, used, float(self.l_clamp))
            if w > 0.0:
                ax, ay, ah = px + bi * self.sxy, py + bj * self.sxy, (ph + bk * self.sh) % NANG
            else:
                ax, ay, ah = px, py, ph
            z = self._aligned_estimate(ax, ay, ah)
            e.est[r] = z.astype(np.float32)
            # F3 / F4: the window takes the new pose
            c = int(self.count[r])
            if c == self.L:
                self.x[r, :-1] = self.x[r, 1:].copy()
                self.odo[r, :-1] = self.odo[r, 1:].copy()
                self.scan[r, :-1] = self.scan[r, 1:].copy()
                self.sig[r, :-1] = self.sig[r, 1:].copy()
                self.prior[r] = np.concatenate([self.x[r, 0], 1.0 / self.sig[r, 0]])
                c -= 1
            d, phi = float(o.odo[r, 0]), float(o.odo[r, 1])
            self.odo[r, c - 1] = np.concatenate([[d, 0.0, phi], self.odo_info])
            self.scan[r, c] = np.concatenate([z, w * self.scan_info])
            self.x[r, c] = z
            c += 1
            self.count[r] = c
            x, sigma = S.fixedlag_solve(self.x[r, :c], self.prior[r], self.odo[r, :c - 1], self.scan[r, :c], self.K)
            self.x[r, :c] = x
            self.sig[r, c - 1] = np.diag(sigma)
            e.cov[r] = np.array([sigma[0, 0], sigma[0, 1], sigma[0, 2], sigma[1, 1], sigma[1, 2], sigma[2, 2]],
                                np.float32)
            # F6: weighted integration from the aligned pose
            w_q = int(np.rint(256.0 * (self.floor + (1.0 - self.floor) * w)))
            new, coded = S.integrate(grid, ax, ay, ah, rho, self.a_off, self.rmax_q, self.l_hit, self.l_miss,
                                     self.l_clamp, w_q=w_q)
            grid[:, :] = new
            o.counters[r, 2] = coded
            # F7: Eq. (7) with U_t of the window
            u = O.uncertainty(e.cov[r])
            o.reward[r] = O.paper_reward(self.p, bool(o.collided[r]), float(o.dcells[r]), float(e.u_prev[r]), u,
                                         float(o.d_min[r]))
            e.u_prev[r] = u
        return o

    def observe(self, ranges, crop_side: int = 64):
        return self.env.observe(ranges, crop_side)
