"""Oracle of the fixed-lag SLAM backbone (arXiv 2603.25834, Sec. III-D): correlative scan matching
against the int16 log-odds grid, the scan factor it yields, and the Gauss-Newton solve of the
sliding-window pose graph with the marginal covariance of the newest pose.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU-baseline leg, never by the
product path.  Plain numpy: integer arithmetic for the matcher (exact), FP64 for the graph.

The paper states the method (a candidate lattice around the predicted pose scored on the grid; an
absolute pose measurement whose information is scaled by the normalised score and the margin to
the second-best candidate; a few Gauss-Newton iterations over odometry and scan factors; the
covariance of the newest pose as the last diagonal block of the inverse Hessian) but not its
constants or exact rules; the readings taken here are:

  S1  Scan: per ray the range rho_q (Q16 cells, < 0 = no return) and a heading offset a_r (heading
      steps of the 46080-step table, relative to the robot heading).  The endpoint under a pose
      (x, y in Q16 cells, heading index h) is x + ((rho_q * cos_q) >> 14), y + ((rho_q * sin_q) >> 14),
      with (cos_q, sin_q) the Q14 table entry of (h + a_r) mod 46080; its cell is (ex >> 16, ey >> 16).
  S2  Candidates: (x + i*step_xy, y + j*step_xy, h + k*step_h) for |i|, |j| <= W, |k| <= V; index
      ((k+V)(2W+1) + (j+W))(2W+1) + (i+W).  Score = sum of the log-odds of the endpoint cells of the
      rays with a return that fall inside the grid (an int32 sum).
  S3  Best = highest score, ties to the smallest index.  Second = highest score among candidates at
      lattice Chebyshev distance >= 2 from the best (the next separate peak), INT32_MIN if none.
  S4  Scan factor: the best pose in metres / radians; information diag(w / s_xy^2, w / s_xy^2,
      w / s_th^2) with w = q * m, q = clamp(best / (n_rays_used * L_max), 0, 1) the normalised score
      and m = clamp((best - second) / max(best, 1), 0, 1) the ambiguity margin (w = 0: no factor).
  S5  Graph over L poses: a prior on pose 0 (mean, diagonal information), odometry factors between
      consecutive poses (the relative motion in the frame of the earlier pose, diagonal
      information), scan factors (unary, diagonal information, zero = absent).  Residuals: prior
      and scan x - z with the angle wrapped to [-pi, pi]; odometry (R(th_i)^T (t_{i+1} - t_i) - u_t,
      wrap(th_{i+1} - th_i - u_th)).
  S6  K Gauss-Newton steps x <- x - H^{-1} g (H = sum J^T Omega J, g = sum J^T Omega r, analytic
      Jacobians), then H re-formed at the final estimate; Sigma = the last 3x3 block of H^{-1}.
  S7  wrap(a) = a - 2 pi rint(a / (2 pi)).
  S8  Confidence-weighted map integration: the scan is cast into the grid from the best candidate's
      pose by the exact traversal of the env step's map update (every cell a ray passes up to its
      range is a MISS, the cell where a ray with a return ends is a HIT unless the ray left the grid
      first, HIT beats MISS, rays without a return pass free space up to the maximum range), and each
      coded cell gets one saturating add of the log-odds increment scaled by the scan weight w of S4.
      w is quantised to w_q = rint(256 w) and the increment is floor((w_q l + 128) / 256): at w = 1 the
      update is the unweighted one, at w = 0 the grid is unchanged.  An aligned pose outside the grid
      leaves the grid unchanged.
"""
from __future__ import annotations

import numpy as np

NANG = 46080
INT32_MIN = -(2 ** 31)


def _trig():
    from oracle import oracle as O
    return O.trig_table()


# ------------------------------------------------------------------ correlative scan matching (S1-S3)

def csm_scores(grid: np.ndarray, px: int, py: int, ph: int, rho_q: np.ndarray, a_off: np.ndarray,
               W: int, V: int, step_xy: int, step_h: int, trig=None) -> np.ndarray:
    """Scores of every candidate, shape [2V+1, 2W+1, 2W+1] indexed [k+V, j+W, i+W] (S1, S2)."""
    cq, sq = trig if trig is not None else _trig()
    s = grid.shape[0]
    assert grid.shape == (s, s) and grid.dtype == np.int16
    n = 2 * W + 1
    out = np.zeros((2 * V + 1, n, n), np.int64)
    valid = rho_q >= 0
    rho = rho_q[valid].astype(np.int64)
    aoff = a_off[valid].astype(np.int64)
    G = grid.astype(np.int64)
    for k in range(-V, V + 1):
        h = np.mod(ph + k * step_h + aoff, NANG)
        dx = (rho * cq[h].astype(np.int64)) >> 14
        dy = (rho * sq[h].astype(np.int64)) >> 14
        for j in range(-W, W + 1):
            ey = py + j * step_xy + dy
            cy = ey >> 16
            for i in range(-W, W + 1):
                ex = px + i * step_xy + dx
                cx = ex >> 16
                inside = (cx >= 0) & (cx < s) & (cy >= 0) & (cy < s)
                out[k + V, j + W, i + W] = int(G[cy[inside], cx[inside]].sum())
    return out


def csm_match(grid, px, py, ph, rho_q, a_off, W, V, step_xy, step_h, trig=None):
    """(best_i, best_j, best_k, best_score, second_score, n_used) per S3."""
    sc = csm_scores(grid, px, py, ph, rho_q, a_off, W, V, step_xy, step_h, trig)
    flat = sc.reshape(-1)
    b = int(np.argmax(flat))          # first maximum = smallest index
    n = 2 * W + 1
    bk, rem = divmod(b, n * n)
    bj, bi = divmod(rem, n)
    kk, jj, ii = np.meshgrid(np.arange(2 * V + 1), np.arange(n), np.arange(n), indexing="ij")
    far = np.maximum(np.maximum(np.abs(ii - bi), np.abs(jj - bj)), np.abs(kk - bk)) >= 2
    second = int(sc[far].max()) if far.any() else INT32_MIN
    return bi - W, bj - W, bk - V, int(flat[b]), second, int((rho_q >= 0).sum())


# ------------------------------------------------------------------ scan factor (S4)

def scan_factor(best_i, best_j, best_k, best, second, n_used, px, py, ph, step_xy, step_h, cell_m, l_max,
                sig_xy, sig_th):
    """Measurement (x, y, theta) in metres / radians and the information diagonal."""
    x = (px + best_i * step_xy) / 65536.0 * cell_m
    y = (py + best_j * step_xy) / 65536.0 * cell_m
    h = (ph + best_k * step_h) % NANG
    th = wrap(2.0 * np.pi * h / NANG)
    w = match_weight(best, second, n_used, l_max)
    return np.array([x, y, th]), np.array([w / sig_xy ** 2, w / sig_xy ** 2, w / sig_th ** 2])


def match_weight(best, second, n_used, l_max) -> float:
    """w = q m of S4: the normalised score times the margin to the second peak."""
    q = 0.0 if n_used <= 0 else min(max(best / (n_used * float(l_max)), 0.0), 1.0)
    m = min(max((best - second) / max(float(best), 1.0), 0.0), 1.0)
    return q * m


# ------------------------------------------------------------------ weighted map integration (S8)

def weighted_increment(w_q: int, l: int) -> int:
    """round(w_q l / 256), halves up (S8)."""
    return (int(w_q) * int(l) + 128) >> 8


def integrate(grid: np.ndarray, px: int, py: int, ph: int, rho_q: np.ndarray, a_off: np.ndarray, rmax_q: int,
              l_hit: int, l_miss: int, l_clamp: int, match=None, step_xy: int = 0, step_h: int = 0,
              l_max: float = 1.0, w_q: int | None = None):
    """The grid after integrating the scan from the aligned pose (S8), and the number of coded cells.
    `match` = (best_i, best_j, best_k, best, second, n_used) of csm_match, or None for the update from
    (px, py, ph) itself at weight w_q (256, the unweighted update, when not given)."""
    from oracle import oracle as O
    cq, sq = _trig()
    s = grid.shape[0]
    if match is None:
        ax, ay, ah = px, py, ph
        w_q = 256 if w_q is None else int(w_q)
    else:
        bi, bj, bk, best, second, n_used = (int(v) for v in match)
        ax, ay, ah = px + bi * step_xy, py + bj * step_xy, (ph + bk * step_h) % NANG
        w_q = int(np.rint(256.0 * match_weight(best, second, n_used, l_max)))
    code = np.zeros((s, s), np.int8)
    for k in range(len(rho_q)):
        d = (ah + int(a_off[k])) % NANG
        ret = int(rho_q[k]) >= 0
        cells, _, _, end = O.walk(ax, ay, int(cq[d]), int(sq[d]), 16384, int(rho_q[k]) if ret else rmax_q, s,
                                  max_out=2 * s + 2)   # a walk inside an s x s grid visits at most 2 s + 1 cells
        if len(cells) == 0:
            continue
        code[cells[:, 1], cells[:, 0]] = np.maximum(code[cells[:, 1], cells[:, 0]], 1)
        if ret and end == 0:
            code[cells[-1, 1], cells[-1, 0]] = 2
    inc = np.where(code == 2, weighted_increment(w_q, l_hit), weighted_increment(w_q, l_miss))
    out = grid.astype(np.int64)
    out = np.where(code > 0, np.clip(out + inc, -l_clamp, l_clamp), out)
    return out.astype(np.int16), int((code > 0).sum())


# ------------------------------------------------------------------ fixed-lag graph (S5-S7)

def wrap(a):
    return a - 2.0 * np.pi * np.rint(a / (2.0 * np.pi))


def residuals(x: np.ndarray, prior: np.ndarray, odo: np.ndarray, scan: np.ndarray):
    """Stacked residuals and information diagonals of the window (S5).  x [L,3]; prior [6]; odo [L-1,6];
    scan [L,6]."""
    L = x.shape[0]
    res, info = [], []
    r = x[0] - prior[:3]
    r[2] = wrap(r[2])
    res.append(r); info.append(prior[3:])
    for i in range(L - 1):
        c, s = np.cos(x[i, 2]), np.sin(x[i, 2])
        dt = x[i + 1, :2] - x[i, :2]
        rel = np.array([c * dt[0] + s * dt[1], -s * dt[0] + c * dt[1]])
        r = np.array([rel[0] - odo[i, 0], rel[1] - odo[i, 1], wrap(x[i + 1, 2] - x[i, 2] - odo[i, 2])])
        res.append(r); info.append(odo[i, 3:])
    for i in range(L):
        if np.any(scan[i, 3:] != 0):
            r = x[i] - scan[i, :3]
            r[2] = wrap(r[2])
            res.append(r); info.append(scan[i, 3:])
    return res, info


def normal_equations(x, prior, odo, scan):
    """Dense H (3L x 3L) and g of the window at x, analytic Jacobians (S5, S6)."""
    L = x.shape[0]
    H = np.zeros((3 * L, 3 * L))
    g = np.zeros(3 * L)

    def add(J: np.ndarray, r: np.ndarray, om: np.ndarray):
        Om = np.diag(om)
        H[:] += J.T @ Om @ J
        g[:] += J.T @ Om @ r

    r = x[0] - prior[:3]
    r[2] = wrap(r[2])
    J = np.zeros((3, 3 * L)); J[:, 0:3] = np.eye(3)
    add(J, r, prior[3:])
    for i in range(L - 1):
        th = x[i, 2]
        c, s = np.cos(th), np.sin(th)
        dt = x[i + 1, :2] - x[i, :2]
        rel = np.array([c * dt[0] + s * dt[1], -s * dt[0] + c * dt[1]])
        r = np.array([rel[0] - odo[i, 0], rel[1] - odo[i, 1], wrap(x[i + 1, 2] - x[i, 2] - odo[i, 2])])
        J = np.zeros((3, 3 * L))
        Rt = np.array([[c, s], [-s, c]])
        dRt = np.array([[-s, c], [-c, -s]])          # d R(th)^T / d th
        J[0:2, 3 * i:3 * i + 2] = -Rt
        J[0:2, 3 * i + 2] = dRt @ dt
        J[2, 3 * i + 2] = -1.0
        J[0:2, 3 * (i + 1):3 * (i + 1) + 2] = Rt
        J[2, 3 * (i + 1) + 2] = 1.0
        add(J, r, odo[i, 3:])
    for i in range(L):
        if np.any(scan[i, 3:] != 0):
            r = x[i] - scan[i, :3]
            r[2] = wrap(r[2])
            J = np.zeros((3, 3 * L)); J[:, 3 * i:3 * i + 3] = np.eye(3)
            add(J, r, scan[i, 3:])
    return H, g


def fixedlag_solve(x0: np.ndarray, prior: np.ndarray, odo: np.ndarray, scan: np.ndarray, iters: int):
    """K Gauss-Newton steps and the newest pose's covariance (S6): returns (x [L,3], Sigma [3,3])."""
    x = np.array(x0, dtype=np.float64, copy=True)
    L = x.shape[0]
    for _ in range(iters):
        H, g = normal_equations(x, prior, odo, scan)
        x = x - np.linalg.solve(H, g).reshape(L, 3)
    H, _ = normal_equations(x, prior, odo, scan)
    Sigma = np.linalg.inv(H)[-3:, -3:]
    return x, Sigma
