"""CPU oracle of the batched Active-SLAM environment step (ctypes front end).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  The arithmetic lives
in ``aslam_oracle.c`` (plain C, FP32 state as the workload fixes it, FP64 for
reward and tables); this file only owns numpy state arrays and marshals them.

Method: arXiv 2603.25834, Sec. III-B..III-E and Sec. IV-A (see the C file).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
NANG = 46080


def build_oracle(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math, no FP contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    src = os.path.join(HERE, "aslam_oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrcConfig(ctypes.Structure):
    _fields_ = [
        ("n_rays", ctypes.c_int32), ("loop_closure", ctypes.c_int32),
        ("lc_gap", ctypes.c_int32), ("episode_len", ctypes.c_int32),
        ("cell_m", ctypes.c_float), ("r_max_m", ctypes.c_float), ("dt", ctypes.c_float),
        ("v_max", ctypes.c_float), ("w_max", ctypes.c_float),
        ("sigma_x", ctypes.c_float), ("sigma_y", ctypes.c_float), ("sigma_th", ctypes.c_float),
        ("var0_xy", ctypes.c_float), ("var0_th", ctypes.c_float),
        ("lc_cell_m", ctypes.c_float), ("lc_radius_m", ctypes.c_float), ("lc_sigma_m", ctypes.c_float),
        ("l_hit", ctypes.c_float), ("l_miss", ctypes.c_float), ("l_clamp", ctypes.c_float),
        ("w_entropy", ctypes.c_float), ("w_dopt", ctypes.c_float), ("lambda_col", ctypes.c_float),
        ("fov_steps", ctypes.c_int32), ("reward_mode", ctypes.c_int32),
        ("r_min_m", ctypes.c_float), ("range_sigma_m", ctypes.c_float), ("range_quant_m", ctypes.c_float),
        ("d_crash_m", ctypes.c_float), ("d_full_m", ctypes.c_float),
        ("lambda_explore", ctypes.c_float), ("lambda_abs", ctypes.c_float), ("lambda_delta", ctypes.c_float),
        ("u_hi", ctypes.c_float), ("kappa", ctypes.c_float),
        ("noise_seed", ctypes.c_uint64),
        ("slam_backend", ctypes.c_int32),
    ]


_P = ctypes.c_void_p


class OrcState(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32)] + [(f, _P) for f in (
        "side", "world_off", "cell_off", "visit_off", "world", "belief", "pose", "est", "cov",
        "h_q", "step", "last_lc", "visit_t", "visit_x", "visit_y", "visit_last", "prev_vcell", "u_prev",
        "draws")]


class OrcOut(ctypes.Structure):
    _fields_ = [(f, _P) for f in (
        "ranges", "rho_q", "hit_cell", "reward", "done", "collided", "closed", "r_entropy",
        "logdet", "counters", "odo", "d_min", "dcells")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_oracle()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_trig_table.argtypes = [_P, _P]
        L.orc_logodds_q.argtypes = [ctypes.c_float]
        L.orc_logodds_q.restype = ctypes.c_int32
        L.orc_entropy_table.argtypes = [ctypes.c_int32, _P]
        L.orc_heading_index.argtypes = [ctypes.c_float]
        L.orc_heading_index.restype = ctypes.c_int32
        L.orc_walk.argtypes = [ctypes.c_int64] * 6 + [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32, _P]
        L.orc_walk.restype = ctypes.c_int32
        L.orc_reset.argtypes = [ctypes.POINTER(OrcConfig), ctypes.POINTER(OrcState), _P, _P]
        L.orc_step.argtypes = [ctypes.POINTER(OrcConfig), ctypes.POINTER(OrcState), _P, _P,
                               ctypes.POINTER(OrcOut), ctypes.c_int32]
        L.orc_observe.argtypes = [ctypes.POINTER(OrcConfig), ctypes.POINTER(OrcState), _P, _P,
                                  ctypes.c_int32, _P, _P, _P, ctypes.c_double]
        L.orc_noise_width.argtypes = [ctypes.POINTER(OrcConfig)]
        L.orc_noise_width.restype = ctypes.c_int32
        L.orc_paper_reward.argtypes = [ctypes.POINTER(OrcConfig), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double]
        L.orc_paper_reward.restype = ctypes.c_double
        L.orc_philox4x64.argtypes = [_P, _P, _P]
        L.orc_normal.argtypes = [ctypes.c_uint64] * 5
        L.orc_normal.restype = ctypes.c_float
        L.orc_permute.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, _P]
        L.orc_to_q16.argtypes = [ctypes.c_float, ctypes.c_float]
        L.orc_to_q16.restype = ctypes.c_int64
        L.orc_uncertainty.argtypes = [_P]
        L.orc_uncertainty.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def trig_table():
    cq = np.zeros(NANG, np.int32)
    sq = np.zeros(NANG, np.int32)
    lib().orc_trig_table(_ptr(cq), _ptr(sq))
    return cq, sq


def logodds_q(x: float) -> int:
    return int(lib().orc_logodds_q(x))


def entropy_table(lc: int) -> np.ndarray:
    hq = np.zeros(2 * lc + 1, np.uint32)
    lib().orc_entropy_table(lc, _ptr(hq))
    return hq


def heading_index(theta: float) -> int:
    return int(lib().orc_heading_index(np.float32(theta)))


def walk(ox, oy, a, b, scale, lim, s, max_out=1 << 16):
    """Exact traversal: returns (cells [n,2], entry distances E [n], axis [n], end_reason)."""
    cx = np.zeros(max_out, np.int32)
    cy = np.zeros(max_out, np.int32)
    e = np.zeros(max_out, np.int64)
    ax = np.zeros(max_out, np.int32)
    end = np.zeros(1, np.int32)
    n = lib().orc_walk(int(ox), int(oy), int(a), int(b), int(scale), int(lim), int(s),
                       _ptr(cx), _ptr(cy), _ptr(e), _ptr(ax), max_out, _ptr(end))
    return np.stack([cx[:n], cy[:n]], 1), e[:n], ax[:n], int(end[0])


def make_config(p: dict) -> OrcConfig:
    c = OrcConfig()
    for name, _ in OrcConfig._fields_:
        setattr(c, name, p.get(name, 0) if name in ("noise_seed", "slam_backend") else p[name])
    return c


DOMAIN_ENV, DOMAIN_ACTION, DOMAIN_PERM = 1, 2, 3


def philox4x64(ctr, key) -> np.ndarray:
    """Philox4x64-10 block at a 4-word counter under a 2-word key (the oracle's own C implementation)."""
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def normal(seed: int, domain: int, c0: int, c1: int, c2: int) -> np.float32:
    """Irwin-Hall(12) standard normal of the block at counter (c0, c1, c2, 0) under key (seed, domain)."""
    return np.float32(lib().orc_normal(seed, domain, c0, c1, c2))


def normals(seed: int, domain: int, c0: int, rows: int, cols: int) -> np.ndarray:
    """[rows, cols] draws: entry (b, d) at counter (c0, b, d)."""
    out = np.zeros((rows, cols), np.float32)
    for b in range(rows):
        for d in range(cols):
            out[b, d] = lib().orc_normal(seed, domain, c0, b, d)
    return out


def permute(n: int, seed: int, counter: int) -> np.ndarray:
    """Keyed permutation of [0, n) (Feistel network with cycle walking), out[j] = image of j."""
    out = np.zeros(max(n, 1), np.int32)
    lib().orc_permute(int(n), seed, counter, _ptr(out))
    return out[:n]


def bridge_alpha(t: int, t_bridge: int) -> float:
    """Blending coefficient of the uncertainty bridge, Sec. III-G, Eq. (21): min(1, t / T_bridge)."""
    return min(1.0, float(t) / float(t_bridge))


def noise_width(p: dict) -> int:
    """Normal draws per robot and step the step expects (5, plus R with range noise)."""
    c = make_config(p)
    return int(lib().orc_noise_width(ctypes.byref(c)))


def to_q16(v: float, cell_m: float) -> int:
    """Q16 cells of a coordinate, as the step forms them (FP32 product, rint, clamp)."""
    return int(lib().orc_to_q16(float(v), float(cell_m)))


def uncertainty(c6: np.ndarray) -> float:
    """U = cbrt(det Sigma) of the 6 unique FP32 covariance entries, as the reward uses it."""
    c = np.ascontiguousarray(c6, np.float32)
    return float(lib().orc_uncertainty(_ptr(c)))


def paper_reward(p: dict, collided: bool, dcells: float, u_prev: float, u: float, d_min: float) -> float:
    """The paper's Eq. (7) reward from its inputs (the oracle's own function)."""
    c = make_config(p)
    return float(lib().orc_paper_reward(ctypes.byref(c), int(bool(collided)), dcells, u_prev, u, d_min))


@dataclass
class StepOut:
    ranges: np.ndarray
    rho_q: np.ndarray
    hit_cell: np.ndarray
    reward: np.ndarray
    done: np.ndarray
    collided: np.ndarray
    closed: np.ndarray
    r_entropy: np.ndarray
    logdet: np.ndarray
    counters: np.ndarray
    odo: np.ndarray
    d_min: np.ndarray
    dcells: np.ndarray


class OracleEnv:
    """Numpy-owned state for a batch of robots, stepped by the C oracle."""

    def __init__(self, params: dict, sides: np.ndarray, world_words: np.ndarray, world_off: np.ndarray):
        self.p = dict(params)
        self.cfg = make_config(self.p)
        self.sides = np.ascontiguousarray(sides, np.int32)
        n = self.n = len(self.sides)
        self.world = np.ascontiguousarray(world_words, np.uint32)
        self.world_off = np.ascontiguousarray(world_off, np.int64)
        cells = self.sides.astype(np.int64) ** 2
        self.cell_off = np.concatenate([[0], np.cumsum(cells)[:-1]]).astype(np.int64)
        self.belief = np.zeros(int(cells.sum()), np.int16)
        nv = np.ceil(self.sides.astype(np.float64) * float(np.float32(self.p["cell_m"]))
                     / float(np.float32(self.p["lc_cell_m"]))).astype(np.int64)
        self.visit_off = np.concatenate([[0], np.cumsum(nv * nv)[:-1]]).astype(np.int64)
        nvt = int((nv * nv).sum())
        self.visit_t = np.full(max(nvt, 1), -1, np.int32)
        self.visit_x = np.zeros(max(nvt, 1), np.float32)
        self.visit_y = np.zeros(max(nvt, 1), np.float32)
        self.visit_last = np.full(max(nvt, 1), -1, np.int32)
        self.prev_vcell = np.full(n, -1, np.int32)
        self.u_prev = np.zeros(n, np.float64)
        self.pose = np.zeros((n, 3), np.float32)
        self.est = np.zeros((n, 3), np.float32)
        self.cov = np.zeros((n, 6), np.float32)
        self.h_q = np.zeros(n, np.int64)
        self.step_ct = np.zeros(n, np.int32)
        self.last_lc = np.zeros(n, np.int32)
        self.draws = np.zeros(n, np.uint64)
        self.R = int(self.p["n_rays"])

    def _state(self) -> OrcState:
        st = OrcState()
        st.n = self.n
        for f, a in (("side", self.sides), ("world_off", self.world_off), ("cell_off", self.cell_off),
                     ("visit_off", self.visit_off), ("world", self.world), ("belief", self.belief),
                     ("pose", self.pose), ("est", self.est), ("cov", self.cov), ("h_q", self.h_q),
                     ("step", self.step_ct), ("last_lc", self.last_lc), ("visit_t", self.visit_t),
                     ("visit_x", self.visit_x), ("visit_y", self.visit_y), ("visit_last", self.visit_last),
                     ("prev_vcell", self.prev_vcell), ("u_prev", self.u_prev), ("draws", self.draws)):
            setattr(st, f, _ptr(a))
        return st

    def reset(self, init_pose: np.ndarray, mask: np.ndarray | None = None):
        ip = np.ascontiguousarray(init_pose, np.float32)
        m = None if mask is None else np.ascontiguousarray(mask, np.uint8)
        st = self._state()
        lib().orc_reset(ctypes.byref(self.cfg), ctypes.byref(st), _ptr(ip), None if m is None else _ptr(m))

    def step(self, actions: np.ndarray, noise: np.ndarray | None, threads: int = 0) -> StepOut:
        """One step; noise None draws the step's own normals (key noise_seed, counter draws[r])."""
        n, R = self.n, self.R
        a = np.ascontiguousarray(actions, np.float32).reshape(n, 2)
        g = None
        if noise is not None:
            g = np.ascontiguousarray(noise, np.float32).reshape(n, int(lib().orc_noise_width(ctypes.byref(self.cfg))))
        o = StepOut(ranges=np.zeros((n, R), np.float32), rho_q=np.zeros((n, R), np.int32),
                    hit_cell=np.zeros((n, R), np.int32), reward=np.zeros(n, np.float64),
                    done=np.zeros(n, np.uint8), collided=np.zeros(n, np.uint8),
                    closed=np.zeros(n, np.uint8), r_entropy=np.zeros(n, np.float64),
                    logdet=np.zeros(n, np.float64), counters=np.zeros((n, 4), np.int64),
                    odo=np.zeros((n, 2), np.float32), d_min=np.zeros(n, np.float64), dcells=np.zeros(n, np.float64))
        co = OrcOut()
        for f in OrcOut._fields_:
            setattr(co, f[0], _ptr(getattr(o, f[0])))
        st = self._state()
        th = threads if threads > 0 else (os.cpu_count() or 1)
        lib().orc_step(ctypes.byref(self.cfg), ctypes.byref(st), _ptr(a), None if g is None else _ptr(g),
                       ctypes.byref(co), th)
        return o

    def observe(self, ranges: np.ndarray, crop_side: int = 64, u_new: np.ndarray | None = None, t: int = 0,
                t_bridge: int = 1):
        """Observation; with u_new (reward_mode 1) the uncertainty entry is bridged with
        alpha = min(1, t / T_bridge) (Sec. III-G)."""
        n, R = self.n, self.R
        rg = np.ascontiguousarray(ranges, np.float32)
        crop = np.zeros((n, crop_side, crop_side), np.int16)
        scan = np.zeros((n, R), np.float32)
        state = np.zeros((n, 12), np.float32)
        st = self._state()
        un = None if u_new is None else np.ascontiguousarray(u_new, np.float32)
        alpha = bridge_alpha(t, t_bridge)
        lib().orc_observe(ctypes.byref(self.cfg), ctypes.byref(st), _ptr(rg), _ptr(crop), crop_side,
                          _ptr(scan), _ptr(state), None if un is None else _ptr(un), alpha)
        return crop, scan, state

    def belief_of(self, i: int) -> np.ndarray:
        s = int(self.sides[i])
        o = int(self.cell_off[i])
        return self.belief[o:o + s * s].reshape(s, s)
