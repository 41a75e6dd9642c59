"""Shared helpers of the GPU-vs-oracle environment tests (oracle side = CPU C oracle)."""
from __future__ import annotations

import sys

import numpy as np

from paper_2603_25834_amd import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Pair:
    """The same robots, stepped by the C-ABI library (GPU) and by the CPU oracle."""

    def __init__(self, name: str, seed: int, robots=None, exec_kw=None, params_over=None, steps: int = 100,
                 oracle: bool = True, own_draws: bool = False):
        """own_draws: both sides take the step's normals from their own counter-based generators
        (params['noise_seed']) instead of the host-drawn rows."""
        import torch

        from oracle import oracle as O
        from paper_2603_25834_amd.env import Env

        self.torch = torch
        self.name = name
        w = synth.WORKLOADS[name]
        self.p = w.params()
        if params_over:
            self.p.update(params_over)
        self.b = synth.make_batch(name, seed, robots)
        self.n = len(self.b.sides)
        self.R = int(self.p["n_rays"])
        self.A = synth.actions(name, seed, steps, robots)
        self.G = synth.noise(name, seed, steps, robots)
        gw = synth.noise_width(self.p)
        if self.G.shape[-1] > gw:          # an override turned the range noise off
            self.G = np.ascontiguousarray(self.G[..., :gw])
        elif self.G.shape[-1] < gw:        # ... or on: draw the ray noise separately
            rng = np.random.default_rng([seed, 5])
            extra = rng.standard_normal(self.G.shape[:-1] + (gw - self.G.shape[-1],), dtype=np.float32)
            self.G = np.ascontiguousarray(np.concatenate([self.G, extra], axis=-1))
        self.orc = None
        if oracle:
            self.orc = O.OracleEnv(self.p, self.b.sides, self.b.world, self.b.world_off)
            self.orc.reset(self.b.start)
        say(f"[pair] {name} seed={seed} n={self.n} R={self.R} exec={exec_kw}")
        self.env = Env(self.p, self.b.sides)
        if exec_kw:
            self.env.set_exec(**exec_kw)
        dev = "cuda"
        self.world = torch.from_numpy(self.b.world.view(np.int32).copy()).to(dev)
        self.start = torch.from_numpy(self.b.start).to(dev)
        self.env.reset(self.world, self.start)
        self.dA = torch.from_numpy(self.A).to(dev)
        self.dG = torch.from_numpy(self.G).to(dev)
        self.ranges = torch.zeros((self.n, self.R), dtype=torch.float32, device=dev)
        self.reward = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.done = torch.zeros(self.n, dtype=torch.uint8, device=dev)
        self.own = own_draws
        self.t = 0
        self.cum = np.zeros((self.n, 3), np.int64)   # oracle work counters since reset

    def reset(self, start, mask=None):
        import torch
        m = None if mask is None else np.asarray(mask, np.uint8)
        if self.orc is not None:
            self.orc.reset(start, m)
        self.env.reset(self.world, torch.from_numpy(np.ascontiguousarray(start, np.float32)).cuda(),
                       None if m is None else torch.from_numpy(m).cuda())
        if m is None:
            self.cum[:] = 0
        else:
            self.cum[m.astype(bool)] = 0

    def step(self):
        g = None if self.own else self.G[self.t]
        o = self.orc.step(self.A[self.t], g) if self.orc is not None else None
        if o is not None:
            self.cum += o.counters[:, [2, 0, 1]]
        self.env.step(self.dA[self.t], None if self.own else self.dG[self.t], self.ranges, self.reward, self.done)
        self.t += 1
        return o

    def gpu_state(self):
        from paper_2603_25834_amd import _lib
        e = self.env
        self.torch.cuda.synchronize()
        return dict(
            pose=e.read(_lib.FIELD_POSE).cpu().numpy(), est=e.read(_lib.FIELD_EST).cpu().numpy(),
            cov=e.read(_lib.FIELD_COV).cpu().numpy(), belief=e.read(_lib.FIELD_BELIEF).cpu().numpy(),
            hq=e.read(_lib.FIELD_ENTROPY_Q).cpu().numpy(), step=e.read(_lib.FIELD_STEP).cpu().numpy(),
            flags=e.read(_lib.FIELD_FLAGS).cpu().numpy(), terms=e.read(_lib.FIELD_TERMS).cpu().numpy(),
            rho=e.read(_lib.FIELD_RHO_Q).cpu().numpy(), hitc=e.read(_lib.FIELD_HIT_CELL).cpu().numpy(),
            counters=e.read(_lib.FIELD_COUNTERS).cpu().numpy(),
            u_prev=e.read(_lib.FIELD_U_PREV).cpu().numpy(), visit_last=e.read(_lib.FIELD_VISIT_LAST).cpu().numpy(),
            ranges=self.ranges.cpu().numpy(), reward=self.reward.cpu().numpy(), done=self.done.cpu().numpy())

    def compare(self, o, rays: bool = True, belief: bool = True, tag: str = ""):
        """GPU state vs the oracle: bit-exact integer and pose state, tolerances for FP reward terms."""
        g = self.gpu_state()
        orc = self.orc
        where = f"{self.name} t={self.t} {tag}"
        assert np.array_equal(g["pose"].view(np.int32), orc.pose.view(np.int32)), f"pose differs {where}"
        assert np.array_equal(g["est"].view(np.int32), orc.est.view(np.int32)), f"estimate differs {where}"
        assert np.array_equal(g["cov"].view(np.int32), orc.cov.view(np.int32)), f"covariance differs {where}"
        assert np.array_equal(g["step"], orc.step_ct), where
        assert np.array_equal(g["flags"][:, 0], o.collided), f"collision flags differ {where}"
        assert np.array_equal(g["flags"][:, 1], o.closed), f"loop-closure flags differ {where}"
        assert np.array_equal(g["done"], o.done), f"done differs {where}"
        # ranges: same FP32 expression of the same integer range -> identical; 1e-5 rel is the contract
        assert np.allclose(g["ranges"], o.ranges, rtol=1e-5, atol=0), f"ranges differ {where}"
        if rays:
            assert np.array_equal(g["rho"], o.rho_q), f"rho_q differs {where}"
            assert np.array_equal(g["hitc"], o.hit_cell), f"hit cells differ {where}"
        if belief:
            bad = np.flatnonzero(g["belief"] != orc.belief)
            assert bad.size == 0, f"belief differs in {bad.size} cells {where} (first {bad[:5]})"
            assert np.array_equal(g["hq"], orc.h_q), f"entropy differs {where}"
        assert np.array_equal(g["counters"], self.cum), f"work counters differ {where}"
        assert np.allclose(g["terms"][:, 0], o.r_entropy, rtol=1e-5, atol=1e-4), f"entropy term {where}"
        assert np.allclose(g["terms"][:, 1], o.logdet, rtol=1e-5, atol=1e-4), f"logdet term {where}"
        assert np.all(np.abs(g["reward"] - o.reward) <= 1e-4 * np.maximum(1.0, np.abs(o.reward))), \
            f"reward differs {where}: max {np.max(np.abs(g['reward'] - o.reward))}"
        if int(self.p.get("reward_mode", 0)) == 1:
            # U = cbrt(det Sigma) of bit-identical covariances: FP64 library cbrt, within a few ulp
            assert np.allclose(g["u_prev"], orc.u_prev, rtol=1e-13, atol=0), f"U_t differs {where}"
            nv = g["visit_last"].size
            assert np.array_equal(g["visit_last"], orc.visit_last[:nv]), f"visit bookkeeping differs {where}"
        return g
