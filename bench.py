"""Benchmark of the batched Active-SLAM hot path on one MI355X.

One step = one environment step of every robot (motion and collision, EKF
predict and loop closure, LiDAR march, log-odds map update, entropy and
D-optimality reward) followed by the observation assembly for the policy.
Inputs (worlds, start poses, actions) are seeded, synthetic and resident in
HBM before the timed region; the normal draws and permutations come from the
library's counter-based generator inside the kernels.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
METRIC = "env-steps/s and rays/s at 750 & 4096 robots; % HBM roofline; PPO fwd+bwd/s"
# The paper's own training-time figures (Sec. IV-A hardware, Sec. IV-B results), quoted as context only:
# a different pipeline (Isaac Sim physics, the fixed-lag SLAM, the GRU policy) on other hardware.
PAPER_CONTEXT = {
    "training_time": "about 4 h to train the evaluated policy with 750 parallel agents (Env 1, episodes of at "
                     "most 2048 steps, PPO with a GRU(256) policy)",
    "hardware": "laptop: Intel Core i7 13th gen, NVIDIA RTX 4060 Laptop GPU 8 GB, 32 GB RAM; Ubuntu 22.04, "
                "Isaac Sim 4.5, Isaac Lab 2.3.2",
    "training_volume": "tens of millions of timesteps in a few hours",
    "derived_rate": "about 0.7k-7k env-steps/s end to end (10-99 M steps over about 4 h; derived here, not stated "
                    "in the paper)",
    "prior_work": "over 50 h for Gazebo-based single-robot training",
}


def alg_bytes_per_robot_step(D: float, R: int, loop_closure: bool, host_draws: int = 0,
                             paper_reward: bool = False) -> float:
    """Algorithmic HBM bytes of one robot-step.

    Map: read + write each coded int16 cell (4 B); world bits of the cells the
    rays cross, taken equal to the coded cells (D/8 B); ranges out (4R B);
    per-robot state and I/O: action 8, true pose r/w 24, estimate r/w 24,
    covariance r/w 48, step r/w 8, entropy r/w 16, draw counter r/w 16,
    reward 4, done 1 (149 B), plus 4 B per normal draw read from the caller
    (none when the step draws its own); loop-closure visit record read 12 B;
    Eq. (7) reward state: U_{t-1} r/w 16, previous visit cell r/w 8, last
    visit r/w 8 (32 B)."""
    return (4.0 * D + D / 8.0 + 4.0 * R + 149.0 + 4.0 * host_draws + (12.0 if loop_closure else 0.0) +
            (32.0 if paper_reward else 0.0))


def noise_seed(seed: int) -> int:
    """Key of the env step's own normal draws for a benchmark seed."""
    return 0x5EED0000 + int(seed)


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("env_kernels.hip", "env_internal.h"):
        with open(os.path.join(ROOT, "paper_2603_25834_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(kernel: str, workload: str, threads: int, mark_seg: int = 0) -> str:
    seg = f"_s{mark_seg}" if mark_seg else ""
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_t{threads}{seg}_{workload}.txt")


def read_summary(path: str) -> dict | None:
    """key: value lines of a committed rocprofv3 counter summary, if it was taken on the current kernel
    source; else None."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("source_digest") == kernel_source_digest() else None


def read_traffic(kernel: str, workload: str, threads: int, mark_seg: int = 0):
    """HBM traffic per launch from the committed rocprofv3 counter summary for this kernel, workload,
    workgroup size and walk form, if it was taken on the current kernel source; else None."""
    kv = read_summary(traffic_file(kernel, workload, threads, mark_seg))
    try:
        return float(kv["hbm_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


# VALU issue peak of the chip: 256 CUs x 4 SIMDs x 16 lanes per cycle x 2.4 GHz (a wave64 instruction
# occupies a SIMD for 4 cycles), in lane-instructions per second.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def valu_roofline(kernel: str, workload: str, threads: int, mark_seg: int, avg_launch_ms: float):
    """VALU issue of the kernel: SQ_INSTS_VALU per launch (committed counter summary of the same shape,
    current source) x 64 lanes over the live average launch time, against the issue peak."""
    seg = f"_s{mark_seg}" if mark_seg else ""
    path = os.path.join(ROOT, "profiles", f"sq_counters_{kernel}_t{threads}{seg}_{workload}.txt")
    kv = read_summary(path)
    if not kv or "SQ_INSTS_VALU" not in kv:
        return None
    lane_ops = float(kv["SQ_INSTS_VALU"]) * 64
    achieved = lane_ops / (avg_launch_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
            "unit": "T lane-instructions/s", "frac": achieved / VALU_PEAK_LANE_OPS,
            "valu_instructions_per_launch": float(kv["SQ_INSTS_VALU"]),
            "wait_share": float(kv["SQ_WAIT_ANY"]) / float(kv["SQ_WAVE_CYCLES"]),
            "source": os.path.basename(path)}


def copy_bandwidth(gib: float = 1.0, reps: int = 10) -> float:
    """Measured device-to-device copy rate (read + write bytes / time) of a gib-GiB buffer, GB/s."""
    import torch
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


class Workbench:
    """One workload on the GPU: env + resident inputs + output buffers."""

    def __init__(self, name: str, seed: int, steps: int, exec_kw: dict):
        import torch

        from paper_2603_25834_amd import synth
        from paper_2603_25834_amd.env import Env
        self.torch = torch
        self.name = name
        w = self.w = synth.WORKLOADS[name]
        self.p = w.params()
        self.p["noise_seed"] = noise_seed(seed)
        t0 = time.time()
        self.b = synth.make_batch(name, seed)
        self.n, self.R = len(self.b.sides), w.n_rays
        A = synth.actions(name, seed, steps)
        self.gen_s = time.time() - t0
        self.env = Env(self.p, self.b.sides)
        self.env.set_exec(**exec_kw)
        self.exec_kw = exec_kw
        dev = "cuda"
        self.world = torch.from_numpy(self.b.world.view(np.int32).copy()).to(dev)
        self.start = torch.from_numpy(self.b.start).to(dev)
        self.dA = torch.from_numpy(A).to(dev)
        self.ranges = torch.zeros((self.n, self.R), device=dev)
        self.reward = torch.zeros(self.n, device=dev)
        self.done = torch.zeros(self.n, dtype=torch.uint8, device=dev)
        self.crop = torch.zeros((self.n, 64, 64), dtype=torch.int16, device=dev)
        self.scan = torch.zeros((self.n, self.R), device=dev)
        self.state = torch.zeros((self.n, 12), device=dev)
        self.env.reset(self.world, self.start)

    def run(self, warmup: int, steps: int, graph: bool = True):
        """Warm up, then time `steps` env steps (one HIP graph, or eager launches)."""
        torch = self.torch
        from paper_2603_25834_amd import _lib
        e = self.env
        n = self.n
        for t in range(warmup):
            e.step(self.dA[t], None, self.ranges, self.reward, self.done)
        if graph:
            e.graph_build(steps, self.dA[warmup:], 2 * n, None, 0, self.ranges, 0, self.reward, 0, self.done, 0)
        torch.cuda.synchronize()
        c0 = e.read(_lib.FIELD_COUNTERS).sum(0).cpu().numpy()
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_start.record()
        if graph:
            e.graph_launch()
        else:
            for t in range(warmup, warmup + steps):
                e.step(self.dA[t], None, self.ranges, self.reward, self.done)
        t_end.record()
        torch.cuda.synchronize()
        ms = t_start.elapsed_time(t_end)
        c1 = e.read(_lib.FIELD_COUNTERS).sum(0).cpu().numpy()
        D = float(c1[0] - c0[0]) / (n * steps)
        vm = float(c1[1] - c0[1]) / (n * steps)
        vu = float(c1[2] - c0[2]) / (n * steps)
        bytes_step = n * alg_bytes_per_robot_step(D, self.R, bool(self.p["loop_closure"]), 0,
                                                  int(self.p.get("reward_mode", 0)) == 1)
        s = ms / 1e3
        return dict(ms=ms, ms_per_step=ms / steps, env_steps_per_s=n * steps / s, rays_per_s=n * steps * self.R / s,
                    coded_cells_per_robot_step=D, march_visits_per_robot_step=vm, update_visits_per_robot_step=vu,
                    alg_bytes_per_step=bytes_step, achieved_gbs=bytes_step * steps / s / 1e9)

    def observe_time(self, reps: int = 20) -> float:
        torch = self.torch
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            self.env.observe(self.ranges, self.crop, self.scan, self.state)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / reps


def slam_time(wb, reps: int = 20, L: int = 10, iters: int = 3) -> dict:
    """The fixed-lag SLAM backbone on the env's state after its timed steps: correlative scan matching of
    every robot's last scan against its belief grid (a 9 x 9 x 11 lattice: one-cell and 64-table-step
    (0.5 degree) steps), the scan factors, and Gauss-Newton over an L-pose window per robot with the
    newest pose's covariance.  Each call timed alone with HIP events on the current stream."""
    torch = wb.torch
    from paper_2603_25834_amd import _lib, slam
    n, R, p = wb.n, wb.R, wb.p
    cell, rmax = float(p["cell_m"]), float(p["r_max_m"])
    nang = 46080
    a_off = (torch.arange(R, dtype=torch.int32, device="cuda") * (nang // R)).contiguous()
    belief = wb.env.read(_lib.FIELD_BELIEF)
    sides = torch.tensor(np.asarray(wb.b.sides, np.int64), device="cuda")
    cell_off = (torch.cumsum(sides * sides, 0) - sides * sides).contiguous()
    side32 = sides.to(torch.int32).contiguous()
    est = wb.env.read(_lib.FIELD_EST).double()
    pose_q = torch.stack([torch.floor(est[:, 0] / cell * 65536), torch.floor(est[:, 1] / cell * 65536),
                          torch.remainder(torch.round(est[:, 2] * (nang / (2 * np.pi))), nang)], 1)
    pose_q = pose_q.to(torch.int32).contiguous()
    rho_q = torch.where(wb.ranges < rmax - 1e-4, torch.round(wb.ranges / cell * 65536),
                        torch.full_like(wb.ranges, -1.0)).to(torch.int32).contiguous()
    cfg = slam.csm_config(4, 5, 65536, 64)
    match = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    # windows: L poses along the estimate, odometry between them, the prior on the oldest
    g = torch.Generator(device="cpu").manual_seed(0)
    x0 = est[:, None, :].repeat(1, L, 1) + 0.01 * torch.randn((n, L, 3), generator=g, dtype=torch.float64).cuda()
    prior = torch.cat([est, torch.full((n, 3), 400.0, dtype=torch.float64, device="cuda")], 1).contiguous()
    odo = torch.cat([torch.zeros((n, L - 1, 3), dtype=torch.float64, device="cuda"),
                     torch.full((n, L - 1, 3), 2500.0, dtype=torch.float64, device="cuda")], 2).contiguous()
    scan = torch.zeros((n, L, 6), dtype=torch.float64, device="cuda")
    xo = torch.empty_like(x0)
    cov = torch.empty((n, 3, 3), dtype=torch.float64, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / reps

    max_side = int(max(wb.b.sides))
    csm_ms = timed(lambda: slam.csm_match(belief, cell_off, side32, pose_q, rho_q, a_off, cfg, out=match,
                                          max_side=max_side))
    meas, info = slam.csm_factor(match, pose_q, cfg, cell, 896.0, 0.05, 0.02)
    fac_ms = timed(lambda: slam.csm_factor(match, pose_q, cfg, cell, 896.0, 0.05, 0.02, meas=meas, info=info))
    scan[:, -1, :3] = meas
    scan[:, -1, 3:] = info
    gn_ms = timed(lambda: slam.fixedlag_solve(x0, prior, odo, scan, iters, x=xo, cov=cov))
    # confidence-weighted integration of each scan from its matched pose, on a copy of the grids
    lq = [int(round(float(p[k]) * 256.0)) for k in ("l_hit", "l_miss", "l_clamp")]
    rmax_q = int(round(rmax / cell * 65536.0))
    bel_w = belief.clone()
    coded = torch.empty(n, dtype=torch.int32, device="cuda")
    int_ms = timed(lambda: slam.csm_integrate(bel_w, cell_off, side32, pose_q, rho_q, a_off, rmax_q, *lq, match=match,
                                              cfg=cfg, l_max=float(lq[2]), coded=coded, max_side=max_side))
    del bel_w
    m = match.cpu().numpy()
    ncand = 9 * 9 * 11
    used = float(m[:, 5].mean())
    return {"robots": n, "rays": R, "lattice": [9, 9, 11], "candidates": ncand,
            "csm_us": csm_ms * 1e3, "factor_us": fac_ms * 1e3, "integrate_us": int_ms * 1e3,
            "fixedlag_us": gn_ms * 1e3, "window_poses": L, "gn_iters": iters,
            "candidate_ray_evals_per_s": n * ncand * used / (csm_ms / 1e3),
            "coded_cells_per_robot": float(coded.double().mean().item()),
            "robots_per_s": n / ((csm_ms + fac_ms + int_ms + gn_ms) / 1e3),
            "rays_with_return": used,
            "mean_best_offset_cells": float(np.abs(m[:, :2]).mean()),
            "factor_weight_mean": float((info[:, 0] * 0.05 ** 2).mean().item())}


def policy_flops(n_scan: int) -> tuple:
    """Algorithmic FLOP per sample of the actor-critic: forward, and backward with the forward recomputed.

    conv1 1->16 (3x3, stride 2) onto 32x32, conv2 16->32 onto 16x16, FC1 (8192 + R + 12)->256, FC2 256->256,
    heads 256->3.  Backward: weight gradients of every layer, input gradients of every layer but conv1, and
    of FC1 only for its conv2 inputs."""
    c1 = 2 * 16 * 32 * 32 * 9
    c2 = 2 * 32 * 16 * 16 * 16 * 9
    k1 = 8192 + n_scan + 12
    f1 = 2 * k1 * 256
    f2 = 2 * 256 * 256
    hd = 2 * 256 * 3
    fwd = c1 + c2 + f1 + f2 + hd
    bwd = fwd + c1 + 2 * c2 + (f1 + 2 * 8192 * 256) + 2 * f2 + 2 * hd
    return float(fwd), float(bwd)


def ppo_time(n_scan: int, batch: int, seed: int, reps: int = 10, precision: int = 0) -> dict:
    """Policy forward and fused loss+backward on one synthetic minibatch resident in HBM (precision 0:
    BF16 operands; 1: split hi + lo forward operands)."""
    import torch

    from paper_2603_25834_amd import synth
    from paper_2603_25834_amd.policy import Policy
    pol = Policy(n_scan, max_batch=batch, precision=precision)
    d = {k: torch.from_numpy(v).cuda() for k, v in synth.policy_batch(batch, n_scan, seed).items()}
    params = torch.from_numpy(synth.init_policy_params(n_scan, seed)).cuda()
    grads = torch.zeros_like(params)
    mu = torch.empty((batch, 2), device="cuda")
    val = torch.empty(batch, device="cuda")
    loss = torch.empty(4, device="cuda")

    def fwd():
        pol.forward(params, d["crop"], d["scan"], d["state"], mu, val)

    def bwd():
        pol.backward(params, d["crop"], d["scan"], d["state"], d["act"], d["old_logp"], d["adv"], d["ret"], grads,
                     loss)

    out = {}
    for name, fn in (("forward", fwd), ("backward", bwd)):
        for _ in range(2):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    f_fwd, f_bwd = policy_flops(n_scan)
    tf_f = f_fwd * batch / (out["forward"] / 1e3) / 1e12
    tf_b = f_bwd * batch / (out["backward"] / 1e3) / 1e12
    pol.close()
    return {"minibatch": batch, "precision": "split" if precision else "bf16",
            "forward_ms": out["forward"], "backward_ms": out["backward"],
            "forward_samples_per_s": batch / (out["forward"] / 1e3),
            "fwd_bwd_samples_per_s": batch / ((out["forward"] + out["backward"]) / 1e3),
            "forward_tflops": tf_f, "backward_tflops": tf_b,
            "mfma_frac_forward": tf_f / BF16_PEAK_TFLOPS, "mfma_frac_backward": tf_b / BF16_PEAK_TFLOPS,
            "flop_per_sample": {"forward": f_fwd, "backward_with_recompute": f_bwd}}


def cpu_full_loop(name: str, seed: int, robots: int, T: int, epochs: int) -> dict:
    """The oracle as it stands running one PPO iteration on the host: C oracle env (all host threads) and
    the FP64 PyTorch policy (forward per step, loss gradient by autograd, Adam), one minibatch per epoch."""
    import torch

    from oracle import oracle as O
    from oracle import policy_ref as PR
    from paper_2603_25834_amd import synth
    w = synth.WORKLOADS[name]
    idx = np.arange(min(robots, w.n_robots))
    n = len(idx)
    b = synth.make_batch(name, seed, idx)
    p = w.params()
    p["noise_seed"] = noise_seed(seed)
    env = O.OracleEnv(p, b.sides, b.world, b.world_off)
    env.reset(b.start)
    shape = PR.PolicyShape(w.n_rays)
    theta = torch.from_numpy(synth.init_policy_params(w.n_rays, seed)).double()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = min(threads, os.cpu_count() or threads)
    ranges = np.zeros((n, w.n_rays), np.float32)
    obs = {"crop": [], "scan": [], "state": []}
    act_l, logp_l, val_l, rew_l, done_l = [], [], [], [], []
    t0 = time.time()
    with torch.no_grad():
        for t in range(T + 1):
            crop, scan, state = env.observe(ranges)
            mu, ls, val = PR.forward(theta, torch.from_numpy(crop), torch.from_numpy(scan), torch.from_numpy(state),
                                     shape)
            val_l.append(val)
            if t == T:
                break
            for k, a in (("crop", crop), ("scan", scan), ("state", state)):
                obs[k].append(a)
            eps = O.normals(seed, O.DOMAIN_ACTION, t, n, 2)
            act = mu + torch.exp(ls) * torch.from_numpy(eps.astype(np.float64))
            act_l.append(act.float())
            logp_l.append(PR.gaussian_logp(mu, ls, act).float())
            o = env.step(act.float().numpy(), None, threads=threads)
            ranges = o.ranges
            rew_l.append(torch.from_numpy(o.reward))
            done_l.append(torch.from_numpy(o.done.astype(np.float64)))
            if o.done.any():
                env.reset(b.start, o.done)
    adv, ret = PR.gae(torch.stack(rew_l), torch.stack(val_l[:T]), torch.stack(done_l), val_l[T])
    flat = lambda xs: torch.from_numpy(np.concatenate(xs, 0))
    crop, scan, state = flat(obs["crop"]), flat(obs["scan"]), flat(obs["state"])
    act, old = torch.cat(act_l, 0), torch.cat(logp_l, 0)
    for e in range(epochs):
        th = theta.clone().requires_grad_(True)
        loss, _ = PR.ppo_loss(th, crop, scan, state, act, old, adv.reshape(-1).float(), ret.reshape(-1).float(),
                              shape)
        (g,) = torch.autograd.grad(loss, th)
        theta, m, v = PR.adam_step(theta, g, m, v, e + 1)
    dt = time.time() - t0
    return {"value": n * T / dt, "unit": "env-steps/s (PPO training loop)", "cores": threads, "kind": "oracle",
            "sample": f"{name}: first {n} robots, one iteration of {T} rollout steps + {epochs} epochs "
                      f"of one {n * T}-sample minibatch, FP64 policy ({dt:.1f} s)"}


def cpu_slam(seed: int, robots: int = 8, windows: int = 64, R: int = 360, L: int = 10, iters: int = 3) -> dict:
    """The SLAM oracle as it stands on a seeded synthetic sample of the benchmark's shapes (256^2 int16 grids
    with walls, 360 rays of up to 10 m at 0.05 m cells, the 9 x 9 x 11 lattice, 10-pose windows): scan
    matching, the oracle's own matches integrated into the grids, and the fixed-lag solve, per robot."""
    from oracle import slam_ref as S
    rng = np.random.default_rng([seed, 11])
    s, nang = 256, S.NANG
    lq = [218, -102, 896]
    rmax_q = 200 * 65536
    a_off = (np.arange(R) * (nang // R)).astype(np.int32)
    grids, poses, rhos = [], [], []
    for _ in range(robots):
        g = rng.integers(-300, 150, (s, s)).astype(np.int16)
        for _ in range(24):   # walls of strong occupied evidence
            y0, x0, ln = int(rng.integers(0, s)), int(rng.integers(0, s)), int(rng.integers(8, 64))
            if rng.random() < 0.5:
                g[y0, x0:x0 + ln] = 880
            else:
                g[y0:y0 + ln, x0] = 880
        rho = (rng.uniform(0.5, 200.0, R) * 65536).astype(np.int32)
        rho[rng.random(R) < 0.05] = -1
        grids.append(g)
        poses.append((int(rng.integers(64, 192)) * 65536 + 32768, int(rng.integers(64, 192)) * 65536 + 32768,
                      int(rng.integers(0, nang))))
        rhos.append(rho)
    trig = S._trig()
    t0 = time.time()
    matches = [S.csm_match(grids[r], *poses[r], rhos[r], a_off, 4, 5, 65536, 64, trig) for r in range(robots)]
    t_csm = (time.time() - t0) / robots
    t0 = time.time()
    for r in range(robots):
        S.integrate(grids[r], *poses[r], rhos[r], a_off, rmax_q, *lq, match=matches[r], step_xy=65536, step_h=64,
                    l_max=float(lq[2]))
    t_int = (time.time() - t0) / robots
    x0 = rng.uniform(-5.0, 5.0, (windows, 1, 3)) + 0.01 * rng.standard_normal((windows, L, 3))
    prior = np.concatenate([x0[:, 0], np.full((windows, 3), 400.0)], 1)
    odo = np.concatenate([np.zeros((windows, L - 1, 3)), np.full((windows, L - 1, 3), 2500.0)], 2)
    scan = np.zeros((windows, L, 6))
    scan[:, -1, :3] = x0[:, -1] + 0.02 * rng.standard_normal((windows, 3))
    scan[:, -1, 3:] = 100.0
    t0 = time.time()
    for w in range(windows):
        S.fixedlag_solve(x0[w], prior[w], odo[w], scan[w], iters)
    t_gn = (time.time() - t0) / windows
    return {"kind": "oracle", "cores": 1, "robots_per_s": 1.0 / (t_csm + t_int + t_gn),
            "csm_ms_per_robot": t_csm * 1e3, "integrate_ms_per_robot": t_int * 1e3,
            "fixedlag_ms_per_window": t_gn * 1e3,
            "sample": f"seeded synthetic: {robots} robots' scan matching and integration (256^2, {R} rays), "
                      f"{windows} windows of {L} poses"}


def cpu_baseline(name: str, seed: int, robots: int, steps: int, threads: int = 0) -> dict:
    """The oracle as it stands, all host threads (or `threads`), on a bounded sample of the workload."""
    from oracle import oracle as O
    from paper_2603_25834_amd import synth
    w = synth.WORKLOADS[name]
    idx = np.arange(min(robots, w.n_robots))
    b = synth.make_batch(name, seed, idx)
    A = synth.actions(name, seed, steps, idx)
    p = w.params()
    p["noise_seed"] = noise_seed(seed)
    env = O.OracleEnv(p, b.sides, b.world, b.world_off)
    env.reset(b.start)
    if threads <= 0:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        threads = min(threads, os.cpu_count() or threads)
    cnt = np.zeros(4, np.int64)
    t0 = time.time()
    for t in range(steps):
        o = env.step(A[t], None, threads=threads)
        cnt += o.counters.sum(0)
    dt = time.time() - t0
    rs = len(idx) * steps
    return {"value": rs / dt, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{name}: first {len(idx)} robots x {steps} steps ({dt:.1f} s)",
            "rays_per_s": rs * w.n_rays / dt,
            "coded_cells_per_robot_step": float(cnt[2]) / rs, "world_cells_read_per_robot_step": float(cnt[3]) / rs}


def train_loop(wb, horizon: int, epochs: int, minibatch: int, warmup: int, iters: int, seed: int,
               recurrent: bool = False, precision: int = 0) -> dict:
    """Time `iters` PPO training iterations on the workbench's env after `warmup` untimed ones (with
    `recurrent`, the GRU policy and sequence minibatches)."""
    import torch

    from paper_2603_25834_amd import synth
    from paper_2603_25834_amd.ppo import PPOTrainer
    wb.env.reset(wb.world, wb.start)
    init = synth.init_recurrent_params if recurrent else synth.init_policy_params
    params = torch.from_numpy(init(wb.R, seed)).cuda()
    tr = PPOTrainer(wb.env, wb.world, wb.start, params, T=horizon, epochs=epochs, minibatch=minibatch,
                    recurrent=recurrent, seed=seed, precision=precision)
    for i in range(warmup):
        tr.iteration()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    phases = [] if not recurrent else None
    e0.record()
    for i in range(warmup, warmup + iters):
        if phases is not None:
            tr.phase_events = tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
            phases.append(tr.phase_events)
        tr.iteration()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    split = {}
    if phases:
        split = {"rollout_ms": float(np.mean([a.elapsed_time(b) for a, b, _ in phases])),
                 "update_ms": float(np.mean([b.elapsed_time(c) for _, b, c in phases]))}
    out = {"ms_per_iteration": ms, "env_steps_per_s": wb.n * horizon / (ms / 1e3),
           "samples_per_iteration": tr.S, "minibatch": tr.mb, "minibatches_per_epoch": tr.n_mb,
           "iterations": iters, "final_loss_terms": [float(x) for x in tr.loss.cpu()],
           "policy_precision": "bf16" if recurrent or not precision else "split", **split}
    del tr
    torch.cuda.empty_cache()
    return out


def autotune_forms(wb) -> tuple:
    """Autotune the fused and the plain form on the workbench's own batch, then reset it."""
    from paper_2603_25834_amd import _lib
    from paper_2603_25834_amd.autotune import THREADS, Candidate, default_candidates, tune
    A = wb.dA[:8]
    out = (wb.ranges, wb.reward, wb.done)
    rf = tune(wb.env, A, None, *out, candidates=default_candidates(wb.env), force=True)
    fused = dict(rf["best"])
    rp = tune(wb.env, A, None, *out, candidates=[Candidate(t, form=_lib.FORM_PLAIN, mark_seg=g) for t in THREADS
                                                  for g in (0, 32)], force=True)
    plain = dict(rp["best"])
    wb.env.set_exec(**fused)
    wb.env.reset(wb.world, wb.start)
    # keys threads/band/grid/mark_seg
    key = lambda c: f"{c['threads']}/{c['band_rows']}/{c['grid']}/{c['mark_seg']}"
    summary = {"fused_us": {key(r["candidate"]): round(r["us_per_step"], 1) for r in rf["table"]
                            if r["us_per_step"] is not None},
               "plain_us": {key(r["candidate"]): round(r["us_per_step"], 1) for r in rp["table"]
                            if r["us_per_step"] is not None}}
    return fused, plain, summary


def side_workload(name: str, args, fused: dict, plain: dict, recurrent: bool = False) -> dict:
    """Env-step timings (fused and plain, each autotuned on this batch) and a few training iterations of a
    workload besides the headline one (with `recurrent`, also with the GRU policy)."""
    import torch
    print(f"[bench] {name}: setting up", file=sys.stderr, flush=True)
    wb2 = Workbench(name, args.seed, args.env_warmup + args.secondary_steps, fused)
    f2, p2, t2 = autotune_forms(wb2) if not args.threads else (fused, plain, {})
    r2 = wb2.run(args.env_warmup, args.secondary_steps)
    wb2.env.set_exec(**p2)
    wb2.env.reset(wb2.world, wb2.start)
    r2p = wb2.run(args.env_warmup, args.secondary_steps)
    res = {
        "workload": name, "robots": wb2.n, "rays": wb2.R, "steps": args.secondary_steps,
        "fused_env_steps_per_s": r2["env_steps_per_s"], "fused_rays_per_s": r2["rays_per_s"],
        "fused_us_per_step": r2["ms_per_step"] * 1e3, "plain_us_per_step": r2p["ms_per_step"] * 1e3,
        "plain_env_steps_per_s": r2p["env_steps_per_s"], "fused_speedup": r2["env_steps_per_s"] / r2p["env_steps_per_s"],
        "fused_hbm_gbs": r2["achieved_gbs"], "fused_hbm_frac": r2["achieved_gbs"] / HBM_PEAK_GBS,
        "coded_cells_per_robot_step": r2["coded_cells_per_robot_step"],
        "fused_exec": f2, "plain_exec": p2, "autotune": t2 or None}
    print(f"[bench] {name}: fused {r2['ms_per_step']*1e3:.1f} us/step, plain "
          f"{r2p['ms_per_step']*1e3:.1f} us/step", file=sys.stderr, flush=True)
    if args.secondary_iters > 0:
        wb2.env.set_exec(**f2)
        l2 = train_loop(wb2, args.horizon, args.epochs, args.minibatch, 1, args.secondary_iters, args.seed,
                        precision=args.precision)
        res["training_loop"] = l2
        print(f"[bench] {name}: training iteration {l2['ms_per_iteration']:.2f} ms", file=sys.stderr, flush=True)
        if recurrent:
            l3 = train_loop(wb2, args.horizon, args.epochs, args.minibatch, 1, args.secondary_iters, args.seed,
                            recurrent=True)
            res["training_loop_gru"] = l3
            print(f"[bench] {name}: training iteration with the GRU policy {l3['ms_per_iteration']:.2f} ms",
                  file=sys.stderr, flush=True)
    del wb2
    torch.cuda.empty_cache()
    return res


def fixedlag_workload(name: str, args, ex: dict) -> dict:
    """The paper's mode with the fixed-lag SLAM backbone in the loop: env steps (a sequence of launches:
    motion, march, scan matching, window, Gauss-Newton, weighted integration, reward) in one HIP graph,
    and training iterations with the split-precision MLP policy."""
    import torch
    from paper_2603_25834_amd import _lib
    print(f"[bench] {name}: setting up", file=sys.stderr, flush=True)
    ex = dict(ex, form=_lib.FORM_FUSED)
    wb = Workbench(name, args.seed, args.env_warmup + args.secondary_steps, ex)
    r = wb.run(args.env_warmup, args.secondary_steps)
    res = {"workload": name, "robots": wb.n, "rays": wb.R, "steps": args.secondary_steps,
           "lag_len": int(wb.p["lag_len"]), "gn_iters": int(wb.p["gn_iters"]),
           "lattice": [2 * int(wb.p["csm_W"]) + 1, 2 * int(wb.p["csm_W"]) + 1, 2 * int(wb.p["csm_V"]) + 1],
           "us_per_step": r["ms_per_step"] * 1e3, "env_steps_per_s": r["env_steps_per_s"],
           "rays_per_s": r["rays_per_s"], "coded_cells_per_robot_step": r["coded_cells_per_robot_step"]}
    print(f"[bench] {name}: {r['ms_per_step']*1e3:.1f} us/step", file=sys.stderr, flush=True)
    if args.secondary_iters > 0:
        lp = train_loop(wb, args.horizon, args.epochs, args.minibatch, 1, args.secondary_iters, args.seed,
                        precision=args.precision)
        res["training_loop"] = lp
        print(f"[bench] {name}: training iteration {lp['ms_per_iteration']:.2f} ms", file=sys.stderr, flush=True)
    del wb
    torch.cuda.empty_cache()
    return res


def full_loop(name: str, args, fused: dict, plain: dict) -> dict:
    """The full training loop on the largest workload: env-step timings (fused and plain, each autotuned on
    this batch) and PPO training iterations (rollout with the policy forward per step, then the update
    epochs with recomputation) with the env in the fused and in the plain form."""
    import torch
    print(f"[bench] {name}: setting up", file=sys.stderr, flush=True)
    wb = Workbench(name, args.seed, args.env_warmup + args.secondary_steps, fused)
    f2, p2, t2 = autotune_forms(wb) if not args.threads else (fused, plain, {})
    r_f = wb.run(args.env_warmup, args.secondary_steps)
    wb.env.set_exec(**p2)
    wb.env.reset(wb.world, wb.start)
    r_p = wb.run(args.env_warmup, args.secondary_steps)
    res = {"workload": name, "robots": wb.n, "rays": wb.R, "grid_side": sorted(set(map(int, wb.b.sides))),
           "r_max_m": wb.p["r_max_m"], "env_steps": args.secondary_steps,
           "fused_us_per_step": r_f["ms_per_step"] * 1e3, "plain_us_per_step": r_p["ms_per_step"] * 1e3,
           "fused_env_steps_per_s": r_f["env_steps_per_s"], "plain_env_steps_per_s": r_p["env_steps_per_s"],
           "fused_speedup": r_f["env_steps_per_s"] / r_p["env_steps_per_s"],
           "fused_hbm_frac": r_f["achieved_gbs"] / HBM_PEAK_GBS,
           "coded_cells_per_robot_step": r_f["coded_cells_per_robot_step"],
           "fused_exec": f2, "plain_exec": p2}
    print(f"[bench] {name}: fused {r_f['ms_per_step']*1e3:.1f} us/step, plain {r_p['ms_per_step']*1e3:.1f} us/step",
          file=sys.stderr, flush=True)
    for form, ex in (("fused", f2), ("plain", p2)):
        wb.env.set_exec(**ex)
        lp = train_loop(wb, args.horizon, args.epochs, args.minibatch, 1, args.full_iters, args.seed,
                        precision=args.precision)
        res[f"training_loop_{form}"] = lp
        print(f"[bench] {name}: training iteration ({form} env) {lp['ms_per_iteration']:.1f} ms "
              f"(rollout {lp.get('rollout_ms', 0):.1f}, update {lp.get('update_ms', 0):.1f})",
              file=sys.stderr, flush=True)
    res["end_to_end_env_steps_per_s"] = res["training_loop_fused"]["env_steps_per_s"]
    res["end_to_end_fused_speedup"] = (res["training_loop_plain"]["ms_per_iteration"] /
                                       res["training_loop_fused"]["ms_per_iteration"])
    del wb
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed PPO training iterations")
    ap.add_argument("--warmup", type=int, default=2, help="untimed PPO training iterations")
    ap.add_argument("--horizon", type=int, default=24, help="rollout steps per iteration")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--minibatch", type=int, default=16384)
    ap.add_argument("--env-steps", type=int, default=1000, help="env-only timing: steps in one HIP graph")
    ap.add_argument("--env-warmup", type=int, default=20)
    ap.add_argument("--workload", default="paper_750x256")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0, help="threads per robot; 0: autotune the launch shape")
    ap.add_argument("--band", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--mark-seg", type=int, default=0, help="with --threads: the map update's walk segments (0: one lane per ray)")
    ap.add_argument("--eager", action="store_true", help="eager launches instead of one HIP graph")
    ap.add_argument("--secondary", default="ragged_4096", help="second workload ('' to skip)")
    ap.add_argument("--secondary-steps", type=int, default=200)
    ap.add_argument("--secondary-iters", type=int, default=2, help="timed training iterations of the secondary")
    ap.add_argument("--paper-mode", default="paper_sensor_750x256",
                    help="workload of the paper's sensor / Eq. (7) reward mode, timed like the secondary ('' to skip)")
    ap.add_argument("--fixedlag", default="paper_fixedlag_750x256",
                    help="workload of the paper's mode with the fixed-lag SLAM backbone in the loop ('' to skip)")
    ap.add_argument("--full-loop", default="full_8192x512",
                    help="workload of the full-loop timing (env fused vs plain, training iterations; '' to skip)")
    ap.add_argument("--full-iters", type=int, default=2, help="timed training iterations of the full loop")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ppo", action="store_true")
    ap.add_argument("--only-ppo", action="store_true", help="time the PPO minibatch alone (profiling)")
    ap.add_argument("--only-env", action="store_true", help="time the env step alone (profiling)")
    ap.add_argument("--only-slam", action="store_true", help="time the SLAM backbone alone (profiling)")
    ap.add_argument("--ppo-batch", type=int, default=16384)
    ap.add_argument("--precision", type=int, default=1,
                    help="policy forward operands: 1 split hi + lo BF16 (gradients within 1e-2 of exact FP64), "
                         "0 BF16")
    ap.add_argument("--cpu-robots", type=int, default=640, help="oracle training-loop sample: robots")
    ap.add_argument("--cpu-env-robots", type=int, default=750, help="oracle env-step sample: robots")
    ap.add_argument("--cpu-env-steps", type=int, default=400, help="oracle env-step sample: steps")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (asked for --gpus {args.gpus}): the robots of a batch are independent "
              "and would be split across GPUs with no exchange, each GPU stepping its own share", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2603_25834_amd import _lib
    from paper_2603_25834_amd.env import device_info
    lds, cus = device_info()

    if args.only_ppo:   # profiling aid: the PPO minibatch timing alone
        print(json.dumps({"ppo": ppo_time(360, args.ppo_batch, args.seed, precision=args.precision)}), flush=True)
        return
    fused = dict(form=_lib.FORM_FUSED, threads=args.threads or 256, band_rows=args.band, grid=args.grid,
                 mark_seg=args.mark_seg)
    plain = dict(form=_lib.FORM_PLAIN, threads=args.threads or 256, band_rows=args.band, mark_seg=args.mark_seg)
    print(f"[bench] {args.workload}: setting up", file=sys.stderr, flush=True)
    wb = Workbench(args.workload, args.seed, args.env_warmup + args.env_steps, fused)
    tuned = {}
    if not args.threads:
        fused, plain, tuned = autotune_forms(wb)
        print(f"[bench] autotuned: fused {fused}, plain {plain}", file=sys.stderr, flush=True)
    # ---- the env step alone: one HIP graph of env_steps fused steps, then the plain form
    res = wb.run(args.env_warmup, args.env_steps, graph=not args.eager)
    print(f"[bench] env step, fused: {res['ms_per_step']*1e3:.1f} us/step", file=sys.stderr, flush=True)
    obs_ms = wb.observe_time()
    wb.env.set_exec(**plain)
    wb.env.reset(wb.world, wb.start)
    res_plain = wb.run(args.env_warmup, args.env_steps, graph=not args.eager)
    print(f"[bench] env step, plain: {res_plain['ms_per_step']*1e3:.1f} us/step", file=sys.stderr, flush=True)
    if args.calib_copy:
        src = torch.ones(args.calib_copy << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    traffic = read_traffic("k_fused", args.workload, fused["threads"], fused.get("mark_seg", 0))
    if args.only_env:   # profiling aid: the env-step timings alone
        print(json.dumps({"env_step_ms": res["ms_per_step"], "plain_step_ms": res_plain["ms_per_step"],
                          "observe_ms": obs_ms, "alg_bytes_per_launch": res["alg_bytes_per_step"],
                          "achieved_gbs": res["achieved_gbs"], "traffic": traffic}), flush=True)
        return
    slam_res = slam_time(wb)
    print(f"[bench] SLAM backbone: scan matching {slam_res['csm_us']:.1f} us, factors {slam_res['factor_us']:.1f} us, "
          f"weighted integration {slam_res['integrate_us']:.1f} us, fixed-lag solve {slam_res['fixedlag_us']:.1f} us for {wb.n} robots", file=sys.stderr, flush=True)
    if args.only_slam:   # profiling aid: the SLAM backbone alone
        print(json.dumps({"slam": slam_res}), flush=True)
        return
    # ---- the bench step: one PPO training iteration (rollout of `horizon` steps + update)
    wb.env.set_exec(**fused)
    loop = train_loop(wb, args.horizon, args.epochs, args.minibatch, args.warmup, args.steps, args.seed,
                      precision=args.precision)
    print(f"[bench] training iteration: {loop['ms_per_iteration']:.2f} ms "
          f"({loop['env_steps_per_s']:.4g} env-steps/s)", file=sys.stderr, flush=True)
    value = loop["env_steps_per_s"]
    loop_other = train_loop(wb, args.horizon, args.epochs, args.minibatch, 1, max(2, args.steps // 2), args.seed,
                            precision=1 - args.precision)
    print(f"[bench] training iteration, {loop_other['policy_precision']} policy: "
          f"{loop_other['ms_per_iteration']:.2f} ms", file=sys.stderr, flush=True)

    copy_gbs = copy_bandwidth()   # after the profiling exits above, so counter passes see only their own copy
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": loop["ms_per_iteration"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+bf16" if args.precision == 0 else "int32+bf16x3",
        "data": "synthetic (seeded worlds, start poses and env-timing actions; odometry, loop-closure and action "
                "noise and minibatch permutations from the library's counter-based generator in the kernels; "
                "random-init policy)",
        "config": {"workload": args.workload, "robots": wb.n, "grid_side": sorted(set(map(int, wb.b.sides))),
                   "rays": wb.R, "r_max_m": wb.p["r_max_m"], "cell_m": wb.p["cell_m"],
                   "loop_closure": int(wb.p["loop_closure"]),
                   "step": f"one PPO iteration: {args.horizon} env steps (fused persistent form) with observe, "
                           f"policy forward and action sampling per step, GAE, {args.epochs} epochs of "
                           f"minibatches <= {args.minibatch} (gather, loss+gradient with recompute, Adam)",
                   "policy_precision": loop["policy_precision"],
                   "horizon": args.horizon, "epochs": args.epochs, "minibatch": loop["minibatch"],
                   "minibatches_per_epoch": loop["minibatches_per_epoch"],
                   "threads": fused["threads"], "band_rows": fused.get("band_rows", 0),
                   "grid": fused.get("grid", 0), "mark_seg": fused.get("mark_seg", 0),
                   "plain_threads": plain["threads"],
                   "lds_bytes": wb.env.get_exec()["lds_bytes"]},
        "rays_per_s": value * wb.R,
        "slam": slam_res,
        "training_loop": loop,
        "training_loop_other_precision": loop_other,
        "env_step_only": {"env_steps_per_s": wb.n / ((res["ms_per_step"] + obs_ms) / 1e3),
                          "rays_per_s": wb.n * wb.R / ((res["ms_per_step"] + obs_ms) / 1e3),
                          "step_ms": res["ms_per_step"], "observe_ms": obs_ms, "steps": args.env_steps,
                          "form": "fused persistent, HIP graph"},
        "plain_form": {"env_steps_per_s": res_plain["env_steps_per_s"], "ms_per_step": res_plain["ms_per_step"],
                       "fused_speedup": res["env_steps_per_s"] / res_plain["env_steps_per_s"]},
        "roofline_valu": valu_roofline("k_fused", args.workload, fused["threads"], fused.get("mark_seg", 0),
                                       res["ms_per_step"]),
        "hbm_copy_gbs": copy_gbs,
        "roofline": {"bound": "hbm", "achieved": res["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": res["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"k_fused<{fused['threads']}, {'true' if fused.get('mark_seg', 0) else 'false'}>",
                     "mark_seg": fused.get("mark_seg", 0), "alg_bytes_per_launch": res["alg_bytes_per_step"],
                     "avg_launch_ms": res["ms_per_step"],
                     "coded_cells_per_robot_step": res["coded_cells_per_robot_step"],
                     "cell_visits_per_robot_step": res["march_visits_per_robot_step"] +
                     res["update_visits_per_robot_step"]},
        "device": {"lds_per_block": lds, "compute_units": cus},
        "autotune": tuned or None,
    }
    del wb
    torch.cuda.empty_cache()
    if not args.no_ppo:
        print(f"[bench] PPO minibatch {args.ppo_batch}", file=sys.stderr, flush=True)
        out["ppo"] = ppo_time(out["config"]["rays"], args.ppo_batch, args.seed, precision=args.precision)
        out["ppo_other_precision"] = ppo_time(out["config"]["rays"], args.ppo_batch, args.seed,
                                              precision=1 - args.precision)
        for k in ("ppo", "ppo_other_precision"):
            print(f"[bench] PPO ({out[k]['precision']}) fwd {out[k]['forward_ms']:.3f} ms, "
                  f"fwd+bwd(recompute) {out[k]['backward_ms']:.3f} ms", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    for key, name in (("secondary", args.secondary), ("paper_mode", args.paper_mode)):
        if name:
            out[key] = side_workload(name, args, fused, plain, recurrent=key == "paper_mode")
    if args.fixedlag:
        ex = out.get("paper_mode", {}).get("fused_exec") or fused
        out.setdefault("paper_mode", {})["fixedlag"] = fixedlag_workload(args.fixedlag, args, ex)
    if args.full_loop:
        out["full_loop"] = full_loop(args.full_loop, args, fused, plain)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_full_loop(args.workload, args.seed, args.cpu_robots, args.horizon, args.epochs)
        out["cpu_baseline"]["env_step_only"] = cpu_baseline(args.workload, args.seed, args.cpu_env_robots,
                                                            args.cpu_env_steps)
        out["cpu_baseline"]["slam"] = cpu_slam(args.seed)
        out["cpu_baseline"]["env_step_single_thread"] = cpu_baseline(args.workload, args.seed, 64, 100, threads=1)
    out["context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
