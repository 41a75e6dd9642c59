"""FP64 CPU oracle of the PPO actor-critic, its loss, GAE and Adam.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product path.  Plain PyTorch CPU ops in float64.

Method: arXiv 2603.25834, Sec. III-F.  PPO's clipped surrogate, Eqs. (18)-(20):
    r_t = pi(a|o) / pi_old(a|o),   rbar_t = clip(r_t, 1-eps, 1+eps),
    L = -E[min(r_t A_t, rbar_t A_t)],
with advantages from Generalized Advantage Estimation (same section).  The
network is the workload's actor-critic (the paper's GRU policy is a later
row): two 3x3 stride-2 convolutions (16 and 32 channels, padding 1, ReLU) on a
64x64 belief crop, the flattened features concatenated with the normalised
scan and the 12-float pose/covariance state, two fully connected layers of 256
(ReLU), a Gaussian policy head (mean of 2 actions, state-independent log std)
and a value head.  The loss adds the usual value and entropy terms:
    total = L_clip + c_v * mean((V - R)^2) - c_e * H[pi].
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

CROP = 64
C1, C2 = 16, 32
HID = 256
NACT = 2
NSTATE = 12


@dataclass(frozen=True)
class PolicyShape:
    n_scan: int = 360

    @property
    def n_feat(self) -> int:
        return C2 * (CROP // 4) * (CROP // 4)

    @property
    def k1(self) -> int:
        return self.n_feat + self.n_scan + NSTATE

    def param_layout(self):
        """(name, shape) in the order of the flat parameter vector."""
        return [
            ("conv1.w", (C1, 1, 3, 3)), ("conv1.b", (C1,)),
            ("conv2.w", (C2, C1, 3, 3)), ("conv2.b", (C2,)),
            ("fc1.w", (HID, self.k1)), ("fc1.b", (HID,)),
            ("fc2.w", (HID, HID)), ("fc2.b", (HID,)),
            ("mu.w", (NACT, HID)), ("mu.b", (NACT,)),
            ("v.w", (1, HID)), ("v.b", (1,)),
            ("log_std", (NACT,)),
        ]

    def n_params(self) -> int:
        return sum(math.prod(s) for _, s in self.param_layout())


def unflatten(theta: torch.Tensor, shape: PolicyShape) -> dict:
    out, o = {}, 0
    for name, shp in shape.param_layout():
        n = math.prod(shp)
        out[name] = theta[o:o + n].view(shp)
        o += n
    assert o == theta.numel()
    return out


def forward(theta: torch.Tensor, crop: torch.Tensor, scan: torch.Tensor, state: torch.Tensor,
            shape: PolicyShape):
    """crop: int16 log-odds [B,64,64] (1/256 nat); scan [B,R]; state [B,12].  Returns (mu, log_std, value)."""
    p = unflatten(theta, shape)
    x = crop.to(torch.float64).unsqueeze(1) / 256.0
    a1 = torch.relu(torch.nn.functional.conv2d(x, p["conv1.w"], p["conv1.b"], stride=2, padding=1))
    a2 = torch.relu(torch.nn.functional.conv2d(a1, p["conv2.w"], p["conv2.b"], stride=2, padding=1))
    feat = torch.cat([a2.flatten(1), scan.to(torch.float64), state.to(torch.float64)], dim=1)
    h1 = torch.relu(feat @ p["fc1.w"].T + p["fc1.b"])
    h2 = torch.relu(h1 @ p["fc2.w"].T + p["fc2.b"])
    mu = h2 @ p["mu.w"].T + p["mu.b"]
    value = (h2 @ p["v.w"].T + p["v.b"]).squeeze(1)
    return mu, p["log_std"], value


def gaussian_logp(mu: torch.Tensor, log_std: torch.Tensor, act: torch.Tensor) -> torch.Tensor:
    """log N(act; mu, diag(exp(log_std))^2), summed over the action dims."""
    z = (act - mu) / torch.exp(log_std)
    return -0.5 * (z * z).sum(-1) - log_std.sum() - 0.5 * act.shape[-1] * math.log(2.0 * math.pi)


def gaussian_entropy(log_std: torch.Tensor) -> torch.Tensor:
    return (log_std + 0.5 * math.log(2.0 * math.pi * math.e)).sum()


def ppo_loss(theta, crop, scan, state, act, old_logp, adv, ret, shape, eps=0.2, c_v=0.5, c_e=0.005):
    """Total loss and its three terms (clipped surrogate, value, entropy), Eqs. (18)-(20) + value/entropy."""
    mu, log_std, value = forward(theta, crop, scan, state, shape)
    logp = gaussian_logp(mu, log_std, act.to(torch.float64))
    ratio = torch.exp(logp - old_logp.to(torch.float64))
    adv = adv.to(torch.float64)
    surr = torch.minimum(ratio * adv, torch.clamp(ratio, 1.0 - eps, 1.0 + eps) * adv)
    l_clip = -surr.mean()
    l_v = ((value - ret.to(torch.float64)) ** 2).mean()
    ent = gaussian_entropy(log_std)
    total = l_clip + c_v * l_v - c_e * ent
    return total, torch.stack([l_clip, l_v, ent])


def gae(rewards, values, dones, last_value, gamma=0.99, lam=0.95):
    """Generalized Advantage Estimation over a [T, N] rollout.

    delta_t = r_t + gamma * V_{t+1} * (1 - d_t) - V_t, A_t = sum_l (gamma lam)^l delta_{t+l}
    with the sum cut at episode ends (d_t = 1 ends the episode after step t).
    Returns (advantages, returns = advantages + values), float64."""
    r = rewards.to(torch.float64)
    v = values.to(torch.float64)
    d = dones.to(torch.float64)
    T = r.shape[0]
    adv = torch.zeros_like(r)
    nxt_v = last_value.to(torch.float64)
    acc = torch.zeros_like(nxt_v)
    for t in range(T - 1, -1, -1):
        nonterm = 1.0 - d[t]
        delta = r[t] + gamma * nxt_v * nonterm - v[t]
        acc = delta + gamma * lam * nonterm * acc
        adv[t] = acc
        nxt_v = v[t]
    return adv, adv + v


def adam_step(theta, grad, m, v, step, lr=3e-4, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): bias-corrected first/second moments; returns new (theta, m, v)."""
    th = theta.to(torch.float64)
    g = grad.to(torch.float64)
    m = beta1 * m.to(torch.float64) + (1.0 - beta1) * g
    v = beta2 * v.to(torch.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    th = th - lr * mhat / (torch.sqrt(vhat) + eps)
    return th, m, v


# ------------------------------------------------------- workload precision
# The workload runs the network with BF16 operands and FP32 accumulation.  The
# functions below evaluate the same network in FP64 with BF16 rounding (round
# to nearest even) applied exactly where the workload stores or feeds BF16
# values: GEMM / convolution weights, the crop and FC1's scan/state inputs, the
# ReLU outputs between layers, and the gradients that the backward pass feeds
# to the next GEMM (the gradient at each hidden ReLU output).  Everything else
# (accumulation, biases, heads, loss) stays FP64.

def round_bf16(x: torch.Tensor) -> torch.Tensor:
    return x.to(torch.bfloat16).to(torch.float64)


class _RoundValue(torch.autograd.Function):
    """Rounds the value; the gradient passes through unchanged."""

    @staticmethod
    def forward(ctx, x):
        return round_bf16(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Leaves the value; rounds the incoming gradient."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return round_bf16(g)


class _RoundBoth(torch.autograd.Function):
    """Rounds the value and the incoming gradient."""

    @staticmethod
    def forward(ctx, x):
        return round_bf16(x)

    @staticmethod
    def backward(ctx, g):
        return round_bf16(g)


def forward_bf16(theta: torch.Tensor, crop: torch.Tensor, scan: torch.Tensor, state: torch.Tensor,
                 shape: PolicyShape, rounding: bool = True):
    """forward() at the workload's precision (see above); rounding=False gives forward() exactly."""
    rv = _RoundValue.apply if rounding else (lambda t: t)
    rg = _RoundGrad.apply if rounding else (lambda t: t)
    rb = _RoundBoth.apply if rounding else (lambda t: t)
    p = unflatten(theta, shape)
    x = crop.to(torch.float64).unsqueeze(1) / 256.0
    x = round_bf16(x) if rounding else x
    a1 = rb(torch.relu(torch.nn.functional.conv2d(x, rv(p["conv1.w"]), p["conv1.b"], stride=2, padding=1)))
    a2 = rb(torch.relu(torch.nn.functional.conv2d(a1, rv(p["conv2.w"]), p["conv2.b"], stride=2, padding=1)))
    sc, st = scan.to(torch.float64), state.to(torch.float64)
    if rounding:
        sc, st = round_bf16(sc), round_bf16(st)
    feat = torch.cat([a2.flatten(1), sc, st], dim=1)
    h1 = rb(torch.relu(feat @ rv(p["fc1.w"]).T + p["fc1.b"]))
    h2 = rg(torch.relu(h1 @ rv(p["fc2.w"]).T + p["fc2.b"]))
    mu = h2 @ p["mu.w"].T + p["mu.b"]
    value = (h2 @ p["v.w"].T + p["v.b"]).squeeze(1)
    return mu, p["log_std"], value


def ppo_loss_bf16(theta, crop, scan, state, act, old_logp, adv, ret, shape, eps=0.2, c_v=0.5, c_e=0.005,
                  rounding: bool = True):
    """ppo_loss() on forward_bf16(); its autograd gradient is the workload-precision gradient."""
    mu, log_std, value = forward_bf16(theta, crop, scan, state, shape, rounding)
    logp = gaussian_logp(mu, log_std, act.to(torch.float64))
    ratio = torch.exp(logp - old_logp.to(torch.float64))
    adv = adv.to(torch.float64)
    surr = torch.minimum(ratio * adv, torch.clamp(ratio, 1.0 - eps, 1.0 + eps) * adv)
    l_clip = -surr.mean()
    l_v = ((value - ret.to(torch.float64)) ** 2).mean()
    ent = gaussian_entropy(log_std)
    total = l_clip + c_v * l_v - c_e * ent
    return total, torch.stack([l_clip, l_v, ent])
