"""FP64 CPU oracle of the recurrent actor-critic (a single-layer GRU of 256 units) and its PPO loss.

TEST INFRASTRUCTURE ONLY: used by tests/ and never by the product path.  Plain PyTorch CPU ops in
float64; the gradient is PyTorch autograd through the whole sequence (backpropagation through time).

Method: arXiv 2603.25834, Sec. III-F ("Recurrent Layer"): the policy carries temporal context in a
single-layer GRU with a hidden size of 256.  Here the GRU takes the place of the second fully
connected layer of the workload's actor-critic (the convolutional encoder of the belief crop, FC1 of
256 with ReLU, then the GRU, then the Gaussian mean and value heads on the GRU state).  The GRU cell
is the standard one (Cho et al. 2014, gate order reset / update / new as in common libraries):
    r = sigmoid(W_ir x + b_ir + W_hr h + b_hr)
    z = sigmoid(W_iz x + b_iz + W_hz h + b_hz)
    n = tanh(W_in x + b_in + r * (W_hn h + b_hn))
    h' = (1 - z) * n + z * h
A sequence runs over the T steps of a rollout for a set of robots; the hidden state is set to zero
before a step that starts a new episode (first[t] = 1), so no state crosses an episode boundary.
The loss is the clipped surrogate of Eqs. (18)-(20) plus the value and entropy terms, averaged over
all T x robots samples, as for the feed-forward policy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from .policy_ref import (C1, C2, CROP, HID, NACT, NSTATE, _RoundBoth, _RoundGrad, _RoundValue, gaussian_entropy,
                         gaussian_logp, round_bf16)

GATES = 3 * HID


@dataclass(frozen=True)
class RecurrentShape:
    n_scan: int = 128

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
            ("gru.w_ih", (GATES, HID)), ("gru.w_hh", (GATES, HID)),
            ("gru.b_ih", (GATES,)), ("gru.b_hh", (GATES,)),
            ("mu.w", (NACT, HID)), ("mu.b", (NACT,)),
            ("v.w", (1, HID)), ("v.b", (1,)),
            ("log_std", (NACT,)),
        ]

    def n_params(self) -> int:
        return sum(math.prod(s) for _, s in self.param_layout())


def unflatten(theta: torch.Tensor, shape: RecurrentShape) -> dict:
    out, o = {}, 0
    for name, shp in shape.param_layout():
        n = math.prod(shp)
        out[name] = theta[o:o + n].view(shp)
        o += n
    assert o == theta.numel()
    return out


def gru_cell(x: torch.Tensor, h: torch.Tensor, w_ih, w_hh, b_ih, b_hh) -> torch.Tensor:
    """One GRU step for a batch: x [B, 256], h [B, 256] -> h' [B, 256] (equations in the module doc)."""
    gi = x @ w_ih.T + b_ih
    gh = h @ w_hh.T + b_hh
    r = torch.sigmoid(gi[:, :HID] + gh[:, :HID])
    z = torch.sigmoid(gi[:, HID:2 * HID] + gh[:, HID:2 * HID])
    n = torch.tanh(gi[:, 2 * HID:] + r * gh[:, 2 * HID:])
    return (1.0 - z) * n + z * h


def _encode(p: dict, crop, scan, state, rounding: bool):
    """FC1 output h1 for a flat batch (conv encoder + FC1 + ReLU), at FP64 or at the workload's precision."""
    rv = _RoundValue.apply if rounding else (lambda t: t)
    rb = _RoundBoth.apply if rounding else (lambda t: t)
    x = crop.to(torch.float64).unsqueeze(1) / 256.0
    x = round_bf16(x) if rounding else x
    a1 = rb(torch.relu(torch.nn.functional.conv2d(x, rv(p["conv1.w"]), p["conv1.b"], stride=2, padding=1)))
    a2 = rb(torch.relu(torch.nn.functional.conv2d(a1, rv(p["conv2.w"]), p["conv2.b"], stride=2, padding=1)))
    sc, st = scan.to(torch.float64), state.to(torch.float64)
    if rounding:
        sc, st = round_bf16(sc), round_bf16(st)
    feat = torch.cat([a2.flatten(1), sc, st], dim=1)
    return rb(torch.relu(feat @ rv(p["fc1.w"]).T + p["fc1.b"]))


def forward_seq(theta: torch.Tensor, crop, scan, state, h0, first, shape: RecurrentShape, rounding: bool = False):
    """A rollout segment: crop [T, nb, 64, 64], scan [T, nb, R], state [T, nb, 12], h0 [nb, 256] the
    hidden state entering step 0, first [T, nb] (1: step t starts an episode, the state is zeroed
    before it).  Returns (mu [T, nb, 2], log_std, value [T, nb], h_T [nb, 256]).

    rounding=True evaluates the workload's precision: BF16 operands for every GEMM (weights, the FC1
    output, the GRU state fed to W_hh) and BF16 gradients wherever the backward feeds a GEMM (the gate
    pre-activation gradients), FP32-class accumulation taken as FP64; rounding=False is exact FP64."""
    T, nb = crop.shape[0], crop.shape[1]
    p = unflatten(theta, shape)
    rv = _RoundValue.apply if rounding else (lambda t: t)
    rg = _RoundGrad.apply if rounding else (lambda t: t)
    h1 = _encode(p, crop.reshape(T * nb, CROP, CROP), scan.reshape(T * nb, -1), state.reshape(T * nb, -1), rounding)
    h1 = h1.view(T, nb, HID)
    w_ih, w_hh = rv(p["gru.w_ih"]), rv(p["gru.w_hh"])
    h = h0.to(torch.float64)
    hs = []
    for t in range(T):
        keep = (1.0 - first[t].to(torch.float64)).unsqueeze(1)
        h = h * keep
        gi = rg(h1[t] @ w_ih.T + p["gru.b_ih"])
        gh = rg(rv(h) @ w_hh.T + p["gru.b_hh"])
        r = torch.sigmoid(gi[:, :HID] + gh[:, :HID])
        z = torch.sigmoid(gi[:, HID:2 * HID] + gh[:, HID:2 * HID])
        n = torch.tanh(gi[:, 2 * HID:] + r * gh[:, 2 * HID:])
        h = (1.0 - z) * n + z * h
        hs.append(h)
    g = torch.stack(hs)
    mu = g @ p["mu.w"].T + p["mu.b"]
    value = (g @ p["v.w"].T + p["v.b"]).squeeze(-1)
    return mu, p["log_std"], value, h


def ppo_loss_seq(theta, crop, scan, state, h0, first, act, old_logp, adv, ret, shape, eps=0.2, c_v=0.5,
                 c_e=0.005, rounding: bool = False):
    """Total loss and its three terms over the T x nb samples of forward_seq (means over all samples)."""
    mu, log_std, value, _ = forward_seq(theta, crop, scan, state, h0, first, shape, rounding)
    logp = gaussian_logp(mu, log_std, act.to(torch.float64))
    ratio = torch.exp(logp - old_logp.to(torch.float64))
    adv = adv.to(torch.float64)
    surr = torch.minimum(ratio * adv, torch.clamp(ratio, 1.0 - eps, 1.0 + eps) * adv)
    l_clip = -surr.mean()
    l_v = ((value - ret.to(torch.float64)) ** 2).mean()
    ent = gaussian_entropy(log_std)
    total = l_clip + c_v * l_v - c_e * ent
    return total, torch.stack([l_clip, l_v, ent])
