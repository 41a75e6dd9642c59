"""Pins of the recurrent-policy oracle (CPU only).

Paper passage: arXiv 2603.25834, Sec. III-F, "Recurrent Layer" (a single-layer GRU of 256 units);
PPO loss Eqs. (18)-(20).  The oracle writes the GRU cell out; it is pinned against PyTorch's own
GRUCell (an independent implementation of the same definition), against the closed form of a
saturated update gate, against the episode-reset semantics (a reset sequence equals a fresh one), and
its backpropagation-through-time gradient against FP64 central differences.
"""
import numpy as np
import pytest
import torch

from oracle import gru_ref as G
from paper_2603_25834_amd import synth

R = 16
SHAPE = G.RecurrentShape(n_scan=R)


def _theta(seed=0):
    th = synth.init_recurrent_params(R, seed)
    assert th.size == SHAPE.n_params()
    assert [n for n, _ in synth.recurrent_param_layout(R)] == [n for n, _ in SHAPE.param_layout()]
    return torch.from_numpy(th).double()


def _batch(T, nb, seed=0, reset_p=0.0):
    d = synth.recurrent_batch(T, nb, R, seed, reset_p)
    return {k: torch.from_numpy(v) for k, v in d.items()}


def test_cell_matches_torch_grucell():
    torch.manual_seed(0)
    cell = torch.nn.GRUCell(256, 256).double()
    x = torch.randn(7, 256, dtype=torch.float64)
    h = torch.randn(7, 256, dtype=torch.float64)
    want = cell(x, h)
    got = G.gru_cell(x, h, cell.weight_ih, cell.weight_hh, cell.bias_ih, cell.bias_hh)
    assert torch.allclose(got, want, rtol=1e-12, atol=1e-13)


def test_reset_restarts_the_sequence():
    """first[k] = 1 zeroes the state before step k: steps k.. equal a fresh sequence from h = 0."""
    th = _theta(1)
    d = _batch(6, 3, 1)
    first = torch.zeros(6, 3, dtype=torch.uint8)
    first[3] = 1
    mu, _, v, _ = G.forward_seq(th, d["crop"], d["scan"], d["state"], d["h0"], first, SHAPE)
    mu2, _, v2, _ = G.forward_seq(th, d["crop"][3:], d["scan"][3:], d["state"][3:], torch.zeros(3, 256),
                                  torch.zeros(3, 3, dtype=torch.uint8), SHAPE)
    assert torch.allclose(mu[3:], mu2, rtol=1e-13, atol=1e-14) and torch.allclose(v[3:], v2, rtol=1e-13, atol=1e-14)
    # and the steps before it do depend on h0
    mu3, _, _, _ = G.forward_seq(th, d["crop"], d["scan"], d["state"], torch.zeros(3, 256), first, SHAPE)
    assert not torch.allclose(mu[:3], mu3[:3])


def test_saturated_update_gate_carries_the_state():
    """With b_iz = +60 the update gate is 1 (to FP64 precision): h_t = h_0 at every step, so the heads see
    the entering state: mu_t = W_mu h0 + b_mu for all t."""
    th = _theta(2)
    p = G.unflatten(th, SHAPE)
    p["gru.b_ih"][256:512] = 60.0
    d = _batch(4, 2, 2)
    mu, _, v, hT = G.forward_seq(th, d["crop"], d["scan"], d["state"], d["h0"], torch.zeros(4, 2), SHAPE)
    h0 = d["h0"].double()
    want = h0 @ p["mu.w"].T + p["mu.b"]
    assert torch.allclose(mu, want.expand_as(mu), rtol=1e-12, atol=1e-12)
    assert torch.allclose(hT, h0, rtol=0, atol=1e-20)


def test_workload_precision_is_close_and_reduces_exactly():
    th = _theta(3)
    d = _batch(5, 3, 3, 0.2)
    a = G.forward_seq(th, d["crop"], d["scan"], d["state"], d["h0"], d["first"], SHAPE, rounding=False)
    b = G.forward_seq(th, d["crop"], d["scan"], d["state"], d["h0"], d["first"], SHAPE, rounding=True)
    for x, y in ((a[0], b[0]), (a[2], b[2])):
        assert torch.linalg.norm(x - y) / torch.linalg.norm(x) < 2e-2


def test_bptt_gradient_central_differences():
    """The autograd gradient of the sequence loss (exact FP64) along random directions equals central
    differences of the loss; the directions cover the GRU, FC1 and head parameters."""
    th = _theta(4)
    d = _batch(3, 2, 4, 0.3)
    d["first"][1, 0] = 1
    args = (d["crop"], d["scan"], d["state"], d["h0"], d["first"], d["act"], d["old_logp"], d["adv"], d["ret"], SHAPE)
    t = th.clone().requires_grad_(True)
    loss, _ = G.ppo_loss_seq(t, *args)
    (g,) = torch.autograd.grad(loss, t)
    rng = np.random.default_rng(4)
    lay = SHAPE.param_layout()
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in lay])
    for name in ("gru.w_hh", "gru.w_ih", "gru.b_hh", "fc1.w", "mu.w"):
        k = [n for n, _ in lay].index(name)
        u = torch.zeros_like(th)
        u[offs[k]:offs[k + 1]] = torch.from_numpy(rng.standard_normal(offs[k + 1] - offs[k]))
        u /= torch.linalg.norm(u)
        eps = 1e-5
        lp, _ = G.ppo_loss_seq(th + eps * u, *args)
        lm, _ = G.ppo_loss_seq(th - eps * u, *args)
        fd = (lp - lm) / (2 * eps)
        an = torch.dot(g, u)
        assert abs(float(fd - an)) <= 1e-6 * max(1.0, abs(float(an))), (name, float(fd), float(an))
