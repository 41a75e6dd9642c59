"""GPU recurrent policy (GRU of 256 units, Sec. III-F) vs the CPU oracle, through the C-ABI.

Bar (as for the feed-forward policy): rollout outputs within 3e-3 (relative L2) and every mu, V and
state element within 2e-3 of the workload-precision oracle (BF16 operands at the same points; FP32 vs
FP64 gate math and state over the steps), 3e-2 of exact FP64 both ways; the backpropagation-through-
time gradient per parameter tensor within 1e-2 (relative L2) of the workload-precision oracle's
autograd gradient, two runs bit-identical; against the exact FP64 network on coherent minibatches
(advantages +1) within 5e-2 (conv tensors) / 2e-2 (the rest) by autograd, and within 1e-2 per tensor
by central differences along each tensor's gradient.
"""
import numpy as np
import pytest
import torch

from envpair import say
from oracle import gru_ref as G
from paper_2603_25834_amd import synth

pytestmark = pytest.mark.gpu

R = 128
SHAPE = G.RecurrentShape(n_scan=R)


def _seq_case(T, N, seed, reset_p=0.1):
    theta = synth.init_recurrent_params(R, seed)
    d = synth.recurrent_batch(T, N, R, seed, reset_p)
    t = {k: torch.from_numpy(v) for k, v in d.items()}
    with torch.no_grad():
        mu, ls, _, _ = G.forward_seq(torch.from_numpy(theta).double(), t["crop"], t["scan"], t["state"], t["h0"],
                                     t["first"], SHAPE)
        logp = -0.5 * (((t["act"].double() - mu) / torch.exp(ls)) ** 2).sum(-1) - ls.sum() - np.log(2 * np.pi)
    rng = np.random.default_rng([seed, 98])
    shift = np.where(rng.random((T, N)) < 0.7, rng.uniform(-0.1, 0.1, (T, N)), rng.choice([-0.5, 0.5], (T, N)))
    t["old_logp"] = (logp - torch.from_numpy(shift)).float()
    return theta, t


def _policy(max_batch):
    from paper_2603_25834_amd.policy import Policy
    return Policy(R, max_batch=max_batch, recurrent=True)


def test_rollout_steps_match_oracle():
    """Six rollout steps of 200 robots, the state fed back, episode starts zeroing it."""
    T, N = 6, 200
    theta, t = _seq_case(T, N, 1, 0.15)
    pol = _policy(N)
    params = torch.from_numpy(theta).cuda()
    dev = {k: v.cuda().contiguous() for k, v in t.items()}
    eps = torch.from_numpy(np.random.default_rng(1).normal(size=(T, N, 2)).astype(np.float32)).cuda()
    h = dev["h0"].clone()
    mus, vals = [], []
    pol.prepare(params)
    for s in range(T):
        mu = torch.empty((N, 2), device="cuda")
        v, a, lp, h = pol.act_rnn(params, dev["crop"][s], dev["scan"][s], dev["state"][s], h, dev["first"][s],
                                  eps[s], mu=mu, h_out=h, prepared=True)
        mus.append(mu)
        vals.append(v)
        # the sample uses the mean and the log std exactly as aslam_policy_sample does
        ls = params[-2:]
        assert torch.allclose(a, mu + torch.exp(ls) * eps[s], rtol=1e-6, atol=1e-6)
    torch.cuda.synchronize()
    gm = torch.stack(mus).cpu().double()
    gv = torch.stack(vals).cpu().double()
    with torch.no_grad():
        th = torch.from_numpy(theta).double()
        mb, _, vb, hb = G.forward_seq(th, t["crop"], t["scan"], t["state"], t["h0"], t["first"], SHAPE, rounding=True)
        me, _, ve, he = G.forward_seq(th, t["crop"], t["scan"], t["state"], t["h0"], t["first"], SHAPE)
    rel = lambda x, y: float(torch.linalg.norm(x - y) / torch.linalg.norm(y))
    eb = max(rel(gm, mb), rel(gv, vb), rel(h.cpu().double(), hb))
    ee = max(rel(gm, me), rel(gv, ve), rel(h.cpu().double(), he))
    # per element: every mu, V and final-state entry, relative to its magnitude plus the batch's mean
    # magnitude (an output near zero is compared at the batch's scale)
    def elem(x, y):
        x, y = x.numpy(), y.numpy()
        return float(np.max(np.abs(x - y) / (np.abs(y) + np.mean(np.abs(y)))))
    pb = max(elem(gm, mb), elem(gv, vb), elem(h.cpu().double(), hb))
    pe = max(elem(gm, me), elem(gv, ve), elem(h.cpu().double(), he))
    say(f"[gru] rollout rel err vs workload precision {eb:.2e} (per element {pb:.2e}), "
        f"vs FP64 {ee:.2e} (per element {pe:.2e})")
    assert eb < 3e-3 and ee < 3e-2
    assert pb < 2e-3 and pe < 3e-2   # measured 4.6e-4 and 7.6e-3


def test_act_rnn_prepared_aliasing_and_errors():
    from paper_2603_25834_amd import _lib
    from paper_2603_25834_amd.policy import Policy
    N = 70
    theta, t = _seq_case(1, N, 2)
    pol = _policy(N)
    params = torch.from_numpy(theta).cuda()
    dev = {k: v.cuda().contiguous() for k, v in t.items()}
    eps = torch.zeros((N, 2), device="cuda")
    args = (params, dev["crop"][0], dev["scan"][0], dev["state"][0])
    with pytest.raises(_lib.AslamError) as ei:
        pol.act_rnn(*args, dev["h0"], None, eps, prepared=True)
    assert ei.value.code == -4
    v1, a1, l1, h1 = pol.act_rnn(*args, dev["h0"], dev["first"][0], eps)
    pol.prepare(params)
    h = dev["h0"].clone()
    v2, a2, l2, h2 = pol.act_rnn(*args, h, dev["first"][0], eps, h_out=h, prepared=True)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2) and torch.equal(a1, a2) and torch.equal(l1, l2) and torch.equal(h1, h2)
    # a reset row starts from zero: equal to the same row with h_in = 0
    z = dev["h0"].clone()
    z[dev["first"][0].bool()] = 0.0
    v3, _, _, h3 = pol.act_rnn(*args, z, None, eps)
    torch.cuda.synchronize()
    assert torch.equal(v3, v1) and torch.equal(h3, h1)
    # each handle type takes its own calls only
    ff = Policy(R, max_batch=8)
    with pytest.raises(_lib.AslamError):
        ff.act_rnn(torch.zeros(ff.n_params, device="cuda"), dev["crop"][0][:1], dev["scan"][0][:1],
                   dev["state"][0][:1], dev["h0"][:1], None, eps[:1])
    with pytest.raises(_lib.AslamError):
        pol.forward(*args)


@pytest.mark.parametrize("T,N,nb", [(6, 40, 24), (24, 64, 64)])
def test_bptt_gradient_matches_workload_precision(T, N, nb):
    theta, t = _seq_case(T, N, 3 + T, 0.1)
    pol = _policy(T * nb)
    params = torch.from_numpy(theta).cuda()
    dev = {k: v.cuda().contiguous() for k, v in t.items()}
    robots = np.sort(np.random.default_rng(T).permutation(N)[:nb]).astype(np.int32)
    drob = torch.from_numpy(robots).cuda()
    say(f"[gru] backward_seq T={T} N={N} nb={nb}")
    g1, g2 = torch.zeros_like(params), torch.zeros_like(params)
    loss = pol.backward_seq(params, dev["crop"], dev["scan"], dev["state"], dev["h0"], dev["first"], dev["act"],
                            dev["old_logp"], dev["adv"], dev["ret"], drob, g1)
    loss2 = pol.backward_seq(params, dev["crop"], dev["scan"], dev["state"], dev["h0"], dev["first"], dev["act"],
                             dev["old_logp"], dev["adv"], dev["ret"], drob, g2)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(loss, loss2)
    sel = {k: (v[:, robots] if k not in ("h0",) else v[robots]) for k, v in t.items()}
    th = torch.from_numpy(theta).double().requires_grad_(True)
    lr, terms = G.ppo_loss_seq(th, sel["crop"], sel["scan"], sel["state"], sel["h0"], sel["first"], sel["act"],
                               sel["old_logp"], sel["adv"], sel["ret"], SHAPE, rounding=True)
    (gr,) = torch.autograd.grad(lr, th)
    gr = gr.numpy()
    g = g1.cpu().double().numpy()
    o = 0
    worst = 0.0
    for name, shp in SHAPE.param_layout():
        n = int(np.prod(shp))
        a, b = g[o:o + n], gr[o:o + n]
        e = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        say(f"[gru]   {name:10s} rel err {e:.2e}")
        worst = max(worst, e)
        o += n
    lt = loss.cpu().double().numpy()
    assert np.allclose(lt[1:3], terms.detach().numpy()[:2], rtol=1e-3, atol=1e-5)
    assert worst < 1e-2


def _coherent_seq(T, N, seed):
    """A sequence minibatch whose advantages are all +1 and whose old log-probs sit at the current
    policy's (ratios near 1, inside the clip): the loss gradient is a coherent sum over samples."""
    theta, t = _seq_case(T, N, seed, 0.1)
    with torch.no_grad():
        mu, ls, _, _ = G.forward_seq(torch.from_numpy(theta).double(), t["crop"], t["scan"], t["state"], t["h0"],
                                     t["first"], SHAPE)
        logp = -0.5 * (((t["act"].double() - mu) / torch.exp(ls)) ** 2).sum(-1) - ls.sum() - np.log(2 * np.pi)
    t["old_logp"] = logp.float()
    t["adv"] = torch.ones_like(t["adv"])
    return theta, t


def _bptt(theta, t, T, N):
    pol = _policy(T * N)
    params = torch.from_numpy(theta).cuda()
    dev = {k: v.cuda().contiguous() for k, v in t.items()}
    g = torch.zeros_like(params)
    pol.backward_seq(params, dev["crop"], dev["scan"], dev["state"], dev["h0"], dev["first"], dev["act"],
                     dev["old_logp"], dev["adv"], dev["ret"], torch.arange(N, dtype=torch.int32, device="cuda"), g)
    torch.cuda.synchronize()
    return g.cpu().double().numpy()


def test_bptt_gradient_vs_exact_fp64_coherent():
    """BPTT over 12 steps of 32 robots against the exact FP64 network's autograd gradient (no rounding
    anywhere).  The recurrent handle computes with BF16 operands; as for the feed-forward policy, BF16
    rounding flips a few ReLU pre-activations, which random-sign advantages turn into large relative
    errors of a cancelling sum, so the bar is a coherent minibatch: per tensor within 5e-2 for the
    encoder's conv tensors and 2e-2 for the others (measured below 1.2e-2 / 0.6e-2)."""
    T, N = 12, 32
    theta, t = _coherent_seq(T, N, 21)
    g = _bptt(theta, t, T, N)
    th = torch.from_numpy(theta).double().requires_grad_(True)
    loss, _ = G.ppo_loss_seq(th, t["crop"], t["scan"], t["state"], t["h0"], t["first"], t["act"], t["old_logp"],
                             t["adv"], t["ret"], SHAPE)
    (gr,) = torch.autograd.grad(loss, th)
    gr = gr.numpy()
    o = 0
    for name, shp in SHAPE.param_layout():
        n = int(np.prod(shp))
        e = float(np.linalg.norm(g[o:o + n] - gr[o:o + n]) / max(np.linalg.norm(gr[o:o + n]), 1e-30))
        say(f"[gru] coherent vs exact FP64 {name:10s} {e:.2e}")
        assert e < (5e-2 if name.startswith("conv") else 2e-2), (name, e)
        o += n


def test_bptt_gradient_against_central_differences():
    """The directional derivative of the exact FP64 sequence loss along each tensor's GPU gradient,
    by central differences, against the GPU gradient's norm (both are g . u, u the unit GPU direction,
    up to the gradient's error): within 1e-2 per tensor (measured at most 2.2e-3) on a coherent
    minibatch of 6 steps x 16 robots (random-sign advantages leave the BF16 kink flips' O(5%) residue
    in the conv tensors, as in the coherent test above)."""
    T, N = 6, 16
    theta, t = _coherent_seq(T, N, 31)
    g = _bptt(theta, t, T, N)
    th0 = torch.from_numpy(theta).double()

    def loss_at(th):
        with torch.no_grad():
            v, _ = G.ppo_loss_seq(th, t["crop"], t["scan"], t["state"], t["h0"], t["first"], t["act"],
                                  t["old_logp"], t["adv"], t["ret"], SHAPE)
        return float(v)

    o = 0
    for name, shp in SHAPE.param_layout():
        n = int(np.prod(shp))
        d = np.zeros_like(theta, dtype=np.float64)
        d[o:o + n] = g[o:o + n]
        nd = np.linalg.norm(d)
        if nd == 0.0:
            o += n
            continue
        u = torch.from_numpy(d / nd)
        h = 1e-4 * max(1.0, float(np.linalg.norm(theta[o:o + n])))
        fd = (loss_at(th0 + h * u) - loss_at(th0 - h * u)) / (2 * h)   # d loss along u = g_true . u
        e = abs(fd - nd) / nd                                          # g_gpu . u = |g_gpu|
        say(f"[gru] central differences {name:10s} {e:.2e}")
        assert e < 1e-2, (name, fd, nd)
        o += n
