"""PPO actor-critic on the GPU (thin wrapper over the C-ABI) and autograd glue.

Method: arXiv 2603.25834 Sec. III-F (PPO clipped surrogate, Eqs. 18-20, with
GAE).  Every forward, loss, gradient, GAE and Adam computation runs in the
library's kernels; this module only marshals torch device tensors.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import PolicyConfig, check, lib


def _p(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def num_params(n_scan: int) -> int:
    return int(lib().aslam_policy_num_params(n_scan))


class Policy:
    def __init__(self, n_scan: int = 360, max_batch: int = 16384, clip_eps: float = 0.2, c_value: float = 0.5,
                 c_entropy: float = 0.005, recurrent: bool = False, precision: int = 0):
        """precision 0: BF16 operands; 1: split (hi + lo BF16) forward operands, FP32-accurate ReLU
        pre-activations (feed-forward policy only)."""
        self.n_scan, self.max_batch, self.recurrent = n_scan, max_batch, bool(recurrent)
        self.precision = int(precision)
        self.cfg = PolicyConfig(n_scan, max_batch, clip_eps, c_value, c_entropy, int(self.recurrent), self.precision)
        h = ctypes.c_void_p()
        check(lib().aslam_policy_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self.h = h
        self.n_params = int(lib().aslam_policy_param_count(ctypes.byref(self.cfg)))

    def close(self):
        if getattr(self, "h", None):
            lib().aslam_policy_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_obs(self, params, crop, scan, state):
        B = crop.shape[0]
        assert params.dtype == torch.float32 and params.numel() == self.n_params
        assert crop.dtype == torch.int16 and crop.shape[1:] == (64, 64)
        assert scan.dtype == torch.float32 and scan.shape == (B, self.n_scan)
        assert state.dtype == torch.float32 and state.shape == (B, 12)
        return B

    def forward(self, params, crop, scan, state, mu=None, value=None):
        B = self._check_obs(params, crop, scan, state)
        mu = torch.empty((B, 2), device=crop.device) if mu is None else mu
        value = torch.empty(B, device=crop.device) if value is None else value
        check(lib().aslam_policy_forward(self.h, _p(params), _p(crop), _p(scan), _p(state), B, _p(mu), _p(value),
                                         _stream()))
        return mu, value

    def prepare(self, params):
        """Form the BF16 weight copies of the forward from `params` (for act(prepared=True))."""
        assert params.dtype == torch.float32 and params.numel() == self.n_params
        check(lib().aslam_policy_prepare(self.h, _p(params), _stream()))

    def act(self, params, crop, scan, state, eps, value=None, act=None, logp=None, mu=None, prepared=False,
            seed=0, counter=0):
        """Forward + Gaussian sample in one call: value [B], act [B, 2], logp [B] (and mu [B, 2] if given).
        eps [B, 2] standard normals, or None for the library's own draws at (seed, counter).
        prepared=True reuses the weight copies of the last prepare/forward/act/backward call; the caller
        guarantees that `params` has not changed since."""
        B = self._check_obs(params, crop, scan, state)
        assert eps is None or (eps.dtype == torch.float32 and tuple(eps.shape) == (B, 2))
        value = torch.empty(B, device=crop.device) if value is None else value
        act = torch.empty((B, 2), device=crop.device) if act is None else act
        logp = torch.empty(B, device=crop.device) if logp is None else logp
        check(lib().aslam_policy_act(self.h, _p(params), int(bool(prepared)), _p(crop), _p(scan), _p(state), B,
                                     _p(eps), int(seed), int(counter), _p(mu), _p(value), _p(act), _p(logp),
                                     _stream()))
        return value, act, logp

    def act_rnn(self, params, crop, scan, state, h_in, first, eps, value=None, act=None, logp=None, h_out=None,
                mu=None, prepared=False, seed=0, counter=0):
        """Recurrent rollout step: the GRU state h_in [B, 256] (zeroed where first [B] uint8 is set, may be
        None) advances to h_out (may be h_in itself); value, action and log-prob as act()."""
        B = self._check_obs(params, crop, scan, state)
        assert h_in.dtype == torch.float32 and tuple(h_in.shape) == (B, 256)
        assert eps is None or (eps.dtype == torch.float32 and tuple(eps.shape) == (B, 2))
        if first is not None:
            assert first.dtype == torch.uint8 and first.numel() == B
        value = torch.empty(B, device=crop.device) if value is None else value
        act = torch.empty((B, 2), device=crop.device) if act is None else act
        logp = torch.empty(B, device=crop.device) if logp is None else logp
        h_out = torch.empty_like(h_in) if h_out is None else h_out
        check(lib().aslam_policy_act_rnn(self.h, _p(params), int(bool(prepared)), _p(crop), _p(scan), _p(state), B,
                                         _p(h_in), _p(first), _p(eps), int(seed), int(counter), _p(mu), _p(value),
                                         _p(act), _p(logp), _p(h_out), _stream()))
        return value, act, logp, h_out

    def backward_seq(self, params, crop, scan, state, h0, first, act, old_logp, adv, ret, robots, grads, loss=None):
        """Recurrent PPO loss gradient over the sequences of `robots` (int32 [nb]) in time-major rollout
        arrays [T, N, ...]; h0 [N, 256] the state entering step 0, first [T, N] episode starts."""
        T, N = crop.shape[0], crop.shape[1]
        assert crop.dtype == torch.int16 and tuple(crop.shape[2:]) == (64, 64)
        assert tuple(scan.shape) == (T, N, self.n_scan) and tuple(state.shape) == (T, N, 12)
        assert tuple(h0.shape) == (N, 256) and first.dtype == torch.uint8 and tuple(first.shape) == (T, N)
        for t_, shp in ((act, (T, N, 2)), (old_logp, (T, N)), (adv, (T, N)), (ret, (T, N))):
            assert t_.dtype == torch.float32 and tuple(t_.shape) == shp
        assert robots.dtype == torch.int32 and robots.dim() == 1
        assert grads.dtype == torch.float32 and grads.numel() == self.n_params
        loss = torch.empty(4, device=crop.device) if loss is None else loss
        check(lib().aslam_policy_backward_seq(self.h, _p(params), _p(crop), _p(scan), _p(state), T, N, _p(robots),
                                              robots.numel(), _p(h0), _p(first), _p(act), _p(old_logp), _p(adv),
                                              _p(ret), _p(grads), _p(loss), _stream()))
        return loss

    def backward(self, params, crop, scan, state, act, old_logp, adv, ret, grads, loss=None, rows=None):
        """Adds the PPO loss gradient of this minibatch to `grads`; returns loss terms [4].  With `rows`
        (int32 [B]) the minibatch is those rows of rollout-sized inputs (no gathered copy)."""
        B = self._check_obs(params, crop, scan, state)
        for t, shp in ((act, (B, 2)), (old_logp, (B,)), (adv, (B,)), (ret, (B,))):
            assert t.dtype == torch.float32 and tuple(t.shape) == shp
        assert grads.dtype == torch.float32 and grads.numel() == self.n_params
        loss = torch.empty(4, device=crop.device) if loss is None else loss
        if rows is None:
            check(lib().aslam_policy_backward(self.h, _p(params), _p(crop), _p(scan), _p(state), B, _p(act),
                                              _p(old_logp), _p(adv), _p(ret), _p(grads), _p(loss), _stream()))
        else:
            assert rows.dtype == torch.int32 and rows.is_cuda and rows.dim() == 1
            check(lib().aslam_policy_backward_rows(self.h, _p(params), _p(crop), _p(scan), _p(state), _p(rows),
                                                   rows.numel(), _p(act), _p(old_logp), _p(adv), _p(ret), _p(grads),
                                                   _p(loss), _stream()))
        return loss


    def sample(self, params, mu, eps, act=None, logp=None, seed=0, counter=0):
        """act = mu + exp(log_std) eps and its log-density; eps are standard normals [B, 2], or None for
        the library's own draws at (seed, counter)."""
        B = mu.shape[0]
        assert mu.dtype == torch.float32 and tuple(mu.shape) == (B, 2)
        assert eps is None or tuple(eps.shape) == (B, 2)
        act = torch.empty_like(mu) if act is None else act
        logp = torch.empty(B, device=mu.device) if logp is None else logp
        check(lib().aslam_policy_sample(self.h, _p(params), _p(mu), _p(eps), int(seed), int(counter), B, _p(act),
                                        _p(logp), _stream()))
        return act, logp


def gather_rows(src, idx, out=None):
    """out[i] = src[idx[i]] along dim 0 (rows of any dtype; row bytes a multiple of 4)."""
    assert idx.dtype == torch.int32 and idx.is_cuda
    n = idx.numel()
    out = torch.empty((n,) + tuple(src.shape[1:]), dtype=src.dtype, device=src.device) if out is None else out
    if n == 0:
        return out
    row_bytes = src[0].numel() * src.element_size()
    check(lib().aslam_gather_rows(_p(src), row_bytes, _p(idx), n, _p(out), _stream()))
    return out


def permutation_work_bytes(n: int) -> int:
    return int(lib().aslam_permutation_work_bytes(int(n)))


def permutation(n: int, seed: int, counter: int, out=None, device="cuda", work=None):
    """Keyed permutation of [0, n) (int32 [n], out[j] = image of j) from the library's generator.
    work: an optional device workspace of permutation_work_bytes(n) bytes (the tabulated form)."""
    out = torch.empty(n, dtype=torch.int32, device=device) if out is None else out
    assert out.dtype == torch.int32 and out.numel() == n and (n == 0 or out.is_cuda)
    wb = 0
    if work is not None:
        assert work.is_cuda and work.is_contiguous()
        wb = work.numel() * work.element_size()
    check(lib().aslam_permutation(int(n), int(seed), int(counter), _p(out) if n else None,
                                  _p(work) if work is not None else None, wb, _stream()))
    return out


def gae(rewards, values, dones, last_value, gamma=0.99, lam=0.95):
    T, N = rewards.shape
    adv = torch.empty_like(rewards)
    ret = torch.empty_like(rewards)
    check(lib().aslam_gae(_p(rewards), _p(values), _p(dones), _p(last_value), T, N, gamma, lam, _p(adv), _p(ret),
                          _stream()))
    return adv, ret


def adam(params, grads, m, v, step, lr=3e-4, beta1=0.9, beta2=0.999, eps=1e-8):
    check(lib().aslam_adam(_p(params), _p(grads), _p(m), _p(v), params.numel(), step, lr, beta1, beta2, eps,
                           _stream()))


class PPOLossFn(torch.autograd.Function):
    """loss = PPOLossFn.apply(params, policy, crop, scan, state, act, old_logp, adv, ret).

    The forward pass runs the fused loss-and-gradient kernels (activations are
    recomputed, only inputs are kept); backward scales the stored gradient."""

    @staticmethod
    def forward(ctx, params, policy, crop, scan, state, act, old_logp, adv, ret):
        grads = torch.zeros_like(params)
        loss = policy.backward(params, crop, scan, state, act, old_logp, adv, ret, grads)
        ctx.save_for_backward(grads)
        return loss[0].clone()

    @staticmethod
    def backward(ctx, g):
        (grads,) = ctx.saved_tensors
        return (grads * g,) + (None,) * 8


class PolicyFn(torch.autograd.Function):
    """(mu, value) = PolicyFn.apply(params, policy, crop, scan, state) for rollouts (no gradient)."""

    @staticmethod
    def forward(ctx, params, policy, crop, scan, state):
        return policy.forward(params, crop, scan, state)

    @staticmethod
    def backward(ctx, gm, gv):
        raise RuntimeError("PolicyFn has no backward; train through PPOLossFn")
