"""The policy forward that allocates nothing (aslam_policy_forward_noalloc) against the handle's
aslam_policy_forward, through the C-ABI (needs an MI355X).

Both run the same kernels in the same order; the allocation-free call keeps its staging in the
library's static device array.  Two calls in a row (the second on a smaller batch and a shorter scan,
so the array holds the first call's larger contents) must each equal the handle's forward bit for
bit; sizes beyond the array's limits are rejected."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2603_25834_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _handle_forward(R, d, params, B):
    L = _lib.lib()
    cfg = _lib.PolicyConfig(R, B, 0.2, 0.5, 0.005, 0, 0)
    h = ctypes.c_void_p()
    _lib.check(L.aslam_policy_create(ctypes.byref(cfg), ctypes.byref(h)))
    mu = torch.empty((B, 2), device="cuda")
    val = torch.empty(B, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.aslam_policy_forward(h, _p(params), _p(d["crop"]), _p(d["scan"]), _p(d["state"]), B, _p(mu),
                                      _p(val), st))
    torch.cuda.synchronize()
    L.aslam_policy_destroy(h)
    return mu, val


def _noalloc_forward(R, d, params, B):
    L = _lib.lib()
    mu = torch.full((B, 2), float("nan"), device="cuda")
    val = torch.full((B,), float("nan"), device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.aslam_policy_forward_noalloc(_p(params), R, _p(d["crop"]), _p(d["scan"]), _p(d["state"]), B,
                                              _p(mu), _p(val), st))
    torch.cuda.synchronize()
    return mu, val


def test_noalloc_forward_equals_handle_forward_twice():
    L = _lib.lib()
    ms, mb = ctypes.c_int32(), ctypes.c_int32()
    nbytes = L.aslam_policy_noalloc_limits(ctypes.byref(ms), ctypes.byref(mb))
    assert ms.value == 720 and mb.value == 256 and 0 < nbytes < 32 << 20
    for R, B, seed in ((720, 256, 1), (360, 37, 2)):
        d = {k: torch.from_numpy(v).cuda() for k, v in synth.policy_batch(B, R, seed).items()}
        params = torch.from_numpy(synth.init_policy_params(R, seed)).cuda()
        mu_h, v_h = _handle_forward(R, d, params, B)
        mu_n, v_n = _noalloc_forward(R, d, params, B)
        assert torch.equal(mu_n, mu_h) and torch.equal(v_n, v_h), (R, B)
        assert torch.isfinite(mu_n).all() and torch.isfinite(v_n).all()


def test_noalloc_forward_rejects_sizes_beyond_its_array():
    L = _lib.lib()
    R, B = 360, 8
    d = {k: torch.from_numpy(v).cuda() for k, v in synth.policy_batch(B, R, 3).items()}
    params = torch.from_numpy(synth.init_policy_params(R, 3)).cuda()
    mu = torch.empty((B, 2), device="cuda")
    val = torch.empty(B, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = (_p(d["crop"]), _p(d["scan"]), _p(d["state"]))
    assert L.aslam_policy_forward_noalloc(_p(params), R, *args, 257, _p(mu), _p(val), st) == -1
    assert b"batch" in L.aslam_last_error()
    assert L.aslam_policy_forward_noalloc(_p(params), 721, *args, B, _p(mu), _p(val), st) == -1
    assert L.aslam_policy_forward_noalloc(_p(params), R, *args, 0, _p(mu), _p(val), st) == -1
    assert L.aslam_policy_forward_noalloc(None, R, *args, B, _p(mu), _p(val), st) == -1
