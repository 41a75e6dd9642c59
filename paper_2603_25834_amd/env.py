"""Batched Active-SLAM environment on the GPU (thin wrapper over the C-ABI).

PyTorch provides device memory and the stream; every stage of the step runs in
the library's kernels.  Method: arXiv 2603.25834, Sec. III-B (one POMDP
transition per call), Sec. III-C (action box), Sec. III-D (log-odds grid and
pose covariance), Sec. III-E (collision penalty), Sec. IV-A (LiDAR).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import EnvConfig, ExecConfig, check, lib

_CFG_FIELDS = [f for f, _ in EnvConfig._fields_]


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Env:
    """n robots, each in its own square occupancy world (ragged sides)."""

    def __init__(self, params: dict, sides, device: str | int = "cuda"):
        self.params = dict(params)
        cfg = EnvConfig()
        for f in _CFG_FIELDS:
            setattr(cfg, f, params.get(f, 0) if f == "noise_seed" else params[f])
        self.device = torch.device(device)
        self.sides = np.ascontiguousarray(np.asarray(sides, np.int32))
        self.n = len(self.sides)
        self.R = int(params["n_rays"])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().aslam_env_create(ctypes.byref(cfg), self.n,
                                         self.sides.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self.h = h
        self.cells = int(lib().aslam_env_cells(h))
        self.world_words = int(lib().aslam_env_world_words(h))
        self.visit_cells = int(lib().aslam_env_visit_cells(h))
        self.G = int(lib().aslam_env_noise_width(h))     # normal draws per robot and step
        cells = self.sides.astype(np.int64) ** 2
        self.cell_off = np.concatenate([[0], np.cumsum(cells)[:-1]]).astype(np.int64)

    def close(self):
        if getattr(self, "h", None):
            lib().aslam_env_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ exec form
    def set_exec(self, form: int = _lib.FORM_FUSED, threads: int = 256, band_rows: int = 0, grid: int = 0,
                 record_rays: int = 0, lds_bytes: int = 0, mark_seg: int = 0):
        ex = ExecConfig(form, threads, band_rows, grid, record_rays, lds_bytes, mark_seg)
        check(lib().aslam_env_set_exec(self.h, ctypes.byref(ex)))

    def get_exec(self) -> dict:
        ex = ExecConfig()
        check(lib().aslam_env_get_exec(self.h, ctypes.byref(ex)))
        return {f: getattr(ex, f) for f, _ in ExecConfig._fields_}

    # ------------------------------------------------------------ calls
    def reset(self, world_words: torch.Tensor, init_pose: torch.Tensor, mask: torch.Tensor | None = None):
        assert world_words.dtype == torch.int32 and world_words.numel() == self.world_words
        assert init_pose.dtype == torch.float32 and init_pose.shape == (self.n, 3)
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.numel() == self.n
        check(lib().aslam_env_reset(self.h, _ptr(world_words), _ptr(init_pose), _ptr(mask), _stream()))

    def step(self, actions: torch.Tensor, noise: torch.Tensor | None, ranges: torch.Tensor, reward: torch.Tensor,
             done: torch.Tensor):
        """One step; noise None takes the library's own draws (key params['noise_seed'])."""
        assert actions.dtype == torch.float32 and actions.numel() == 2 * self.n
        assert noise is None or (noise.dtype == torch.float32 and noise.numel() == self.G * self.n)
        assert ranges.dtype == torch.float32 and ranges.numel() == self.R * self.n
        assert reward.dtype == torch.float32 and reward.numel() == self.n
        assert done.dtype == torch.uint8 and done.numel() == self.n
        check(lib().aslam_env_step(self.h, _ptr(actions), _ptr(noise), _ptr(ranges), _ptr(reward), _ptr(done),
                                   _stream()))

    def observe(self, ranges: torch.Tensor, crop: torch.Tensor, scan: torch.Tensor, state: torch.Tensor):
        cs = crop.shape[-1]
        assert crop.dtype == torch.int16 and crop.numel() == self.n * cs * cs
        assert scan.dtype == torch.float32 and scan.numel() == self.n * self.R
        assert state.dtype == torch.float32 and state.numel() == self.n * 12
        check(lib().aslam_env_observe(self.h, _ptr(ranges), _ptr(crop), cs, _ptr(scan), _ptr(state), _stream()))

    def observe_bridge(self, ranges: torch.Tensor, crop: torch.Tensor, scan: torch.Tensor, state: torch.Tensor,
                       u_new: torch.Tensor, t: int, t_bridge: int):
        """Observation with the uncertainty entry bridged towards an external estimator's u_new [n]:
        alpha u_new + (1 - alpha) U_t, alpha = min(1, t / t_bridge) (Sec. III-G)."""
        cs = crop.shape[-1]
        assert crop.dtype == torch.int16 and crop.numel() == self.n * cs * cs
        assert scan.dtype == torch.float32 and scan.numel() == self.n * self.R
        assert state.dtype == torch.float32 and state.numel() == self.n * 12
        assert u_new.dtype == torch.float32 and u_new.numel() == self.n
        check(lib().aslam_env_observe_bridge(self.h, _ptr(ranges), _ptr(crop), cs, _ptr(scan), _ptr(state),
                                             _ptr(u_new), int(t), int(t_bridge), _stream()))

    _FIELDS = {
        _lib.FIELD_BELIEF: (torch.int16, lambda s: (s.cells,)),
        _lib.FIELD_POSE: (torch.float32, lambda s: (s.n, 3)),
        _lib.FIELD_EST: (torch.float32, lambda s: (s.n, 3)),
        _lib.FIELD_COV: (torch.float32, lambda s: (s.n, 6)),
        _lib.FIELD_RHO_Q: (torch.int32, lambda s: (s.n, s.R)),
        _lib.FIELD_HIT_CELL: (torch.int32, lambda s: (s.n, s.R)),
        _lib.FIELD_ENTROPY_Q: (torch.int64, lambda s: (s.n,)),
        _lib.FIELD_STEP: (torch.int32, lambda s: (s.n,)),
        _lib.FIELD_FLAGS: (torch.uint8, lambda s: (s.n, 2)),
        _lib.FIELD_TERMS: (torch.float32, lambda s: (s.n, 2)),
        _lib.FIELD_COUNTERS: (torch.int64, lambda s: (s.n, 3)),
        _lib.FIELD_U_PREV: (torch.float64, lambda s: (s.n,)),
        _lib.FIELD_VISIT_LAST: (torch.int32, lambda s: (s.visit_cells,)),
        _lib.FIELD_DRAWS: (torch.int64, lambda s: (s.n,)),
        _lib.FIELD_MATCH: (torch.int32, lambda s: (s.n, 6)),
    }

    def read(self, field: int) -> torch.Tensor:
        dt, shape = self._FIELDS[field]
        out = torch.empty(shape(self), dtype=dt, device=self.device)
        if out.numel():            # an empty field (no visit grid) has no storage to copy into
            check(lib().aslam_env_read(self.h, field, _ptr(out), _stream()))
        return out

    def graph_build(self, k_steps: int, actions: torch.Tensor, a_stride: int, noise: torch.Tensor | None, g_stride: int,
                    ranges: torch.Tensor, r_stride: int, reward: torch.Tensor, w_stride: int,
                    done: torch.Tensor, d_stride: int):
        # the buffers must hold k_steps strided slices
        for t, st, per in ((actions, a_stride, 2 * self.n), (noise, g_stride, self.G * self.n),
                           (ranges, r_stride, self.R * self.n), (reward, w_stride, self.n), (done, d_stride, self.n)):
            assert t is None or (t.is_contiguous() and t.numel() >= (k_steps - 1) * st + per)
        check(lib().aslam_env_graph_build(self.h, k_steps, _ptr(actions), a_stride, _ptr(noise), g_stride,
                                          _ptr(ranges), r_stride, _ptr(reward), w_stride, _ptr(done), d_stride))

    def graph_launch(self):
        check(lib().aslam_env_graph_launch(self.h, _stream()))


def device_info() -> tuple[int, int]:
    lds = ctypes.c_int32()
    cu = ctypes.c_int32()
    check(lib().aslam_device_info(ctypes.byref(lds), ctypes.byref(cu)))
    return lds.value, cu.value
