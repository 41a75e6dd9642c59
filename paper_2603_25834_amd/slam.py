"""The fixed-lag SLAM backbone (arXiv 2603.25834, Sec. III-D) over the C-ABI: correlative scan
matching, the scan factor of a match, the confidence-weighted integration of the aligned scan into the
grid, and the Gauss-Newton solve of a window of poses with the newest
pose's covariance.  Argument marshalling only: the arithmetic runs in the library's HIP kernels.

The matching and integration calls read the library's direction table through a handle
(``aslam_slam``); this module keeps one per device, created by ``handle()`` on first use -- call it
before capturing these calls into a graph, since creating a handle allocates."""
from __future__ import annotations

import ctypes

import torch

from ._lib import CsmConfig, check, lib


def _p(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_HANDLES: dict = {}


class SlamHandle:
    """An ``aslam_slam`` handle on one device (its direction table)."""

    def __init__(self, device: int):
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            check(lib().aslam_slam_create(ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().aslam_slam_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def handle(device: int | None = None) -> SlamHandle:
    """The module's handle for `device` (default: the current device), created on first use."""
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _HANDLES:
        _HANDLES[dev] = SlamHandle(dev)
    return _HANDLES[dev]


def csm_config(W: int, V: int, step_xy_q: int, step_h: int) -> CsmConfig:
    return CsmConfig(W, V, step_xy_q, step_h)


def csm_match(belief: torch.Tensor, cell_off: torch.Tensor, side: torch.Tensor, pose_q: torch.Tensor,
              rho_q: torch.Tensor, a_off: torch.Tensor, cfg: CsmConfig, out: torch.Tensor | None = None,
              max_side: int | None = None):
    """Best candidate (i, j, k), best and second scores and rays used per robot: int32 [n, 6].  max_side:
    the largest grid side (read from `side` when not given)."""
    if max_side is None:
        max_side = int(side.max().item()) if side.numel() else 0
    n, R = rho_q.shape
    assert belief.dtype == torch.int16 and cell_off.dtype == torch.int64 and side.dtype == torch.int32
    assert pose_q.dtype == torch.int32 and tuple(pose_q.shape) == (n, 3)
    assert rho_q.dtype == torch.int32 and a_off.dtype == torch.int32 and a_off.numel() == R
    out = torch.empty((n, 6), dtype=torch.int32, device=rho_q.device) if out is None else out
    check(lib().aslam_csm_match(handle(belief.device.index).h, _p(belief), _p(cell_off), _p(side), max_side, n, _p(pose_q), _p(rho_q), R,
                                _p(a_off), ctypes.byref(cfg), _p(out), _stream()))
    return out


def csm_factor(match: torch.Tensor, pose_q: torch.Tensor, cfg: CsmConfig, cell_m: float, l_max: float,
               sigma_xy: float, sigma_th: float, meas: torch.Tensor | None = None, info: torch.Tensor | None = None):
    """Scan factor of each match: measurement (x, y, theta) [n, 3] and information diagonal [n, 3], FP64
    (written into `meas` / `info` when given)."""
    n = match.shape[0]
    if meas is None:
        meas = torch.empty((n, 3), dtype=torch.float64, device=match.device)
    if info is None:
        info = torch.empty((n, 3), dtype=torch.float64, device=match.device)
    for t in (meas, info):
        if t.shape != (n, 3) or t.dtype != torch.float64 or not t.is_contiguous() or t.device != match.device:
            raise ValueError("csm_factor: outputs must be contiguous float64 [n, 3] on the match's device")
    check(lib().aslam_csm_factor(_p(match), _p(pose_q), n, ctypes.byref(cfg), cell_m, l_max, sigma_xy, sigma_th,
                                 _p(meas), _p(info), _stream()))
    return meas, info


def csm_integrate(belief: torch.Tensor, cell_off: torch.Tensor, side: torch.Tensor, pose_q: torch.Tensor,
                  rho_q: torch.Tensor, a_off: torch.Tensor, rmax_q: int, l_hit: int, l_miss: int, l_clamp: int,
                  match: torch.Tensor | None = None, cfg: CsmConfig | None = None, l_max: float = 1.0,
                  coded: torch.Tensor | None = None, max_side: int | None = None):
    """Integrate each robot's scan into its grid, in place, from the matched pose with increments scaled by
    the match weight (unweighted from pose_q when `match` is None).  Returns the coded cells per robot,
    int32 [n].  max_side: the largest grid side (read from `side` when not given)."""
    if max_side is None:
        max_side = int(side.max().item()) if side.numel() else 0
    n, R = rho_q.shape
    assert belief.dtype == torch.int16 and cell_off.dtype == torch.int64 and side.dtype == torch.int32
    assert pose_q.dtype == torch.int32 and tuple(pose_q.shape) == (n, 3)
    assert rho_q.dtype == torch.int32 and a_off.dtype == torch.int32 and a_off.numel() == R
    if match is not None:
        assert match.dtype == torch.int32 and tuple(match.shape) == (n, 6) and cfg is not None
    coded = torch.empty(n, dtype=torch.int32, device=rho_q.device) if coded is None else coded
    check(lib().aslam_csm_integrate(handle(belief.device.index).h, _p(belief), _p(cell_off), _p(side), n, _p(pose_q), _p(rho_q), R, _p(a_off),
                                    int(max_side), int(rmax_q), _p(match), None if cfg is None else ctypes.byref(cfg), float(l_max),
                                    int(l_hit), int(l_miss), int(l_clamp), _p(coded), _stream()))
    return coded


def fixedlag_solve(x0: torch.Tensor, prior: torch.Tensor, odo: torch.Tensor | None, scan: torch.Tensor, iters: int,
                   x: torch.Tensor | None = None, cov: torch.Tensor | None = None):
    """Gauss-Newton over n windows of L poses: (x [n, L, 3], newest pose's covariance [n, 3, 3]), FP64."""
    n, L, _ = x0.shape
    for t in (x0, prior, scan) + ((odo,) if odo is not None else ()):
        assert t.dtype == torch.float64
    x = torch.empty_like(x0) if x is None else x
    cov = torch.empty((n, 3, 3), dtype=torch.float64, device=x0.device) if cov is None else cov
    check(lib().aslam_fixedlag_solve(n, L, _p(x0), _p(prior), _p(odo), _p(scan), iters, _p(x), _p(cov), _stream()))
    return x, cov
