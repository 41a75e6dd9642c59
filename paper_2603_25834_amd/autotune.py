"""Autotuner of the batched env step's launch shape.

The step's cost depends on how a robot's ray fan is spread over a workgroup
(threads per robot, i.e. rays per lane and waves per robot), on the band of
code-window rows staged in LDS at once, on the persistent grid size, and on
whether the map update walks one ray per lane or shares segments of all rays
out over the lanes (shorter walks per lane, a setup per segment).  The
best choice moves with the grid sides, the ray count and the range, so it is
measured: every candidate runs a few steps of the caller's own batch, timed
with HIP events on the stream the steps are launched on, and the fastest one
is kept.  Results are cached in memory and, if a path is given, in a JSON
file keyed by the workload signature (device, sides histogram, rays, range,
loop closure), so a later run with the same signature skips the sweep.

Tuning advances the environment by the steps it times; call ``Env.reset``
afterwards to start the real run from its initial state.  Every candidate
computes the same results (the step is exact integer arithmetic), so the
choice affects time only.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass

import numpy as np
import torch

from . import _lib
from .env import Env, device_info

THREADS = (128, 192, 256, 384, 512)


@dataclass(frozen=True)
class Candidate:
    threads: int
    band_rows: int = 0      # 0: the largest band the LDS budget allows
    grid: int = 0           # 0: one workgroup per robot
    form: int = _lib.FORM_FUSED
    mark_seg: int = 0       # map update's walk: 0 one lane per ray, else segments of this many steps


def signature(env: Env) -> str:
    """Workload key: device (CUs, LDS), sides histogram, rays, range, cell size, loop closure, fan width,
    reward mode and range noise."""
    lds, cus = device_info()
    sides, counts = np.unique(env.sides, return_counts=True)
    p = env.params
    parts = [f"cu{cus}", f"lds{lds}", "sides" + ",".join(f"{s}x{c}" for s, c in zip(sides, counts)),
             f"R{p['n_rays']}", f"r{p['r_max_m']:g}", f"c{p['cell_m']:g}", f"lc{int(p['loop_closure'])}",
             f"fov{int(p.get('fov_steps', 0))}", f"rm{int(p.get('reward_mode', 0))}",
             f"sn{p.get('range_sigma_m', 0.0):g}"]
    return "/".join(parts)


MARK_SEGS = (32, 64)


def default_candidates(env: Env) -> list[Candidate]:
    """Threads per robot over the supported set, each with one lane per ray and with segmented walks in
    the map update; for grids whose code window needs several bands, also half-height bands; a
    persistent grid of a few workgroups per CU besides one workgroup per robot."""
    _, cus = device_info()
    cands = [Candidate(t) for t in THREADS] + [Candidate(t, mark_seg=g) for t in THREADS for g in MARK_SEGS]
    if env.n > 4 * cus:
        cands += [Candidate(t, grid=k * cus, mark_seg=g) for t in (256, 512) for k in (2, 4) for g in (0, 32)]
    env.set_exec(form=_lib.FORM_FUSED, threads=256)
    band = env.get_exec()["band_rows"]
    if band < int(env.sides.max()) and band >= 16:
        cands += [Candidate(t, band_rows=band // 2, mark_seg=g) for t in (256, 512) for g in (0, 32)]
    return cands


class _Cache:
    def __init__(self, path: str | None):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as fh:
                self.data = json.load(fh)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(self.data, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


_MEMO: dict = {}


def _time_candidate(env: Env, c: Candidate, actions, noise, ranges, reward, done, warmup: int, steps: int) -> float:
    env.set_exec(form=c.form, threads=c.threads, band_rows=c.band_rows, grid=c.grid, mark_seg=c.mark_seg)
    for t in range(warmup):
        env.step(actions[t % len(actions)], None if noise is None else noise[t % len(noise)], ranges, reward, done)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for t in range(steps):
        k = (warmup + t) % len(actions)
        env.step(actions[k], None if noise is None else noise[k], ranges, reward, done)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(env: Env, actions: torch.Tensor, noise: torch.Tensor | None, ranges: torch.Tensor, reward: torch.Tensor,
         done: torch.Tensor, candidates: list[Candidate] | None = None, warmup: int = 3, steps: int = 10,
         cache_path: str | None = None, force: bool = False) -> dict:
    """Pick the fastest launch shape for this env's batch and apply it with ``Env.set_exec``.

    actions [T, n, 2] and noise [T, n, env.G] (or None: the step draws its own) are device tensors of per-step inputs
    (cycled if T is short).  Returns {"signature", "best", "table"} with the
    per-candidate time in microseconds per step."""
    key = signature(env)
    cache = _Cache(cache_path)
    hit = None if force else (_MEMO.get(key) or cache.get(key))
    if hit is not None:
        best = Candidate(**hit["best"])
        env.set_exec(form=best.form, threads=best.threads, band_rows=best.band_rows, grid=best.grid,
                     mark_seg=best.mark_seg)
        return dict(hit, cached=True)
    cands = candidates if candidates is not None else default_candidates(env)
    table = []
    for c in cands:
        try:
            us = _time_candidate(env, c, actions, noise, ranges, reward, done, warmup, steps) * 1e3
        except _lib.AslamError as err:   # e.g. a band that does not fit the LDS budget
            table.append({"candidate": asdict(c), "us_per_step": None, "error": str(err)})
            continue
        table.append({"candidate": asdict(c), "us_per_step": us})
    timed = [r for r in table if r["us_per_step"] is not None]
    if not timed:
        raise RuntimeError("autotune: no candidate ran")
    best_row = min(timed, key=lambda r: r["us_per_step"])
    best = Candidate(**best_row["candidate"])
    env.set_exec(form=best.form, threads=best.threads, band_rows=best.band_rows, grid=best.grid,
                     mark_seg=best.mark_seg)
    out = {"signature": key, "best": asdict(best), "us_per_step": best_row["us_per_step"], "table": table}
    _MEMO[key] = out
    cache.put(key, out)
    return dict(out, cached=False)
