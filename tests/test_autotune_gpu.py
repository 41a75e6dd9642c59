"""Autotuner of the env step's launch shape, through the C-ABI (needs an MI355X).

Checks: the sweep applies its fastest candidate, a second call with the same
workload signature is served from the JSON cache, and every launch shape
gives bit-identical state after the same steps (the choice changes time only).
"""
import numpy as np
import pytest
import torch

from envpair import say
from paper_2603_25834_amd import _lib, synth
from paper_2603_25834_amd.autotune import Candidate, tune
from paper_2603_25834_amd.env import Env

pytestmark = pytest.mark.gpu


def _setup():
    sides = synth.draw_sides(synth.WORKLOADS["ragged_4096"], 0)
    robots = np.array(sorted(sum((list(np.flatnonzero(sides == s)[:6]) for s in (128, 192, 256, 384, 512)), [])))
    b = synth.make_batch("ragged_4096", 0, robots)
    p = synth.WORKLOADS["ragged_4096"].params()
    env = Env(p, b.sides)
    n, R = len(robots), p["n_rays"]
    dev = "cuda"
    world = torch.from_numpy(b.world.view(np.int32).copy()).to(dev)
    start = torch.from_numpy(b.start).to(dev)
    A = torch.from_numpy(synth.actions("ragged_4096", 0, 12, robots)).to(dev)
    G = torch.from_numpy(synth.noise("ragged_4096", 0, 12, robots)).to(dev)
    out = (torch.zeros((n, R), device=dev), torch.zeros(n, device=dev), torch.zeros(n, dtype=torch.uint8, device=dev))
    return env, world, start, A, G, out


def _run(env, world, start, A, G, out, k):
    env.reset(world, start)
    for t in range(k):
        env.step(A[t], G[t], *out)
    torch.cuda.synchronize()
    return [env.read(f).cpu().numpy() for f in (_lib.FIELD_BELIEF, _lib.FIELD_POSE, _lib.FIELD_EST, _lib.FIELD_COV,
                                                _lib.FIELD_ENTROPY_Q)] + [out[0].cpu().numpy().copy()]


def test_tune_applies_best_and_caches(tmp_path):
    env, world, start, A, G, out = _setup()
    env.reset(world, start)
    cands = [Candidate(128), Candidate(256), Candidate(512), Candidate(256, grid=7), Candidate(256, band_rows=8),
             Candidate(512, mark_seg=32)]
    cache = str(tmp_path / "tune.json")
    res = tune(env, A, G, *out, candidates=cands, warmup=1, steps=3, cache_path=cache)
    say(f"[autotune] {res['signature']}: best {res['best']} "
        + " ".join(f"{r['candidate']['threads']}/{r['candidate']['band_rows']}/{r['candidate']['grid']}="
                   f"{r['us_per_step']:.0f}us" for r in res["table"] if r["us_per_step"]))
    assert not res["cached"] and len(res["table"]) == len(cands)
    ex = env.get_exec()
    assert ex["threads"] == res["best"]["threads"] and ex["grid"] == res["best"]["grid"]
    times = [r["us_per_step"] for r in res["table"] if r["us_per_step"] is not None]
    assert res["us_per_step"] == min(times)
    env.set_exec(form=_lib.FORM_PLAIN, threads=128)
    again = tune(env, A, G, *out, candidates=cands, cache_path=cache)
    assert again["cached"] and again["best"] == res["best"]
    assert env.get_exec()["threads"] == res["best"]["threads"]


def test_every_launch_shape_gives_identical_state():
    env, world, start, A, G, out = _setup()
    ref = None
    for c in (Candidate(128), Candidate(384), Candidate(512, grid=5), Candidate(256, band_rows=8),
              Candidate(256, form=_lib.FORM_PLAIN), Candidate(512, mark_seg=32), Candidate(128, mark_seg=8),
              Candidate(256, band_rows=8, mark_seg=16), Candidate(512, grid=5, mark_seg=64),
              Candidate(192, form=_lib.FORM_PLAIN, mark_seg=1024)):
        env.set_exec(form=c.form, threads=c.threads, band_rows=c.band_rows, grid=c.grid, mark_seg=c.mark_seg)
        got = _run(env, world, start, A, G, out, 10)
        if ref is None:
            ref = got
            continue
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), c
