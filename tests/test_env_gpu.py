"""GPU environment step vs the CPU oracle, through the C-ABI (needs an MI355X).

Bar: bit-exact poses, estimates, covariances, ranges in 1/65536 cell, hit
cells, int16 log-odds and the Q32 map entropy; rewards within 1e-4
(relative above 1); ranges within 1e-5 relative.  Paper passages: Sec. III-B
(one POMDP transition), III-C (action box), III-D (log-odds grid, pose
covariance), III-E (collision penalty), IV-A (LiDAR) of arXiv 2603.25834.
"""
import numpy as np
import pytest

from envpair import Pair, say
from paper_2603_25834_amd import synth

pytestmark = pytest.mark.gpu

PLAIN = dict(form=0, threads=256)
FUSED = dict(form=1, threads=256, record_rays=1)


@pytest.mark.parametrize("exec_kw", [PLAIN, FUSED], ids=["plain", "fused"])
def test_small_16x64_every_step(exec_kw):
    """16 robots, 64x64 worlds, 180 rays, 5 m, 100 steps: every step compared."""
    pr = Pair("small_16x64", 0, exec_kw=exec_kw, steps=100)
    for t in range(100):
        o = pr.step()
        pr.compare(o)


@pytest.mark.parametrize("exec_kw", [PLAIN, FUSED, dict(FUSED, mark_seg=32)], ids=["plain", "fused", "fused_seg32"])
def test_paper_750x256_subset_loop_closure(exec_kw):
    """24 robots of the 750-robot 256x256 scene, 360 rays, 10 m, loop closure, 240 steps."""
    pr = Pair("paper_750x256", 1, robots=np.arange(0, 750, 31)[:24], exec_kw=exec_kw, steps=240)
    closed = 0
    for t in range(240):
        o = pr.step()
        closed += int(o.closed.sum())
        if t % 20 == 19 or o.closed.any():
            pr.compare(o)
    assert closed > 0, "no loop closure happened; the case does not cover the fix"


def _ragged_robots():
    sides = synth.draw_sides(synth.WORKLOADS["ragged_4096"], 0)
    pick = []
    for s in (128, 192, 256, 384, 512):
        pick += list(np.flatnonzero(sides == s)[:4])
    return np.array(sorted(pick))


@pytest.mark.parametrize("exec_kw", [
    dict(form=0, threads=128), dict(form=1, threads=512, record_rays=1),
    dict(form=1, threads=256, record_rays=1, band_rows=8),
    dict(form=1, threads=256, record_rays=1, grid=7),
    dict(form=1, threads=256, record_rays=1, mark_seg=32), dict(form=1, threads=512, record_rays=1, mark_seg=8),
    dict(form=1, threads=256, record_rays=1, band_rows=8, mark_seg=16), dict(form=0, threads=192, mark_seg=64)],
    ids=["plain128", "fused512", "fused_band8", "fused_grid7", "fused_seg32", "fused512_seg8", "fused_band8_seg16",
         "plain192_seg64"])
def test_ragged_sides(exec_kw):
    """Robots of every side in {128,...,512}; tiny bands force the multi-pass code window; the map update's
    walk one lane per ray or in segments of 8 to 64 steps."""
    pr = Pair("ragged_4096", 0, robots=_ragged_robots(), exec_kw=exec_kw, steps=40)
    for t in range(40):
        o = pr.step()
        if t % 8 == 7:
            pr.compare(o)


def test_plain_and_fused_identical_and_deterministic():
    robots = _ragged_robots()
    outs = []
    for kw in (PLAIN, FUSED, dict(form=1, threads=128, grid=3, record_rays=1), FUSED):
        pr = Pair("ragged_4096", 2, robots=robots, exec_kw=kw, steps=30, oracle=False)
        for t in range(30):
            pr.step()
        outs.append(pr.gpu_state())
    for g in outs[1:]:
        for k in ("pose", "est", "cov", "belief", "hq", "rho", "hitc", "ranges", "reward", "done"):
            assert np.array_equal(g[k], outs[0][k]), k


def test_observe_matches_oracle():
    import torch
    pr = Pair("small_16x64", 4, exec_kw=FUSED, steps=20)
    for t in range(20):
        o = pr.step()
    crop = torch.zeros((pr.n, 64, 64), dtype=torch.int16, device="cuda")
    scan = torch.zeros((pr.n, pr.R), dtype=torch.float32, device="cuda")
    state = torch.zeros((pr.n, 12), dtype=torch.float32, device="cuda")
    pr.env.observe(pr.ranges, crop, scan, state)
    torch.cuda.synchronize()
    c2, s2, st2 = pr.orc.observe(o.ranges)
    assert np.array_equal(crop.cpu().numpy(), c2)
    assert np.array_equal(scan.cpu().numpy(), s2)
    assert np.array_equal(state.cpu().numpy(), st2)


def test_edge_cases_collision_nan_masked_reset_episode():
    """Robot driven into a wall, NaN actions, a masked reset mid-run, episode length."""
    import torch
    pr = Pair("small_16x64", 5, exec_kw=FUSED, steps=60, params_over=dict(episode_len=25))
    pr.A[:, 0, 0] = np.nan        # robot 0: NaN speed -> 0
    pr.A[:, 1, :] = [0.5, 0.0]    # robot 1: full speed straight ahead, will hit a wall
    pr.dA.copy_(torch.from_numpy(pr.A))
    for t in range(60):
        o = pr.step()
        pr.compare(o)
        if t == 30:
            mask = np.zeros(pr.n, np.uint8)
            mask[[1, 3, 7]] = 1
            pr.reset(pr.b.start, mask)
    assert pr.gpu_state()["done"].dtype == np.uint8


def test_degenerate_start_poses():
    """A robot starting off the grid (no march, no update, always blocked) and one inside a wall cell."""
    import torch
    pr = Pair("small_16x64", 6, exec_kw=FUSED, steps=12)
    start = pr.b.start.copy()
    start[2] = [-1.0, 3.0, 0.3]              # off the map
    occ = synth.draw_world(synth.WORKLOADS["small_16x64"], 64, 6, int(pr.b.index[5]))
    j, i = np.argwhere(occ)[100]
    start[5] = [(i + 0.5) * 0.1, (j + 0.5) * 0.1, 1.0]   # inside an occupied cell
    pr.reset(start)
    for t in range(12):
        o = pr.step()
        pr.compare(o)
        assert o.collided[2] == 1 and o.collided[5] == 1
        assert np.all(o.hit_cell[2] == -1) and np.all(o.rho_q[5] == 0)


def test_errors_through_the_abi():
    from paper_2603_25834_amd import _lib
    from paper_2603_25834_amd.env import Env
    p = synth.WORKLOADS["small_16x64"].params()
    with pytest.raises(_lib.AslamError) as ei:
        Env(p, np.array([64, 70], np.int32))
    assert ei.value.code == -1
    bad = dict(p, n_rays=7)
    with pytest.raises(_lib.AslamError):
        Env(bad, np.array([64], np.int32))
    import torch
    env = Env(p, np.array([64], np.int32))
    z = torch.zeros(8, device="cuda")
    with pytest.raises(_lib.AslamError) as ei:
        env.step(z[:2], z[:5], torch.zeros(180, device="cuda"), z[:1], torch.zeros(1, dtype=torch.uint8,
                                                                                  device="cuda"))
    assert ei.value.code == -4
    with pytest.raises(_lib.AslamError):
        env.set_exec(form=1, threads=96)


@pytest.mark.parametrize("form", [0, 1], ids=["plain", "fused"])
def test_graph_replay_matches_eager(form):
    """One graph of K captured steps, replayed 3 times with eager work in between, equals eager steps."""
    import torch
    robots = _ragged_robots()
    K = 6
    kw = dict(form=form, threads=256, record_rays=1)
    eager = Pair("ragged_4096", 3, robots=robots, exec_kw=kw, steps=K, oracle=False)
    graph = Pair("ragged_4096", 3, robots=robots, exec_kw=kw, steps=K, oracle=False)
    n, R = graph.n, graph.R
    rng = torch.zeros((K, n, R), device="cuda")
    rew = torch.zeros((K, n), device="cuda")
    dn = torch.zeros((K, n), dtype=torch.uint8, device="cuda")
    graph.env.graph_build(K, graph.dA, 2 * n, graph.dG, graph.env.G * n, rng, n * R, rew, n, dn, n)
    for rep in range(3):
        say(f"[graph] form={form} replay {rep}")
        graph.env.graph_launch()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        for k in range(K):
            eager.env.step(eager.dA[k], eager.dG[k], eager.ranges, eager.reward, eager.done)
            torch.cuda.synchronize()
            assert torch.equal(eager.ranges, rng[k]) and torch.equal(eager.reward, rew[k]), (rep, k)
            assert torch.equal(eager.done, dn[k])
        ge, gg = eager.gpu_state(), graph.gpu_state()
        for key in ("pose", "est", "cov", "belief", "hq", "rho", "hitc"):
            assert np.array_equal(ge[key], gg[key]), (rep, key)
        del junk


@pytest.mark.parametrize("name,steps,exec_kw", [
    ("paper_750x256", 1000, dict(form=1, threads=512)),
    ("ragged_4096", 1000, dict(form=1, threads=512)),
    ("ragged_4096", 1000, dict(form=1, threads=256, band_rows=203, mark_seg=32)),
    ("full_8192x512", 30, dict(form=1, threads=512))],
    ids=["paper_750x256_T1000", "ragged_4096_T1000", "ragged_4096_T1000_t256_band203_seg32", "full_8192x512"])
def test_full_batch_sampled(name, steps, exec_kw):
    """The whole batch stepped in the fused launches the benchmark times (the shapes its autotuner picks:
    512 threads per robot at 750 robots; 256 threads, 203-row bands and 32-step walk segments for the
    ragged batch; also 512 threads there), steps captured in one HIP graph: the 750-robot and the ragged
    4096-robot scenes for their full 1000 steps, and 30 steps of the 8192-robot, 512^2, 720-ray, 15 m
    scene.  16 sampled robots re-run alone by the oracle (robots are independent, so a sample sees the
    same inputs) and compared bit for bit at every step (ranges, rewards, done) and at the end (poses,
    covariances, beliefs, entropies)."""
    import torch
    from oracle import oracle as O
    from paper_2603_25834_amd import _lib
    full = Pair(name, 8, exec_kw=exec_kw, steps=steps, oracle=False)
    n = full.n
    pick = np.unique(np.linspace(3, n - 1, 16).astype(np.int64))
    b = synth.make_batch(name, 8, pick)
    orc = O.OracleEnv(full.p, b.sides, b.world, b.world_off)
    orc.reset(b.start)
    A = synth.actions(name, 8, steps, pick)
    G = synth.noise(name, 8, steps, pick)
    rng_ = torch.zeros((steps, n, full.R), device="cuda")
    rew = torch.zeros((steps, n), device="cuda")
    dn = torch.zeros((steps, n), dtype=torch.uint8, device="cuda")
    full.env.graph_build(steps, full.dA, 2 * n, full.dG, full.env.G * n, rng_, n * full.R, rew, n, dn, n)
    full.env.graph_launch()
    torch.cuda.synchronize()
    say(f"[full] {name}: {steps} graph steps of {n} robots, sample {len(pick)}")
    ip = torch.from_numpy(pick).cuda()
    gr, gw, gd = rng_[:, ip].cpu().numpy(), rew[:, ip].cpu().numpy(), dn[:, ip].cpu().numpy()
    del rng_
    for t in range(steps):
        o = orc.step(A[t], G[t])
        assert np.array_equal(gr[t], o.ranges), t
        assert np.all(np.abs(gw[t] - o.reward) <= 1e-4 * np.maximum(1.0, np.abs(o.reward))), t
        assert np.array_equal(gd[t], o.done), t
    e = full.env
    assert np.array_equal(e.read(_lib.FIELD_POSE).cpu().numpy()[pick].view(np.int32), orc.pose.view(np.int32))
    assert np.array_equal(e.read(_lib.FIELD_COV).cpu().numpy()[pick].view(np.int32), orc.cov.view(np.int32))
    assert np.array_equal(e.read(_lib.FIELD_ENTROPY_Q).cpu().numpy()[pick], orc.h_q)
    bel = e.read(_lib.FIELD_BELIEF).cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(full.b.sides.astype(np.int64) ** 2)])
    got = np.concatenate([bel[offs[i]:offs[i + 1]] for i in pick])
    assert np.array_equal(got, orc.belief)
