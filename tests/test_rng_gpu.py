"""The library's counter-based draws vs the oracle's own generator (needs an MI355X).

The workload's odometry and loop-closure noise, the paper's range noise (Sec. IV-A), PPO's action
samples and minibatch shuffles (Sec. III-F) are drawn inside the kernels from Philox4x64-10 blocks
(Irwin-Hall normals, a keyed Feistel permutation).  The oracle implements the same published
generator on its own (pinned against numpy's Philox in test_oracle_rng.py); here the two sides draw
independently and must agree bit for bit:
  * env steps taking their own draws (plain and fused forms, loop closures firing, the paper's range
    noise of 5 + R draws per robot-step, a masked reset keeping the counter, graph replays drawing
    new numbers) equal the oracle stepping with its own draws;
  * action samples at log std 0 and mean 0 are the normals themselves; the fused rollout call with
    its own draws equals the same call fed the oracle's normals;
  * permutations equal the oracle's for ragged sizes.
"""
import numpy as np
import pytest
import torch

from envpair import Pair, say
from paper_2603_25834_amd import _lib, synth

pytestmark = pytest.mark.gpu

SEED = 0x1234ABCD


@pytest.mark.parametrize("exec_kw", [dict(form=0, threads=256), dict(form=1, threads=128, record_rays=1),
                                     dict(form=1, threads=256, record_rays=1, grid=5)],
                         ids=["plain", "fused128", "fused_grid5"])
def test_env_own_draws_small(exec_kw):
    """The small workload with loop closure on (gap 5, so fixes fire and draws 3 and 4 are used),
    every step compared; a masked reset half way keeps the draw counter."""
    pr = Pair("small_16x64", 4, exec_kw=exec_kw, steps=60, own_draws=True,
              params_over=dict(loop_closure=1, lc_gap=5, lc_radius_m=0.6, noise_seed=SEED))
    closed = 0
    for t in range(60):
        o = pr.step()
        closed += int(o.closed.sum())
        pr.compare(o)
        if t == 29:
            m = np.zeros(pr.n, np.uint8)
            m[::3] = 1
            pr.reset(pr.b.start, m)
    draws = pr.env.read(_lib.FIELD_DRAWS).cpu().numpy()
    assert np.all(draws == 60) and np.array_equal(draws.astype(np.uint64), pr.orc.draws)
    say(f"[rng] loop closures fired: {closed}")
    assert closed > 0
    # the draws moved the true poses off the noise-free estimates
    assert np.all(np.abs(pr.orc.pose[:, :2] - pr.orc.est[:, :2]).max(axis=1) > 0)


def test_env_own_draws_paper_sensor():
    """The paper's sensor mode (range noise: draws 5 .. 5 + R - 1 per robot-step), fused 256."""
    pick = np.arange(0, 750, 53)[:12]
    pr = Pair("paper_sensor_750x256", 2, robots=pick, exec_kw=dict(form=1, threads=256, record_rays=1), steps=40,
              own_draws=True, params_over=dict(noise_seed=SEED + 1))
    assert pr.env.G == 5 + pr.R
    for t in range(40):
        o = pr.step()
        if t % 5 == 4:
            pr.compare(o)


def test_env_graph_replays_draw_new_numbers():
    """A captured sequence of steps with the library's draws: two replays equal 2 x K eager steps (the
    counters live on the device) and the oracle's 2 x K steps."""
    K = 6
    pr = Pair("small_16x64", 5, exec_kw=dict(form=1, threads=256, record_rays=1), steps=2 * K, own_draws=True,
              params_over=dict(noise_seed=SEED + 2))
    e = pr.env
    A = pr.dA
    e.graph_build(K, A, 2 * pr.n, None, 0, pr.ranges, 0, pr.reward, 0, pr.done, 0)
    e.graph_launch()
    torch.cuda.synchronize()
    for t in range(K):
        o = pr.orc.step(pr.A[t], None)
        pr.cum += o.counters[:, [2, 0, 1]]
    pr.t = K
    pr.compare(o, rays=True, tag="after replay 1")
    # the second replay re-reads actions 0..K-1; the oracle follows the same actions
    e.graph_launch()
    torch.cuda.synchronize()
    for t in range(K):
        o = pr.orc.step(pr.A[t], None)
        pr.cum += o.counters[:, [2, 0, 1]]
    pr.compare(o, rays=True, tag="after replay 2")
    assert np.all(e.read(_lib.FIELD_DRAWS).cpu().numpy() == 2 * K)


def test_action_draws_are_the_oracle_normals(oracle_mod):
    """sample() with mean 0 and log std 0 returns the normals themselves: equal to the oracle's draws
    (seed, action domain, counter, row, dimension) bit for bit, for several counters."""
    from paper_2603_25834_amd.policy import Policy, num_params
    O = oracle_mod
    B, R = 3000, 180
    pol = Policy(R, max_batch=16)
    params = torch.zeros(num_params(R), device="cuda")
    mu = torch.zeros((B, 2), device="cuda")
    for counter in (0, 1, 77, 2 ** 40 + 5):
        act, logp = pol.sample(params, mu, None, seed=SEED, counter=counter)
        torch.cuda.synchronize()
        want = O.normals(SEED, O.DOMAIN_ACTION, counter, B, 2)
        assert np.array_equal(act.cpu().numpy().view(np.int32), want.view(np.int32)), counter
        lp = -0.5 * (want[:, 0].astype(np.float64) ** 2 + want[:, 1] ** 2) - np.log(2 * np.pi)
        assert np.allclose(logp.cpu().numpy(), lp, rtol=1e-5, atol=1e-5)
    pol.close()


def test_rollout_call_own_draws_equal_fed_draws(oracle_mod):
    """The fused rollout call (forward + sample) with its own draws equals the same call fed the
    oracle's normals for that (seed, counter), bit for bit."""
    from paper_2603_25834_amd.policy import Policy
    O = oracle_mod
    B, R = 200, 360
    d = {k: torch.from_numpy(v).cuda() for k, v in synth.policy_batch(B, R, 3).items()}
    params = torch.from_numpy(synth.init_policy_params(R, 3)).cuda()
    pol = Policy(R, max_batch=B)
    v1, a1, l1 = pol.act(params, d["crop"], d["scan"], d["state"], None, seed=SEED, counter=9)
    eps = torch.from_numpy(O.normals(SEED, O.DOMAIN_ACTION, 9, B, 2)).cuda()
    v2, a2, l2 = pol.act(params, d["crop"], d["scan"], d["state"], eps)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2) and torch.equal(a1, a2) and torch.equal(l1, l2)
    v3, a3, _ = pol.act(params, d["crop"], d["scan"], d["state"], None, seed=SEED, counter=10)
    torch.cuda.synchronize()
    assert torch.equal(v1, v3) and not torch.equal(a1, a3)
    pol.close()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 1000, 18000, 98304, 131073])
def test_permutation_equals_oracle(oracle_mod, n):
    from paper_2603_25834_amd.policy import permutation, permutation_work_bytes
    p = permutation(n, SEED, 3).cpu().numpy()
    want = oracle_mod.permute(n, SEED, 3)
    assert np.array_equal(p, want)
    assert np.array_equal(np.sort(p), np.arange(n))
    # the tabulated form (workspace of the whole Feistel domain) is the same permutation
    wb = permutation_work_bytes(n)
    b = 2
    while (1 << b) < n:
        b += 2
    assert wb == 4 << b
    work = torch.full((wb // 4 + 3,), -1, dtype=torch.int32, device="cuda")
    q = permutation(n, SEED, 3, work=work[:wb // 4]).cpu().numpy()
    assert np.array_equal(q, want)
    assert int(work[wb // 4:].min()) == -1 and int(work[wb // 4:].max()) == -1   # nothing past the workspace
    with pytest.raises(Exception, match="work_bytes"):
        permutation(n, SEED, 3, work=work[:wb // 4 - 1])
