"""One PPO training iteration over the batched env, end to end on the GPU (needs an MI355X).

The stages are checked one by one elsewhere (env step, forward, loss gradient, sampling, gather,
GAE, Adam); here: the iteration runs on the small workload, the losses stay finite, the parameters
move, and two runs from the same state with the same draws end bit-identical."""
import numpy as np
import pytest
import torch

from envpair import say
from paper_2603_25834_amd import synth
from paper_2603_25834_amd.env import Env
from paper_2603_25834_amd.ppo import PPOTrainer

pytestmark = pytest.mark.gpu


def _trainer(seed):
    w = synth.WORKLOADS["small_16x64"]
    b = synth.make_batch("small_16x64", seed)
    env = Env(w.params(), b.sides)
    env.set_exec(form=1, threads=128)
    world = torch.from_numpy(b.world.view(np.int32).copy()).cuda()
    start = torch.from_numpy(b.start).cuda()
    env.reset(world, start)
    params = torch.from_numpy(synth.init_policy_params(w.n_rays, seed)).cuda()
    tr = PPOTrainer(env, world, start, params, T=6, epochs=2, minibatch=40, lr=1e-3)
    return tr, params.clone()


def test_iteration_runs_and_is_deterministic():
    finals = []
    for _ in range(2):
        tr, p0 = _trainer(3)
        noise, eps, perm = tr.draws(2, seed=5)
        for i in range(2):
            tr.iteration(noise[i], eps[i], perm[i])
        torch.cuda.synchronize()
        loss = tr.loss.cpu().numpy()
        say(f"[ppo] minibatches/epoch {tr.n_mb} of {tr.mb}; last loss terms {loss}")
        assert np.all(np.isfinite(loss))
        assert not torch.equal(tr.params, p0)
        assert tr.step_count == 2 * tr.epochs * tr.n_mb
        finals.append(tr.params.cpu().numpy().copy())
    assert np.array_equal(finals[0], finals[1])
