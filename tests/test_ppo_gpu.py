"""One PPO training iteration over the batched env, end to end on the GPU (needs an MI355X).

The stages are checked one by one elsewhere (env step, forward, loss gradient, sampling, gather,
GAE, Adam); here: the iteration runs on the small workload, the losses stay finite, the parameters
move, and two runs from the same state with the same seed end bit-identical (every draw comes from
the library's counter-based generator), while another seed ends elsewhere."""
import numpy as np
import pytest
import torch

from envpair import say
from paper_2603_25834_amd import synth
from paper_2603_25834_amd.env import Env
from paper_2603_25834_amd.ppo import PPOTrainer

pytestmark = pytest.mark.gpu


def _trainer(seed, recurrent=False, name="small_16x64", draw_seed=5):
    w = synth.WORKLOADS[name]
    b = synth.make_batch(name, seed, np.arange(16) if w.n_robots > 16 else None)
    p = w.params()
    p["noise_seed"] = 1000 + draw_seed
    env = Env(p, b.sides)
    env.set_exec(form=1, threads=128)
    world = torch.from_numpy(b.world.view(np.int32).copy()).cuda()
    start = torch.from_numpy(b.start).cuda()
    env.reset(world, start)
    init = synth.init_recurrent_params if recurrent else synth.init_policy_params
    params = torch.from_numpy(init(w.n_rays, seed)).cuda()
    tr = PPOTrainer(env, world, start, params, T=6, epochs=2, minibatch=40, lr=1e-3, recurrent=recurrent,
                    seed=draw_seed)
    return tr, params.clone()


@pytest.mark.parametrize("recurrent,name", [(False, "small_16x64"), (True, "paper_sensor_750x256")],
                         ids=["mlp", "gru_paper_mode"])
def test_iteration_runs_and_is_deterministic(recurrent, name):
    """The feed-forward policy on the small workload, and the GRU policy in the paper's sensor / reward
    mode on 16 robots of the 750-robot scene (minibatches of whole robot sequences, BPTT)."""
    finals = []
    for draw_seed in (5, 5, 6):
        tr, p0 = _trainer(3, recurrent, name, draw_seed)
        for i in range(2):
            tr.iteration()
        torch.cuda.synchronize()
        loss = tr.loss.cpu().numpy()
        say(f"[ppo] minibatches/epoch {tr.n_mb} of {tr.mb}; last loss terms {loss}")
        assert np.all(np.isfinite(loss))
        assert not torch.equal(tr.params, p0)
        assert tr.step_count == 2 * tr.epochs * tr.n_mb
        finals.append(tr.params.cpu().numpy().copy())
    assert np.array_equal(finals[0], finals[1])
    assert not np.array_equal(finals[0], finals[2])
