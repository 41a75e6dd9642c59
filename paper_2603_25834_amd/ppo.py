"""PPO training iteration over the batched environment (rollout + update), on the library's kernels.

Method: arXiv 2603.25834 Sec. III-F (PPO with the clipped surrogate of Eqs. 18-20 and GAE) driving the
batched POMDP step of Sec. III-B.  One iteration:

  rollout, t = 0 .. T-1:  observe (scan, pose + covariance, 64x64 belief crop) -> policy forward and
      Gaussian action sample in one call (value, action, log-prob; the BF16 weight copies are formed
      once per rollout) -> env step (reward, done) -> masked reset of the robots whose episode ended;
  bootstrap value of the last observation; GAE over the [T, N] rollout;
  update: `epochs` passes over the T*N samples in shuffled minibatches: fused loss and gradient over
      the minibatch's rows of the rollout arrays, read in place (activations recomputed from the stored
      inputs) -> Adam.

With `recurrent` the policy is the GRU actor-critic of Sec. III-F ("Recurrent Layer"): the rollout
carries each robot's GRU state from step to step (zeroed at the first step of an episode), and the
update takes minibatches of whole robot sequences (all T steps of a shuffled set of robots) through
backpropagation through time, starting from the state each robot had entering the rollout.

Every stage runs in the library's kernels; torch provides device memory, the stream, the
gradient accumulator's `zero_()` fill and a few small device copies (recurrent bookkeeping).
Random draws come from the library's counter-based generator inside the kernels that use them: the
env step's odometry (and range) noise under the env's own key, the action samples under (seed,
iteration * (T + 1) + t) and one minibatch permutation per epoch under (seed, iteration * epochs + e),
so an iteration is deterministic given the trainer's seed and iteration count.
"""
from __future__ import annotations

import torch

from .policy import Policy, adam, gae, permutation, permutation_work_bytes


class PPOTrainer:
    def __init__(self, env, world: torch.Tensor, start: torch.Tensor, params: torch.Tensor, T: int = 24,
                 epochs: int = 4, minibatch: int = 16384, lr: float = 3e-4, gamma: float = 0.99, lam: float = 0.95,
                 seed: int = 0, crop: int = 64, recurrent: bool = False, precision: int = 0):
        """precision: the feed-forward policy's forward operands, 0 BF16, 1 split hi + lo BF16 (the
        gradients then follow the exact network to 1e-2)."""
        self.env, self.world, self.start = env, world, start
        self.n, self.R = env.n, env.R
        self.T, self.epochs = T, epochs
        self.recurrent = bool(recurrent)
        self.S = T * self.n
        if self.recurrent:
            # minibatches of whole sequences: equal sets of at most minibatch // T robots
            self.n_mb = max(1, -(-self.n // max(1, minibatch // T)))
            self.mb = -(-self.n // self.n_mb)          # robots per minibatch
            max_b = max(self.mb * T, self.n)
        else:
            self.n_mb = max(1, -(-self.S // minibatch))
            self.mb = -(-self.S // self.n_mb)          # equal minibatches of at most `minibatch`
            max_b = max(self.mb, self.n)
        self.lr, self.gamma, self.lam = lr, gamma, lam
        dev = params.device
        self.policy = Policy(self.R, max_batch=max_b, recurrent=self.recurrent,
                             precision=0 if self.recurrent else precision)
        self.params = params
        self.grads = torch.zeros_like(params)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step_count = 0
        self.seed = int(seed)
        self.iters = 0                                   # iterations run (counter of the draws)
        T, n, R = self.T, self.n, self.R
        self.units = n if self.recurrent else self.S     # what a minibatch permutation shuffles
        self.phase_events = None   # set to (start, rollout done, end) torch.cuda.Events to time the phases
        # set to a callable hook(epoch, k, rows, flat, grads, params) to see each minibatch's gradient
        # before its Adam step (feed-forward policy; flat holds the rollout arrays, adv and ret)
        self.minibatch_hook = None
        self.perm = torch.zeros(self.units, dtype=torch.int32, device=dev)
        self.perm_work = torch.zeros(max(1, permutation_work_bytes(self.units) // 4), dtype=torch.int32, device=dev)
        # rollout storage (time-major)
        self.crop = torch.zeros((T + 1, n, crop, crop), dtype=torch.int16, device=dev)
        self.scan = torch.zeros((T + 1, n, R), device=dev)
        self.state = torch.zeros((T + 1, n, 12), device=dev)
        self.act_boot = torch.zeros((n, 2), device=dev)   # the bootstrap step's sample (unused)
        self.logp_boot = torch.zeros(n, device=dev)
        self.act = torch.zeros((T, n, 2), device=dev)
        self.logp = torch.zeros((T, n), device=dev)
        self.value = torch.zeros((T + 1, n), device=dev)
        self.reward = torch.zeros((T, n), device=dev)
        self.done = torch.zeros((T, n), dtype=torch.uint8, device=dev)
        self.ranges = torch.zeros((n, R), device=dev)
        self.loss = torch.zeros(4, device=dev)
        if self.recurrent:
            self.h = torch.zeros((n, 256), device=dev)            # GRU state after the last step
            self.h0 = torch.zeros((n, 256), device=dev)           # state entering step 0 of this rollout
            self.h_boot = torch.zeros((n, 256), device=dev)       # the bootstrap step's state (unused)
            self.first = torch.ones((T + 1, n), dtype=torch.uint8, device=dev)   # episode starts per step

    def _shuffle(self, it: int, e: int) -> torch.Tensor:
        """The permutation of epoch e of iteration `it` (library generator, into self.perm)."""
        return permutation(self.units, self.seed, it * self.epochs + e, out=self.perm, work=self.perm_work)

    def iteration(self) -> None:
        """One rollout of T steps and `epochs` update passes (all launches on the current stream)."""
        it = self.iters
        self.iters += 1
        if self.recurrent:
            return self._iteration_recurrent(it)
        env, pol, p, sd = self.env, self.policy, self.params, self.seed
        c0 = it * (self.T + 1)
        ev = self.phase_events
        if ev:
            ev[0].record()
        pol.prepare(p)   # the parameters are fixed during the rollout
        for t in range(self.T):
            env.observe(self.ranges, self.crop[t], self.scan[t], self.state[t])
            pol.act(p, self.crop[t], self.scan[t], self.state[t], None, self.value[t], self.act[t], self.logp[t],
                    prepared=True, seed=sd, counter=c0 + t)
            env.step(self.act[t], None, self.ranges, self.reward[t], self.done[t])
            env.reset(self.world, self.start, mask=self.done[t])
        env.observe(self.ranges, self.crop[self.T], self.scan[self.T], self.state[self.T])
        pol.act(p, self.crop[self.T], self.scan[self.T], self.state[self.T], None, self.value[self.T],
                self.act_boot, self.logp_boot, prepared=True, seed=sd, counter=c0 + self.T)
        adv, ret = gae(self.reward, self.value[:self.T].contiguous(), self.done, self.value[self.T],
                       self.gamma, self.lam)
        if ev:
            ev[1].record()
        flat = {
            "crop": self.crop[:self.T].reshape(self.S, *self.crop.shape[2:]),
            "scan": self.scan[:self.T].reshape(self.S, self.R),
            "state": self.state[:self.T].reshape(self.S, 12),
            "act": self.act.reshape(self.S, 2),
            "logp": self.logp.reshape(self.S),
            "adv": adv.reshape(self.S),
            "ret": ret.reshape(self.S),
        }
        for e in range(self.epochs):
            perm = self._shuffle(it, e)
            for k in range(self.n_mb):
                lo = k * self.mb
                idx = perm[lo:min(self.S, lo + self.mb)]
                self.grads.zero_()
                # the minibatch is the rows idx of the rollout arrays: the kernels read them in place
                pol.backward(p, flat["crop"], flat["scan"], flat["state"], flat["act"], flat["logp"], flat["adv"],
                             flat["ret"], self.grads, self.loss, rows=idx)
                if self.minibatch_hook is not None:
                    self.minibatch_hook(e, k, idx, flat, self.grads, p)
                self.step_count += 1
                adam(p, self.grads, self.m, self.v, self.step_count, lr=self.lr)
        if ev:
            ev[2].record()

    def _iteration_recurrent(self, it: int) -> None:
        env, pol, p, T, sd = self.env, self.policy, self.params, self.T, self.seed
        c0 = it * (T + 1)
        pol.prepare(p)
        self.h0.copy_(self.h)
        self.first[0].copy_(self.first[T])     # episode starts carried over from the last rollout's end
        for t in range(T):
            env.observe(self.ranges, self.crop[t], self.scan[t], self.state[t])
            pol.act_rnn(p, self.crop[t], self.scan[t], self.state[t], self.h, self.first[t], None, self.value[t],
                        self.act[t], self.logp[t], h_out=self.h, prepared=True, seed=sd, counter=c0 + t)
            env.step(self.act[t], None, self.ranges, self.reward[t], self.done[t])
            env.reset(self.world, self.start, mask=self.done[t])
            self.first[t + 1].copy_(self.done[t])
        env.observe(self.ranges, self.crop[T], self.scan[T], self.state[T])
        pol.act_rnn(p, self.crop[T], self.scan[T], self.state[T], self.h, self.first[T], None, self.value[T],
                    self.act_boot, self.logp_boot, h_out=self.h_boot, prepared=True, seed=sd, counter=c0 + T)
        adv, ret = gae(self.reward, self.value[:T].contiguous(), self.done, self.value[T], self.gamma, self.lam)
        first = self.first[:T]
        for e in range(self.epochs):
            perm = self._shuffle(it, e)
            for k in range(self.n_mb):
                lo = k * self.mb
                robots = perm[lo:min(self.n, lo + self.mb)]
                self.grads.zero_()
                pol.backward_seq(p, self.crop[:T], self.scan[:T], self.state[:T], self.h0, first, self.act,
                                 self.logp, adv, ret, robots, self.grads, self.loss)
                self.step_count += 1
                adam(p, self.grads, self.m, self.v, self.step_count, lr=self.lr)
