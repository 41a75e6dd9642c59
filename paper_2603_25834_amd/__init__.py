"""MI355X-native (gfx950) hot path of "Massive Parallel Deep Reinforcement Learning
for Active SLAM" (arXiv 2603.25834): the batched environment step and the PPO
actor-critic, behind the C-ABI library ``libaslam.so``.

Submodules are imported on demand: ``env`` (GPU environment), ``synth``
(seeded synthetic inputs), ``_lib`` (ctypes binding), ``build`` (hipcc step).
"""
__all__ = ["env", "synth", "build"]
