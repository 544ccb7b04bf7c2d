"""PPO driver for the batched economy (argument marshalling around the C ABI).

Rollout: every step the shared policy samples all agents' actions
(ej_policy_forward) and the economy step (ej_env_step, which also draws the
government's uniform tax levels) writes rewards, done flags and the next
observation and mask straight into the rollout storage.  Update: GAE (ej_gae), then epochs x
minibatches of the hand-written backward (ej_ppo_backward) and Adam
(ej_adam), with the bf16 work copy refreshed after every step
(ej_mlp_sync_weights).  Table 2 of the paper lists the PPO settings; the
entropy coefficient is annealed linearly over 90 % of training and the
learning rate over all of it.

`PPOLoss` exposes the backward kernel as a torch.autograd.Function: its
forward runs the fused kernel (which produces the loss terms and the
gradient in one pass) and its backward hands the stored gradient to
autograd.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding


def economy_groups(env, groups: int):
    """Split the economies into `groups` contiguous ranges:
    [(e_begin, e_end, row_begin, row_end)] (rows from the env's row offsets)."""
    E = env.E
    groups = max(1, min(int(groups), E))
    out = []
    for g in range(groups):
        e0, e1 = E * g // groups, E * (g + 1) // groups
        out.append((e0, e1, int(env.row_offsets[e0]), int(env.row_offsets[e1])))
    return out


class GroupStreams:
    """One stream per economy group (default priority).  Economies never
    interact, so each group's policy -> step chain runs on its own stream and
    one group's policy overlaps another's economy step.  fork() / join()
    order the streams after / before the current stream's work (also inside
    graph capture)."""

    def __init__(self, n: int):
        self.streams = [torch.cuda.Stream() for _ in range(n)] if n > 1 else []

    def fork(self):
        cur = torch.cuda.current_stream()
        for st in self.streams:
            st.wait_stream(cur)

    def join(self):
        cur = torch.cuda.current_stream()
        for st in self.streams:
            cur.wait_stream(st)

    def stream(self, g: int):
        return torch.cuda.stream(self.streams[g]) if self.streams else torch.cuda.stream(torch.cuda.current_stream())


class PPOLoss(torch.autograd.Function):
    """loss = surrogate + c_v * value - c_e * entropy of one minibatch, as a
    function of the flat parameter vector `params` (= mlp.params)."""

    @staticmethod
    def forward(ctx, params, mlp, storage, M_total, perm_a, perm_c, row_begin, rows, hp, workspace):
        grads = torch.empty_like(params)
        terms = torch.empty(binding.PPO_LOSS_TERMS, device=params.device)
        binding.ppo_backward(mlp, storage, M_total, perm_a, perm_c, row_begin, rows, hp, workspace, grads, terms)
        ctx.save_for_backward(grads)
        ctx.terms = terms
        return terms[4]  # the kernel's minibatch loss

    @staticmethod
    def backward(ctx, grad_out):
        (grads,) = ctx.saved_tensors
        return (grad_out * grads,) + (None,) * 9


class RolloutStorage:
    def __init__(self, T: int, M: int, Ds: int, W: int, device="cuda"):
        self.T, self.M = T, M
        z = dict(device=device)
        self.obs = torch.zeros((T + 1, M, Ds), dtype=torch.int16, **z)  # obs[T] = the state after the rollout
        self.mask = torch.zeros((T + 1, M, W), dtype=torch.int32, **z)
        self.act = torch.zeros((T, M), dtype=torch.int32, **z)
        self.logp = torch.zeros((T, M), **z)
        self.val = torch.zeros((T, M), **z)
        self.ent = torch.zeros((T, M), **z)
        self.rew = torch.zeros((T, M), **z)
        self.done = torch.zeros((T, M), dtype=torch.uint8, **z)
        self.adv = torch.zeros((T, M), **z)
        self.ret = torch.zeros((T, M), **z)
        self.last_val = torch.zeros(M, **z)
        self.scratch_act = torch.zeros(M, dtype=torch.int32, **z)
        self.scratch = torch.zeros((2, M), **z)

    def flat(self) -> dict:
        T, M = self.T, self.M
        return dict(obs=self.obs[:T].reshape(T * M, -1), mask=self.mask[:T].reshape(T * M, -1),
                    act=self.act.reshape(-1), logp_old=self.logp.reshape(-1), val_old=self.val.reshape(-1),
                    adv=self.adv.reshape(-1), ret=self.ret.reshape(-1))


class PPOTrainer:
    def __init__(self, env_cfg: dict, scales: dict, hidden: int, rollout: int, epochs: int, minibatches: int,
                 gamma: float, lam: float, clip: float, vf_coef: float, vclip: float, ent_coef: float, lr: float,
                 seed: int = 0, weights: dict | None = None, n_per_env=None, total_updates: int = 1,
                 groups: int = 1):
        import workloads as W
        self.env = binding.Env(env_cfg, scales, n_per_env)
        e = self.env
        self.M, self.A, self.D, self.Ds, self.Wm = e.M, e.A, e.D, e.Ds, e.W
        if weights is None:
            weights = W.policy_weights(e.D, hidden, e.A, seed=seed)
        self.mlp = binding.Mlp(e.D, e.Ds, hidden, e.A, weights)
        self.T, self.epochs, self.minibatches = rollout, epochs, minibatches
        self.gamma, self.lam, self.lr0, self.ent0 = gamma, lam, lr, ent_coef
        self.hp = dict(clip=clip, vclip=vclip, vf_coef=vf_coef, ent_coef=ent_coef)
        self.seed = seed
        self.total_updates = total_updates
        self.store = RolloutStorage(rollout, self.M, self.Ds, self.Wm)
        self.gov = torch.zeros(max(e.E * e.K, 1), dtype=torch.int32, device="cuda")
        self.gov_rew = torch.zeros(e.E, device="cuda")
        n = self.mlp.layout["n_params"]
        self.grads = torch.zeros(n, device="cuda")
        self.adam_m = torch.zeros(n, device="cuda")
        self.adam_v = torch.zeros(n, device="cuda")
        self.loss_terms = torch.zeros(binding.PPO_LOSS_TERMS, device="cuda")
        self.M_total = rollout * self.M
        self.mb_rows = self.M_total // minibatches
        self.workspace = torch.zeros(binding.ppo_workspace_bytes(self.mlp, self.mb_rows), dtype=torch.uint8,
                                     device="cuda")
        # sampling counter on the device: a step's uniforms use (base + t); the
        # base moves by T + 1 after each rollout, so a replayed graph draws fresh ones
        self.ctr_base = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.updates = 0
        self.adam_step = 0
        self.graph = None
        self.groups = economy_groups(self.env, groups)  # rollout pipelined over economy groups
        self.group_streams = GroupStreams(len(self.groups))
        self.env.set_gov_draw(True, seed + 1)
        self.env.observe(self.store.obs[0], self.store.mask[0])

    # ---- rollout ----
    def rollout_step(self, t: int):
        """Policy and economy step for every group (the government's uniform
        levels are drawn inside the step, seed + 1).  A group's rows are a
        slice of the batch; row_base keeps the sampler's row numbering, so
        any grouping gives the same rollout."""
        s = self.store
        for g, (e0, e1, r0, r1) in enumerate(self.groups):
            with self.group_streams.stream(g):
                self.mlp.forward(s.obs[t][r0:r1], s.mask[t][r0:r1], r1 - r0, self.seed, t, s.act[t][r0:r1],
                                 s.logp[t][r0:r1], s.val[t][r0:r1], s.ent[t][r0:r1], ctr_base=self.ctr_base,
                                 row_base=r0)
                self.env.step(s.act[t], None, s.rew[t], self.gov_rew, s.done[t], s.obs[t + 1], s.mask[t + 1],
                              economies=(e0, e1))

    def _collect_launches(self):
        self.group_streams.fork()
        for t in range(self.T):
            self.rollout_step(t)
        self.group_streams.join()
        s = self.store
        self.mlp.forward(s.obs[self.T], s.mask[self.T], self.M, self.seed, self.T, s.scratch_act, s.scratch[0],
                         s.last_val, s.scratch[1], ctr_base=self.ctr_base)
        binding.gae(s.rew, s.val, s.done, s.last_val, self.T, self.M, self.gamma, self.lam, s.adv, s.ret)
        binding.counter_add(self.ctr_base, self.T + 1)

    def collect(self, graph: bool = False):
        """One rollout of T steps, then GAE.  graph=True replays the whole
        rollout as one captured HIP graph (captured on first use; the kernels
        must have run once before, so the first call with graph=True runs the
        plain launches and captures afterwards)."""
        if not graph:
            self._collect_launches()
            return
        if self.graph is None:
            self._collect_launches()
            torch.cuda.synchronize()
            # record the rollout for the following calls (capture executes nothing)
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self._collect_launches()
        else:
            self.graph.replay()

    # ---- update ----
    def schedules(self):
        frac = self.updates / max(self.total_updates, 1)
        lr = self.lr0 * max(1.0 - frac, 0.0)
        ent = self.ent0 * max(1.0 - frac / 0.9, 0.0)
        return lr, ent

    def update(self):
        import workloads as W
        lr, ent = self.schedules()
        hp = dict(self.hp, ent_coef=ent)
        flat = self.store.flat()
        for epoch in range(self.epochs):
            a, c = W.affine_permutation(self.M_total, self.updates * self.epochs + epoch, seed=self.seed)
            for mb in range(self.minibatches):
                binding.ppo_backward(self.mlp, flat, self.M_total, a, c, mb * self.mb_rows, self.mb_rows, hp,
                                     self.workspace, self.grads, self.loss_terms)
                self.adam_step += 1
                binding.adam(self.mlp.params, self.grads, self.adam_m, self.adam_v, self.adam_step, max(lr, 1e-12))
                self.mlp.sync()
        self.updates += 1
        self.next_rollout()

    def next_rollout(self):
        """The next rollout starts from the state after this one."""
        self.store.obs[0].copy_(self.store.obs[self.T])
        self.store.mask[0].copy_(self.store.mask[self.T])

    def close(self):
        self.env.close()
