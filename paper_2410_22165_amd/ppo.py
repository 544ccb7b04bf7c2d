"""PPO driver for the batched economy (argument marshalling around the C ABI).

Rollout: every step the shared policy samples all agents' actions
(ej_policy_forward) and the economy step (ej_env_step, which also draws the
government's uniform tax levels) writes rewards, done flags and the next
observation and mask straight into the rollout storage; the library captures
the whole rollout as one HIP graph (ej_rollout_capture).  Update: GAE (ej_gae), then epochs x
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
    def __init__(self, T: int, M: int, Ds: int, W: int, E: int, device="cuda"):
        self.T, self.M = T, M
        z = dict(device=device)
        self.gov_rew = torch.zeros((T, E), **z)
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
        self.tmp = torch.zeros(3 * M, **z)  # discarded outputs of the last-value forward

    def buffers(self, ctr) -> dict:
        """The arrays ej_rollout_capture writes (the graph keeps them)."""
        return dict(obs=self.obs, mask=self.mask, act=self.act, logp=self.logp, val=self.val, ent=self.ent,
                    rew=self.rew, done=self.done, gov_rew=self.gov_rew, last_val=self.last_val, adv=self.adv,
                    ret=self.ret, tmp=self.tmp, ctr=ctr)

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
        self.store = RolloutStorage(rollout, self.M, self.Ds, self.Wm, e.E)
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
        self.env.set_gov_draw(True, seed + 1)
        self.env.observe(self.store.obs[0], self.store.mask[0])
        # the whole rollout as one HIP graph captured by the library, the
        # economies pipelined over `groups` streams
        self.rollout = binding.Rollout(self.env, self.mlp, self.store.buffers(self.ctr_base), rollout, seed,
                                       groups=groups, last_value=True, gamma=gamma, lam=lam)

    # ---- rollout ----
    def collect(self, graph: bool = False):
        """One rollout of T steps (policy forward and economy step of every
        group per step; the government's uniform levels are drawn inside the
        step, seed + 1), the last value and GAE.  graph=True replays the
        captured HIP graph; graph=False issues the same launches one by one
        (identical results)."""
        if graph:
            self.rollout.launch()
        else:
            self.rollout.launch_plain()

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
        self.rollout.close()
        self.env.close()
