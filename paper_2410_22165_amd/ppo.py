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
                 groups: int = 1, gov_learning: bool = False, gov_hidden: int = 128):
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
        # every sample of a rollout packed into one record (ej_ppo_pack), so that a
        # minibatch row's gather touches one cache-line-aligned block
        self.records = torch.empty(self.M_total * binding.ppo_record_bytes(self.mlp), dtype=torch.uint8,
                                   device="cuda")
        # sampling counter on the device: a step's uniforms use (base + t); the
        # base moves by T + 1 after each rollout, so a replayed graph draws fresh ones
        self.ctr_base = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.updates = 0
        self.adam_step = 0
        self.gov = None
        if gov_learning:
            self.gov = GovLearner(self, env_cfg, gov_hidden, seed)
            self.rollout = None
        else:
            self.env.set_gov_draw(True, seed + 1)
        self.env.observe(self.store.obs[0], self.store.mask[0])
        if not gov_learning:
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
        if self.gov is not None:
            self.gov.collect()
        elif graph:
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
        binding.ppo_pack(self.mlp, flat, self.M_total, self.records)
        for epoch in range(self.epochs):
            a, c = W.affine_permutation(self.M_total, self.updates * self.epochs + epoch, seed=self.seed)
            for mb in range(self.minibatches):
                binding.ppo_backward(self.mlp, flat, self.M_total, a, c, mb * self.mb_rows, self.mb_rows, hp,
                                     self.workspace, self.grads, self.loss_terms, records=self.records)
                self.adam_step += 1
                binding.adam(self.mlp.params, self.grads, self.adam_m, self.adam_v, self.adam_step, max(lr, 1e-12))
                self.mlp.sync()
        if self.gov is not None:
            self.gov.update(lr, ent)
        self.updates += 1
        self.next_rollout()

    def next_rollout(self):
        """The next rollout starts from the state after this one."""
        self.store.obs[0].copy_(self.store.obs[self.T])
        self.store.mask[0].copy_(self.store.mask[self.T])

    def close(self):
        if self.rollout is not None:
            self.rollout.close()
        self.env.close()


class GovLearner:
    """The government agent trained at the same time as the population
    (Sec. 3 "Government Agent", "Setting tax rates"; Sec. 4 "Experimental
    details"): at the first step of every tax period its policy
    (ej_gov_policy_forward) reads each economy's government observation and
    sets the K bracket levels the economy step applies.  A decision's reward
    is the sum of the per-step government rewards until the next decision
    (ej_sum_steps, within the rollout); GAE runs over the decisions of the
    rollout (ej_gae), bootstrapped with the value of the state after it, and
    the update is the PPO loss of the K-head policy (ej_gov_ppo_backward) with
    Adam.  The rollout is issued from the host, one launch per kernel."""

    def __init__(self, tr: "PPOTrainer", env_cfg: dict, hidden: int, seed: int):
        import workloads as W
        e = tr.env
        self.tr, self.K = tr, e.K
        self.Dg = e.Dg
        self.Dgs = (e.Dg + 7) // 8 * 8
        self.E, self.P_tax, self.T_ep = e.E, env_cfg["P_tax"], env_cfg["T"]
        self.seed = seed + 2
        A = 21 * self.K
        self.mlp = binding.Mlp(self.Dg, self.Dgs, hidden, A, W.policy_weights(self.Dg, hidden, A, seed=seed + 3))
        self.scale = torch.from_numpy(W.gov_obs_scales(env_cfg)).cuda()
        z = dict(device="cuda")
        T = tr.T
        self.Dmax = T // self.P_tax + 2  # decisions per rollout at most
        D, E, K = self.Dmax, self.E, self.K
        self.obs = torch.zeros((D, E, self.Dgs), dtype=torch.int16, **z)
        self.lv = torch.zeros((D, E, K), dtype=torch.int32, **z)
        self.logp = torch.zeros((D, E), **z)
        self.val = torch.zeros((D, E), **z)
        self.ent = torch.zeros((D, E), **z)
        self.rew = torch.zeros((D, E), **z)
        self.done = torch.zeros((D, E), dtype=torch.uint8, **z)
        self.adv = torch.zeros((D, E), **z)
        self.ret = torch.zeros((D, E), **z)
        self.last_val = torch.zeros(E, **z)
        self.gov_obs = torch.zeros((E, self.Dg), **z)
        self.scratch_obs = torch.zeros((tr.M, tr.Ds), dtype=torch.int16, **z)
        self.scratch_mask = torch.zeros((tr.M, tr.Wm), dtype=torch.int32, **z)
        self.tmp_i = torch.zeros((E, K), dtype=torch.int32, **z)
        self.tmp_f = torch.zeros((3, E), **z)
        n = self.mlp.layout["n_params"]
        self.grads = torch.zeros(n, **z)
        self.adam_m = torch.zeros(n, **z)
        self.adam_v = torch.zeros(n, **z)
        self.adam_step = 0
        self.loss_terms = torch.zeros(binding.PPO_LOSS_TERMS, **z)
        self.t_env = int(e.get_state()["t"][0])  # every economy shares the episode clock
        self.levels = torch.zeros(max(E * K, 1), dtype=torch.int32, **z)  # the levels in force
        self.n_dec = 0
        self.decisions = 0  # sampling counter

    def _observe(self):
        tr = self.tr
        tr.env.observe(self.scratch_obs, self.scratch_mask, self.gov_obs)

    def collect(self):
        tr, s = self.tr, self.tr.store
        starts = []
        for t in range(tr.T):
            if self.t_env % self.P_tax == 0:
                d = len(starts)
                self._observe()
                binding.gov_policy_forward(self.mlp, self.K, self.gov_obs, self.scale, self.E, self.seed,
                                           self.decisions, self.lv[d], self.logp[d], self.val[d], self.ent[d],
                                           obs_bf16=self.obs[d])
                self.levels.copy_(self.lv[d].reshape(-1))
                self.decisions += 1
                starts.append(t)
            tr.mlp.forward(s.obs[t], s.mask[t], tr.M, tr.seed, t, s.act[t], s.logp[t], s.val[t], s.ent[t],
                           ctr_base=tr.ctr_base)
            tr.env.step(s.act[t], self.levels, s.rew[t], s.gov_rew[t], s.done[t], s.obs[t + 1], s.mask[t + 1])
            self.t_env = (self.t_env + 1) % self.T_ep
        tr.mlp.forward(s.obs[tr.T], s.mask[tr.T], tr.M, tr.seed, tr.T, s.tmp[2 * tr.M:].view(torch.int32),
                       s.tmp[:tr.M], s.last_val, s.tmp[tr.M:2 * tr.M], ctr_base=tr.ctr_base)
        binding.gae(s.rew, s.val, s.done, s.last_val, tr.T, tr.M, tr.gamma, tr.lam, s.adv, s.ret)
        binding.counter_add(tr.ctr_base, tr.T + 1)
        # decisions: rewards summed over their periods, episode ends, bootstrap value
        self.n_dec = len(starts)
        ends = starts[1:] + [tr.T]
        done_host = s.done[:, 0].cpu().numpy()  # every economy ends its episode at the same step
        for d, (a, b) in enumerate(zip(starts, ends)):
            binding.sum_steps(s.gov_rew, a, b, self.E, self.rew[d])
            self.done[d].fill_(1 if done_host[a:b].any() else 0)
        if self.n_dec:
            self._observe()
            binding.gov_policy_forward(self.mlp, self.K, self.gov_obs, self.scale, self.E, self.seed, 0, self.tmp_i,
                                       self.tmp_f[0], self.last_val, self.tmp_f[1])
            binding.gae(self.rew, self.val, self.done, self.last_val, self.n_dec, self.E, self.tr.gamma,
                        self.tr.lam, self.adv, self.ret)

    def update(self, lr: float, ent: float):
        import workloads as W
        if self.n_dec == 0:
            return
        tr = self.tr
        hp = dict(tr.hp, ent_coef=ent)
        n = self.n_dec * self.E
        flat = dict(obs=self.obs[:self.n_dec].reshape(n, -1), act=self.lv[:self.n_dec].reshape(n, -1),
                    logp_old=self.logp[:self.n_dec].reshape(-1), val_old=self.val[:self.n_dec].reshape(-1),
                    adv=self.adv[:self.n_dec].reshape(-1), ret=self.ret[:self.n_dec].reshape(-1))
        mbs = max(1, min(tr.minibatches, n // 64))
        rows = n // mbs
        ws = torch.zeros(binding.gov_ppo_workspace_bytes(self.mlp, self.K, rows), dtype=torch.uint8, device="cuda")
        for epoch in range(tr.epochs):
            a, c = W.affine_permutation(n, tr.updates * tr.epochs + epoch, seed=self.seed)
            for mb in range(mbs):
                binding.gov_ppo_backward(self.mlp, self.K, flat, n, a, c, mb * rows, rows, hp, ws, self.grads,
                                         self.loss_terms)
                self.adam_step += 1
                binding.adam(self.mlp.params, self.grads, self.adam_m, self.adam_v, self.adam_step, max(lr, 1e-12))
                self.mlp.sync()


class MultiAgentTrainer:
    """PPO with per-agent weight sets (Sec. 5, methods 2 and 3): layout
    "ippo" gives every agent index its own policy and value network (agent g
    of every economy acts with set g); "mappo" gives every agent its own
    policy and all agents one shared value network that sees the same
    per-agent observation.  The rollout runs the grouped policy forward
    (ej_policy_forward_grouped: one launch, 64-row tiles of one set each)
    and, for "mappo", the shared value network; each agent's update reads its
    own samples of the shared storage (batch row_stride = N, row_offset =
    agent), and one Adam step covers every stacked set.  Economies have N
    agents each; launches are issued from the host."""

    def __init__(self, env_cfg: dict, scales: dict, layout: str, hidden: int, rollout: int, epochs: int,
                 minibatches: int, gamma: float, lam: float, clip: float, vf_coef: float, vclip: float,
                 ent_coef: float, lr: float, seed: int = 0, total_updates: int = 1):
        import workloads as W
        if layout not in ("ippo", "mappo"):
            raise ValueError(layout)
        self.layout = layout
        self.env = binding.Env(env_cfg, scales)
        e = self.env
        self.E, self.N = e.E, env_cfg["N"]
        self.M, self.A, self.D, self.Ds, self.Wm = e.M, e.A, e.D, e.Ds, e.W
        assert self.M == self.E * self.N
        self.T, self.epochs, self.minibatches = rollout, epochs, minibatches
        self.gamma, self.lam, self.lr0, self.ent0 = gamma, lam, lr, ent_coef
        self.hp = dict(clip=clip, vclip=vclip, vf_coef=vf_coef, ent_coef=ent_coef)
        self.seed, self.total_updates = seed, total_updates
        self.pol = binding.GroupedMlp(e.D, e.Ds, hidden, e.A, self.N,
                                      [W.policy_weights(e.D, hidden, e.A, seed=seed * 1000 + g) for g in range(self.N)])
        z = dict(device="cuda")
        self.grads = torch.zeros_like(self.pol.params)
        self.adam_m = torch.zeros_like(self.pol.params)
        self.adam_v = torch.zeros_like(self.pol.params)
        self.store = RolloutStorage(rollout, self.M, self.Ds, self.Wm, e.E)
        self.ctr_base = torch.zeros(1, dtype=torch.int64, **z)
        self.loss_terms = torch.zeros(binding.PPO_LOSS_TERMS, **z)
        self.S_agent = rollout * self.E  # one agent's samples per rollout
        self.mb_rows = self.S_agent // minibatches
        self.workspace = torch.zeros(binding.ppo_workspace_bytes(self.pol._one, self.mb_rows), dtype=torch.uint8, **z)
        if layout == "mappo":
            self.vnet = binding.Mlp(e.D, e.Ds, hidden, 1, W.policy_weights(e.D, hidden, 1, seed=seed + 7))
            self.vmask = torch.ones((rollout + 1, self.M, 1), dtype=torch.int32, **z)  # the one dummy action
            self.vzero_i = torch.zeros((rollout, self.M), dtype=torch.int32, **z)
            self.vzero_f = torch.zeros((rollout, self.M), **z)
            self.vtmp = torch.zeros((4, self.M), **z)
            self.vgrads = torch.zeros_like(self.vnet.params)
            self.vadam_m = torch.zeros_like(self.vnet.params)
            self.vadam_v = torch.zeros_like(self.vnet.params)
            self.v_rows = rollout * self.M // minibatches
            self.vworkspace = torch.zeros(binding.ppo_workspace_bytes(self.vnet, self.v_rows), dtype=torch.uint8, **z)
            self.vloss = torch.zeros(binding.PPO_LOSS_TERMS, **z)
        self.updates = 0
        self.adam_step = 0
        self.env.set_gov_draw(True, seed + 1)
        self.env.observe(self.store.obs[0], self.store.mask[0])

    def _values(self, t, out):
        s = self.store
        self.vnet.forward(s.obs[t], self.vmask[t], self.M, self.seed + 9, t, self.vtmp[0].view(torch.int32),
                          self.vtmp[1], out, self.vtmp[2], ctr_base=self.ctr_base)

    def collect(self):
        s = self.store
        for t in range(self.T):
            self.pol.forward(s.obs[t], s.mask[t], self.E, self.N, self.seed, t, s.act[t], s.logp[t], s.val[t],
                             s.ent[t], ctr_base=self.ctr_base)
            if self.layout == "mappo":
                self._values(t, s.val[t])
            self.env.step(s.act[t], None, s.rew[t], s.gov_rew[t], s.done[t], s.obs[t + 1], s.mask[t + 1])
        if self.layout == "mappo":
            self._values(self.T, s.last_val)
        else:
            self.pol.forward(s.obs[self.T], s.mask[self.T], self.E, self.N, self.seed, self.T,
                             s.tmp[2 * self.M:].view(torch.int32), s.tmp[:self.M], s.last_val, s.tmp[self.M:2 * self.M],
                             ctr_base=self.ctr_base)
        binding.gae(s.rew, s.val, s.done, s.last_val, self.T, self.M, self.gamma, self.lam, s.adv, s.ret)
        binding.counter_add(self.ctr_base, self.T + 1)

    def update(self):
        import workloads as W
        frac = self.updates / max(self.total_updates, 1)
        lr = self.lr0 * max(1.0 - frac, 0.0)
        ent = self.ent0 * max(1.0 - frac / 0.9, 0.0)
        hp = dict(self.hp, ent_coef=ent)
        if self.layout == "mappo":
            hp = dict(hp, vf_coef=0.0)  # the policies carry no value head of their own
        flat = self.store.flat()
        n = self.pol.layout["n_params"]
        for epoch in range(self.epochs):
            a, c = W.affine_permutation(self.S_agent, self.updates * self.epochs + epoch, seed=self.seed)
            if self.layout == "mappo":
                av, cv = W.affine_permutation(self.T * self.M, self.updates * self.epochs + epoch, seed=self.seed + 5)
            for mb in range(self.minibatches):
                for g in range(self.N):
                    binding.ppo_backward(self.pol._one, flat, self.S_agent, a, c, mb * self.mb_rows, self.mb_rows, hp,
                                         self.workspace, self.grads[g * self.pol.ps:g * self.pol.ps + n],
                                         self.loss_terms, row_stride=self.N, row_offset=g,
                                         params=self.pol.params_ptr(g), work=self.pol.work_ptr(g))
                self.adam_step += 1
                binding.adam(self.pol.params, self.grads, self.adam_m, self.adam_v, self.adam_step, max(lr, 1e-12))
                self.pol.sync()
                if self.layout == "mappo":
                    vflat = dict(flat, mask=self.vmask[:self.T].reshape(self.T * self.M, 1),
                                 act=self.vzero_i.reshape(-1), logp_old=self.vzero_f.reshape(-1),
                                 adv=self.vzero_f.reshape(-1))
                    vhp = dict(self.hp, ent_coef=0.0)
                    binding.ppo_backward(self.vnet, vflat, self.T * self.M, av, cv, mb * self.v_rows, self.v_rows,
                                         vhp, self.vworkspace, self.vgrads, self.vloss)
                    binding.adam(self.vnet.params, self.vgrads, self.vadam_m, self.vadam_v, self.adam_step,
                                 max(lr, 1e-12))
                    self.vnet.sync()
        self.updates += 1
        self.store.obs[0].copy_(self.store.obs[self.T])
        self.store.mask[0].copy_(self.store.mask[self.T])

    def close(self):
        self.env.close()
