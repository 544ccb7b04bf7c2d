"""Per-agent weight sets (Sec. 5, methods 2 and 3: iPPO and MAPPO) on the
GPU: the grouped policy forward against the oracle network of each agent's
own weights, a grouped call with one set equal to the shared-layout call bit
for bit, each agent's strided backward equal to the backward of its gathered
samples bit for bit and to the oracle gradient element by element, and both
trainers end to end."""
import numpy as np
import pytest

import workloads as W
from oracle import env as oe
from oracle import policy as op

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _set_weights(D, H, A, seed):
    rng = np.random.default_rng(seed)
    w = W.policy_weights(D, H, A, seed=seed)
    for k in ("b1", "b2", "b3"):
        w[k] = (rng.standard_normal(w[k].shape) * 0.1).astype(np.float32)
    return w


@pytest.mark.parametrize("case", [(35, 40, 256, 125, 70, 5), (11, 16, 64, 30, 130, 3), (49, 56, 128, 507, 40, 4)])
def test_grouped_forward_matches_each_agents_oracle_network(case):
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, E, N = case
    M = E * N
    ws = [_set_weights(D, H, A, 100 + g) for g in range(N)]
    pol = binding.GroupedMlp(D, Ds, H, A, N, ws)
    obs = W.synthetic_obs(M, D, Ds, seed=E)
    mask = W.synthetic_masks(M, A, seed=E)
    out = dict(act=torch.zeros(M, dtype=torch.int32, device="cuda"), logp=torch.zeros(M, device="cuda"),
               val=torch.zeros(M, device="cuda"), ent=torch.zeros(M, device="cuda"))
    logits = torch.zeros((M, A), device="cuda")
    print(f"[gpu] grouped forward D={D} H={H} A={A} E={E} N={N}", flush=True)
    pol.forward(_t(obs.view(np.int16)), _t(mask.view(np.int32)), E, N, 31, 4, out["act"], out["logp"], out["val"],
                out["ent"], logits=logits)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    lg = logits.cpu().numpy()
    NC = (A + 1 + 127) // 128
    for a in range(N):
        rows = np.arange(E) * N + a
        x = oe.bf16_bits_to_f32(obs[rows, :D]).astype(np.float64)
        wb = op.bf16_weights(ws[a])
        lo, vo = op.mlp(x, wb)
        assert np.abs(lg[rows] - lo).max() <= 2e-2, a
        assert np.abs(g["val"][rows] - vo).max() <= 2e-2, a
        allowed = op.unpack_mask(mask[rows], A)
        lp = op.masked_log_softmax(lo, allowed)
        assert np.abs(g["logp"][rows] - lp[np.arange(E), g["act"][rows]]).max() <= 2e-2
        assert np.abs(g["ent"][rows] - op.entropy(lp)).max() <= 2e-2
        lp16 = op.masked_log_softmax(op.mlp(x, wb, bf16_hidden=True)[0], allowed)
        u1, u2 = oe.sample_uniforms(31, rows, 4, NC)  # keyed by the global row
        a_o, margin = op.sample_chunked(np.concatenate([lp16, np.full((E, NC * 128 - A), -np.inf)], 1), u1, u2)
        safe = margin > 1e-4
        assert safe.mean() > 0.9
        assert np.array_equal(g["act"][rows][safe], a_o[safe]), a


def test_one_group_equals_the_shared_call():
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 125, 1000
    w = _set_weights(D, H, A, 5)
    pol = binding.GroupedMlp(D, Ds, H, A, 1, [w])
    mlp = binding.Mlp(D, Ds, H, A, w)
    obs, mask = _t(W.synthetic_obs(M, D, Ds, seed=2).view(np.int16)), _t(W.synthetic_masks(M, A, seed=2).view(np.int32))
    outs = [[torch.zeros(M, dtype=torch.int32, device="cuda")] + [torch.zeros(M, device="cuda") for _ in range(3)]
            for _ in range(2)]
    pol.forward(obs, mask, M, 1, 3, 5, *outs[0])
    mlp.forward(obs, mask, M, 3, 5, *outs[1])
    torch.cuda.synchronize()
    for x, y in zip(*outs):
        assert torch.equal(x, y)


def test_strided_agent_backward_equals_gathered_and_matches_oracle():
    """Agent g's samples inside a rollout stored for every agent (batch
    row_stride = N, row_offset = g, its own weights) give exactly the gradient
    of the same samples gathered into their own storage, and that gradient
    matches the oracle element by element (1e-2 relative + 2^-7 B)."""
    import torch
    from paper_2410_22165_amd import binding
    from test_gpu_ppo import HP, assert_elementwise, kink_free_storage, reference_with_bounds
    D, Ds, H, A, N = 35, 40, 128, 125, 4
    w_all, st_all = [], []
    for g in range(N):
        w, st, _ = kink_free_storage(D, Ds, H, A, 800, seed=40 + g, hp=HP)
        assert len(st["act"]) >= 600
        w_all.append(w)
        st_all.append({k: v[:600] for k, v in st.items()})
    S = 600
    inter = {k: np.stack([st_all[g][k] for g in range(N)], axis=1).reshape(S * N, *st_all[0][k].shape[1:])
             for k in st_all[0]}
    pol = binding.GroupedMlp(D, Ds, H, A, N, w_all)
    dev = {k: _t(v.view(np.int16) if k == "obs" else (v.view(np.int32) if k == "mask" else v)) for k, v in inter.items()}
    rows = 400
    ws = torch.zeros(binding.ppo_workspace_bytes(pol._one, rows), dtype=torch.uint8, device="cuda")
    loss = torch.zeros(binding.PPO_LOSS_TERMS, device="cuda")
    a, c = W.affine_permutation(S, 1, seed=3)
    n = pol.layout["n_params"]
    for g in range(N):
        print(f"[gpu] strided backward agent {g}", flush=True)
        gs = torch.zeros(n, device="cuda")
        binding.ppo_backward(pol._one, dev, S, a, c, 50, rows, HP, ws, gs, loss, row_stride=N, row_offset=g,
                             params=pol.params_ptr(g), work=pol.work_ptr(g))
        mlp = binding.Mlp(D, Ds, H, A, w_all[g])
        own = {k: _t(v.view(np.int16) if k == "obs" else (v.view(np.int32) if k == "mask" else v))
               for k, v in st_all[g].items()}
        gg_ref = torch.zeros(n, device="cuda")
        binding.ppo_backward(mlp, own, S, a, c, 50, rows, HP, ws, gg_ref, loss)
        torch.cuda.synchronize()
        assert torch.equal(gs, gg_ref), g
        if g == N - 1:
            idx = (a * (50 + np.arange(rows)) + c) % S
            sub = {k: v[idx] for k, v in st_all[g].items()}
            _, _, g_o, B = reference_with_bounds(w_all[g], sub, D, HP)
            assert_elementwise(mlp.unflat(gs.cpu().numpy()), g_o, B, where=f"agent {g}")


@pytest.mark.parametrize("layout,R", [("ippo", 4), ("mappo", 4), ("ippo", 12), ("mappo", 12)])
def test_multi_agent_trainers(layout, R):
    """The variant economy with 4 resources (30 actions) and with 12 (86
    actions, 91-feature observations: the 128-column first layer): two
    updates of each layout; finite losses, every agent's policy moves away
    from the others' (independent sets), the shared value network moves
    (MAPPO)."""
    import torch
    from paper_2410_22165_amd.ppo import MultiAgentTrainer
    cfg = W.variant_config(R=R, N=6, E=16, X=6, T=30, seed=1)
    tr = MultiAgentTrainer(cfg, W.obs_scales(cfg), layout, hidden=64 if R <= 8 else 128, rollout=12, epochs=2,
                           minibatches=2, gamma=0.99,
                           lam=0.95, clip=0.2, vf_coef=0.25, vclip=10.0, ent_coef=0.01, lr=3e-3, seed=2,
                           total_updates=4)
    p0 = tr.pol.params.clone()
    v0 = tr.vnet.params.clone() if layout == "mappo" else None
    for _ in range(2):
        tr.collect()
        tr.update()
    torch.cuda.synchronize()
    assert np.isfinite(tr.loss_terms.cpu().numpy()).all()
    d = (tr.pol.params - p0).abs()
    for g in range(tr.N):
        assert d[g * tr.pol.ps:g * tr.pol.ps + tr.pol.layout["n_params"]].max() > 0, g
    if layout == "mappo":
        assert not torch.equal(v0, tr.vnet.params)
        assert np.isfinite(tr.vloss.cpu().numpy()).all()
    assert np.isfinite(tr.store.adv.cpu().numpy()).all()
    tr.close()
