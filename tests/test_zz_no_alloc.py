"""The allocation-free PPO backward (ej_ppo_backward_static, workspace in the
library's static device array) against ej_ppo_backward with a caller
workspace: identical gradients and loss terms on two calls in a row, the
second with a smaller minibatch, and a clean rejection of a minibatch whose
workspace would not fit."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HP = dict(clip=0.2, vclip=0.5, vf_coef=0.25, ent_coef=0.1)


def _storage(D, Ds, A, M, seed):
    import torch
    rng = np.random.default_rng(seed)
    obs = W.synthetic_obs(M, D, Ds, seed=seed)
    mask = W.synthetic_masks(M, A, seed=seed)
    act = np.array([rng.choice(np.flatnonzero((mask[m, np.arange(A) // 32] >> (np.arange(A) % 32)) & 1))
                    for m in range(M)], np.int32)
    host = dict(obs=obs.view(np.int16), mask=mask.view(np.int32), act=act,
                logp_old=(-np.log(A / 2) + rng.normal(size=M) * 0.3).astype(np.float32),
                val_old=rng.normal(size=M).astype(np.float32), adv=rng.normal(size=M).astype(np.float32),
                ret=rng.normal(size=M).astype(np.float32))
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for k, v in host.items()}


def test_static_scratch_backward_equals_workspace_backward():
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 125, 2000
    mlp = binding.Mlp(D, Ds, H, A, W.policy_weights(D, H, A, seed=7))
    st = _storage(D, Ds, A, M, seed=7)
    n = mlp.layout["n_params"]
    for call, (rows, begin) in enumerate([(1500, 0), (333, 1100)]):
        print(f"[gpu] ppo_backward_static call {call} rows={rows}", flush=True)
        a, c = W.affine_permutation(M, epoch=call, seed=7)
        ws = torch.zeros(binding.ppo_workspace_bytes(mlp, rows), dtype=torch.uint8, device="cuda")
        g_ref = torch.zeros(n, device="cuda")
        l_ref = torch.zeros(binding.PPO_LOSS_TERMS, device="cuda")
        binding.ppo_backward(mlp, st, M, a, c, begin, rows, HP, ws, g_ref, l_ref)
        g = torch.full((n,), 3.0, device="cuda")
        loss = torch.full((binding.PPO_LOSS_TERMS,), 3.0, device="cuda")
        binding.ppo_backward_static(mlp, st, M, a, c, begin, rows, HP, g, loss)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), call
        assert torch.equal(loss, l_ref), call
        assert torch.isfinite(g).all() and g.abs().max() > 0


def test_static_scratch_rejects_a_minibatch_that_does_not_fit():
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 125, 256
    mlp = binding.Mlp(D, Ds, H, A, W.policy_weights(D, H, A, seed=8))
    rows = 100000
    assert binding.ppo_workspace_bytes(mlp, rows) > binding.PPO_STATIC_SCRATCH_BYTES
    st = _storage(D, Ds, A, M, seed=8)
    g = torch.full((mlp.layout["n_params"],), 3.0, device="cuda")
    loss = torch.zeros(binding.PPO_LOSS_TERMS, device="cuda")
    b = binding.EjPpoBatch(*(binding.ptr(st[k]) for k in ("obs", "mask", "act", "logp_old", "val_old", "adv",
                                                           "ret")), M, 1, 0, 0, rows)
    h = binding.EjPpoHparams(HP["clip"], HP["vclip"], HP["vf_coef"], HP["ent_coef"])
    rc = binding.lib().ej_ppo_backward_static(C.byref(mlp.desc), binding.ptr(mlp.params), binding.ptr(mlp.work),
                                              C.byref(b), C.byref(h), binding.ptr(g), binding.ptr(loss), None)
    assert rc == binding.EJ_ESCRATCH
    assert binding.lib().ej_strerror(rc).startswith(b"request larger")
    torch.cuda.synchronize()
    assert (g.cpu() == 3.0).all()
