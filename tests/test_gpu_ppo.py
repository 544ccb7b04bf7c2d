"""GPU parity of the learner (C ABI): GAE, Adam, and the PPO minibatch
backward against the float64 oracle (reference autograd gradient and float64
finite differences), 1e-2 relative."""
import numpy as np
import pytest

import workloads as W
from oracle import env as oe
from oracle import policy as op

pytestmark = pytest.mark.gpu

HP = dict(clip=0.2, vclip=10.0, vf_coef=0.25, ent_coef=0.1)


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda") if dtype is None else t.to("cuda", dtype)


def test_gae_parity():
    from paper_2410_22165_amd import binding
    rng = np.random.default_rng(0)
    T, M = 37, 1000
    rew = rng.normal(size=(T, M)).astype(np.float32)
    val = rng.normal(size=(T, M)).astype(np.float32)
    done = (rng.random((T, M)) < 0.05).astype(np.uint8)
    last = rng.normal(size=M).astype(np.float32)
    import torch
    adv = torch.zeros((T, M), device="cuda")
    ret = torch.zeros((T, M), device="cuda")
    binding.gae(_t(rew), _t(val), _t(done), _t(last), T, M, 0.99, 0.95, adv, ret)
    a_o, r_o = op.gae(rew, val, done, last, 0.99, 0.95)
    assert np.allclose(adv.cpu().numpy(), a_o, rtol=1e-4, atol=1e-4)
    assert np.allclose(ret.cpu().numpy(), r_o, rtol=1e-4, atol=1e-4)


def test_adam_parity():
    import torch
    from paper_2410_22165_amd import binding
    rng = np.random.default_rng(1)
    n = 10007
    w0 = rng.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    pw = _t(w0.astype(np.float32))
    pm, pv = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    w = w0.astype(np.float32).astype(np.float64)
    for step in range(1, 6):
        g = rng.normal(size=n) * 0.1
        binding.adam(pw, _t(g.astype(np.float32)), pm, pv, step, 5e-4)
        w, m, v = op.adam_step(w, g.astype(np.float32).astype(np.float64), m, v, step, 5e-4)
    assert np.allclose(pw.cpu().numpy(), w, rtol=1e-5, atol=1e-7)


def make_storage(D, Ds, H, A, M, seed, ratio_noise=0.3):
    """A synthetic rollout store with logp_old near the current policy (so
    that some ratios leave the clip range; ratio_noise = 0 puts every ratio
    at 1, far from the clip thresholds)."""
    rng = np.random.default_rng(seed)
    w = W.policy_weights(D, H, A, seed=seed)
    for k in ("b1", "b2", "b3"):
        w[k] = (rng.standard_normal(w[k].shape) * 0.1).astype(np.float32)
    obs = W.synthetic_obs(M, D, Ds, seed=seed)
    mask = W.synthetic_masks(M, A, seed=seed)
    x = oe.bf16_bits_to_f32(obs[:, :D]).astype(np.float64)
    logits, value = op.mlp(x, op.bf16_weights(w))
    allowed = op.unpack_mask(mask, A)
    lp = op.masked_log_softmax(logits, allowed)
    act = np.array([rng.choice(np.flatnonzero(allowed[m])) for m in range(M)], np.int32)
    logp_old = (lp[np.arange(M), act] + rng.normal(size=M) * ratio_noise).astype(np.float32)
    val_old = (value + rng.normal(size=M) * 0.5).astype(np.float32)
    adv = rng.normal(size=M).astype(np.float32)
    ret = (value + rng.normal(size=M)).astype(np.float32)
    return w, dict(obs=obs, mask=mask, act=act, logp_old=logp_old, val_old=val_old, adv=adv, ret=ret)


def gpu_backward(w, st, D, Ds, H, A, M, a, c, begin, rows, hp=HP):
    import torch
    from paper_2410_22165_amd import binding
    print(f"[gpu] ppo_backward D={D} H={H} A={A} M={M} rows={rows}", flush=True)
    mlp = binding.Mlp(D, Ds, H, A, w)
    dev = {k: _t(v.view(np.int16) if k == "obs" else (v.view(np.int32) if k == "mask" else v)) for k, v in st.items()}
    ws = torch.zeros(binding.ppo_workspace_bytes(mlp, rows), dtype=torch.uint8, device="cuda")
    grads = torch.zeros(mlp.layout["n_params"], device="cuda")
    loss = torch.zeros(4, device="cuda")
    binding.ppo_backward(mlp, dev, M, a, c, begin, rows, hp, ws, grads, loss)
    torch.cuda.synchronize()
    return mlp, grads.cpu().numpy(), loss.cpu().numpy()


def rel_err(g, r):
    return np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)


@pytest.mark.parametrize("case", [(35, 40, 256, 125, 3000, 1000), (11, 16, 64, 9, 500, 77),
                                  (49, 56, 512, 507, 1200, 300), (64, 64, 128, 300, 700, 700)])
def test_ppo_backward_matches_reference_autograd(case):
    D, Ds, H, A, M, rows = case
    w, st = make_storage(D, Ds, H, A, M, seed=rows)
    a, c = W.affine_permutation(M, epoch=1, seed=rows)
    begin = 17 if rows < M else 0
    mlp, g, loss = gpu_backward(w, st, D, Ds, H, A, M, a, c, begin, rows)
    idx = (a * (begin + np.arange(rows)) + c) % M
    sub = {k: v[idx] for k, v in st.items()}
    x = oe.bf16_bits_to_f32(sub["obs"][:, :D]).astype(np.float64)
    # the clip decisions of every row are taken in the kernel's precision (bf16 hidden activations)
    l_o, terms, g_o = op.ppo_grads(w, x, sub["mask"], sub["act"], sub["logp_old"], sub["val_old"], sub["adv"],
                                   sub["ret"], HP, bf16_hidden=True)
    gg = mlp.unflat(g)
    errs = {k: rel_err(gg[k].astype(np.float64), g_o[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3")}
    print("relative gradient errors", errs, flush=True)
    for k, e in errs.items():
        assert e <= 1e-2, (k, e)
    assert abs(loss[0] - terms["pg"]) <= 1e-2 * max(1.0, abs(terms["pg"]))
    assert abs(loss[1] - terms["vf"]) <= 1e-2 * max(1.0, abs(terms["vf"]))
    assert abs(loss[2] - terms["ent"]) <= 1e-2 * max(1.0, abs(terms["ent"]))


def test_ppo_backward_finite_differences_one_economy_slice():
    """100 rows (one economy of the 100-agent workload): GPU gradient entries
    against float64 central differences of the oracle loss."""
    import torch
    D, Ds, H, A, M = 35, 40, 256, 125, 100
    # ratios at 1: no row sits near a clip threshold, so the float64 loss is
    # smooth around the weights and central differences are meaningful
    w, st = make_storage(D, Ds, H, A, M, seed=11, ratio_noise=0.0)
    mlp, g, _ = gpu_backward(w, st, D, Ds, H, A, M, 1, 0, 0, M)
    gg = mlp.unflat(g)
    wb = op.bf16_weights(w)
    x = oe.bf16_bits_to_f32(st["obs"][:, :D]).astype(np.float64)
    allowed = op.unpack_mask(st["mask"], A)

    def f(params):
        p = {k: torch.tensor(v, dtype=torch.float64) for k, v in params.items()}
        return float(op.ppo_loss_torch(p, x, allowed, st["act"], st["logp_old"], st["val_old"], st["adv"],
                                       st["ret"], HP)[0])

    rng = np.random.default_rng(3)
    h = 1e-5
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = np.abs(gg[k]).ravel()
        order = np.argsort(-flat)[:40]
        got, want = [], []
        for pos in rng.choice(order, size=6, replace=False):
            idx = np.unravel_index(pos, gg[k].shape)
            pp = {kk: vv.copy() for kk, vv in wb.items()}
            pm = {kk: vv.copy() for kk, vv in wb.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            want.append((f(pp) - f(pm)) / (2 * h))
            got.append(float(gg[k][idx]))
        got, want = np.array(got), np.array(want)
        assert np.linalg.norm(got - want) <= 1e-2 * np.linalg.norm(want), (k, got, want)


def test_ppo_backward_deterministic():
    D, Ds, H, A, M = 35, 40, 256, 125, 2000
    w, st = make_storage(D, Ds, H, A, M, seed=5)
    a, c = W.affine_permutation(M, 0, seed=5)
    _, g1, l1 = gpu_backward(w, st, D, Ds, H, A, M, a, c, 0, 1500)
    _, g2, l2 = gpu_backward(w, st, D, Ds, H, A, M, a, c, 0, 1500)
    assert np.array_equal(g1, g2) and np.array_equal(l1, l2)


def test_ppo_backward_rejects_misaligned_arrays():
    """A gradient, workspace or observation array that is not 16-byte aligned
    returns EJ_EINVAL before anything is launched."""
    import ctypes as C
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 125, 256
    w, st = make_storage(D, Ds, H, A, M, seed=3)
    a, c = W.affine_permutation(M, 0, seed=3)
    mlp = binding.Mlp(D, Ds, H, A, w)
    dev = {k: _t(v.view(np.int16) if k == "obs" else (v.view(np.int32) if k == "mask" else v)) for k, v in st.items()}
    nbytes = binding.ppo_workspace_bytes(mlp, M)
    ws = torch.zeros(nbytes + 16, dtype=torch.uint8, device="cuda")
    grads = torch.full((mlp.layout["n_params"] + 4,), 7.0, device="cuda")
    loss = torch.zeros(4, device="cuda")
    h = binding.EjPpoHparams(HP["clip"], HP["vclip"], HP["vf_coef"], HP["ent_coef"])
    L = binding.lib()
    P = lambda t, off=0: C.c_void_p(t.data_ptr() + off)

    def call(obs_off=0, ws_off=0, g_off=0):
        b = binding.EjPpoBatch(P(dev["obs"], obs_off), *(P(dev[k]) for k in ("mask", "act", "logp_old", "val_old",
                                                                              "adv", "ret")), M, a, c, 0, M)
        return L.ej_ppo_backward(C.byref(mlp.desc), P(mlp.params), P(mlp.work), C.byref(b), C.byref(h),
                                 P(ws, ws_off), nbytes, P(grads, g_off), P(loss), None)

    assert call(g_off=4) == -1
    assert call(ws_off=8) == -1
    assert call(obs_off=8) == -1
    torch.cuda.synchronize()
    assert (grads.cpu() == 7.0).all()
