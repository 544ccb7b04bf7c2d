"""GPU parity of the learner (C ABI): GAE, Adam, and the PPO minibatch
backward against the float64 oracle, element by element: the reference
autograd gradient and float64 finite differences at 1e-2 relative plus an
absolute floor derived from the kernel's bf16 roundings, on rows clear of
the loss's kinks (ReLU, surrogate clip, value clip)."""
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


def _forward_margins(w, st, D, hp, bf16_hidden):
    """Per-row distances of the oracle forward from every kink of the loss:
    the ReLU pre-activations (relative to the sum of |terms| that forms
    them), the surrogate clip thresholds 1 +- clip and the value clip
    thresholds (and, for a clipped value, the switch of the max)."""
    wb = op.bf16_weights(w)
    x = oe.bf16_bits_to_f32(st["obs"][:, :D]).astype(np.float64)
    z1 = x @ wb["W1"] + wb["b1"]
    s1 = np.abs(x) @ np.abs(wb["W1"]) + np.abs(wb["b1"])
    h1 = np.maximum(z1, 0.0)
    if bf16_hidden:
        h1 = op.bf16_round(h1.astype(np.float32)).astype(np.float64)
    z2 = h1 @ wb["W2"] + wb["b2"]
    s2 = h1 @ np.abs(wb["W2"]) + np.abs(wb["b2"])
    h2 = np.maximum(z2, 0.0)
    if bf16_hidden:
        h2 = op.bf16_round(h2.astype(np.float32)).astype(np.float64)
    out = h2 @ wb["W3"] + wb["b3"]
    A = out.shape[1] - 1
    lp = op.masked_log_softmax(out[:, :-1], op.unpack_mask(st["mask"], A))
    M = len(x)
    ratio = np.exp(lp[np.arange(M), st["act"]] - st["logp_old"].astype(np.float64))
    dv = out[:, -1] - st["val_old"].astype(np.float64)
    R = st["ret"].astype(np.float64)
    vc = st["val_old"] + np.clip(dv, -hp["vclip"], hp["vclip"])
    l1, l2 = (out[:, -1] - R) ** 2, (vc - R) ** 2
    return dict(relu1=np.min(np.abs(z1) / (s1 + 1e-30), axis=1), relu2=np.min(np.abs(z2) / (s2 + 1e-30), axis=1),
                pat1=z1 > 0, pat2=z2 > 0, ratio=ratio,
                clip=np.minimum(np.abs(ratio - (1 - hp["clip"])), np.abs(ratio - (1 + hp["clip"]))),
                vclip=np.abs(np.abs(dv) - hp["vclip"]),
                vmax=np.where(np.abs(dv) > hp["vclip"], np.abs(l1 - l2) / (l1 + l2 + 1e-30), np.inf))


def clear_of_kinks(w, st, D, hp, relu_margin=2.0 ** -13, clip_margin=1e-3, fd=False):
    """Rows whose loss is smooth around the oracle's forward in the kernel's
    precision (bf16 hidden activations): no ReLU pre-activation within
    relu_margin (relative) of 0, no ratio within clip_margin of 1 +- clip,
    no value difference within 1e-3 of the value clip, no clipped value whose
    two squared errors are within 1e-3 (relative) of each other.  fd=True
    also requires the float64 forward (no bf16 rounding) to take every
    decision the same way, so that central differences of the float64 loss
    see the function the kernel differentiates."""
    a = _forward_margins(w, st, D, hp, bf16_hidden=True)
    keep = (a["relu1"] > relu_margin) & (a["relu2"] > relu_margin) & (a["clip"] > clip_margin) & \
        (a["vclip"] > 1e-3) & (a["vmax"] > 1e-3)
    if fd:
        b = _forward_margins(w, st, D, hp, bf16_hidden=False)
        keep &= (b["relu1"] > relu_margin) & (b["relu2"] > relu_margin) & (b["clip"] > clip_margin) & \
            (b["vclip"] > 1e-3) & (b["vmax"] > 1e-3)
        keep &= (a["pat1"] == b["pat1"]).all(axis=1) & (a["pat2"] == b["pat2"]).all(axis=1)
        lo, hi = 1 - hp["clip"], 1 + hp["clip"]
        keep &= ((a["ratio"] < lo) == (b["ratio"] < lo)) & ((a["ratio"] > hi) == (b["ratio"] > hi))
    return keep, a


def kink_free_storage(D, Ds, H, A, M_gen, seed, hp, ratio_noise=0.3, fd=False, **kw):
    """make_storage restricted to the rows clear_of_kinks keeps."""
    w, st = make_storage(D, Ds, H, A, M_gen, seed, ratio_noise=ratio_noise)
    keep, a = clear_of_kinks(w, st, D, hp, fd=fd, **kw)
    st = {k: np.ascontiguousarray(v[keep]) for k, v in st.items()}
    ratio = a["ratio"][keep]
    return w, st, ratio


def gpu_backward(w, st, D, Ds, H, A, M, a, c, begin, rows, hp=HP):
    import torch
    from paper_2410_22165_amd import binding
    print(f"[gpu] ppo_backward D={D} H={H} A={A} M={M} rows={rows} hp={hp}", flush=True)
    mlp = binding.Mlp(D, Ds, H, A, w)
    dev = {k: _t(v.view(np.int16) if k == "obs" else (v.view(np.int32) if k == "mask" else v)) for k, v in st.items()}
    ws = torch.zeros(binding.ppo_workspace_bytes(mlp, rows), dtype=torch.uint8, device="cuda")
    grads = torch.zeros(mlp.layout["n_params"], device="cuda")
    loss = torch.zeros(binding.PPO_LOSS_TERMS, device="cuda")
    binding.ppo_backward(mlp, dev, M, a, c, begin, rows, hp, ws, grads, loss)
    torch.cuda.synchronize()
    return mlp, grads.cpu().numpy(), loss.cpu().numpy()


def rel_err(g, r):
    return np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)


def reference_with_bounds(w, sub, D, hp):
    """The float64 reference autograd (decisions in bf16 hidden precision)
    and, per gradient element, the sum of |terms| that the kernel's bf16
    roundings act on: B = |X|^T |Y| for each weight-gradient product, where
    |Y| propagates |dY| through |W3|^T and |W2|^T under the ReLU masks, and
    the column sums of |Y| for the biases.  Each bf16 rounding on the way
    (dY, dh2, dh1 and the back-propagated products) is relative 2^-9, so
    2^-7 B bounds their joint effect on an element."""
    x = oe.bf16_bits_to_f32(sub["obs"][:, :D]).astype(np.float64)
    cap = {}
    l_o, terms, g_o = op.ppo_grads(w, x, sub["mask"], sub["act"], sub["logp_old"], sub["val_old"], sub["adv"],
                                   sub["ret"], hp, bf16_hidden=True, capture=cap)
    wb = op.bf16_weights(w)
    dY = np.abs(cap["out"].grad.numpy())
    h1, h2 = cap["h1"].detach().numpy(), cap["h2"].detach().numpy()
    m1, m2 = cap["z1"].detach().numpy() > 0, cap["z2"].detach().numpy() > 0
    a2 = (dY @ np.abs(wb["W3"]).T) * m2
    a1 = (a2 @ np.abs(wb["W2"]).T) * m1
    B = dict(W3=np.abs(h2).T @ dY, b3=dY.sum(0), W2=np.abs(h1).T @ a2, b2=a2.sum(0), W1=np.abs(x).T @ a1,
             b1=a1.sum(0))
    return l_o, terms, g_o, B


def assert_elementwise(got, want, B, rtol=1e-2, floor=2.0 ** -7, where=""):
    """|got - want| <= rtol |want| + floor B for every element."""
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        g = np.asarray(got[k], np.float64)
        r = np.asarray(want[k], np.float64)
        tol = rtol * np.abs(r) + floor * B[k]
        bad = np.abs(g - r) > tol
        assert not bad.any(), (f"{where} {k}: {int(bad.sum())} of {bad.size} elements out of tolerance; first at "
                               f"{np.argwhere(bad)[:3].tolist()}: gpu {g[bad][:3]} ref {r[bad][:3]} tol {tol[bad][:3]}")


@pytest.mark.parametrize("case", [(35, 40, 256, 125, 3000, 1000, 10.0), (11, 16, 64, 9, 500, 77, 10.0),
                                  (49, 56, 512, 507, 1200, 300, 10.0), (64, 64, 128, 300, 700, 700, 10.0),
                                  (35, 40, 256, 125, 3000, 1000, 0.2), (49, 56, 512, 507, 1200, 300, 0.2),
                                  (91, 96, 256, 86, 2000, 700, 10.0), (122, 128, 256, 114, 2000, 700, 0.2),
                                  (35, 40, 256, 125, 8000, 120, 10.0)])
def test_ppo_backward_matches_reference_autograd(case):
    """Every gradient element against the float64 reference autograd at
    1e-2 relative plus the bf16 floor 2^-7 B (reference_with_bounds), on
    rows clear of every kink of the loss.  vclip 0.2 makes the value clip
    bind on most rows; ratio noise puts a share of rows outside the
    surrogate clip.  The advantage statistics take the streaming pass for
    minibatches of at least 1/32 of the batch and the per-row gather below
    (the last case).  The 122 -> 256 -> 256 -> 114 + 1 network is the
    16-resource variant's."""
    D, Ds, H, A, M_gen, rows, vclip = case
    hp = dict(HP, vclip=vclip)
    w, st, ratio = kink_free_storage(D, Ds, H, A, M_gen, seed=rows, hp=hp)
    M = len(st["act"])
    rows = min(rows, M - 17)
    if M_gen == 8000:
        assert rows * 32 < M, "this case exercises the gathered advantage statistics"
    a, c = W.affine_permutation(M, epoch=1, seed=rows)
    begin = 17 if rows < M else 0
    mlp, g, loss = gpu_backward(w, st, D, Ds, H, A, M, a, c, begin, rows, hp)
    idx = (a * (begin + np.arange(rows)) + c) % M
    sub = {k: v[idx] for k, v in st.items()}
    outside = np.abs(ratio[idx] - 1) > hp["clip"]
    assert outside.mean() > 0.05, "the surrogate clip must be active on some rows"
    l_o, terms, g_o, B = reference_with_bounds(w, sub, D, hp)
    if vclip < 1:
        dv = np.abs(op.mlp(oe.bf16_bits_to_f32(sub["obs"][:, :D]).astype(np.float64), op.bf16_weights(w),
                           bf16_hidden=True)[1] - sub["val_old"])
        assert (dv > vclip).mean() > 0.3, "the value clip must bind"
    gg = mlp.unflat(g)
    print("relative gradient errors", {k: rel_err(gg[k].astype(np.float64), g_o[k]) for k in g_o}, flush=True)
    assert_elementwise(gg, g_o, B, where=f"case {case}")
    assert abs(loss[0] - terms["pg"]) <= 1e-3 * max(1.0, abs(terms["pg"]))
    assert abs(loss[1] - terms["vf"]) <= 1e-3 * max(1.0, abs(terms["vf"]))
    assert abs(loss[2] - terms["ent"]) <= 1e-3 * max(1.0, abs(terms["ent"]))
    assert abs(loss[3] - outside.mean()) <= 1e-6
    assert abs(loss[4] - l_o) <= 1e-3 * max(1.0, abs(l_o))


def test_rows_without_allowed_actions_contribute_nothing():
    """Rows whose mask allows no action (policy and entropy undefined) add
    nothing to the loss terms or the gradients, whatever their observation,
    action, old log-probability, old value and return: two batches that differ
    only there give bit-identical, finite results.  Their advantages stay (the
    minibatch statistics count every row)."""
    D, Ds, H, A, M = 35, 40, 256, 125, 3000
    w, st = make_storage(D, Ds, H, A, M, seed=5)
    empty = np.random.default_rng(7).random(M) < 0.1
    st["mask"][empty] = 0
    other = make_storage(D, Ds, H, A, M, seed=6)[1]
    st2 = {k: v.copy() for k, v in st.items()}
    for k in ("obs", "act", "logp_old", "val_old", "ret"):
        st2[k][empty] = other[k][empty]
    a, c = W.affine_permutation(M, epoch=0, seed=3)
    rows = 1200
    idx = (a * np.arange(rows) + c) % M
    assert empty[idx].sum() > 50
    _, g1, l1 = gpu_backward(w, st, D, Ds, H, A, M, a, c, 0, rows)
    _, g2, l2 = gpu_backward(w, st2, D, Ds, H, A, M, a, c, 0, rows)
    assert np.isfinite(g1).all() and np.isfinite(l1).all()
    assert np.array_equal(g1, g2) and np.array_equal(l1, l2)


@pytest.mark.parametrize("A", [125, 507])
def test_peaked_policy_backward_is_finite(A):
    """Head weights scaled by 300 (logits over hundreds of units: every
    allowed weight but the largest underflows to 0 in fp32, in one chunk and
    across four): gradients and loss terms stay finite, and the surrogate,
    value and entropy terms equal the reference's (bf16 hidden activations,
    as in the kernel)."""
    D, Ds, H, M = 35, 40, 256, 3000
    w, st = make_storage(D, Ds, H, A, M, seed=8)
    w["W3"] = w["W3"].copy()
    w["W3"][:, :A] *= 300.0
    a, c = W.affine_permutation(M, epoch=0, seed=4)
    rows = 1500
    _, g, loss = gpu_backward(w, st, D, Ds, H, A, M, a, c, 0, rows)
    assert np.isfinite(g).all() and np.isfinite(loss).all()
    idx = (a * np.arange(rows) + c) % M
    sub = {k: v[idx] for k, v in st.items()}
    x = oe.bf16_bits_to_f32(sub["obs"][:, :D]).astype(np.float64)
    _, terms, _ = op.ppo_grads(w, x, sub["mask"], sub["act"], sub["logp_old"], sub["val_old"], sub["adv"],
                               sub["ret"], HP, bf16_hidden=True)
    print("loss terms", loss[:3], terms["pg"], terms["vf"], terms["ent"], flush=True)
    assert abs(loss[0] - terms["pg"]) <= 1e-3 * max(1.0, abs(terms["pg"]))
    assert abs(loss[1] - terms["vf"]) <= 1e-3 * max(1.0, abs(terms["vf"]))
    assert abs(loss[2] - terms["ent"]) <= 1e-3


@pytest.mark.parametrize("case", [(35, 40, 256, 125, 64000, 40000), (35, 40, 64, 125, 330000, 300000)])
def test_ppo_backward_many_mblocks_per_split(case):
    """Minibatches large enough that every weight-gradient split accumulates
    several 32-row m-blocks (40 000 rows: about five per split; 300 000
    rows at hidden 64: about 37) and the advantage statistics loop over more
    rows than the grid has threads (more than 262 144).  Every element
    against the reference autograd, as above."""
    D, Ds, H, A, M_gen, rows = case
    w, st, _ = kink_free_storage(D, Ds, H, A, M_gen, seed=H, hp=HP)
    M = len(st["act"])
    assert M >= rows
    a, c = W.affine_permutation(M, epoch=2, seed=H)
    mlp, g, loss = gpu_backward(w, st, D, Ds, H, A, M, a, c, 0, rows)
    idx = (a * np.arange(rows) + c) % M
    sub = {k: v[idx] for k, v in st.items()}
    l_o, terms, g_o, B = reference_with_bounds(w, sub, D, HP)
    gg = mlp.unflat(g)
    assert_elementwise(gg, g_o, B, where=f"case {case}")
    assert abs(loss[4] - l_o) <= 1e-3 * max(1.0, abs(l_o))


def _fd_check(D, Ds, H, A, M_gen, seed, n_pick=8, h=1e-5):
    """GPU gradient entries against float64 central differences of the
    oracle loss (no bf16 rounding), element by element: |g - fd| <= 1e-2 |fd|
    + 2^-5 B.  The rows are those on which the float64 and the bf16-hidden
    forwards take every ReLU and clip decision the same way, with margins
    far wider than the perturbation; ratio noise leaves a share of them
    clipped.  Half the entries are among the largest of each tensor, half
    drawn uniformly."""
    import torch
    w, st, ratio = kink_free_storage(D, Ds, H, A, M_gen, seed=seed, hp=HP, fd=True)
    M = len(st["act"])
    assert (np.abs(ratio - 1) > HP["clip"]).mean() > 0.05, "some rows must be clipped"
    mlp, g, _ = gpu_backward(w, st, D, Ds, H, A, M, 1, 0, 0, M)
    gg = mlp.unflat(g)
    _, _, _, B = reference_with_bounds(w, st, D, HP)
    wb = op.bf16_weights(w)
    x = oe.bf16_bits_to_f32(st["obs"][:, :D]).astype(np.float64)
    allowed = op.unpack_mask(st["mask"], A)

    def f(params):
        p = {k: torch.tensor(v, dtype=torch.float64) for k, v in params.items()}
        return float(op.ppo_loss_torch(p, x, allowed, st["act"], st["logp_old"], st["val_old"], st["adv"],
                                       st["ret"], HP)[0])

    rng = np.random.default_rng(seed)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = np.abs(gg[k]).ravel()
        picks = list(rng.choice(np.argsort(-flat)[:40], size=n_pick // 2, replace=False))
        picks += list(rng.choice(flat.size, size=n_pick - n_pick // 2, replace=False))
        for pos in picks:
            idx = np.unravel_index(pos, gg[k].shape)
            pp = {kk: vv.copy() for kk, vv in wb.items()}
            pm = {kk: vv.copy() for kk, vv in wb.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (f(pp) - f(pm)) / (2 * h)
            got = float(gg[k][idx])
            tol = 1e-2 * abs(fd) + 2.0 ** -5 * float(B[k][idx])
            assert abs(got - fd) <= tol, (k, idx, got, fd, tol)


def test_ppo_backward_finite_differences_one_economy_slice():
    """The 35 -> 256 -> 256 -> 125 + 1 network on one economy's worth of
    rows (100-agent economies; 200 generated, the kink-free ones kept)."""
    _fd_check(35, 40, 256, 125, 200, seed=11)


def test_ppo_backward_finite_differences_large_action_space():
    """The 49 -> 512 -> 512 -> 507 + 1 network of the 1000-agent, 5-resource,
    50-price workload, on one minibatch of one economy's rows (1000-agent
    economies; 2000 generated, the kink-free ones kept)."""
    _fd_check(49, 56, 512, 507, 2000, seed=12, n_pick=6)


def test_ppo_backward_finite_differences_wide_rows():
    """The 91 -> 256 -> 256 -> 86 + 1 network of the 12-resource multi-agent
    economy (a 128-column first layer)."""
    _fd_check(91, 96, 256, 86, 300, seed=13)


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
    loss = torch.zeros(binding.PPO_LOSS_TERMS, device="cuda")
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


@pytest.mark.parametrize("case", [(35, 40, 256, 125, 30000, 1, 0), (35, 40, 256, 125, 24000, 3, 2),
                                  (91, 96, 256, 86, 5000, 1, 0), (49, 56, 512, 507, 3000, 1, 0)])
def test_ppo_records_equal_arrays(case):
    """ej_ppo_pack writes each sample's observation row, mask words and five
    scalars into one record (checked byte by byte against the arrays), and
    the backward that gathers the records gives the gradient and loss of the
    one that gathers the arrays, bit for bit: ragged minibatches, several
    m-blocks per weight-gradient split, a strided (per-agent) batch, the
    wide-row and 507-action networks."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M_gen, stride, offset = case
    print(f"[gpu] records D={D} H={H} A={A} M={M_gen} stride={stride}", flush=True)
    w, st = make_storage(D, Ds, H, A, M_gen, seed=21)
    mlp = binding.Mlp(D, Ds, H, A, w)
    dev = {k: _t(v.view(np.int16) if k == "obs" else (v.view(np.int32) if k == "mask" else v)) for k, v in st.items()}
    M = (M_gen - 1 - offset) // stride + 1
    rb = binding.ppo_record_bytes(mlp)
    Wm = (A + 31) // 32
    rmask = (2 * Ds + 15) // 16 * 16
    rsc = rmask + 4 * Wm
    assert rb % 128 == 0 and rb >= rsc + 20
    rec = torch.full((M * rb,), 0xAB, dtype=torch.uint8, device="cuda")
    binding.ppo_pack(mlp, dev, M, rec, row_stride=stride, row_offset=offset)
    torch.cuda.synchronize()
    R = rec.view(M, rb).cpu().numpy()
    idx = np.arange(M) * stride + offset
    assert np.array_equal(R[:, :2 * Ds], st["obs"][idx].view(np.uint8).reshape(M, -1))
    assert not R[:, 2 * Ds:rmask].any() and not R[:, rsc + 20:].any()
    assert np.array_equal(R[:, rmask:rsc], st["mask"][idx].view(np.uint8).reshape(M, -1))
    for k, name in enumerate(("act", "logp_old", "val_old", "adv", "ret")):
        assert np.array_equal(R[:, rsc + 4 * k:rsc + 4 * k + 4], st[name][idx].view(np.uint8).reshape(M, 4)), name
    rows_all = [(0, M // 3), (M // 3, M - M // 3 - 5)]
    for epoch, (begin, rows) in enumerate(rows_all):
        a, c = W.affine_permutation(M, epoch, seed=5)
        out = []
        for r in (None, rec):
            ws = torch.zeros(binding.ppo_workspace_bytes(mlp, rows), dtype=torch.uint8, device="cuda")
            grads = torch.zeros(mlp.layout["n_params"], device="cuda")
            loss = torch.zeros(binding.PPO_LOSS_TERMS, device="cuda")
            binding.ppo_backward(mlp, dev, M, a, c, begin, rows, HP, ws, grads, loss, row_stride=stride,
                                 row_offset=offset, records=r)
            torch.cuda.synchronize()
            out.append((grads.cpu(), loss.cpu()))
        assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1]), (case, begin, rows)
