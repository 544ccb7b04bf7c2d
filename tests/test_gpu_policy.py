"""GPU parity of the policy forward (C ABI) against the oracle network.

Logits and values within 2e-2 absolute of the float64 oracle (bf16 weights);
sampled actions identical to the oracle's sampler where the decision is not
within rounding distance of a threshold (the oracle then takes it in the
kernel's precision: bf16 hidden activations); masked actions never drawn;
the sampler's distribution matches the softmax (chi-square)."""
import numpy as np
import pytest

import workloads as W
from oracle import env as oe
from oracle import policy as op

pytestmark = pytest.mark.gpu

CASES = [  # (D, Ds, H, A, M)
    (11, 16, 64, 9, 300),
    (35, 40, 256, 125, 1000),      # shape of the 1024 x 100 economy's policy
    (49, 56, 512, 507, 333),       # 1000-agent economy: 5 resources, 50 prices
    (64, 64, 128, 300, 129),
    (35, 40, 256, 125, 1),
    (64, 64, 256, 1000, 200),      # 64 features and 8 action chunks
    (91, 96, 256, 86, 500),        # 12-resource multi-agent economy: a 128-column first layer
    (128, 128, 512, 300, 129),     # widest input (128 features)
    (122, 128, 256, 114, 300),     # 16-resource multi-agent economy (the largest resource count)
]


def run_forward(D, Ds, H, A, M, seed=0, with_logits=True):
    import torch
    from paper_2410_22165_amd import binding
    print(f"[gpu] policy D={D} H={H} A={A} M={M}", flush=True)
    w = W.policy_weights(D, H, A, seed=seed)
    rng = np.random.default_rng(seed)
    for k in ("b1", "b2", "b3"):
        w[k] = (rng.standard_normal(w[k].shape) * 0.1).astype(np.float32)
    mlp = binding.Mlp(D, Ds, H, A, w)
    obs = W.synthetic_obs(M, D, Ds, seed=seed)
    mask = W.synthetic_masks(M, A, seed=seed)
    dev = "cuda"
    t_obs = torch.from_numpy(obs.view(np.int16)).to(dev)
    t_mask = torch.from_numpy(mask.view(np.int32)).to(dev)
    out = dict(act=torch.zeros(M, dtype=torch.int32, device=dev), logp=torch.zeros(M, device=dev),
               val=torch.zeros(M, device=dev), ent=torch.zeros(M, device=dev),
               logits=torch.zeros((M, A), device=dev) if with_logits else None)
    mlp.forward(t_obs, t_mask, M, 1234, 7, out["act"], out["logp"], out["val"], out["ent"], out["logits"])
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    return w, obs, mask, res


@pytest.mark.parametrize("case", CASES)
def test_policy_forward_parity(case):
    D, Ds, H, A, M = case
    w, obs, mask, g = run_forward(D, Ds, H, A, M)
    x = oe.bf16_bits_to_f32(obs[:, :D]).astype(np.float64)
    wb = op.bf16_weights(w)
    logits, value = op.mlp(x, wb)
    allowed = op.unpack_mask(mask, A)
    # logits and values: 2e-2 absolute against the float64 network
    assert np.abs(g["logits"] - logits).max() <= 2e-2, np.abs(g["logits"] - logits).max()
    assert np.abs(g["val"] - value).max() <= 2e-2
    lp = op.masked_log_softmax(logits, allowed)
    ent = op.entropy(lp)
    assert np.abs(g["ent"] - ent).max() <= 2e-2
    # every sampled action is allowed, and its log-probability is consistent
    assert allowed[np.arange(M), g["act"]].all()
    assert np.abs(g["logp"] - lp[np.arange(M), g["act"]]).max() <= 2e-2
    # decisions: the oracle samples from bf16-hidden logits with the same uniforms
    l16, _ = op.mlp(x, wb, bf16_hidden=True)
    lp16 = op.masked_log_softmax(l16, allowed)
    NC = (A + 1 + 127) // 128
    u1, u2 = oe.sample_uniforms(1234, np.arange(M), 7, NC)
    pad = NC * 128 - A
    lp16p = np.concatenate([lp16, np.full((M, pad), -np.inf)], axis=1)
    a_o, margin = op.sample_chunked(lp16p, u1, u2)
    safe = margin > 1e-4
    assert safe.mean() > 0.97, safe.mean()  # about 1 - 2e-4 per near-threshold candidate
    assert np.array_equal(g["act"][safe], a_o[safe]), np.flatnonzero(g["act"][safe] != a_o[safe])[:10]


def test_sampler_distribution_chi_square():
    """Many rows with the same observation: the empirical action histogram
    matches the softmax of the oracle logits."""
    import scipy.stats
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 125, 200000
    w = W.policy_weights(D, H, A, seed=3)
    w["W3"] *= 3.0  # a peaked, non-uniform distribution
    mlp = binding.Mlp(D, Ds, H, A, w)
    obs1 = W.synthetic_obs(1, D, Ds, seed=3)
    mask1 = W.synthetic_masks(1, A, seed=3, p_allow=0.3)
    obs = np.repeat(obs1, M, axis=0)
    mask = np.repeat(mask1, M, axis=0)
    dev = "cuda"
    act = torch.zeros(M, dtype=torch.int32, device=dev)
    f = [torch.zeros(M, device=dev) for _ in range(3)]
    mlp.forward(torch.from_numpy(obs.view(np.int16)).to(dev), torch.from_numpy(mask.view(np.int32)).to(dev), M, 99, 0,
                act, *f)
    counts = np.bincount(act.cpu().numpy(), minlength=A)
    allowed = op.unpack_mask(mask1, A)[0]
    assert counts[~allowed].sum() == 0
    x = oe.bf16_bits_to_f32(obs1[:, :D]).astype(np.float64)
    logits, _ = op.mlp(x, op.bf16_weights(w), bf16_hidden=True)
    p = np.exp(op.masked_log_softmax(logits, allowed[None])[0])
    exp_c = p[allowed] * M
    keep = exp_c > 5
    chi = scipy.stats.chisquare(counts[allowed][keep], exp_c[keep] * counts[allowed][keep].sum() / exp_c[keep].sum())
    assert chi.pvalue > 1e-4, chi


def test_sampler_multi_chunk_distribution():
    """507 actions (4 chunks of 128): the chunk reservoir draws each chunk
    with its total probability."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 49, 56, 512, 507, 100000
    w = W.policy_weights(D, H, A, seed=4)
    mlp = binding.Mlp(D, Ds, H, A, w)
    obs1 = W.synthetic_obs(1, D, Ds, seed=4)
    mask1 = W.synthetic_masks(1, A, seed=4, p_allow=0.5)
    dev = "cuda"
    act = torch.zeros(M, dtype=torch.int32, device=dev)
    f = [torch.zeros(M, device=dev) for _ in range(3)]
    mlp.forward(torch.from_numpy(np.repeat(obs1, M, 0).view(np.int16)).to(dev),
                torch.from_numpy(np.repeat(mask1, M, 0).view(np.int32)).to(dev), M, 5, 0, act, *f)
    a = act.cpu().numpy()
    x = oe.bf16_bits_to_f32(obs1[:, :D]).astype(np.float64)
    logits, _ = op.mlp(x, op.bf16_weights(w), bf16_hidden=True)
    allowed = op.unpack_mask(mask1, A)[0]
    p = np.exp(op.masked_log_softmax(logits, allowed[None])[0])
    for c in range(4):
        frac = ((a >= 128 * c) & (a < 128 * (c + 1))).mean()
        pc = p[128 * c:128 * (c + 1)].sum()
        assert abs(frac - pc) < 5 * np.sqrt(pc * (1 - pc) / M) + 1e-3, (c, frac, pc)


def test_row_tile_variants_are_bit_identical():
    """64-row and 128-row tiles compute every row with the same k order:
    actions, log-probabilities, values and entropies agree bit for bit."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 125, 777
    w = W.policy_weights(D, H, A, seed=8)
    outs = []
    for rows in (128, 64):
        mlp = binding.Mlp(D, Ds, H, A, w, tile_rows=rows)
        o = [torch.zeros(M, dtype=torch.int32, device="cuda")] + [torch.zeros(M, device="cuda") for _ in range(3)]
        mlp.forward(torch.from_numpy(W.synthetic_obs(M, D, Ds, 8).view(np.int16)).cuda(),
                    torch.from_numpy(W.synthetic_masks(M, A, 8).view(np.int32)).cuda(), M, 3, 4, *o)
        outs.append([t.cpu() for t in o])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_empty_batch_is_a_no_op():
    """M = 0 rows: the call succeeds and writes nothing."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A = 35, 40, 256, 125
    mlp = binding.Mlp(D, Ds, H, A, W.policy_weights(D, H, A, seed=1))
    o = [torch.full((4,), 7, dtype=torch.int32, device="cuda")] + [torch.full((4,), 7.0, device="cuda") for _ in range(3)]
    obs = torch.zeros((4, Ds), dtype=torch.int16, device="cuda")
    mask = torch.zeros((4, 4), dtype=torch.int32, device="cuda")
    mlp.forward(obs, mask, 0, 1, 0, *o)
    torch.cuda.synchronize()
    assert all((t.cpu() == 7).all() for t in o)


def test_row_slices_with_row_base_equal_one_call():
    """Three slices drawn separately (row_base = first row) give bit for bit
    the results of one call over the whole batch."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 125, 700
    mlp = binding.Mlp(D, Ds, H, A, W.policy_weights(D, H, A, seed=2))
    obs = torch.from_numpy(W.synthetic_obs(M, D, Ds, 2).view(np.int16)).cuda()
    mask = torch.from_numpy(W.synthetic_masks(M, A, 2).view(np.int32)).cuda()
    full = [torch.zeros(M, dtype=torch.int32, device="cuda")] + [torch.zeros(M, device="cuda") for _ in range(3)]
    part = [torch.zeros_like(t) for t in full]
    mlp.forward(obs, mask, M, 11, 3, *full)
    for r0, r1 in ((0, 129), (129, 500), (500, 700)):
        mlp.forward(obs[r0:r1], mask[r0:r1], r1 - r0, 11, 3, *[t[r0:r1] for t in part], row_base=r0)
    torch.cuda.synchronize()
    for a, b in zip(full, part):
        assert torch.equal(a, b)


def test_misaligned_parameters_are_rejected():
    """A parameter or observation pointer that is not 16-byte aligned returns
    EJ_EINVAL before anything is launched; the outputs stay untouched."""
    import ctypes as C
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A = 35, 40, 256, 125
    mlp = binding.Mlp(D, Ds, H, A, W.policy_weights(D, H, A, seed=1))
    M = 64
    obs = torch.zeros((M + 1, Ds), dtype=torch.int16, device="cuda")
    mask = torch.full((M, 4), -1, dtype=torch.int32, device="cuda")
    o = [torch.full((M,), 7, dtype=torch.int32, device="cuda")] + [torch.full((M,), 7.0, device="cuda") for _ in range(3)]
    L = binding.lib()
    P = lambda t, off=0: C.c_void_p(t.data_ptr() + off)
    outs = [P(t) for t in o]
    rc = L.ej_policy_forward(C.byref(mlp.desc), P(mlp.params, 4), P(mlp.work), P(obs), P(mask), M, 0, 1, 0, None,
                             *outs, None, None)
    assert rc == -1
    rc = L.ej_policy_forward(C.byref(mlp.desc), P(mlp.params), P(mlp.work), P(obs, 8), P(mask), M, 0, 1, 0, None,
                             *outs, None, None)
    assert rc == -1
    torch.cuda.synchronize()
    assert all((t.cpu() == 7).all() for t in o)


def test_sparse_masks_single_actions_and_empty_chunks():
    """Masks that leave a single action (at either end of the action space or
    at a 128-action chunk edge), or that empty whole chunks: a single allowed
    action is always drawn with log-probability 0 and entropy 0; otherwise the
    draw, its log-probability and the entropy agree with the oracle."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, A, M = 35, 40, 256, 300, 384  # three chunks, the last one partial
    w = W.policy_weights(D, H, A, seed=9)
    mlp = binding.Mlp(D, Ds, H, A, w)
    obs = W.synthetic_obs(M, D, Ds, seed=9)
    rng = np.random.default_rng(9)
    allowed = np.zeros((M, A), bool)
    singles = [0, A - 1, 127, 128, 255, 256]
    for i in range(M):
        kind = i % 4
        if kind == 0:  # exactly one action
            allowed[i, singles[(i // 4) % len(singles)]] = True
        elif kind == 1:  # only the first chunk
            allowed[i, :128] = rng.random(128) < 0.3
            allowed[i, rng.integers(0, 128)] = True
        elif kind == 2:  # only the last (partial) chunk
            allowed[i, 256:] = rng.random(A - 256) < 0.5
            allowed[i, rng.integers(256, A)] = True
        else:  # the middle chunk, every action
            allowed[i, 128:256] = True
    Wd = (A + 31) // 32
    mask = np.zeros((M, Wd), np.uint32)
    for a in range(A):
        mask[:, a // 32] |= allowed[:, a].astype(np.uint32) << np.uint32(a % 32)
    dev = "cuda"
    out = dict(act=torch.zeros(M, dtype=torch.int32, device=dev), logp=torch.zeros(M, device=dev),
               val=torch.zeros(M, device=dev), ent=torch.zeros(M, device=dev))
    mlp.forward(torch.from_numpy(obs.view(np.int16)).to(dev), torch.from_numpy(mask.view(np.int32)).to(dev), M,
                77, 3, out["act"], out["logp"], out["val"], out["ent"])
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert allowed[np.arange(M), g["act"]].all()
    one = allowed.sum(axis=1) == 1
    assert np.array_equal(g["act"][one], np.argmax(allowed[one], axis=1))
    assert np.abs(g["logp"][one]).max() <= 1e-6 and np.abs(g["ent"][one]).max() <= 1e-6
    x = oe.bf16_bits_to_f32(obs[:, :D]).astype(np.float64)
    wb = op.bf16_weights(w)
    logits, _ = op.mlp(x, wb)
    lp = op.masked_log_softmax(logits, allowed)
    assert np.abs(g["ent"] - op.entropy(lp)).max() <= 2e-2
    assert np.abs(g["logp"] - lp[np.arange(M), g["act"]]).max() <= 2e-2
    l16, _ = op.mlp(x, wb, bf16_hidden=True)
    lp16 = op.masked_log_softmax(l16, allowed)
    NC = (A + 1 + 127) // 128
    u1, u2 = oe.sample_uniforms(77, np.arange(M), 3, NC)
    lp16p = np.concatenate([lp16, np.full((M, NC * 128 - A), -np.inf)], axis=1)
    a_o, margin = op.sample_chunked(lp16p, u1, u2)
    safe = margin > 1e-4
    assert safe.mean() > 0.97, safe.mean()  # about 1 - 2e-4 per near-threshold candidate
    assert np.array_equal(g["act"][safe], a_o[safe]), np.flatnonzero(g["act"][safe] != a_o[safe])[:10]


@pytest.mark.parametrize("A", [125, 507])
def test_rows_without_allowed_actions(A):
    """A row whose mask allows no action gets action 0, log-probability 0
    and entropy 0 (its value head is still computed), and the other rows
    are bit for bit those of the same call with that row's mask full."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, M = 35, 40, 256, 300
    mlp = binding.Mlp(D, Ds, H, A, W.policy_weights(D, H, A, seed=4))
    obs = torch.from_numpy(W.synthetic_obs(M, D, Ds, 4).view(np.int16)).cuda()
    masks = W.synthetic_masks(M, A, 4)
    empty = np.zeros(M, bool)
    empty[[0, 63, 64, 130, 299]] = True
    cut = masks.copy()
    cut[empty] = 0
    outs = []
    for mk in (masks, cut):
        o = [torch.zeros(M, dtype=torch.int32, device="cuda")] + [torch.zeros(M, device="cuda") for _ in range(3)]
        mlp.forward(obs, torch.from_numpy(mk.view(np.int32)).cuda(), M, 9, 2, *o)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in o])
    (act0, lp0, val0, ent0), (act1, lp1, val1, ent1) = outs
    assert (act1[empty] == 0).all() and (lp1[empty] == 0).all() and (ent1[empty] == 0).all()
    assert np.array_equal(val1, val0)
    keep = ~empty
    for x, y in ((act0, act1), (lp0, lp1), (ent0, ent1)):
        assert np.array_equal(x[keep], y[keep])


@pytest.mark.parametrize("A", [125, 507])
def test_peaked_distributions(A):
    """Head weights scaled by 300, so that the logits spread over hundreds of
    units and every allowed weight but the largest underflows to 0 in fp32
    (within the chunk and across the chunks' reservoir).  The draw is the
    best allowed action wherever its margin over the runner-up exceeds the
    bf16 rounding of the logits; with a margin above 30 its log-probability
    and the entropy are 0 to within 1e-3; the value column is not scaled and
    stays within 2e-2."""
    import torch
    from paper_2410_22165_amd import binding
    D, Ds, H, M = 35, 40, 256, 400
    print(f"[gpu] peaked policy A={A} M={M}", flush=True)
    w = W.policy_weights(D, H, A, seed=9)
    w["W3"] = w["W3"].copy()
    w["W3"][:, :A] *= 300.0
    mlp = binding.Mlp(D, Ds, H, A, w)
    obs = W.synthetic_obs(M, D, Ds, seed=9)
    mask = W.synthetic_masks(M, A, seed=9)
    o = [torch.zeros(M, dtype=torch.int32, device="cuda")] + [torch.zeros(M, device="cuda") for _ in range(3)]
    mlp.forward(torch.from_numpy(obs.view(np.int16)).cuda(), torch.from_numpy(mask.view(np.int32)).cuda(), M,
                5, 1, *o)
    torch.cuda.synchronize()
    act, logp, val, ent = (t.cpu().numpy() for t in o)
    x = oe.bf16_bits_to_f32(obs[:, :D]).astype(np.float64)
    logits, value = op.mlp(x, op.bf16_weights(w), bf16_hidden=True)
    allowed = op.unpack_mask(mask, A)
    z = np.where(allowed, logits, -np.inf)
    best = np.argmax(z, axis=1)
    top2 = -np.sort(-z, axis=1)[:, :2]
    gap = top2[:, 0] - top2[:, 1]
    clear = gap > 0.01 * np.abs(z[np.isfinite(z)]).max() + 1.0
    assert clear.mean() > 0.5
    assert np.array_equal(act[clear], best[clear])
    wide = gap > 30.0
    assert wide.sum() > 20
    assert np.abs(logp[wide]).max() <= 1e-3 and np.abs(ent[wide]).max() <= 1e-3
    assert np.abs(val - value).max() <= 2e-2
