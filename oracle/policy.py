"""Oracle of the shared population policy and of the PPO learner.

TEST INFRASTRUCTURE: see the package docstring.

The paper trains every population agent with one shared actor-critic network
(Sec. 4 "Experimental details": all population agents share the weights of
the policy and value networks; PPO, Table 2) and masks invalid actions to
probability zero (Sec. 3 "Action masking").  The network here is the one the
synthetic workload names: d_in -> H -> H -> (A logits, 1 value), ReLU.
Weights are the bf16-rounded values of the float32 inputs; the arithmetic
is float64 throughout, with no blocking or fusion.
"""
from __future__ import annotations

import numpy as np
import torch


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def bf16_weights(w: dict) -> dict:
    """The values the network computes with: bf16 matrices, float32 biases."""
    out = {}
    for k, v in w.items():
        out[k] = bf16_round(v).astype(np.float64) if k.startswith("W") else np.asarray(v, np.float64)
    return out


def unpack_mask(mask_words: np.ndarray, A: int) -> np.ndarray:
    """Bit a of word a // 32 says whether action a is allowed."""
    m = np.asarray(mask_words, dtype=np.uint32)
    a = np.arange(A)
    return ((m[:, a // 32] >> (a % 32).astype(np.uint32)) & 1).astype(bool)


def mlp(obs: np.ndarray, w: dict, bf16_hidden: bool = False):
    """Logits [M, A] and values [M] of the two-hidden-layer ReLU network.
    bf16_hidden rounds the hidden activations to bf16 (the precision in
    which a bf16 kernel feeds them to the next layer), so that a sampling
    decision can be taken in the kernel's precision."""
    x = np.asarray(obs, dtype=np.float64)
    h1 = np.maximum(x @ w["W1"] + w["b1"], 0.0)
    if bf16_hidden:
        h1 = bf16_round(h1.astype(np.float32)).astype(np.float64)
    h2 = np.maximum(h1 @ w["W2"] + w["b2"], 0.0)
    if bf16_hidden:
        h2 = bf16_round(h2.astype(np.float32)).astype(np.float64)
    out = h2 @ w["W3"] + w["b3"]
    return out[:, :-1], out[:, -1]


def masked_log_softmax(logits: np.ndarray, allowed: np.ndarray) -> np.ndarray:
    """log pi(a) over the allowed actions; -inf for masked ones."""
    z = np.where(allowed, logits, -np.inf)
    zmax = z.max(axis=1, keepdims=True)
    lse = zmax + np.log(np.exp(z - zmax).sum(axis=1, keepdims=True))
    return z - lse


def entropy(logp: np.ndarray) -> np.ndarray:
    finite = np.isfinite(logp)
    safe = np.where(finite, logp, 0.0)
    return -(np.exp(safe) * safe * finite).sum(axis=1)


def sample_inverse_cdf(logp: np.ndarray, u: np.ndarray):
    """Action = the first index whose cumulative probability exceeds u.
    Also returns the distance of u from the nearest cumulative boundary, so
    a test can tell a decision that rounding could flip from one it cannot."""
    p = np.exp(logp)
    cdf = np.cumsum(p, axis=1)
    M, A = p.shape
    act = np.empty(M, np.int64)
    margin = np.empty(M)
    for m in range(M):
        uu = u[m] * cdf[m, -1]
        idx = int(np.searchsorted(cdf[m], uu, side="right"))
        idx = min(idx, A - 1)
        while p[m, idx] == 0.0 and idx > 0:  # never land on a masked action
            idx -= 1
        act[m] = idx
        lo = cdf[m, idx - 1] if idx > 0 else 0.0
        margin[m] = min(abs(uu - lo), abs(cdf[m, idx] - uu))
    return act, margin


def chunk_walk_order(chunk: int = 128) -> np.ndarray:
    """Order in which the actions of one chunk are walked by the inverse CDF:
    action order."""
    return np.arange(chunk, dtype=np.int64)


def sample_chunked(logp: np.ndarray, u1: np.ndarray, u2: np.ndarray, chunk: int = 128):
    """Exact categorical sampling in chunks of `chunk` actions: chunk c (total
    probability S_c) becomes the candidate when u1_c * (S_0 + ... + S_c) < S_c
    (weighted reservoir); inside the candidate the actions are walked in the
    fixed order of chunk_walk_order and the first whose cumulative
    probability exceeds u2_c * S_c is drawn.  Any fixed walk order samples the
    same distribution.  Returns the actions and the smallest distance of any
    of the row's decisions from its threshold (relative to the quantity
    compared)."""
    p = np.exp(logp)
    M, A = p.shape
    NC = (A + chunk - 1) // chunk
    order = chunk_walk_order(chunk)
    act = np.zeros(M, np.int64)
    margin = np.full(M, np.inf)
    for m in range(M):
        W = 0.0
        for c in range(NC):
            pc = np.zeros(chunk)
            seg = p[m, c * chunk:(c + 1) * chunk]
            pc[:len(seg)] = seg
            pc = pc[order]
            Sc = pc.sum()
            if Sc <= 0.0:
                continue
            W += Sc
            lhs = u1[m, c] * W
            if c > 0:
                margin[m] = min(margin[m], abs(lhs - Sc) / W)
            if lhs < Sc:
                cdf = np.cumsum(pc)
                target = u2[m, c] * Sc
                j = int(np.searchsorted(cdf, target, side="right"))
                j = min(j, len(pc) - 1)
                while pc[j] == 0.0 and j > 0:
                    j -= 1
                act[m] = c * chunk + order[j]
                lo = cdf[j - 1] if j > 0 else 0.0
                margin[m] = min(margin[m], abs(target - lo) / Sc, abs(cdf[j] - target) / Sc)
    return act, margin


def uniform_from_word(w: np.ndarray) -> np.ndarray:
    """u = (top 24 bits + 1/2) / 2^24, exactly representable in float32."""
    top = (np.asarray(w, dtype=np.uint64) >> np.uint64(40)).astype(np.float64)
    return (top + 0.5) / 16777216.0


def policy_forward(obs, mask_words, w_f32: dict, u: np.ndarray):
    """Sampled actions, their log-probabilities, values and entropies."""
    w = bf16_weights(w_f32)
    A = w["W3"].shape[1] - 1
    logits, value = mlp(obs, w)
    logp = masked_log_softmax(logits, unpack_mask(mask_words, A))
    act, margin = sample_inverse_cdf(logp, u)
    return dict(logits=logits, value=value, logp_all=logp, act=act,
                logp=logp[np.arange(len(act)), act], entropy=entropy(logp), margin=margin)


# ---------------------------------------------------------------------------
# PPO (Schulman et al. 2017) as configured in Table 2: clipped surrogate,
# clipped value loss with coefficient c_v, entropy bonus c_e, GAE(gamma, lambda).
# ---------------------------------------------------------------------------
def gae(rew, val, done, last_val, gamma: float, lam: float):
    """Generalised advantage estimation, reverse over time.
    rew, val, done: [T, M]; done[t] = 1 when step t ended an episode;
    last_val: [M], the value of the state after the last step."""
    rew = np.asarray(rew, np.float64)
    val = np.asarray(val, np.float64)
    done = np.asarray(done, np.float64)
    T = rew.shape[0]
    adv = np.zeros_like(rew)
    nxt_adv = np.zeros(rew.shape[1])
    nxt_val = np.asarray(last_val, np.float64)
    for t in range(T - 1, -1, -1):
        nonterm = 1.0 - done[t]
        delta = rew[t] + gamma * nxt_val * nonterm - val[t]
        nxt_adv = delta + gamma * lam * nonterm * nxt_adv
        adv[t] = nxt_adv
        nxt_val = val[t]
    return adv, adv + val


def _round_bf16_straight_through(h):
    """Values rounded to bf16 (via float32, ties to even); gradient passed
    through unchanged."""
    r = h.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64)
    return h + (r - h.detach())


def ppo_loss_torch(params: dict, obs, allowed, act, logp_old, val_old, adv, ret, hp: dict,
                   bf16_hidden: bool = False, capture: dict | None = None):
    """PPO minibatch loss in float64 torch ops; returns (loss, terms).

    Advantages are normalised over the minibatch (population standard
    deviation, + 1e-8).  loss = mean(-min(rho A, clip(rho) A))
                              + c_v mean(1/2 max((V-R)^2, (Vclip-R)^2))
                              - c_e mean(H).
    bf16_hidden rounds the hidden activations to bf16 in the forward pass
    (straight-through in the backward pass): the clip decisions are then
    taken in the precision of a bf16 kernel.  `capture`, when given,
    receives the intermediate tensors (pre-activations z1, z2, activations
    h1, h2, outputs out, ratio, V) for a test's tolerance bookkeeping; out
    keeps its gradient after backward()."""
    x = torch.as_tensor(np.asarray(obs, np.float64))
    z1 = x @ params["W1"] + params["b1"]
    h1 = torch.relu(z1)
    if bf16_hidden:
        h1 = _round_bf16_straight_through(h1)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = torch.relu(z2)
    if bf16_hidden:
        h2 = _round_bf16_straight_through(h2)
    out = h2 @ params["W3"] + params["b3"]
    if capture is not None and out.requires_grad:
        out.retain_grad()
    logits, v = out[:, :-1], out[:, -1]
    allowed_t = torch.as_tensor(allowed)
    z = logits.masked_fill(~allowed_t, float("-inf"))
    logp_all = torch.log_softmax(z, dim=1)
    p = torch.exp(logp_all)
    ent = -(p * logp_all.masked_fill(~allowed_t, 0.0)).sum(dim=1)
    a = torch.as_tensor(np.asarray(act, np.int64))
    logp = logp_all.gather(1, a[:, None])[:, 0]
    A = torch.as_tensor(np.asarray(adv, np.float64))
    A = (A - A.mean()) / (torch.sqrt(((A - A.mean()) ** 2).mean()) + 1e-8)
    ratio = torch.exp(logp - torch.as_tensor(np.asarray(logp_old, np.float64)))
    eps = hp["clip"]
    pg = -torch.minimum(ratio * A, torch.clamp(ratio, 1.0 - eps, 1.0 + eps) * A).mean()
    vo = torch.as_tensor(np.asarray(val_old, np.float64))
    R = torch.as_tensor(np.asarray(ret, np.float64))
    v_clip = vo + torch.clamp(v - vo, -hp["vclip"], hp["vclip"])
    vl = 0.5 * torch.maximum((v - R) ** 2, (v_clip - R) ** 2).mean()
    en = ent.mean()
    loss = pg + hp["vf_coef"] * vl - hp["ent_coef"] * en
    if capture is not None:
        capture.update(z1=z1, z2=z2, h1=h1, h2=h2, out=out, ratio=ratio, V=v)
    return loss, dict(pg=pg, vf=vl, ent=en)


def ppo_grads(w_f32: dict, obs, mask_words, act, logp_old, val_old, adv, ret, hp: dict,
              bf16_hidden: bool = False, capture: dict | None = None):
    """Float64 loss and autograd gradients with respect to the bf16 weights."""
    w = bf16_weights(w_f32)
    A = w["W3"].shape[1] - 1
    params = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in w.items()}
    loss, terms = ppo_loss_torch(params, obs, unpack_mask(mask_words, A), act, logp_old, val_old, adv,
                                 ret, hp, bf16_hidden=bf16_hidden, capture=capture)
    loss.backward()
    return (float(loss.detach()), {k: float(v.detach()) for k, v in terms.items()},
            {k: params[k].grad.numpy().copy() for k in params})


def adam_step(w, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# The government agent (Sec. 3 "Government Agent", "Setting tax rates"): one
# level in 0..20 per tax bracket, K independent categorical heads on the same
# kind of network, trained with the same PPO loss (Sec. 4: the government
# learns at the same time as the population).
# ---------------------------------------------------------------------------
GOV_LEVELS = 21


def gov_obs_rows(gov_obs, scale, Ds: int) -> np.ndarray:
    """bf16 bit patterns [E, Ds] of the government features times their
    scale (the product in float32, then rounded to bf16; zero padding)."""
    x = np.asarray(gov_obs, np.float32) * np.asarray(scale, np.float32)[None, :]
    b = bf16_round(x).view(np.uint32) >> 16
    out = np.zeros((x.shape[0], Ds), np.uint16)
    out[:, :x.shape[1]] = b.astype(np.uint16)
    return out


def gov_head_log_softmax(logits: np.ndarray, K: int) -> np.ndarray:
    """log pi_k(level) [E, K, 21] of every bracket head."""
    z = np.asarray(logits, np.float64)[:, :K * GOV_LEVELS].reshape(-1, K, GOV_LEVELS)
    m = z.max(axis=2, keepdims=True)
    return z - (m + np.log(np.exp(z - m).sum(axis=2, keepdims=True)))


def gov_forward(x, w: dict, K: int, u: np.ndarray, bf16_hidden: bool = False):
    """Levels drawn head by head (inverse CDF in level order at u[e, k]),
    their summed log-probability, the summed entropy, the value; plus the
    smallest distance of any draw from its threshold (relative to the head's
    total), so that a test can skip decisions rounding could flip."""
    logits, value = mlp(x, w, bf16_hidden=bf16_hidden)
    lp = gov_head_log_softmax(logits, K)
    p = np.exp(lp)
    E = lp.shape[0]
    levels = np.zeros((E, K), np.int64)
    margin = np.full((E, K), np.inf)
    for e in range(E):
        for k in range(K):
            cdf = np.cumsum(p[e, k])
            j = int(np.searchsorted(cdf, u[e, k] * cdf[-1], side="right"))
            j = min(j, GOV_LEVELS - 1)
            levels[e, k] = j
            lo = cdf[j - 1] if j > 0 else 0.0
            margin[e, k] = min(abs(u[e, k] * cdf[-1] - lo), abs(cdf[j] - u[e, k] * cdf[-1])) / cdf[-1]
    logp = np.take_along_axis(lp, levels[:, :, None], axis=2)[:, :, 0].sum(axis=1)
    ent = -(p * lp).sum(axis=(1, 2))
    return dict(logits=logits, value=value, levels=levels, logp=logp, entropy=ent, margin=margin.min(axis=1),
                margin_heads=margin)


def gov_ppo_loss_torch(params: dict, obs, levels, logp_old, val_old, adv, ret, hp: dict, K: int,
                       bf16_hidden: bool = False, capture: dict | None = None):
    """The PPO loss of ppo_loss_torch with the multi-discrete policy: the
    ratio uses the sum over brackets of log pi_k(level_k), the entropy is the
    sum of the brackets' entropies."""
    x = torch.as_tensor(np.asarray(obs, np.float64))
    z1 = x @ params["W1"] + params["b1"]
    h1 = torch.relu(z1)
    if bf16_hidden:
        h1 = _round_bf16_straight_through(h1)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = torch.relu(z2)
    if bf16_hidden:
        h2 = _round_bf16_straight_through(h2)
    out = h2 @ params["W3"] + params["b3"]
    if capture is not None and out.requires_grad:
        out.retain_grad()
    heads = out[:, :K * GOV_LEVELS].reshape(-1, K, GOV_LEVELS)
    v = out[:, K * GOV_LEVELS]
    lp_all = torch.log_softmax(heads, dim=2)
    lv = torch.as_tensor(np.asarray(levels, np.int64))
    logp = lp_all.gather(2, lv[:, :, None])[:, :, 0].sum(dim=1)
    ent = -(torch.exp(lp_all) * lp_all).sum(dim=(1, 2))
    A = torch.as_tensor(np.asarray(adv, np.float64))
    A = (A - A.mean()) / (torch.sqrt(((A - A.mean()) ** 2).mean()) + 1e-8)
    ratio = torch.exp(logp - torch.as_tensor(np.asarray(logp_old, np.float64)))
    eps = hp["clip"]
    pg = -torch.minimum(ratio * A, torch.clamp(ratio, 1.0 - eps, 1.0 + eps) * A).mean()
    vo = torch.as_tensor(np.asarray(val_old, np.float64))
    R = torch.as_tensor(np.asarray(ret, np.float64))
    v_clip = vo + torch.clamp(v - vo, -hp["vclip"], hp["vclip"])
    vl = 0.5 * torch.maximum((v - R) ** 2, (v_clip - R) ** 2).mean()
    en = ent.mean()
    loss = pg + hp["vf_coef"] * vl - hp["ent_coef"] * en
    if capture is not None:
        capture.update(z1=z1, z2=z2, h1=h1, h2=h2, out=out, ratio=ratio, V=v)
    return loss, dict(pg=pg, vf=vl, ent=en)


def gov_ppo_grads(w_f32: dict, obs, levels, logp_old, val_old, adv, ret, hp: dict, K: int,
                  bf16_hidden: bool = False, capture: dict | None = None):
    """Float64 loss and autograd gradients with respect to the bf16 weights."""
    w = bf16_weights(w_f32)
    params = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in w.items()}
    loss, terms = gov_ppo_loss_torch(params, obs, levels, logp_old, val_old, adv, ret, hp, K,
                                     bf16_hidden=bf16_hidden, capture=capture)
    loss.backward()
    return (float(loss.detach()), {k: float(v.detach()) for k, v in terms.items()},
            {k: params[k].grad.numpy().copy() for k in params})
