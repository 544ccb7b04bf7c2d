"""Pins of the policy / PPO oracle that do not come from the oracle itself
(CPU only): hand-computed network outputs with non-zero biases, the chunked
sampler against the softmax (chi-square over several chunks, sparse and empty
chunks) and against the plain inverse CDF, the reservoir's chunk choice in
closed form, the bf16 straight-through rounding on hand-rounded values, and
every branch of the PPO loss (Table 2: clip 0.2, value clip, value and
entropy coefficients) through hand-derived closed forms of the loss and of its
gradient."""
import math

import numpy as np
import pytest
import scipy.stats
import torch

from oracle import policy as op


# ---------------------------------------------------------------------------
# network: biases, ReLU and the W[in][out] orientation by hand
# ---------------------------------------------------------------------------
def test_mlp_hand_computed_with_biases():
    """x = (1, 2); pre-activations and outputs worked out by hand (every value
    exact in bf16 and in binary floating point):
      layer 1: (1*1 + 2*2 + 0.5, 1*(-1) + 2*0.5 - 3) = (5.5, -3) -> relu (5.5, 0)
      layer 2: (5.5*1 + 0*(-2) - 5, 5.5*0.25 + 0*1 + 1) = (0.5, 2.375)
      head:    (0.5*2 + 2.375*0 + 0.25, 0.5*0 + 2.375*4 - 0.5, 0.5*1 + 2.375*(-1) + 1)
             = (1.25, 9.0 | value -0.875)"""
    w = dict(W1=np.array([[1.0, -1.0], [2.0, 0.5]]), b1=np.array([0.5, -3.0]),
             W2=np.array([[1.0, 0.25], [-2.0, 1.0]]), b2=np.array([-5.0, 1.0]),
             W3=np.array([[2.0, 0.0, 1.0], [0.0, 4.0, -1.0]]), b3=np.array([0.25, -0.5, 1.0]))
    wb = op.bf16_weights({k: v.astype(np.float32) for k, v in w.items()})
    logits, value = op.mlp(np.array([[1.0, 2.0]]), wb)
    assert logits.tolist() == [[1.25, 9.0]]
    assert value.tolist() == [-0.875]
    # the same through the torch loss path (logits of the taken action, value)
    params = {k: torch.tensor(v, dtype=torch.float64) for k, v in wb.items()}
    _, terms = op.ppo_loss_torch(params, np.array([[1.0, 2.0]]), np.array([[True, True]]), [1], [0.0], [-0.875],
                                 [0.0], [-0.875], dict(clip=0.2, vclip=10.0, vf_coef=1.0, ent_coef=0.0))
    assert terms["vf"].item() == 0.0


# ---------------------------------------------------------------------------
# bf16 rounding with a straight-through gradient
# ---------------------------------------------------------------------------
def test_bf16_straight_through_values_and_gradient():
    """Forward: round to the nearest bf16, ties to even (values rounded by
    hand: 8 significant bits).  Backward: the identity."""
    x = torch.tensor([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.0 - 2 ** -7, 0.0,
                      1000.5], dtype=torch.float64, requires_grad=True)
    want = [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -3.0, 0.0, 1000.0]
    y = op._round_bf16_straight_through(x)
    assert y.detach().tolist() == want
    c = torch.tensor([1.0, -2.0, 3.0, 0.5, 7.0, -1.0, 2.0], dtype=torch.float64)
    (y * c).sum().backward()
    assert x.grad.tolist() == c.tolist()


# ---------------------------------------------------------------------------
# the chunked sampler
# ---------------------------------------------------------------------------
def _pad(lp, chunk=128):
    M, A = lp.shape
    NC = (A + chunk - 1) // chunk
    return np.concatenate([lp, np.full((M, NC * chunk - A), -np.inf)], axis=1)


def test_sample_chunked_single_chunk_equals_inverse_cdf():
    """With one chunk the reservoir always keeps chunk 0 and the draw is the
    plain inverse CDF at u2 (action order): identical actions."""
    rng = np.random.default_rng(11)
    M, A = 400, 97
    z = rng.normal(size=(M, A)) * 2.0
    allowed = rng.random((M, A)) < 0.5
    allowed[np.arange(M), rng.integers(0, A, M)] = True
    lp = op.masked_log_softmax(z, allowed)
    u1, u2 = rng.random((M, 1)), rng.random((M, 1))
    a_c, _ = op.sample_chunked(_pad(lp), u1, u2)
    a_i, _ = op.sample_inverse_cdf(lp, u2[:, 0])
    assert np.array_equal(a_c, a_i)
    assert allowed[np.arange(M), a_c].all()


def test_sample_chunked_reservoir_chooses_chunks_in_proportion():
    """Two chunks, one allowed action in each (probabilities p0, p1): chunk 1
    is kept exactly when u1 of chunk 1 is below p1 / (p0 + p1); on a fine
    grid of u1 the kept fraction is that ratio."""
    A = 200
    z = np.full((1, A), -np.inf)
    allowed = np.zeros((1, A), bool)
    allowed[0, 5] = allowed[0, 150] = True
    z[0, 5], z[0, 150] = 0.0, math.log(3.0)  # p = (1/4, 3/4)
    lp = op.masked_log_softmax(np.where(allowed, z, 0.0), allowed)
    n = 1000
    u1 = np.stack([np.full(n, 0.5), (np.arange(n) + 0.5) / n], axis=1)
    u2 = np.full((n, 2), 0.5)
    act, _ = op.sample_chunked(_pad(np.repeat(lp, n, axis=0)), u1, u2)
    assert set(np.unique(act)) == {5, 150}
    assert np.array_equal(act == 150, u1[:, 1] < 0.75)


def test_sample_chunked_chi_square_three_chunks_sparse_and_empty():
    """Three chunks (300 actions, the last one partial), the middle chunk
    entirely masked and the others sparse: the histogram of many draws
    matches the softmax (chi-square), and no masked action is ever drawn."""
    rng = np.random.default_rng(12)
    A = 300
    allowed = np.zeros(A, bool)
    allowed[rng.choice(128, 6, replace=False)] = True
    allowed[256 + rng.choice(A - 256, 5, replace=False)] = True
    z = rng.normal(size=A) * 1.5
    lp1 = op.masked_log_softmax(z[None], allowed[None])
    M = 40000
    u1, u2 = rng.random((M, 3)), rng.random((M, 3))
    act, _ = op.sample_chunked(_pad(np.repeat(lp1, M, axis=0)), u1, u2)
    counts = np.bincount(act, minlength=A)
    assert counts[~allowed].sum() == 0
    p = np.exp(lp1[0, allowed])
    chi = scipy.stats.chisquare(counts[allowed], p * M)
    assert chi.pvalue > 1e-4, chi


def test_sample_chunked_chi_square_many_chunks_dense():
    """Four chunks (507 actions, the workload with 5 resources and 50 prices),
    about half the actions allowed: chunk frequencies and the per-action
    histogram match the softmax."""
    rng = np.random.default_rng(13)
    A = 507
    allowed = rng.random(A) < 0.5
    z = rng.normal(size=A) * 0.7
    z[:64] += 2.0  # a peaked region
    lp1 = op.masked_log_softmax(z[None], allowed[None])
    M = 30000
    u1, u2 = rng.random((M, 4)), rng.random((M, 4))
    act, _ = op.sample_chunked(_pad(np.repeat(lp1, M, axis=0)), u1, u2)
    p = np.exp(lp1[0])
    for c in range(4):
        frac = ((act >= 128 * c) & (act < 128 * (c + 1))).mean()
        pc = p[128 * c:128 * (c + 1)].sum()
        assert abs(frac - pc) < 5 * math.sqrt(pc * (1 - pc) / M) + 1e-4, (c, frac, pc)
    counts = np.bincount(act, minlength=A)
    exp_c = p * M
    keep = exp_c > 5
    chi = scipy.stats.chisquare(counts[keep], exp_c[keep] * counts[keep].sum() / exp_c[keep].sum())
    assert chi.pvalue > 1e-4, chi


# ---------------------------------------------------------------------------
# PPO loss branches (Table 2 settings) in closed form
# ---------------------------------------------------------------------------
def _bias_only_params(b3, H=4, D=3, b2=None):
    """W1 = W2 = W3 = 0: logits and value are the head bias b3 for every row;
    h2 = relu(b2) (constant)."""
    A1 = len(b3)
    b2 = np.zeros(H) if b2 is None else np.asarray(b2, np.float64)
    p = dict(W1=np.zeros((D, H)), b1=np.ones(H), W2=np.zeros((H, H)), b2=b2, W3=np.zeros((H, A1)),
             b3=np.asarray(b3, np.float64))
    return {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}


def _loss(params, M, allowed, act, logp_old, val_old, adv, ret, hp):
    obs = np.zeros((M, params["W1"].shape[0]))
    loss, terms = op.ppo_loss_torch(params, obs, np.repeat(allowed[None], M, axis=0), act, logp_old, val_old, adv,
                                    ret, hp)
    loss.backward()
    return loss.item(), {k: v.item() for k, v in terms.items()}


def test_ppo_clipped_surrogate_branches_closed_form():
    """Four rows, ratios 1.5, 1.5, 0.5, 0.5 with advantages +1, -1, +1, -1
    (normalised: mean 0, population std 1).  Per row -min(rho A, clip(rho) A):
      rho 1.5, A +1: min(1.5, 1.2) = 1.2 (clipped)     -> -1.2, no gradient
      rho 1.5, A -1: min(-1.5, -1.2) = -1.5 (unclipped) -> +1.5
      rho 0.5, A +1: min(0.5, 0.8) = 0.5 (unclipped)   -> -0.5
      rho 0.5, A -1: min(-0.5, -0.8) = -0.8 (clipped)  -> +0.8, no gradient
    Surrogate = (-1.2 + 1.5 - 0.5 + 0.8) / 4 = 0.15.  Gradient with respect to
    the logits z (d log pi(a) / dz_j = [j = a] - p_j) of the unclipped rows:
    -A rho ([j = a] - p_j) / 4."""
    b = np.array([0.3, -0.2, 0.9, 0.1, 0.0])  # 4 logits + value
    allowed = np.array([True, True, True, True])
    z = b[:4]
    logp = z - np.log(np.exp(z).sum())
    p = np.exp(logp)
    act = np.array([2, 0, 1, 3])
    rho = np.array([1.5, 1.5, 0.5, 0.5])
    A = np.array([1.0, -1.0, 1.0, -1.0])
    logp_old = logp[act] - np.log(rho)
    hp = dict(clip=0.2, vclip=10.0, vf_coef=0.0, ent_coef=0.0)
    params = _bias_only_params(b)
    loss, terms = _loss(params, 4, allowed, act, logp_old, np.zeros(4), A, np.zeros(4), hp)
    s = 1.0 / (1.0 + 1e-8)  # normalisation: std 1, + 1e-8
    assert terms["pg"] == pytest.approx(0.15 * s, abs=1e-12)
    assert loss == pytest.approx(0.15 * s, abs=1e-12)
    g = np.zeros(4)
    for m in (1, 2):  # the unclipped rows
        onehot = np.eye(4)[act[m]]
        g += -(A[m] * s) * rho[m] * (onehot - p) / 4
    assert np.allclose(params["b3"].grad.numpy()[:4], g, atol=1e-12)
    assert params["b3"].grad.numpy()[4] == 0.0
    # reversed signs of the advantages flip which rows are clipped
    params = _bias_only_params(b)
    _, terms = _loss(params, 4, allowed, act, logp_old, np.zeros(4), -A, np.zeros(4), hp)
    # rho 1.5 A -1: -(-1.5) = 1.5; rho 1.5 A +1: -1.2; rho 0.5 A -1: 0.8; rho 0.5 A +1: -0.5
    assert terms["pg"] == pytest.approx((1.5 - 1.2 + 0.8 - 0.5) / 4 * s, abs=1e-12)


def test_ppo_clip_epsilon_changes_the_clipped_value():
    """clip = 0.4: rho 1.5 with A = +1 clips at 1.4 instead of 1.2."""
    b = np.array([0.0, 0.0, 0.0])
    act = np.array([0, 1])
    logp = np.log(0.5)
    rho = np.array([1.5, 1.0])
    A = np.array([1.0, -1.0])
    hp = dict(clip=0.4, vclip=10.0, vf_coef=0.0, ent_coef=0.0)
    params = _bias_only_params(b)
    _, terms = _loss(params, 2, np.array([True, True]), act, logp - np.log(rho), np.zeros(2), A, np.zeros(2), hp)
    s = 1.0 / (1.0 + 1e-8)
    assert terms["pg"] == pytest.approx((-1.4 + 1.0) / 2 * s, abs=1e-12)


def test_ppo_value_clip_binds_closed_form():
    """Value V = b3[value] = 0.7 on every row, value clip 0.5, c_v = 0.25:
      row 0: V_old = V - 2 -> V_clip = V - 1.5; R = V + 1: (V-R)^2 = 1, (V_clip-R)^2 = 6.25
             -> the clipped term wins, no gradient
      row 1: V_old = V - 2, R = V - 3: 9 against 2.25 -> unclipped, dL/dV = (V - R) = 3
      row 2: V_old = V (inside the clip), R = V + 0.5: 0.25 both, dL/dV = -0.5
      row 3: V_old = V + 0.2 (inside), R = V: 0
    value term = mean(1/2 max(...)) = (6.25 + 9 + 0.25 + 0) / 8 = 1.9375;
    dL/db3[value] = c_v (0 + 3 - 0.5 + 0) / 4 = 0.15625."""
    V = 0.7
    b = np.array([0.1, -0.3, V])
    vo = np.array([V - 2, V - 2, V, V + 0.2])
    R = np.array([V + 1, V - 3, V + 0.5, V])
    act = np.zeros(4, np.int64)
    logp = b[0] - np.log(np.exp(b[:2]).sum())
    hp = dict(clip=0.2, vclip=0.5, vf_coef=0.25, ent_coef=0.0)
    params = _bias_only_params(b)
    loss, terms = _loss(params, 4, np.array([True, True]), act, np.full(4, logp), vo, np.array([1.0, -1, 1, -1]), R,
                        hp)
    assert terms["vf"] == pytest.approx(1.9375, abs=1e-12)
    assert params["b3"].grad.numpy()[2] == pytest.approx(0.25 * (3.0 - 0.5) / 4, abs=1e-12)
    assert loss == pytest.approx(terms["pg"] + 0.25 * 1.9375, abs=1e-12)


def test_ppo_entropy_bonus_sign_and_gradient_closed_form():
    """c_e = 0.1, ratios 1 and zero advantages: loss = -c_e H.  For logits z
    over the allowed actions, H = -sum p log p and dH/dz_j = -p_j (log p_j + H),
    so dL/dz_j = c_e p_j (log p_j + H); a masked action has no gradient.
    The loss falls as the entropy rises (the bonus has a negative sign)."""
    b = np.array([0.5, -1.0, 2.0, 0.25, 3.0])
    allowed = np.array([True, True, True, False])
    z = b[:4][allowed]
    logp = z - np.log(np.exp(z).sum())
    p = np.exp(logp)
    H = -(p * logp).sum()
    act = np.array([0, 2])
    hp = dict(clip=0.2, vclip=10.0, vf_coef=0.0, ent_coef=0.1)
    params = _bias_only_params(b)
    lp_full = np.full(4, -np.inf)
    lp_full[allowed] = logp
    loss, terms = _loss(params, 2, allowed, act, lp_full[act], np.zeros(2), np.zeros(2), np.zeros(2), hp)
    assert terms["ent"] == pytest.approx(H, abs=1e-12)
    assert loss == pytest.approx(-0.1 * H, abs=1e-12)
    g = np.zeros(4)
    g[allowed] = 0.1 * p * (logp + H)
    assert np.allclose(params["b3"].grad.numpy()[:4], g, atol=1e-12)
    # a flatter distribution (higher entropy) gives a lower loss
    b_flat = b.copy()
    b_flat[:4] = 0.0
    params = _bias_only_params(b_flat)
    lp_flat = np.full(4, -np.inf)
    lp_flat[allowed] = -np.log(3.0)
    loss_flat, _ = _loss(params, 2, allowed, act, lp_flat[act], np.zeros(2), np.zeros(2), np.zeros(2), hp)
    assert loss_flat == pytest.approx(-0.1 * np.log(3.0), abs=1e-12) and loss_flat < loss


def test_ppo_head_weight_gradient_is_outer_product_of_h2():
    """With W1 = W2 = W3 = 0 the second hidden layer is relu(b2) on every row,
    so dL/dW3 = relu(b2) (outer) dL/db3: a check of the chain through the
    head's weights."""
    b = np.array([0.3, -0.2, 0.9, 0.1, 0.4])
    b2 = np.array([1.5, -1.0, 0.25, 2.0])
    act = np.array([2, 0, 1, 3])
    z = b[:4]
    logp = z - np.log(np.exp(z).sum())
    hp = dict(clip=0.2, vclip=0.5, vf_coef=0.25, ent_coef=0.1)
    params = _bias_only_params(b, b2=b2)
    _loss(params, 4, np.array([True] * 4), act, logp[act] - np.log([1.5, 0.5, 1.1, 0.9]), np.array([-2, 0, 1, 0.4]),
          np.array([1.0, -0.5, 0.3, 2.0]), np.array([1.0, 2.0, -1.0, 0.0]), hp)
    h2 = np.maximum(b2, 0.0)
    assert np.allclose(params["W3"].grad.numpy(), np.outer(h2, params["b3"].grad.numpy()), atol=1e-12)
