"""Pins of the government-policy oracle (Sec. 3 "Government Agent", "Setting
tax rates"): K independent categorical heads of 21 tax levels, whose
log-probabilities and entropies add up; hand-computed heads, the inverse-CDF
draw at chosen quantiles, chi-square of the draws, the surrogate's gradient
in closed form, and the worked tax example of the paper (brackets 0-50,
50-100, 100+, rates 10 %, 30 %, 50 %, income 130 -> 35) driven by levels the
policy draws."""
import json
import math
import os

import numpy as np
import scipy.stats
import torch

from oracle import env as oe
from oracle import policy as op

L = op.GOV_LEVELS


def _bias_only_net(D, H, K, b3):
    """A network whose weights are all zero: every row's logits are b3."""
    return dict(W1=np.zeros((D, H), np.float32), b1=np.zeros(H, np.float32), W2=np.zeros((H, H), np.float32),
                b2=np.zeros(H, np.float32), W3=np.zeros((H, K * L + 1), np.float32), b3=np.asarray(b3, np.float32))


def _peaked(K, favourite, weight=3.0, value=0.5):
    """Head k: all levels logit 0 except `favourite[k]` with logit log(weight)."""
    b3 = np.zeros(K * L + 1, np.float32)
    for k, f in enumerate(favourite):
        b3[k * L + f] = math.log(weight)
    b3[-1] = value
    return b3


def test_heads_add_their_log_probabilities_and_entropies():
    """K = 3 heads, each with one level of weight 3 and twenty of weight 1
    (probabilities 3/23 and 1/23): log pi(levels) = sum of the heads' terms and
    the entropy is three times one head's."""
    K, D, H = 3, 5, 8
    w = op.bf16_weights(_bias_only_net(D, H, K, _peaked(K, [2, 6, 10], 3.0)))
    x = np.zeros((4, D))
    u = np.array([[0.1, 0.1, 0.1], [0.9, 0.9, 0.9], [0.0001, 0.5, 0.99], [0.2, 0.3, 0.4]])
    g = op.gov_forward(x, w, K, u)
    assert np.allclose(g["value"], 0.5)
    wf = math.exp(float(np.float32(math.log(3.0))))  # the weight the float32 bias holds (3 to 7 digits)
    pf, po = wf / (wf + 20), 1 / (wf + 20)
    h1 = -(pf * math.log(pf) + 20 * po * math.log(po))
    assert np.allclose(g["entropy"], 3 * h1, rtol=1e-12, atol=0)
    for e in range(4):
        want = sum(math.log(pf if g["levels"][e, k] == f else po) for k, f in enumerate([2, 6, 10]))
        assert abs(g["logp"][e] - want) < 1e-12
    # inverse CDF in level order: cumulative weights 1, 2, 5, 6, ... (head 0);
    # u S = 0.1 * 23 = 2.3 falls in level 2; 0.9 * 23 = 20.7 in level 18
    assert g["levels"][0].tolist() == [2, 2, 2]  # heads 1, 2: cum 1..6 then 9 at level 6 -> 2.3 in level 2
    assert g["levels"][1].tolist() == [18, 18, 18]
    assert g["levels"][2, 0] == 0


def test_draws_follow_each_head_softmax_chi_square():
    K, D, H, E = 2, 4, 8, 40000
    rng = np.random.default_rng(1)
    b3 = np.zeros(K * L + 1, np.float32)
    b3[:K * L] = rng.normal(size=K * L).astype(np.float32)
    w = op.bf16_weights(_bias_only_net(D, H, K, b3))
    u = oe.gov_uniforms(7, np.arange(E), 3, K)
    g = op.gov_forward(np.zeros((E, D)), w, K, u)
    p = np.exp(op.gov_head_log_softmax(np.tile(b3.astype(np.float64), (1, 1)), K))[0]
    for k in range(K):
        counts = np.bincount(g["levels"][:, k], minlength=L)
        chi = scipy.stats.chisquare(counts, p[k] * E)
        assert chi.pvalue > 1e-4, (k, chi)


def test_surrogate_gradient_of_the_head_biases_closed_form():
    """W = 0, ratios 1, c_v = c_e = 0: the loss is -mean(A_hat rho) and
    dL/db3[21 k + j] = -(1/n) sum_m A_hat_m (1[j = a_mk] - p_kj)."""
    K, D, H, n = 2, 3, 4, 6
    rng = np.random.default_rng(2)
    b3 = np.zeros(K * L + 1, np.float32)
    b3[:K * L] = rng.normal(size=K * L).astype(np.float32) * 0.5
    w = _bias_only_net(D, H, K, b3)
    wb = op.bf16_weights(w)
    lp_heads = op.gov_head_log_softmax(wb["b3"][None, :], K)[0]
    levels = rng.integers(0, L, size=(n, K))
    logp_old = np.array([lp_heads[np.arange(K), levels[m]].sum() for m in range(n)])
    adv = rng.normal(size=n)
    hp = dict(clip=0.2, vclip=10.0, vf_coef=0.0, ent_coef=0.0)
    _, _, g = op.gov_ppo_grads(w, np.zeros((n, D)), levels, logp_old, np.zeros(n), adv, np.zeros(n), hp, K)
    ah = (adv - adv.mean()) / (np.sqrt(((adv - adv.mean()) ** 2).mean()) + 1e-8)
    p = np.exp(lp_heads)
    want = np.zeros(K * L + 1)
    for k in range(K):
        for j in range(L):
            want[k * L + j] = -np.mean(ah * ((levels[:, k] == j).astype(float) - p[k, j]))
    assert np.allclose(g["b3"], want, atol=1e-12)
    assert not g["W3"].any() and not g["W1"].any()


def test_entropy_bonus_gradient_closed_form():
    """c_e = 0.3 alone (zero advantages): dL/dz_kj = c_e p_kj (log p_kj + H_k)."""
    K, D, H, n = 3, 2, 4, 5
    rng = np.random.default_rng(3)
    b3 = np.zeros(K * L + 1, np.float32)
    b3[:K * L] = rng.normal(size=K * L).astype(np.float32)
    w = _bias_only_net(D, H, K, b3)
    lp = op.gov_head_log_softmax(op.bf16_weights(w)["b3"][None, :], K)[0]
    levels = np.zeros((n, K), np.int64)
    logp_old = np.full(n, lp[:, 0].sum())
    hp = dict(clip=0.2, vclip=10.0, vf_coef=0.0, ent_coef=0.3)
    _, terms, g = op.gov_ppo_grads(w, np.zeros((n, D)), levels, logp_old, np.zeros(n), np.zeros(n), np.zeros(n),
                                   hp, K)
    p = np.exp(lp)
    Hk = -(p * lp).sum(axis=1)
    assert abs(terms["ent"] - Hk.sum()) < 1e-12
    want = np.concatenate([(0.3 * p * (lp + Hk[:, None])).ravel(), [0.0]])
    assert np.allclose(g["b3"], want, atol=1e-12)


def test_paper_tax_example_from_levels_the_policy_draws():
    """A policy peaked at levels 2, 6 and 10 (10 %, 30 %, 50 %) on three
    brackets draws them at every row for mid quantiles, and those levels tax
    an income of 130 with cutoffs 50 and 100 at 35 coin, the paper's worked
    example (golden value)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")) as f:
        gold = json.load(f)
    K, D, H = 3, 4, 8
    w = op.bf16_weights(_bias_only_net(D, H, K, _peaked(K, [2, 6, 10], weight=1e6)))
    u = oe.gov_uniforms(11, np.arange(50), 0, K)
    g = op.gov_forward(np.zeros((50, D)), w, K, u)
    assert (g["levels"] == np.array([2, 6, 10])).all()
    ex = gold["tax_example"]
    tax = oe.bracket_tax(ex["income"], g["levels"][0], ex["cutoffs"])
    assert tax == ex["tax"] == 35


def test_gov_obs_rows_round_scaled_features_to_bf16():
    obs = np.array([[1.0, 2.0, 300.0], [0.1, -7.0, 0.0]], np.float32)
    sc = np.array([0.5, 1.0, 2 ** -7], np.float32)
    rows = op.gov_obs_rows(obs, sc, 8)
    vals = (rows.astype(np.uint32) << 16).view(np.float32)
    assert vals[0, :3].tolist() == [0.5, 2.0, 2.34375]
    assert vals[1, 1] == -7.0 and vals[1, 2] == 0.0 and not vals[:, 3:].any()
    assert abs(vals[1, 0] - 0.05) < 0.05 * 2 ** -8
