"""Pins of the policy / PPO oracle: library routines for the softmax and
entropy, closed forms of the uniform policy, the sampler's distribution,
GAE special cases and brute force, and float64 finite differences of the
PPO loss (CPU only)."""
import numpy as np
import pytest
import scipy.special
import scipy.stats

import workloads as W
from oracle import policy as op


def test_bf16_round_ties_to_even_and_exact_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 0.0], np.float32)
    r = op.bf16_round(x)
    assert list(r) == [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5, 0.0]


def test_masked_log_softmax_matches_scipy():
    rng = np.random.default_rng(0)
    z = rng.normal(size=(50, 37)) * 3
    allowed = rng.random((50, 37)) < 0.6
    allowed[:, 0] = True
    lp = op.masked_log_softmax(z, allowed)
    for m in range(50):
        ref = scipy.special.log_softmax(z[m, allowed[m]])
        assert np.allclose(lp[m, allowed[m]], ref, rtol=0, atol=1e-12)
        assert np.all(np.isneginf(lp[m, ~allowed[m]]))
        assert op.entropy(lp[m:m + 1])[0] == pytest.approx(scipy.stats.entropy(np.exp(ref)), abs=1e-12)


def test_uniform_policy_closed_form():
    w = W.policy_weights(11, 16, 9, seed=1)
    w["W3"][:] = 0
    w["b3"][:] = 0.25
    obs = np.random.default_rng(1).normal(size=(20, 11))
    mask = np.zeros((20, 1), np.uint32)
    mask[:, 0] = 0b101101011
    out = op.policy_forward(obs, mask, w, np.full(20, 0.5))
    n_valid = bin(0b101101011).count("1")
    assert np.allclose(out["logp"], -np.log(n_valid))
    assert np.allclose(out["entropy"], np.log(n_valid))
    assert np.allclose(out["value"], 0.25)
    assert all((0b101101011 >> int(a)) & 1 for a in out["act"])


def test_relu_positive_homogeneity():
    w = W.policy_weights(8, 16, 5, seed=2)
    wb = op.bf16_weights(w)
    x = np.random.default_rng(2).normal(size=(10, 8))
    l1, v1 = op.mlp(x, wb)
    l2, v2 = op.mlp(3.0 * x, wb)  # zero biases: f(3x) = 3 f(x)
    assert np.allclose(l2, 3 * l1, atol=1e-12) and np.allclose(v2, 3 * v1, atol=1e-12)


def test_sampler_distribution_chi_square():
    rng = np.random.default_rng(3)
    z = np.array([[0.3, -1.0, 2.0, 0.0, 0.5, -0.2]])
    allowed = np.array([[True, True, True, False, True, True]])
    lp = op.masked_log_softmax(z, allowed)
    M = 200000
    u = rng.random(M)
    act, _ = op.sample_inverse_cdf(np.repeat(lp, M, axis=0), u)
    counts = np.bincount(act, minlength=6)
    assert counts[3] == 0
    p = np.exp(lp[0, allowed[0]])
    chi2 = scipy.stats.chisquare(counts[allowed[0]], p * M)
    assert chi2.pvalue > 1e-4


def test_gae_special_cases_and_brute_force():
    rng = np.random.default_rng(4)
    T, M = 13, 6
    rew, val = rng.normal(size=(T, M)), rng.normal(size=(T, M))
    done = (rng.random((T, M)) < 0.15).astype(np.float64)
    last = rng.normal(size=M)
    g = 0.97
    # lambda = 0 -> one-step TD residual
    adv, ret = op.gae(rew, val, done, last, g, 0.0)
    nxt = np.vstack([val[1:], last[None]])
    assert np.allclose(adv, rew + g * nxt * (1 - done) - val)
    assert np.allclose(ret, adv + val)
    # lambda = 1, no terminations -> discounted Monte-Carlo return (bootstrapped) - V
    adv1, _ = op.gae(rew, val, np.zeros_like(done), last, g, 1.0)
    for t in range(T):
        mc = sum(g ** (k - t) * rew[k] for k in range(t, T)) + g ** (T - t) * last
        assert np.allclose(adv1[t], mc - val[t])
    # brute force: A_t = sum_l (g lam)^l delta_{t+l}, cut at the first termination
    lam = 0.9
    adv2, _ = op.gae(rew, val, done, last, g, lam)
    delta = rew + g * nxt * (1 - done) - val
    for m in range(M):
        for t in range(T):
            acc, coef = 0.0, 1.0
            for k in range(t, T):
                acc += coef * delta[k, m]
                if done[k, m]:
                    break
                coef *= g * lam
            assert adv2[t, m] == pytest.approx(acc, abs=1e-12)


def _ppo_case(seed, M=24, D=7, H=8, A=6):
    rng = np.random.default_rng(seed)
    w = W.policy_weights(D, H, A, seed=seed)
    for k in ("b1", "b2", "b3"):
        w[k] = rng.normal(size=w[k].shape).astype(np.float32) * 0.1
    obs = rng.normal(size=(M, D))
    mask = np.zeros((M, 1), np.uint32)
    for m in range(M):
        bits = rng.random(A) < 0.7
        bits[rng.integers(A)] = True
        mask[m, 0] = sum(1 << a for a in range(A) if bits[a])
    allowed = op.unpack_mask(mask, A)
    act = np.array([rng.choice(np.flatnonzero(allowed[m])) for m in range(M)])
    logp_old = rng.normal(size=M) * 0.3 - 1.5
    val_old = rng.normal(size=M)
    adv = rng.normal(size=M)
    ret = rng.normal(size=M) * 2
    return w, obs, mask, act, logp_old, val_old, adv, ret


def test_ppo_gradient_finite_differences():
    hp = dict(clip=0.2, vclip=0.5, vf_coef=0.25, ent_coef=0.1)
    w, obs, mask, act, lpo, vo, adv, ret = _ppo_case(5)
    loss, _, grads = op.ppo_grads(w, obs, mask, act, lpo, vo, adv, ret, hp)
    import torch
    wb = op.bf16_weights(w)
    allowed = op.unpack_mask(mask, wb["W3"].shape[1] - 1)

    def f(params):
        p = {k: torch.tensor(v, dtype=torch.float64) for k, v in params.items()}
        return float(op.ppo_loss_torch(p, obs, allowed, act, lpo, vo, adv, ret, hp)[0])

    rng = np.random.default_rng(6)
    h = 1e-6
    for k in wb:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in wb[k].shape)
            pp = {kk: vv.copy() for kk, vv in wb.items()}
            pm = {kk: vv.copy() for kk, vv in wb.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (f(pp) - f(pm)) / (2 * h)
            assert grads[k][idx] == pytest.approx(fd, rel=1e-4, abs=1e-8), (k, idx)
    assert np.isfinite(loss)


def test_ppo_loss_closed_forms_at_ratio_one():
    """With logp_old equal to the current log-probabilities and V_old = V, the
    surrogate is -mean(normalised A) = 0 and the value loss is mean((V-R)^2)/2."""
    hp = dict(clip=0.2, vclip=10.0, vf_coef=1.0, ent_coef=0.0)
    w, obs, mask, act, _, _, adv, ret = _ppo_case(7)
    out = op.policy_forward(obs, mask, w, np.full(len(act), 0.5))
    lp_cur = out["logp_all"][np.arange(len(act)), act]
    loss, terms, _ = op.ppo_grads(w, obs, mask, act, lp_cur, out["value"], adv, ret, hp)
    assert terms["pg"] == pytest.approx(0.0, abs=1e-12)
    assert terms["vf"] == pytest.approx(0.5 * np.mean((out["value"] - ret) ** 2), rel=1e-12)


def test_adam_first_step_is_signed_lr():
    w = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.1, 0.0])
    w1, m, v = op.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> w - lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8))
