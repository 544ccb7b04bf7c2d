"""Pins of the oracle's economy step: invariants that the paper's rules fix
(escrow accounting, conservation of coin and resources, tax collected equals
tax redistributed), bounds (gathering), the paper's crafting and tax
examples run through the whole step, expiry, masking, auto-reset and
checkpoint/resume (CPU only)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import env as oe

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def decode(cfg, a):
    R, P = cfg["R"], cfg["P"]
    if a == 0:
        return ("noop", 0, 0)
    if 1 <= a <= R:
        return ("gather", a - 1, 0)
    if a == R + 1:
        return ("craft", 0, 0)
    b = a - (R + 2)
    if b < R * P:
        return ("buy", b // P, b % P)
    b -= R * P
    return ("sell", b // P, b % P)


def live_orders(cfg, st):
    out = []
    X, N, R = cfg["X"], cfg["N"], cfg["R"]
    for s in range(X):
        for i in range(N):
            code = st["orders"][s, i]
            if code >= 0:
                out.append((i, code & 1, (code >> 1) % R, (code >> 1) // R))
    return out


def check_invariants(cfg, st):
    prices = cfg["prices"]
    N, R = cfg["N"], cfg["R"]
    orders = live_orders(cfg, st)
    esc_c = np.zeros(N, np.int64)
    esc_r = np.zeros((R, N), np.int64)
    n_act = np.zeros(N, np.int64)
    for i, side, r, p in orders:
        n_act[i] += 1
        if side == 0:
            esc_c[i] += prices[p]
        else:
            esc_r[r, i] += 1
    assert np.array_equal(esc_c, st["coin_esc"]), "coin escrow != sum of own live bids"
    assert np.array_equal(esc_r, st["res_esc"]), "resource escrow != own live asks"
    assert np.array_equal(n_act, st["n_active"])
    assert (st["coin_inv"] >= 0).all() and (st["res_inv"] >= 0).all()
    assert (n_act <= max(cfg["max_orders"], 0) + 0).all() or cfg["max_orders"] >= cfg["X"]
    # the book is uncrossed per resource
    for r in range(R):
        bids = [prices[p] for (_, s, rr, p) in orders if rr == r and s == 0]
        asks = [prices[p] for (_, s, rr, p) in orders if rr == r and s == 1]
        if bids and asks:
            assert max(bids) < min(asks)


def masked_random_actions(cfg, env, rng):
    """Uniform over the allowed actions of each agent (from the oracle's own mask)."""
    _, mask, _ = env.observe(W.obs_scales(cfg), W.obs_stride(cfg), with_gov=False)
    A = W.num_actions(cfg)
    bits = ((mask[:, np.arange(A) // 32] >> (np.arange(A) % 32).astype(np.uint32)) & 1).astype(bool)
    return np.array([rng.choice(np.flatnonzero(bits[i])) for i in range(cfg["N"])], np.int32), bits


CONFIGS = [
    W.env_config(N=4, R=2, P=10, X=10, P_tax=10, K=7, T=100),
    W.env_config(N=7, R=3, P=4, X=3, max_orders=2, P_tax=5, K=3, T=37, R_d=2),
    W.env_config(N=5, R=1, P=3, X=1, P_tax=4, K=1, T=20, R_d=1, R_kappa=1),
    W.env_config(N=6, R=5, P=3, X=30, max_orders=15, P_tax=7, K=0, T=50, R_d=3, allow_noop=0),
]


@pytest.mark.parametrize("ci", range(len(CONFIGS)))
def test_invariants_and_conservation(ci):
    cfg = CONFIGS[ci]
    rng = np.random.default_rng(ci)
    env = oe.OracleEnv(cfg, e=3, seed=11)
    N, R = cfg["N"], cfg["R"]
    u0 = None
    ret = np.zeros(N)
    for step in range(cfg["T"] * 2 + 3):
        st = env.state()
        check_invariants(cfg, st)
        if rng.random() < 0.5:
            act, bits = masked_random_actions(cfg, env, rng)
        else:
            act = rng.integers(0, W.num_actions(cfg), size=N).astype(np.int32)
            _, bits = masked_random_actions(cfg, env, rng)
        gov = rng.integers(0, 21, size=max(cfg["K"], 1)).astype(np.int32)
        C0 = st["coin_inv"].astype(np.int64) + st["coin_esc"]
        res0 = (st["res_inv"] + st["res_esc"]).astype(np.int64)
        coins_expected = C0.sum()
        res_delta = np.zeros(R, np.int64)
        gathers = []
        for i in range(N):
            a = int(act[i])
            if not bits[i, a]:
                continue
            kind, r, p = decode(cfg, a)
            if kind == "craft":
                coins_expected += (int(st["sc"][i]) * cfg["kappa_c"]) >> 16
                res_delta -= 0  # per-type split checked below in total
            if kind == "gather":
                gathers.append((i, r))
        rew, grew, done = env.step(act, gov)
        st1 = env.state()
        if done:
            assert st1["t"] == 0 and st1["ep"] == st["ep"] + 1
            ret[:] = 0
            continue
        C1 = st1["coin_inv"].astype(np.int64) + st1["coin_esc"]
        assert C1.sum() == coins_expected, "coin is created only by crafting"
        res1 = (st1["res_inv"] + st1["res_esc"]).astype(np.int64)
        n_craft = sum(1 for i in range(N) if bits[i, act[i]] and decode(cfg, int(act[i]))[0] == "craft")
        gained = res1.sum() - res0.sum() + n_craft * cfg["R_kappa"] * cfg["R_d"]
        # gathering bounds floor(SG) <= amount <= floor(SG + 1.1)
        lo = sum(int(st["sg"][r, i]) >> 16 for i, r in gathers)
        hi = sum((int(st["sg"][r, i]) + 72090) >> 16 for i, r in gathers)
        assert lo <= gained <= hi
        # rewards are utility differences (Eq. (2)) of the step's endpoints
        for i in range(N):
            du = oe.utility(C1[i], st1["labor"][i], cfg["eta"]) - oe.utility(C0[i], st["labor"][i], cfg["eta"])
            assert rew[i] == np.float32(du)
        ug = oe.social_welfare(C1, cfg["omega"]) - oe.social_welfare(C0, cfg["omega"])
        assert grew == np.float32(ug)
        # invalid actions cost nothing: labor only grows by the allowed action's cost
        for i in range(N):
            kind = decode(cfg, int(act[i]))[0] if bits[i, act[i]] else "noop"
            cost = dict(noop=0, gather=cfg["labor_gather"], craft=cfg["labor_craft"],
                        buy=cfg["labor_trade"], sell=cfg["labor_trade"])[kind]
            assert st1["labor"][i] - st["labor"][i] == cost
        ret += rew


def test_tax_collected_equals_redistributed_and_example():
    """The paper's worked example through a whole step: an agent that earned
    130 in the period pays 35 and gets its 1/n share back."""
    ex = GOLDEN["tax_example"]
    cfg = W.env_config(N=5, R=2, P=5, X=4, P_tax=10, K=3, T=100, cutoffs=ex["cutoffs"])
    env = oe.OracleEnv(cfg, seed=1)
    st = env.state()
    st["t"] = 9  # last step of the first period
    st["rates"] = np.array(ex["levels_5pct"], np.int32)
    st["snap"] = np.array([15, 15, 15, 15, 15], np.int32)
    st["coin_inv"] = np.array([15 + ex["income"], 15, 20, 15, 15], np.int32)
    env.set_state(st)
    act = np.zeros(5, np.int32)  # NOOP
    rew, grew, done = env.step(act, np.zeros(3, np.int32))
    st1 = env.state()
    taxes = [ex["tax"], 0, 0, 0, 0]  # agent 2 earned 5 -> floor(2 * 5 / 20) = 0
    pool = sum(taxes)
    # 35 = 7 * 5: every agent gets 7 back, no remainder
    expect = np.array([145 - 35 + 7, 15 + 7, 20 + 7, 15 + 7, 15 + 7])
    assert pool == 35
    assert np.array_equal(st1["coin_inv"], expect)
    assert np.array_equal(st1["snap"], expect)  # next period's earnings start here


def test_redistribution_remainder_rotates():
    cfg = W.env_config(N=4, R=1, P=3, X=2, P_tax=3, K=1, T=100, cutoffs=[])
    env = oe.OracleEnv(cfg, seed=1)
    st = env.state()
    st["t"] = 5  # last step of period 1
    st["rates"] = np.array([20], np.int32)  # 100 %: all income is taxed
    st["snap"] = np.zeros(4, np.int32)
    st["coin_inv"] = np.array([3, 2, 0, 1], np.int32)  # pool 6 = 4 * 1 + 2
    env.set_state(st)
    env.step(np.zeros(4, np.int32), np.zeros(1, np.int32))
    st1 = env.state()
    # period index 1: agents with (i - 1) mod 4 < 2, i.e. 1 and 2, get the extra unit
    assert list(st1["coin_inv"]) == [1, 2, 2, 1]
    assert st1["coin_inv"].sum() == 6


def test_crafting_example_fullest_types_first():
    ex = GOLDEN["craft_example"]
    cfg = W.env_config(N=2, R=ex["R"], P=3, X=3, P_tax=50, K=1, T=100, R_kappa=ex["R_kappa"],
                       R_d=ex["R_d"], cutoffs=[])
    env = oe.OracleEnv(cfg, seed=4)
    st = env.state()
    st["res_inv"] = np.array([[5, 9], [2, 1], [3, 1], [1, 1], [2, 1]], np.int32)
    env.set_state(st)
    craft = cfg["R"] + 1
    env.step(np.array([craft, craft], np.int32), np.zeros(1, np.int32))
    st1 = env.state()
    # agent 0: eligible 5, 2, 3, -, 2 -> the three fullest are 0, 2 and (tie 1 vs 4 -> 1)
    assert list(st1["res_inv"][:, 0]) == [3, 0, 1, 1, 2]
    assert st1["coin_inv"][0] == 15 + ((int(st["sc"][0]) * cfg["kappa_c"]) >> 16)
    assert st1["labor"][0] == cfg["labor_craft"]
    # agent 1 has only one type with 2 units: crafting is masked, the action becomes NOOP
    assert list(st1["res_inv"][:, 1]) == [9, 1, 1, 1, 1] and st1["labor"][1] == 0
    assert env.invalid_counts()[0] == 1


def test_order_expiry_after_x_clearings():
    cfg = W.env_config(N=2, R=1, P=3, X=3, P_tax=100, K=1, T=100, cutoffs=[])
    env = oe.OracleEnv(cfg, seed=2)
    sell_top = 2 + 1 + 3 + 2  # sell r=0 at the highest price, nobody buys
    act = np.array([sell_top, 0], np.int32)
    st = env.state()
    st["res_inv"] = np.array([[1, 0]], np.int32)
    env.set_state(st)
    env.step(act, [0])
    for k in range(cfg["X"] - 1):
        s = env.state()
        assert s["res_esc"][0, 0] == 1 and s["n_active"][0] == 1
        env.step(np.zeros(2, np.int32), [0])
    s = env.state()
    assert s["res_esc"][0, 0] == 0 and s["res_inv"][0, 0] == 1 and s["n_active"][0] == 0


def test_max_orders_mask_binds():
    cfg = W.env_config(N=1, R=1, P=3, X=5, max_orders=2, P_tax=100, K=1, T=100, cutoffs=[])
    env = oe.OracleEnv(cfg, seed=2)
    buy_low = 2 + 1  # buy r=0 at price 2; nobody sells
    for k in range(4):
        env.step(np.array([buy_low], np.int32), [0])
    s = env.state()
    assert s["n_active"][0] == 2 and s["coin_esc"][0] == 4
    assert env.invalid_counts()[0] == 2


def test_matching_inside_env_and_price_paid():
    cfg = W.env_config(N=2, R=1, P=3, X=5, P_tax=100, K=1, T=100, prices=[2, 4, 6], cutoffs=[])
    env = oe.OracleEnv(cfg, seed=5)
    st = env.state()
    st["res_inv"] = np.array([[3, 0]], np.int32)
    env.set_state(st)
    sell_2 = 2 + 1 + 3 + 0  # ask at price 2, placed first
    buy_6 = 2 + 1 + 2       # bid at price 6, placed later -> trades at 6
    env.step(np.array([sell_2, 0], np.int32), [0])
    env.step(np.array([0, buy_6], np.int32), [0])
    s = env.state()
    assert s["coin_inv"][0] == 15 + 6 and s["res_esc"][0, 0] == 0 and s["res_inv"][0, 0] == 2
    assert s["coin_inv"][1] == 15 - 6 and s["coin_esc"][1] == 0 and s["res_inv"][0, 1] == 1
    assert s["n_active"].sum() == 0


def test_auto_reset_and_determinism():
    cfg = W.workload("econ_e1_n4")["env"]
    a = oe.OracleEnv(cfg, e=2, seed=9)
    b = oe.OracleEnv(cfg, e=2, seed=9)
    r_a, r_b = [], []
    for t in range(cfg["T"] + 5):
        act, gov = a.random_actions(123)
        act2, gov2 = b.random_actions(123)
        assert np.array_equal(act, act2)
        ra, ga, da = a.step(act, gov)
        rb, gb, db = b.step(act2, gov2)
        r_a.append(ra)
        r_b.append(rb)
        assert da == db == (1 if t == cfg["T"] - 1 else 0)
    assert np.array_equal(np.array(r_a), np.array(r_b))
    sa, sb = a.state(), b.state()
    assert sa["ep"] == 1 and sa["t"] == 5
    for k in sa:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k]))


def test_checkpoint_resume_bit_identical():
    cfg = W.env_config(N=6, R=2, P=5, X=4, P_tax=7, K=3, T=60)
    act, gov = W.uniform_actions(cfg, 80, E=1, seed=3)
    ref = oe.OracleEnv(cfg, seed=13)
    for t in range(80):
        ref.step(act[t, 0], gov[t, 0])
    first = oe.OracleEnv(cfg, seed=13)
    for t in range(33):
        first.step(act[t, 0], gov[t, 0])
    saved = first.state()
    resumed = oe.OracleEnv(cfg, seed=13)
    resumed.set_state(saved)
    for t in range(33, 80):
        resumed.step(act[t, 0], gov[t, 0])
    s1, s2 = ref.state(), resumed.state()
    for k in s1:
        assert np.array_equal(np.asarray(s1[k]), np.asarray(s2[k])), k


def test_skills_pareto_range_and_tail():
    cfg = W.env_config(N=1000, R=3, P=3, X=2, P_tax=10, K=1, T=10)
    env = oe.OracleEnv(cfg, seed=0)
    st = env.state()
    x = np.concatenate([st["sg"].ravel(), st["sc"]]) / 65536.0
    assert x.min() >= 1.0 and x.max() <= 5.0
    # Pareto(4): P(X > 2) = 2^-4 = 1/16, P(X >= 5) = 5^-4 (clipped mass)
    assert abs((x > 2.0).mean() - 1 / 16) < 0.01
    assert abs((x >= 5.0).mean() - 5.0 ** -4) < 0.002
    assert abs(np.minimum(x, 2.0).mean() - (4 / 3) * (1 - 2.0 ** -3) - 2.0 * 2.0 ** -4) < 0.01


def test_observation_layout_and_mask():
    cfg = W.env_config(N=3, R=2, P=4, X=3, P_tax=10, K=2, T=50, cutoffs=[20])
    env = oe.OracleEnv(cfg, seed=0)
    sc = W.obs_scales(cfg)
    obs, mask, gov = env.observe(sc, W.obs_stride(cfg))
    assert obs.shape == (3, W.obs_stride(cfg)) and gov.shape == (W.gov_obs_dim(cfg),)
    f = oe.bf16_bits_to_f32(obs)
    assert (f[:, W.obs_dim(cfg):] == 0).all()
    assert f[0, 0] == np.float32(15 * sc["coin"])
    A = W.num_actions(cfg)
    bits = ((mask[:, np.arange(A) // 32] >> (np.arange(A) % 32).astype(np.uint32)) & 1).astype(bool)
    # at reset: NOOP, gathers allowed; craft and sells masked; buys allowed where the price is affordable
    assert bits[:, 0].all() and bits[:, 1:3].all() and not bits[:, 3].any()
    buy = bits[:, 4:4 + 2 * 4]
    assert (buy == np.array([p <= 15 for p in cfg["prices"]] * 2)).all()
    assert not bits[:, 4 + 2 * 4:].any()
    assert gov[0] == 15.0 and gov[1] == 0.0 and gov[2] == 15.0
