"""Pins of the oracle's episode statistics (the measures the paper reports
at the end of an episode, Sec. 4 results: productivity, equality 1 - gini,
government utility Eq * Prod, mean and median episode return, actions taken,
trades and their prices), against what the definitions fix: a hand-built
two-agent episode with one trade, and brute-force recomputation from the
pre-reset state of a twin economy whose episode is one step longer."""
import numpy as np

import workloads as W
from oracle import env as oe


def _record_fields(m, R):
    return dict(ep=m[0], prod=m[1], eq=m[2], ug=m[3], mean=m[4], median=m[5], hist=m[6:9 + 3 * R],
                trades=m[9 + 3 * R:9 + 4 * R], psum=m[9 + 4 * R:9 + 5 * R])


def test_metrics_before_any_episode_end():
    cfg = W.env_config(E=1, N=3, R=2, P=4, X=3, P_tax=5, K=2, T=10)
    o = oe.OracleEnv(cfg, e=0, seed=1)
    m = o.episode_metrics()
    assert len(m) == 5 * 2 + 9
    assert m[0] == -1 and not m[1:].any()


def test_two_agent_episode_with_one_trade_by_hand():
    """T = 4, one resource, prices 2 and 4.  Step 0: agent 0 gathers (its
    skill is at least 1, so it holds a unit), agent 1 waits.  Step 1: agent 0
    asks at price 2, agent 1 bids at 4: one trade at the price of whichever
    order counts as placed later.  Steps 2, 3: both wait.  The record holds one
    gather, one buy, one sell, five NOOPs, no rejection, one trade whose
    price is the seller's coin gain, and the end state's welfare measures."""
    cfg = W.env_config(E=1, N=2, R=1, P=2, X=3, P_tax=100, K=0, T=4)
    o = oe.OracleEnv(cfg, e=0, seed=3)
    A = o.num_actions if hasattr(o, "num_actions") else oe.num_actions(1, 2)
    R, P = 1, 2
    gather0, sell_p0, buy_p1 = 1, 2 + R + R * P + 0 * P + 0, 2 + R + 0 * P + 1
    assert A == 2 + R + 2 * R * P
    o.step(np.array([gather0, 0], np.int32), np.zeros(0, np.int32))
    coin_before = o.state()["coin_inv"].copy()
    o.step(np.array([sell_p0, buy_p1], np.int32), np.zeros(0, np.int32))
    st = o.state()
    q = int(st["coin_inv"][0] - coin_before[0])
    assert q in (2, 4)
    assert st["res_inv"][0, 1] == 1  # the buyer holds the unit
    coins_end = (st["coin_inv"] + st["coin_esc"]).astype(np.int64)
    labor_end = st["labor"].astype(np.int64)
    for _ in range(2):
        _, _, done = o.step(np.zeros(2, np.int32), np.zeros(0, np.int32))
    assert done
    f = _record_fields(o.episode_metrics(), R)
    assert f["ep"] == 0
    assert f["hist"].tolist() == [5, 1, 0, 1, 1, 0]  # NOOP, gather, craft, buy, sell, rejected
    assert f["trades"].tolist() == [1] and f["psum"].tolist() == [q]
    prod = int(coins_end.sum())
    assert f["prod"] == prod
    gini = abs(coins_end[0] - coins_end[1]) * 2 / (2 * 2 * prod)  # sum_i sum_j |x_i - x_j| / (2 n sum x)
    assert abs(f["eq"] - (1 - gini)) < 1e-15
    assert abs(f["ug"] - (1 - gini) * prod) < 1e-12 * prod
    u0 = oe.utility(15, 0, 0.27)
    ret = sorted(oe.utility(int(coins_end[i]), int(labor_end[i]), 0.27) - u0 for i in range(2))
    assert abs(f["mean"] - (ret[0] + ret[1]) / 2) < 1e-12
    assert f["median"] == ret[0]  # lower median of two


def test_random_episodes_match_brute_force_from_the_pre_reset_state():
    """Two episodes of uniform random actions (invalid ones included).  A
    twin economy with T + 1 steps per episode replays the same actions: its
    state after step T is the pre-reset state of the original, from which
    productivity, the O(N^2) Gini, Eq * Prod and the returns are recomputed;
    the returns also equal each agent's summed rewards (Eq. (2) telescopes),
    the action counts add up to N T, the rejections to the invalid counter's
    increase, and every resource's price sum lies between its trade count
    times the lowest and the highest price."""
    T, N = 25, 9
    cfg = W.env_config(E=1, N=N, R=3, P=5, X=4, P_tax=6, K=3, T=T)
    twin_cfg = dict(cfg, T=T + 1)
    R = cfg["R"]
    rng = np.random.default_rng(5)
    o = oe.OracleEnv(cfg, e=0, seed=2)
    for ep in range(2):
        twin = oe.OracleEnv(twin_cfg, e=0, seed=2)
        twin.set_state(dict(o.state(), t=0))
        inv0 = o.invalid_counts()[0]
        rsum = np.zeros(N)
        for t in range(T):
            a = rng.integers(-1, oe.num_actions(R, cfg["P"]) + 1, size=N).astype(np.int32)
            g = rng.integers(0, 21, size=3).astype(np.int32)
            r, _, done = o.step(a, g)
            twin.step(a, g)
            rsum += r
        assert done
        f = _record_fields(o.episode_metrics(), R)
        st = twin.state()
        C = (st["coin_inv"] + st["coin_esc"]).astype(np.int64)
        assert f["ep"] == ep
        assert f["prod"] == C.sum()
        brute = np.abs(C[:, None] - C[None, :]).sum() / (2 * N * C.sum())
        assert abs(f["eq"] - (1 - brute)) < 1e-12
        assert abs(f["ug"] - (1 - brute) * C.sum()) < 1e-9 * C.sum()
        u0 = oe.utility(cfg["start_coin"], 0, cfg["eta"])
        ret = np.array([oe.utility(int(C[i]), int(st["labor"][i]), cfg["eta"]) - u0 for i in range(N)])
        assert abs(f["mean"] - ret.mean()) < 1e-12
        assert f["median"] == np.sort(ret)[(N - 1) // 2]
        assert np.allclose(np.sort(ret), np.sort(rsum), atol=1e-4)
        assert f["hist"].sum() == N * T
        assert f["hist"][-1] == o.invalid_counts()[0] - inv0
        prices = np.asarray(cfg["prices"][:cfg["P"]])
        assert (f["psum"] >= f["trades"] * prices.min()).all() and (f["psum"] <= f["trades"] * prices.max()).all()
