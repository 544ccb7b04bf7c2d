"""Pins of the oracle's multi-agent variant (Sec. 5): skills drawn near 1
with spread 1 and growing by 0.5 % per use, shrinking to nothing at the
maximum 5; R_d from the number of resources; the 30- and 86-action spaces
with the three prices 3, 6, 9."""
import math

import numpy as np
import scipy.stats

import workloads as W
from oracle import env as oe

SMAX = 5 * 65536


def _grow(q):
    return min(SMAX, q + max(0, (q * (SMAX - q)) // (200 * SMAX)))


def test_skill_growth_on_gathering_and_crafting_follows_the_definition():
    """One agent gathers its only resource 400 times, then crafts: each use
    adds floor(s (5 - s) / 1000) in Q16 -- within 2^-16 of s + 0.005 s (1 - s/5)
    -- the skill never exceeds 5, and the other skill does not move."""
    cfg = W.env_config(E=1, N=1, R=1, P=3, X=4, P_tax=100, K=0, T=2000, R_kappa=1, R_d=1, prices=[3, 6, 9],
                       skill_mode=3, seed=4)
    o = oe.OracleEnv(cfg, e=0, seed=4)
    s0 = o.state()
    sg, sc = int(s0["sg"][0, 0]), int(s0["sc"][0])
    for k in range(400):
        o.step(np.array([1], np.int32), np.zeros(0, np.int32))
        new = int(o.state()["sg"][0, 0])
        x = sg / 65536
        assert new == _grow(sg)
        assert abs(new / 65536 - (x + 0.005 * x * (1 - x / 5))) <= 2 ** -16
        assert new <= SMAX
        sg = new
    assert int(o.state()["sc"][0]) == sc
    o.step(np.array([2], np.int32), np.zeros(0, np.int32))  # craft (R_kappa = R_d = 1)
    assert int(o.state()["sc"][0]) == _grow(sc)
    assert int(o.state()["sg"][0, 0]) == sg


def test_skill_growth_fixed_points_and_monotone_approach():
    assert _grow(0) == 0 and _grow(SMAX) == SMAX
    q = 65536
    for _ in range(5000):
        nq = _grow(q)
        assert q <= nq <= SMAX
        q = nq
    assert q > 4.9 * 65536  # approaches the maximum


def test_normal_skills_match_a_unit_normal_around_one_clipped():
    """20 480 skill draws (1024 agents, 4 resources + crafting, 4 episodes):
    the share clipped to 0 is Phi(-1) and the CDF inside (0, 5) follows
    N(1, 1) within 0.01 (the twelve-uniform sum approximates the normal to
    about 0.002 in the CDF); the mean equals that of N(1, 1) clipped to [0, 5]."""
    cfg = W.env_config(E=1, N=1024, R=4, P=3, X=4, P_tax=100, K=0, T=5, R_d=2, prices=[3, 6, 9], skill_mode=1,
                       seed=9)
    o = oe.OracleEnv(cfg, e=0, seed=9)
    vals = []
    for ep in range(4):
        o.reset(ep)
        st = o.state()
        vals.append(st["sg"].ravel())
        vals.append(st["sc"].ravel())
    x = np.concatenate(vals).astype(np.float64) / 65536
    assert len(x) == 1024 * 5 * 4
    assert x.min() >= 0 and x.max() <= 5
    assert abs((x == 0).mean() - scipy.stats.norm.cdf(-1)) < 0.01
    for v in (0.5, 1.0, 1.5, 2.0, 3.0):
        assert abs((x <= v).mean() - scipy.stats.norm.cdf(v - 1)) < 0.01, v
    z = scipy.stats.norm
    clipped_mean = (5 * z.sf(4) + (z.expect(lambda t: t + 1, lb=-1, ub=4)))
    assert abs(x.mean() - clipped_mean) < 0.02


def test_variant_configuration():
    """R_d = max(1, floor(log2 R)) (the printed 'min' read as max, since
    min(1, .) would never exceed one type); prices 3, 6, 9; 30 and 86 actions
    at 4 and 12 resources."""
    for R, rd, A in ((4, 2, 30), (12, 3, 86), (1, 1, 9), (2, 1, 16)):
        cfg = W.variant_config(R=R, N=10, E=1)
        assert cfg["R_d"] == rd == max(1, int(math.floor(math.log2(R))))
        assert cfg["prices"][:3] == [3, 6, 9] and cfg["P"] == 3 and cfg["K"] == 0
        assert cfg["skill_mode"] == 3
        assert W.num_actions(cfg) == A == oe.num_actions(R, 3)
