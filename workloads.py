"""Synthetic workloads: configuration tables and seeded input generators.

This module holds no arithmetic of the economy or of the learner.  It only
names the shapes of the five synthetic economies (shaped like the paper's
Table 2: 100 agents, 1000-step episodes, 100-step tax periods) and draws
seeded inputs that both the GPU library and the CPU oracle consume unchanged
(action arrays for small cases, policy weights, minibatch permutations).
Randomness that the economy itself draws (skills, gathering luck, order tie
keys) is not here: each side derives it from the counter-based generator.
"""
from __future__ import annotations

import copy
import math

import numpy as np

GOV_LEVELS = 21  # tax levels 0 %, 5 %, ..., 100 %


def default_cutoffs(p_tax: int, k: int) -> list[int]:
    """Bracket thresholds (the paper does not print its own): (P_tax / 2) * 2^b."""
    return [(p_tax // 2) * (1 << b) for b in range(max(k - 1, 0))]


def default_prices(p: int) -> list[int]:
    """Price grid 2, 4, ..., 2P (Table 2 lists 2, 4, 6, 8, 10 for P = 5)."""
    return [2 * (i + 1) for i in range(p)]


def env_config(E=1, N=4, R=2, P=10, X=10, max_orders=15, P_tax=10, K=7, T=100, R_kappa=2, R_d=2,
               kappa_c=10, start_coin=15, labor_gather=20, labor_craft=20, labor_trade=1,
               allow_noop=1, eta=0.27, omega=1.0, prices=None, cutoffs=None, seed=0, skill_mode=0):
    cfg = dict(E=E, N=N, R=R, P=P, X=X, max_orders=max_orders, P_tax=P_tax, K=K, T=T,
               R_kappa=R_kappa, R_d=R_d, kappa_c=kappa_c, start_coin=start_coin,
               labor_gather=labor_gather, labor_craft=labor_craft, labor_trade=labor_trade,
               allow_noop=allow_noop, eta=eta, omega=omega, seed=seed, skill_mode=skill_mode)
    cfg["prices"] = list(prices) if prices is not None else default_prices(P)
    cfg["cutoffs"] = list(cutoffs) if cutoffs is not None else default_cutoffs(P_tax, K)
    return cfg


SKILL_NORMAL, SKILL_GROWTH = 1, 2


def variant_config(R: int, N: int = 100, E: int = 1, X: int = 30, T: int = 1000, seed: int = 0):
    """The multi-agent experiments' economy (Sec. 5): R resources, taxes off,
    R_d = max(1, floor(log2 R)), trade prices 3, 6 and 9, skills near 1 with
    spread 1 that grow with use; otherwise Table 2 (order lifetime 30)."""
    return env_config(E=E, N=N, R=R, P=3, X=X, P_tax=100, K=0, T=T, R_d=max(1, int(math.floor(math.log2(R)))),
                      prices=[3, 6, 9], seed=seed, skill_mode=SKILL_NORMAL | SKILL_GROWTH)


def num_actions(cfg) -> int:
    return 2 + cfg["R"] + 2 * cfg["R"] * cfg["P"]


def obs_dim(cfg) -> int:
    return 7 + 7 * cfg["R"] + cfg["K"]


def gov_obs_dim(cfg) -> int:
    return 3 * (3 + cfg["R"]) + cfg["K"] + 1 + 4 * cfg["R"]


def obs_stride(cfg) -> int:
    return (obs_dim(cfg) + 7) // 8 * 8


def mask_words(cfg) -> int:
    return (num_actions(cfg) + 31) // 32


def obs_scales(cfg) -> dict:
    """Float32 scale of every observation feature group (inputs to both sides)."""
    f32 = np.float32
    return dict(coin=float(f32(2.0 ** -7)), labor=float(f32(2.0 ** -11)), orders=float(f32(0.125)),
                res=float(f32(2.0 ** -4)), skill=float(f32(2.0 ** -16)), rate=float(f32(0.05)),
                phase=float(f32(1.0) / f32(cfg["P_tax"])),
                price=float(f32(1.0) / f32(cfg["prices"][-1])),
                count=float(f32(1.0) / f32(cfg["N"])))


# ---------------------------------------------------------------------------
# The five synthetic workloads.
# ---------------------------------------------------------------------------
WORKLOADS = {
    # parity case: one economy, 4 agents, 2 resources, 10 prices, 7 brackets, 100 steps
    "econ_e1_n4": dict(env=env_config(E=1, N=4, R=2, P=10, X=10, P_tax=10, K=7, T=100), steps=100),
    # env-only throughput: 1024 economies x 100 agents, 3 resources, 20 prices
    "econ_e1024_n100": dict(env=env_config(E=1024, N=100, R=3, P=20, X=10, P_tax=100, K=7, T=1000),
                            steps=1000),
    # rollout + PPO: 4096 x 100 with a 35 -> 256 -> 256 -> (125 + 1) policy
    "econ_e4096_n100_ppo": dict(env=env_config(E=4096, N=100, R=3, P=20, X=10, P_tax=100, K=7, T=1000),
                                hidden=256, rollout=128, epochs=4, minibatches=8, gamma=0.99,
                                lam=0.95, clip=0.2, vf_coef=0.25, vclip=10.0, ent_coef=0.1,
                                lr=5e-4),
    # uneven populations: 512 economies, N_e in 10..500
    "econ_e512_uneven": dict(env=env_config(E=512, N=500, R=3, P=20, X=10, P_tax=100, K=7, T=1000),
                             n_min=10, n_max=500, steps=1000),
    # large population / large action space: 256 x 1000, 5 resources, 50 prices
    "econ_e256_n1000_ppo": dict(env=env_config(E=256, N=1000, R=5, P=50, X=10, P_tax=100, K=7, T=1000),
                                hidden=512, rollout=256, epochs=4, minibatches=8, gamma=0.99,
                                lam=0.95, clip=0.2, vf_coef=0.25, vclip=10.0, ent_coef=0.1,
                                lr=5e-4),
}


def workload(name: str) -> dict:
    return copy.deepcopy(WORKLOADS[name])


def uneven_populations(E: int, n_min: int, n_max: int, seed: int = 0) -> np.ndarray:
    """Per-economy population sizes, uniform over n_min..n_max (fixed seed)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x4E53]))
    return rng.integers(n_min, n_max + 1, size=E).astype(np.int32)


def uniform_actions(cfg, steps: int, E: int | None = None, seed: int = 0):
    """Seeded uniform action arrays [steps][E][N] and government levels
    [steps][E][K] for small cases (both sides read the same arrays)."""
    E = cfg["E"] if E is None else E
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xAC7]))
    act = rng.integers(0, num_actions(cfg), size=(steps, E, cfg["N"])).astype(np.int32)
    gov = rng.integers(0, GOV_LEVELS, size=(steps, E, max(cfg["K"], 1))).astype(np.int32)
    return act, gov


def policy_weights(d_in: int, hidden: int, n_act: int, seed: int = 0) -> dict:
    """Float32 MLP weights d_in -> hidden -> hidden -> (n_act logits + 1 value),
    N(0, 1/fan_in), zero biases.  W[k][n] maps input k to output n."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x3E16]))

    def layer(k, n):
        return (rng.standard_normal((k, n)) / math.sqrt(k)).astype(np.float32)

    return dict(W1=layer(d_in, hidden), b1=np.zeros(hidden, np.float32),
                W2=layer(hidden, hidden), b2=np.zeros(hidden, np.float32),
                W3=layer(hidden, n_act + 1), b3=np.zeros(n_act + 1, np.float32))


def affine_permutation(M: int, epoch: int, seed: int = 0):
    """Multiplier and offset of the row shuffle j -> (a j + c) mod M used to
    cut an epoch into minibatches (a is coprime with M)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5EED, epoch]))
    while True:
        a = int(rng.integers(1, max(M, 2)))
        if math.gcd(a, M) == 1:
            break
    c = int(rng.integers(0, max(M, 1)))
    return a, c


def gov_obs_scales(cfg) -> np.ndarray:
    """Float32 scale of every government observation feature (the layout of
    ej_env_observe: mean, std, median of coin, period income, labor and each
    inventory; the K rates; the phase; best bid, best ask, #bids, #asks per
    resource).  Inputs to both sides."""
    R, K = cfg["R"], cfg["K"]
    stats = [2.0 ** -7, 2.0 ** -6, 2.0 ** -11] + [2.0 ** -4] * R
    s = []
    for v in stats:
        s += [v, v, v]
    s += [1.0] * K + [1.0]
    for _ in range(R):
        s += [1.0 / cfg["prices"][cfg["P"] - 1]] * 2 + [1.0 / cfg["N"]] * 2
    return np.asarray(s, np.float32)


def synthetic_obs(M: int, D: int, Ds: int, seed: int = 0) -> np.ndarray:
    """Observation rows as bf16 bit patterns [M, Ds]: values k/16 with
    k in -40..40 (exact in bf16), zero padding beyond D."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x0B5]))
    v = (rng.integers(-40, 41, size=(M, D)) / 16.0).astype(np.float32)
    bits = np.zeros((M, Ds), np.uint16)
    bits[:, :D] = (v.view(np.uint32) >> 16).astype(np.uint16)
    return bits


def synthetic_masks(M: int, A: int, seed: int = 0, p_allow: float = 0.4) -> np.ndarray:
    """Action-mask words [M, ceil(A/32)]; every row allows at least one action."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x3A5C]))
    allow = rng.random((M, A)) < p_allow
    allow[np.arange(M), rng.integers(0, A, size=M)] = True
    W = (A + 31) // 32
    words = np.zeros((M, W), np.uint32)
    for a in range(A):
        words[:, a // 32] |= allow[:, a].astype(np.uint32) << np.uint32(a % 32)
    return words
