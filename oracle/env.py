"""ctypes wrapper of the C economy oracle (econ_oracle.c).

TEST INFRASTRUCTURE: see the package docstring.  The economy's rules live in
the C file; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_MAXR, _MAXP, _MAXK = 16, 128, 16


class OcConfig(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("N", "R", "P", "X", "max_orders", "P_tax", "K", "T", "R_kappa",
                                          "R_d", "kappa_c", "start_coin", "labor_gather", "labor_craft",
                                          "labor_trade", "allow_noop", "skill_mode")] + [
        ("eta", C.c_double), ("omega", C.c_double),
        ("prices", C.c_int32 * _MAXP), ("cutoffs", C.c_int32 * _MAXK)]


class OcOrder(C.Structure):
    _fields_ = [("agent", C.c_int32), ("side", C.c_int32), ("r", C.c_int32), ("p", C.c_int32),
                ("t0", C.c_int32), ("key", C.c_uint32)]


class OcObsScales(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("coin", "labor", "orders", "res", "skill", "rate", "phase",
                                          "price", "count")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        P64, P32, PU16, PU32, PF = (C.POINTER(C.c_uint64), C.POINTER(C.c_int32), C.POINTER(C.c_uint16),
                                    C.POINTER(C.c_uint32), C.POINTER(C.c_float))
        L.oc_philox4x64.argtypes = [P64, P64, P64]
        L.oc_utility.argtypes = [C.c_int64, C.c_int64, C.c_double]
        L.oc_utility.restype = C.c_double
        L.oc_gini_numerator.argtypes = [C.POINTER(C.c_int64), C.c_int32]
        L.oc_gini_numerator.restype = C.c_int64
        L.oc_social_welfare.argtypes = [C.POINTER(C.c_int64), C.c_int32, C.c_double]
        L.oc_social_welfare.restype = C.c_double
        L.oc_bracket_tax.argtypes = [C.c_int64, P32, P32, C.c_int32]
        L.oc_bracket_tax.restype = C.c_int64
        L.oc_num_actions.argtypes = [C.c_int32, C.c_int32]
        L.oc_num_actions.restype = C.c_int32
        L.oc_env_create.argtypes = [C.POINTER(OcConfig), C.c_uint64, C.c_int32]
        L.oc_env_create.restype = C.c_void_p
        L.oc_env_destroy.argtypes = [C.c_void_p]
        L.oc_env_reset.argtypes = [C.c_void_p, C.c_int32]
        L.oc_env_step.argtypes = [C.c_void_p, P32, P32, PF, PF, P32]
        L.oc_clear_orders.argtypes = [C.POINTER(OcOrder), C.c_int32, C.c_int32, P32, P32, P32, P32]
        L.oc_clear_orders.restype = C.c_int32
        L.oc_env_observe.argtypes = [C.c_void_p, C.POINTER(OcObsScales), C.c_int32, PU16, PU32, PF]
        L.oc_env_get_state.argtypes = [C.c_void_p] + [P32] * 11
        L.oc_env_set_state.argtypes = [C.c_void_p] + [P32] * 10
        L.oc_env_invalid_actions.argtypes = [C.c_void_p]
        L.oc_env_invalid_actions.restype = C.c_int64
        L.oc_env_invalid_gov.argtypes = [C.c_void_p]
        L.oc_env_invalid_gov.restype = C.c_int64
        L.oc_random_actions.argtypes = [C.POINTER(OcConfig), C.c_uint64, C.c_int32, C.c_int32, C.c_int32,
                                        P32, P32]
        L.oc_env_run_random.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(C.c_double)]
        L.oc_metrics_len.argtypes = [C.c_int32]
        L.oc_metrics_len.restype = C.c_int32
        L.oc_env_episode_metrics.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def make_config(cfg: dict) -> OcConfig:
    c = OcConfig()
    for n in ("N", "R", "P", "X", "max_orders", "P_tax", "K", "T", "R_kappa", "R_d", "kappa_c",
              "start_coin", "labor_gather", "labor_craft", "labor_trade", "allow_noop"):
        setattr(c, n, int(cfg[n]))
    c.skill_mode = int(cfg.get("skill_mode", 0))
    c.eta = float(cfg["eta"])
    c.omega = float(cfg["omega"])
    for i, v in enumerate(cfg["prices"]):
        c.prices[i] = int(v)
    for i, v in enumerate(cfg["cutoffs"]):
        c.cutoffs[i] = int(v)
    return c


# ---------------------------------------------------------------------------
# primitive definitions
# ---------------------------------------------------------------------------
def philox4x64(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, np.uint64)
    lib().oc_philox4x64(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def sample_uniforms(seed: int, rows, ctr: int, n_chunks: int):
    """The two uniforms per (row, 128-action chunk) of the policy sampler:
    words 2(c mod 2) and 2(c mod 2) + 1 of Philox(seed, purpose 5;
    row, ctr, c / 2, 0); u = (top 24 bits + 1/2) / 2^24."""
    rows = np.asarray(rows, dtype=np.int64)
    u1 = np.zeros((len(rows), n_chunks))
    u2 = np.zeros((len(rows), n_chunks))
    for m, r in enumerate(rows):
        for c in range(n_chunks):
            w = philox4x64([int(r), int(ctr), c // 2, 0], [int(seed), 5])
            u1[m, c] = ((int(w[2 * (c % 2)]) >> 40) + 0.5) / 16777216.0
            u2[m, c] = ((int(w[2 * (c % 2) + 1]) >> 40) + 0.5) / 16777216.0
    return u1, u2


def gov_uniforms(seed: int, rows, ctr: int, K: int) -> np.ndarray:
    """The government sampler's uniform per (economy row, bracket k): word
    k mod 4 of Philox(seed, purpose 6; row, ctr, k / 4, 0),
    u = (top 24 bits + 1/2) / 2^24."""
    rows = np.asarray(rows, dtype=np.int64)
    u = np.zeros((len(rows), K))
    for m, r in enumerate(rows):
        for q in range((K + 3) // 4):
            w = philox4x64([int(r), int(ctr), q, 0], [int(seed), 6])
            for j in range(4):
                if 4 * q + j < K:
                    u[m, 4 * q + j] = ((int(w[j]) >> 40) + 0.5) / 16777216.0
    return u


def utility(coin: int, labor_q: int, eta: float) -> float:
    return lib().oc_utility(int(coin), int(labor_q), float(eta))


def gini_numerator(x) -> int:
    a = np.ascontiguousarray(x, dtype=np.int64)
    return int(lib().oc_gini_numerator(_p(a, C.c_int64), len(a)))


def social_welfare(x, omega: float) -> float:
    a = np.ascontiguousarray(x, dtype=np.int64)
    return float(lib().oc_social_welfare(_p(a, C.c_int64), len(a), float(omega)))


def bracket_tax(income: int, levels, cutoffs) -> int:
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    ct = np.ascontiguousarray(list(cutoffs) + [0], dtype=np.int32)
    return int(lib().oc_bracket_tax(int(income), _p(lv, C.c_int32), _p(ct, C.c_int32), len(lv)))


def num_actions(R: int, P: int) -> int:
    return int(lib().oc_num_actions(R, P))


def clear_orders(orders, r: int, prices):
    """orders: list of (agent, side, r, p, t0, key).  Returns (filled, price, partner) arrays."""
    n = len(orders)
    arr = (OcOrder * max(n, 1))()
    for j, o in enumerate(orders):
        arr[j] = OcOrder(*[int(v) for v in o])
    pr = np.ascontiguousarray(prices, dtype=np.int32)
    filled = np.zeros(max(n, 1), np.int32)
    paid = np.zeros(max(n, 1), np.int32)
    partner = np.zeros(max(n, 1), np.int32)
    k = lib().oc_clear_orders(arr, n, r, _p(pr, C.c_int32), _p(filled, C.c_int32), _p(paid, C.c_int32),
                              _p(partner, C.c_int32))
    return int(k), filled[:n], paid[:n], partner[:n]


# ---------------------------------------------------------------------------
# one economy
# ---------------------------------------------------------------------------
class OracleEnv:
    """One economy (index `e` of a batch) of the oracle."""

    def __init__(self, cfg: dict, e: int = 0, seed: int | None = None, n_agents: int | None = None):
        self.cfg = dict(cfg)
        if n_agents is not None:
            self.cfg["N"] = int(n_agents)
        self.e = e
        self.seed = int(cfg.get("seed", 0) if seed is None else seed)
        self._c = make_config(self.cfg)
        self._h = lib().oc_env_create(C.byref(self._c), self.seed, e)
        self.N, self.R, self.K, self.X = self.cfg["N"], self.cfg["R"], self.cfg["K"], self.cfg["X"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oc_env_destroy(h)
            self._h = None

    def reset(self, ep: int = 0):
        lib().oc_env_reset(self._h, ep)

    def step(self, act, gov):
        a = np.ascontiguousarray(act, dtype=np.int32)
        g = np.ascontiguousarray(list(np.asarray(gov).ravel()) + [0], dtype=np.int32)
        rew = np.zeros(self.N, np.float32)
        grew = np.zeros(1, np.float32)
        done = np.zeros(1, np.int32)
        lib().oc_env_step(self._h, _p(a, C.c_int32), _p(g, C.c_int32), _p(rew, C.c_float),
                          _p(grew, C.c_float), _p(done, C.c_int32))
        return rew, float(grew[0]), int(done[0])

    def state(self) -> dict:
        N, R, X, K = self.N, self.R, self.X, self.K
        sc = np.zeros(2 + max(K, 1), np.int32)
        f = {k: np.zeros(N, np.int32) for k in ("coin_inv", "coin_esc", "labor", "snap", "n_active", "sc")}
        for k in ("res_inv", "res_esc", "sg"):
            f[k] = np.zeros((R, N), np.int32)
        orders = np.zeros((X, N), np.int32)
        lib().oc_env_get_state(self._h, _p(sc, C.c_int32), *[_p(f[k], C.c_int32) for k in (
            "coin_inv", "coin_esc", "labor", "snap", "n_active", "res_inv", "res_esc", "sg", "sc")],
            _p(orders, C.c_int32))
        f["t"], f["ep"], f["rates"] = int(sc[0]), int(sc[1]), sc[2:2 + K].copy()
        f["orders"] = orders
        return f

    def set_state(self, st: dict):
        K = self.K
        sc = np.zeros(2 + max(K, 1), np.int32)
        sc[0], sc[1] = st["t"], st["ep"]
        sc[2:2 + K] = st["rates"]
        arrs = [np.ascontiguousarray(st[k], dtype=np.int32) for k in (
            "coin_inv", "coin_esc", "labor", "snap", "res_inv", "res_esc", "sg", "sc", "orders")]
        lib().oc_env_set_state(self._h, _p(sc, C.c_int32), *[_p(a, C.c_int32) for a in arrs])

    def observe(self, scales: dict, stride: int, with_gov: bool = True):
        N, R, K = self.N, self.R, self.K
        A = num_actions(R, self.cfg["P"])
        W = (A + 31) // 32
        s = OcObsScales(**{k: float(v) for k, v in scales.items()})
        obs = np.zeros((N, stride), np.uint16)
        mask = np.zeros((N, W), np.uint32)
        gdim = 3 * (3 + R) + K + 1 + 4 * R
        gov = np.zeros(gdim, np.float32)
        lib().oc_env_observe(self._h, C.byref(s), stride, _p(obs, C.c_uint16), _p(mask, C.c_uint32),
                             _p(gov, C.c_float) if with_gov else None)
        return obs, mask, gov

    def episode_metrics(self) -> np.ndarray:
        """Record of the last completed episode (layout in econ_oracle.c:
        episode, productivity, equality, government utility, mean and median
        return, action counts per category, trades and price sums per
        resource)."""
        out = np.zeros(lib().oc_metrics_len(self.R), np.float64)
        lib().oc_env_episode_metrics(self._h, _p(out, C.c_double))
        return out

    def invalid_counts(self):
        return int(lib().oc_env_invalid_actions(self._h)), int(lib().oc_env_invalid_gov(self._h))

    def random_actions(self, act_seed: int, t: int | None = None, ep: int | None = None):
        st = self.state()
        t = st["t"] if t is None else t
        ep = st["ep"] if ep is None else ep
        act = np.zeros(self.N, np.int32)
        gov = np.zeros(max(self.K, 1), np.int32)
        lib().oc_random_actions(C.byref(self._c), int(act_seed), self.e, ep, t, _p(act, C.c_int32),
                                _p(gov, C.c_int32))
        return act, gov[:self.K]

    def run_random(self, act_seed: int, steps: int) -> float:
        acc = C.c_double(0.0)
        lib().oc_env_run_random(self._h, int(act_seed), int(steps), C.byref(acc))
        return acc.value


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)
