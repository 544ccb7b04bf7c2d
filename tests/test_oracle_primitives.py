"""Pins of the oracle's primitive definitions against the paper's worked
examples, closed forms, brute force and library routines (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import env as oe

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


# --- counter-based generator: the library implementation of Philox4x64-10 ---
def test_philox_matches_numpy_bitgenerator():
    """numpy.random.Philox is Philox4x64-10; it increments its 256-bit
    counter before each block, so block c is produced from counter c - 1."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)
        ctr = rng.integers(1, 2 ** 63, size=4, dtype=np.uint64)
        prev = ctr.copy()
        prev[0] -= np.uint64(1)
        bg = np.random.Philox(key=key, counter=prev)
        assert np.array_equal(oe.philox4x64(ctr, key), bg.random_raw(4).astype(np.uint64))


def test_philox_counter_zero_and_carry():
    key = np.array([0, 0], np.uint64)
    # counter 0 = numpy counter (2^256 - 1) + 1 with full carry
    ones = np.array([2 ** 64 - 1] * 4, np.uint64)
    bg = np.random.Philox(key=key, counter=ones)
    assert np.array_equal(oe.philox4x64(np.zeros(4, np.uint64), key), bg.random_raw(4).astype(np.uint64))


# --- tax (Sec. 3 "Setting tax rates") ---
def test_tax_worked_example():
    ex = GOLDEN["tax_example"]
    assert oe.bracket_tax(ex["income"], ex["levels_5pct"], ex["cutoffs"]) == ex["tax"]


def _tax_per_unit(income, levels, cutoffs):
    """Brute force: every unit of income pays the rate of the bracket it falls in."""
    total = 0
    for c in range(max(income, 0)):
        b = sum(1 for x in cutoffs if c >= x)
        total += levels[b]
    return total // 20


def test_tax_brute_force_and_special_cases():
    rng = np.random.default_rng(1)
    for _ in range(300):
        K = int(rng.integers(1, 8))
        cut = sorted(set(int(x) for x in rng.integers(1, 400, size=K - 1)))
        K = len(cut) + 1
        lv = [int(x) for x in rng.integers(0, 21, size=K)]
        inc = int(rng.integers(-50, 900))
        assert oe.bracket_tax(inc, lv, cut) == _tax_per_unit(inc, lv, cut)
    cut = [5, 10, 20, 40, 80, 160]
    for inc in (0, 1, 7, 99, 1000):
        assert oe.bracket_tax(inc, [0] * 7, cut) == 0
        assert oe.bracket_tax(inc, [20] * 7, cut) == inc
    for k in range(21):
        assert oe.bracket_tax(137, [k], []) == (k * 137) // 20


# --- action space (Sec. 5) ---
def test_action_counts_from_paper():
    for case in GOLDEN["action_counts"]["cases"]:
        assert oe.num_actions(case["R"], case["P"]) == case["A"]


# --- Gini and social welfare (Eqs. (3)-(5)) ---
def test_gini_numerator_brute_force():
    rng = np.random.default_rng(2)
    for n in (1, 2, 3, 5, 17, 100):
        for _ in range(20):
            x = rng.integers(0, 1000, size=n)
            brute = sum(abs(int(a) - int(b)) for a in x for b in x)  # sum_i sum_j |xi - xj|
            assert 2 * oe.gini_numerator(x) == brute


def test_gini_special_cases():
    n = 10
    assert oe.gini_numerator([7] * n) == 0
    x = [0] * (n - 1) + [50]
    g = oe.gini_numerator(x) / (n * 50)
    assert g == pytest.approx((n - 1) / n, abs=1e-15)


def test_social_welfare_closed_forms():
    x = [3, 9, 27, 81]
    S = sum(x)
    G = sum(abs(a - b) for a in x for b in x) / (2 * len(x) * S)
    assert oe.social_welfare(x, 1.0) == pytest.approx(S * (1 - G), rel=1e-14)
    assert oe.social_welfare(x, 0.0) == pytest.approx(S, rel=1e-15)
    assert oe.social_welfare([5, 5, 5], 1.0) == pytest.approx(15.0, rel=1e-15)
    assert oe.social_welfare([0, 0], 1.0) == 0.0


# --- utility (Eq. (1)) ---
def test_utility_special_cases():
    eta = 0.27
    assert oe.utility(1, 0, eta) == 0.0
    for L in (1, 20, 377):
        assert oe.utility(1, L, eta) == pytest.approx(-L / 20.0, abs=1e-15)
        assert oe.utility(40, L, eta) - oe.utility(40, 0, eta) == pytest.approx(-L / 20.0, abs=1e-12)
    # eta = 0 makes the utility linear in coin
    for Cc in (0, 1, 15, 999):
        assert oe.utility(Cc, 0, 0.0) == pytest.approx(Cc - 1.0, abs=1e-12)
    # marginal utility ~ C^-eta, decreasing (concavity)
    d = [oe.utility(c + 1, 0, eta) - oe.utility(c, 0, eta) for c in (10, 100, 1000)]
    assert d[0] > d[1] > d[2]
    assert d[2] == pytest.approx(1000.5 ** -eta, rel=1e-4)
    assert oe.utility(0, 0, eta) == pytest.approx(-1.0 / (1.0 - eta), abs=1e-15)
