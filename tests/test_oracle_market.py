"""Pins of the oracle's market clearing (Sec. 3 "Trading", Appendix A):
brute-force greedy matching, the crossing-count formula, exhaustive small
books, and the properties every clearing must leave behind (CPU only)."""
import itertools

import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import env as oe

PRICES = [2, 4, 6, 8, 10, 12]


def brute_force_clear(orders, r, prices):
    """Evaluate the best remaining bid against the best remaining ask, one
    pair at a time, by linear scans (high bids / low asks first, then older,
    then by the random key, then agent id)."""
    alive = [j for j, o in enumerate(orders) if o[2] == r]
    filled, paid = {}, {}

    def bid_key(j):
        a, s, _, p, t0, key = orders[j]
        return (-prices[p], t0, key, a)

    def ask_key(j):
        a, s, _, p, t0, key = orders[j]
        return (prices[p], t0, key, a)

    while True:
        bids = [j for j in alive if orders[j][1] == 0]
        asks = [j for j in alive if orders[j][1] == 1]
        if not bids or not asks:
            break
        b = min(bids, key=bid_key)
        s = min(asks, key=ask_key)
        if prices[orders[b][3]] < prices[orders[s][3]]:
            break
        later = b if (orders[b][4], orders[b][5], orders[b][0]) > (orders[s][4], orders[s][5], orders[s][0]) else s
        q = prices[orders[later][3]]
        filled[b] = filled[s] = 1
        paid[b] = paid[s] = q
        alive.remove(b)
        alive.remove(s)
    return filled, paid


def crossing_count(orders, r, prices):
    """k = max over price levels of min(#bids >= level, #asks <= level)."""
    bids = [prices[o[3]] for o in orders if o[2] == r and o[1] == 0]
    asks = [prices[o[3]] for o in orders if o[2] == r and o[1] == 1]
    return max([0] + [min(sum(b >= lv for b in bids), sum(a <= lv for a in asks)) for lv in prices])


def check_book(orders, prices, r=0):
    k, filled, paid, partner = oe.clear_orders(orders, r, prices)
    bf, bp = brute_force_clear(orders, r, prices)
    assert k == crossing_count(orders, r, prices)
    assert sorted(j for j in range(len(orders)) if filled[j]) == sorted(bf)
    for j in bf:
        assert paid[j] == bp[j]
    # what stays is uncrossed
    rest_b = [prices[o[3]] for j, o in enumerate(orders) if o[2] == r and o[1] == 0 and not filled[j]]
    rest_a = [prices[o[3]] for j, o in enumerate(orders) if o[2] == r and o[1] == 1 and not filled[j]]
    if rest_b and rest_a:
        assert max(rest_b) < min(rest_a)
    # each pair: bid >= ask, the trade price lies between them and is one of the two
    for j in range(len(orders)):
        if filled[j] and orders[j][1] == 0:
            s = partner[j]
            pb, ps = prices[orders[j][3]], prices[orders[s][3]]
            assert pb >= ps and paid[j] in (pb, ps) and paid[s] == paid[j]
    # other resources untouched
    for j, o in enumerate(orders):
        if o[2] != r:
            assert not filled[j]
    return k


def test_exhaustive_small_books():
    """Every book of up to 3 bids and 3 asks over 3 price levels and 3 ages."""
    prices = [3, 6, 9]
    rng = np.random.default_rng(3)
    levels = [(p, t0) for p in range(3) for t0 in range(3)]
    n_books = 0
    for nb in range(4):
        for na in range(4):
            for bids in itertools.combinations_with_replacement(levels, nb):
                for asks in itertools.combinations_with_replacement(levels, na):
                    orders = []
                    agent = 0
                    for p, t0 in bids:
                        orders.append((agent, 0, 0, p, t0, int(rng.integers(0, 2 ** 32))))
                        agent += 1
                    for p, t0 in asks:
                        orders.append((agent, 1, 0, p, t0, int(rng.integers(0, 2 ** 32))))
                        agent += 1
                    check_book(orders, prices)
                    n_books += 1
    assert n_books > 10000


def test_price_rule_placed_last():
    """Appendix A: a matched pair trades at the price of the later order."""
    # resting ask at 4 (t0 = 0), new bid at 10 (t0 = 1): the bid is later -> 10
    orders = [(0, 1, 0, 1, 0, 5), (1, 0, 0, 4, 1, 9)]
    k, filled, paid, _ = oe.clear_orders(orders, 0, PRICES)
    assert k == 1 and paid[0] == paid[1] == PRICES[4]
    # resting bid at 10 (t0 = 0), new ask at 4 (t0 = 1): the ask is later -> 4
    orders = [(0, 0, 0, 4, 0, 5), (1, 1, 0, 1, 1, 9)]
    k, filled, paid, _ = oe.clear_orders(orders, 0, PRICES)
    assert k == 1 and paid[0] == PRICES[1]
    # same step: the larger random key counts as placed later
    orders = [(0, 0, 0, 4, 3, 100), (1, 1, 0, 1, 3, 50)]
    assert oe.clear_orders(orders, 0, PRICES)[2][0] == PRICES[4]
    orders = [(0, 0, 0, 4, 3, 10), (1, 1, 0, 1, 3, 50)]
    assert oe.clear_orders(orders, 0, PRICES)[2][0] == PRICES[1]


def test_priority_price_then_age_then_key():
    # two bids at the same price: the older one trades with the single ask
    orders = [(0, 0, 0, 3, 5, 1), (1, 0, 0, 3, 2, 99), (2, 1, 0, 0, 6, 7)]
    _, filled, _, _ = oe.clear_orders(orders, 0, PRICES)
    assert list(filled) == [0, 1, 1]
    # same price and age: the smaller key wins
    orders = [(0, 0, 0, 3, 2, 50), (1, 0, 0, 3, 2, 49), (2, 1, 0, 0, 6, 7)]
    _, filled, _, _ = oe.clear_orders(orders, 0, PRICES)
    assert list(filled) == [0, 1, 1]
    # a higher bid beats an older one
    orders = [(0, 0, 0, 2, 0, 0), (1, 0, 0, 3, 9, 99), (2, 1, 0, 0, 10, 7)]
    _, filled, _, _ = oe.clear_orders(orders, 0, PRICES)
    assert list(filled) == [0, 1, 1]


order_st = st.tuples(st.integers(0, 1), st.integers(0, 2), st.integers(0, 5), st.integers(0, 6),
                     st.integers(0, 2 ** 32 - 1))


@settings(max_examples=400, deadline=None)
@given(st.lists(order_st, min_size=0, max_size=14))
def test_random_books_multi_resource(raw):
    orders = [(i, s, r, p, t0, key) for i, (s, r, p, t0, key) in enumerate(raw)]
    for r in range(3):
        check_book(orders, PRICES, r)
