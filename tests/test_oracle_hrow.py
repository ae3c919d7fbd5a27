"""Pins for the order of the oracle's inverse-Hessian row products (u = H y
and p = -H g of Sec. III-B, Alg. 4).  The paper fixes no summation order; the
oracle takes fused multiply-add chains over blocks of 16 consecutive columns
with the block sums added pairwise.  The constructed cases below have exact
values that follow from IEEE round-to-nearest-even alone and differ for every
other plausible order (one chain, blocks of another size, block sums added
left to right, another pairwise split), so a mistake in any part of the order
fails one of them.  Integer data and a rounding-error bound against exact
rational arithmetic pin the products themselves (no term dropped, doubled or
taken from the wrong index)."""
from fractions import Fraction

import numpy as np
import pytest

BIG = 2.0 ** 53  # 2^53 + 1 is a tie that rounds to 2^53; 2^53 + 2 is exact


def _row(d, ones_at):
    v = np.zeros(d)
    for i, x in ones_at.items():
        v[i] = x
    return np.ones(d), v


@pytest.mark.parametrize("d, entries, expect", [
    # one block: a chain, 2^53 + 1 + 1 -> 2^53 (pairwise would give 2^53 + 2)
    (16, {0: BIG, 1: 1.0, 2: 1.0}, BIG),
    # the 1s in the second block: 2^53 + (1 + 1) (one chain would give 2^53)
    (32, {0: BIG, 16: 1.0, 17: 1.0}, BIG + 2.0),
    # a block of 8 would split cols 8, 9 from col 0: here they share a chain
    (32, {0: BIG, 8: 1.0, 9: 1.0}, BIG),
    # four blocks (2^53, 0, 1, 1): (b0 + b1) + (b2 + b3) = 2^53 + 2
    # (left to right over the blocks would give 2^53)
    (64, {0: BIG, 32: 1.0, 48: 1.0}, BIG + 2.0),
    # three blocks split 2 | 1: (2^53 + 1) + 1 = 2^53 (a 1 | 2 split gives 2^53 + 2)
    (40, {0: BIG, 16: 1.0, 32: 1.0}, BIG),
    # thirteen blocks split 8 | 5, the 5 as 4 | 1: with 2^53 in block 8 and 1s
    # in blocks 11 and 12, (b8 + .. + b11) absorbs one 1 and the sum then
    # absorbs the other: 2^53 (a 1 | 4 split would give 2^53 + 2)
    (200, {128: BIG, 176: 1.0, 192: 1.0}, BIG),
    # 1s in blocks 8 and 9 pair before meeting 2^53 in the left half: 2^53 + 2
    (200, {0: BIG, 130: 1.0, 150: 1.0}, BIG + 2.0),
    # a 1 in each half: each absorbed in turn, 2^53
    (200, {0: BIG, 16: 1.0, 192: 1.0}, BIG),
])
def test_hrow_order_constructed(oracle_mod, d, entries, expect):
    h, v = _row(d, entries)
    assert oracle_mod.hrow_dot(h, v) == expect
    # the row operand and the vector operand play symmetric roles
    assert oracle_mod.hrow_dot(v, h) == expect


@pytest.mark.parametrize("d", [1, 2, 15, 16, 17, 31, 33, 50, 64, 65, 129, 200, 256])
def test_hrow_integers_exact(oracle_any, d):
    rng = np.random.default_rng(100 + d)
    h = rng.integers(-64, 65, d).astype(np.float64)
    v = rng.integers(-64, 65, d).astype(np.float64)
    exact = int(np.dot(h.astype(np.int64), v.astype(np.int64)))
    assert oracle_any.hrow_dot(h, v) == float(exact)


@pytest.mark.parametrize("d", [3, 16, 50, 200])
def test_hrow_error_bound(oracle_any, d):
    # default build: n roundings along a chain of 16 plus ceil(log2 blocks)
    # levels of adds; plain build: one unfused chain of d products and d - 1
    # adds: |computed - exact| <= gamma * sum |h_c v_c|, gamma = k u / (1 - k u)
    rng = np.random.default_rng(7 + d)
    for _ in range(20):
        h = rng.standard_normal(d) * np.exp(rng.uniform(-5, 5, d))
        v = rng.standard_normal(d)
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(h, v))
        nb = -(-d // 16)
        k = min(d, 16) + int(np.ceil(np.log2(nb))) if nb > 1 else min(d, 16)
        if oracle_any.plain:
            k = d
        u = 2.0 ** -53
        bound = k * u / (1 - k * u) * float(sum(abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(h, v)))
        got = oracle_any.hrow_dot(h, v)
        assert abs(Fraction(got) - exact) <= Fraction(bound)


def test_hrow_empty(oracle_any):
    assert oracle_any.hrow_dot(np.zeros(0), np.zeros(0)) == 0.0


@pytest.mark.parametrize("d, entries, expect", [
    # one chain over the whole row: every 1 after 2^53 is absorbed
    (16, {0: BIG, 1: 1.0, 2: 1.0}, BIG),
    (32, {0: BIG, 16: 1.0, 17: 1.0}, BIG),
    (64, {0: BIG, 32: 1.0, 48: 1.0}, BIG),
    (200, {0: BIG, 130: 1.0, 150: 1.0}, BIG),
    # 1s before 2^53 are summed first: (1 + 1) + 2^53 = 2^53 + 2
    (40, {3: 1.0, 9: 1.0, 39: BIG}, BIG + 2.0),
])
def test_hrow_plain_is_one_chain(d, entries, expect):
    from oracle import oracle as O
    h, v = _row(d, entries)
    assert O.hrow_dot(h, v, plain=True) == expect


def test_hrow_plain_products_are_rounded():
    """The plain build rounds every product before adding it: with
    h = (-1, 1 + 2^-30) and v = (1 + 2^-29, 1 + 2^-30) the second product
    1 + 2^-29 + 2^-60 rounds to 1 + 2^-29 and the sum is 0; a fused
    multiply-add keeps the 2^-60 (the default build's chain)."""
    from oracle import oracle as O
    h = np.array([-1.0, 1.0 + 2.0 ** -30])
    v = np.array([1.0 + 2.0 ** -29, 1.0 + 2.0 ** -30])
    assert O.hrow_dot(h, v, plain=True) == 0.0
    assert O.hrow_dot(h, v) == 2.0 ** -60
