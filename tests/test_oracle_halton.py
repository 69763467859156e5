"""Pins for the oracle's radical inverses and full-screen enumeration (Appendix A.2).

Each check is fixed by the mathematics of the Halton sequence, not by the
oracle's own formula: textbook values, the base-2 bit-reversal identity,
b^k -> b^-(k+1), single digits, stratification of the first b^m points, and
exact rational arithmetic on random 64-bit indices.
"""
import os
import random
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "halton_textbook.txt")


def _exact_bits(i, b, f):
    """floor(2^32 * sum pi(d_k) b^-(k+1)) with Python rationals."""
    x = Fraction(0)
    scale = Fraction(1, b)
    while i:
        i, d = divmod(i, b)
        x += ((f * d) % b) * scale
        scale /= b
    return (x * (1 << 32)).numerator // (x * (1 << 32)).denominator


def test_textbook_values(orc):
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        b, i, num, den = map(int, line.split())
        want = (num << 32) // den
        assert orc.ri_bits(i, b, 1) == want, (b, i)


def test_base2_is_bit_reversal(orc):
    rng = random.Random(7)
    for _ in range(2000):
        i = rng.getrandbits(32)
        rev = int(f"{i:032b}"[::-1], 2)
        assert orc.ri_bits(i, 2, 1) == rev
    # bits above 32 only affect digits beyond 2^-32
    for _ in range(200):
        i = rng.getrandbits(64)
        assert orc.ri_bits(i, 2, 1) == int(f"{i & 0xffffffff:032b}"[::-1], 2)


@pytest.mark.parametrize("b", [2, 3, 5, 7, 11, 13, 97, 673])
def test_powers_and_single_digits(orc, b):
    k = 0
    while b ** k < 2 ** 63:
        assert orc.ri_bits(b ** k, b, 1) == (1 << 32) // b ** (k + 1)
        k += 1
    for i in range(b):
        assert orc.ri_bits(i, b, 1) == (i << 32) // b
        f = orc.scramble_mult(b) if b > 3 else 1
        assert orc.ri_bits(i, b, f) == (((f * i) % b) << 32) // b


def test_scramble_is_permutation(orc):
    for d in range(2, 140):
        b = orc.dim_base(d)
        f = orc.scramble_mult(b)
        perm = sorted((f * a) % b for a in range(b))
        assert perm == list(range(b)), b
        assert (f * 0) % b == 0


@pytest.mark.parametrize("b,m", [(2, 10), (3, 6), (5, 4), (7, 3), (673, 1), (11, 3)])
def test_stratification(orc, b, m):
    """The first b^m points are exactly the grid {k b^-m}, each once, scrambled or not."""
    grid = sorted(((k << 32) // b ** m) for k in range(b ** m))
    for f in (1, orc.scramble_mult(b)):
        got = sorted(orc.ri_bits(i, b, f) for i in range(b ** m))
        assert got == grid


def test_exact_against_rationals(orc):
    rng = random.Random(11)
    for _ in range(3000):
        i = rng.getrandbits(rng.choice([8, 16, 34, 48, 64]))
        d = rng.randrange(2, 140)
        b = orc.dim_base(d)
        f = orc.scramble_mult(b)
        assert orc.ri_bits(i, b, f) == _exact_bits(i, b, f), (i, b)
        assert orc.ri_bits(i, b, 1) == _exact_bits(i, b, 1), (i, b)


def test_dim_bases_are_primes(orc):
    want = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29]
    assert [orc.dim_base(d) for d in range(10)] == want
    assert orc.dim_base(121) == 673  # 122nd prime: last dimension at depth 16


def _digits_rev(v, b, n):
    r = 0
    for _ in range(n):
        v, d = divmod(v, b)
        r = r * b + d
    return r


@pytest.mark.parametrize("W,H", [(5, 4), (128, 128), (1920, 1080), (3840, 2160)])
def test_enumeration_selects_pixel(orc, W, H):
    """floor(2^k RI_2(i)) = px and floor(3^l RI_3(i)) = py for every pass j."""
    k, l, S = orc.enum_params(W, H)
    assert 2 ** k >= W > 2 ** (k - 1) and 3 ** l >= H > 3 ** (l - 1) and S == 2 ** k * 3 ** l
    rng = random.Random(W * 7 + H)
    pts = [(0, 0), (W - 1, H - 1)] + [(rng.randrange(W), rng.randrange(H)) for _ in range(60)]
    for px, py in pts:
        for j in (0, 1, 7, 1023):
            i = orc.pixel_index(W, H, px, py, j)
            x = Fraction(_exact_bits(i, 2, 1), 1 << 32)  # first 32 bits suffice for k <= 12
            assert int(x * 2 ** k) == px
            y3 = Fraction(0)
            v, sc = i, Fraction(1, 3)
            for _ in range(l):
                v, dd = divmod(v, 3)
                y3 += dd * sc
                sc /= 3
            assert int(y3 * 3 ** l) == py
            assert i % S == orc.pixel_index(W, H, px, py, 0)


def test_enumeration_is_bijection_small(orc):
    W, H = 5, 4
    k, l, S = orc.enum_params(W, H)
    seen = set()
    for py in range(H):
        for px in range(W):
            i0 = orc.pixel_index(W, H, px, py, 0)
            assert 0 <= i0 < S
            assert i0 % 2 ** k == _digits_rev(px, 2, k) and i0 % 3 ** l == _digits_rev(py, 3, l)
            seen.add(i0)
    assert len(seen) == W * H


def test_film_offsets_are_remaining_digits(orc):
    """Dim 0/1 samples equal frac(2^k RI_2(i)) and frac(3^l RI_3(i)) to 24+ bits."""
    W, H = 1920, 1080
    k, l, S = orc.enum_params(W, H)
    rng = random.Random(3)
    for _ in range(100):
        px, py, j = rng.randrange(W), rng.randrange(H), rng.randrange(2000)
        i = orc.pixel_index(W, H, px, py, j)
        b0 = int(orc.sample_bits(np.array([i]), np.array([0]), W, H)[0])
        b1 = int(orc.sample_bits(np.array([i]), np.array([1]), W, H)[0])
        # exact fractional parts from rationals with enough digits
        x = Fraction(0)
        v, sc = i, Fraction(1, 2)
        while v:
            v, dd = divmod(v, 2)
            x += dd * sc
            sc /= 2
        fx = x * 2 ** k - int(x * 2 ** k)
        assert b0 == int(fx * 2 ** 32)
        y = Fraction(0)
        v, sc = i, Fraction(1, 3)
        while v:
            v, dd = divmod(v, 3)
            y += dd * sc
            sc /= 3
        fy = y * 3 ** l - int(y * 3 ** l)
        assert b1 == int(fy * 2 ** 32)
