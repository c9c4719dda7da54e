"""Pins of the oracle's acceptance words (Sec. II-B and Sec. III): dyadic
digits, the and/or fold, per-site thresholds and the canonical draw layout."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

DYADIC = [0.5, 0.75, 0.25, 0.9375, 0.625, 0.1875, 0.0625, 0.96875, 0.34375, 1 / 64, 63 / 64]


@pytest.mark.parametrize("r", DYADIC + [0.0, 1.0, 2.0**-32, 1 - 2.0**-32, 0.123046875])
def test_digits_reconstruct_r(orc, r):
    n, b, one = orc.dyadic_digits(r)
    if r == 1.0:
        assert one and n == 0
        return
    assert not one
    assert sum(Fraction(bi, 2**i) for i, bi in enumerate(b, start=1)) == Fraction(r)
    assert n == 0 or b[-1] == 1  # n is the position of the last 1 digit


@pytest.mark.parametrize("r", [0.93, 0.07, 0.95, 0.1, 1 / 3, math.pi / 4])
def test_non_dyadic_detected(orc, r):
    assert orc.dyadic_digits(r) is None


@pytest.mark.parametrize("r", DYADIC + [0.0])
def test_fold_exact_probability_by_enumeration(orc, r):
    """With draw i set to bit i of the bit index, the 64 bit positions run
    through every combination of n <= 6 fair bits, so the fraction of set
    bits in the folded word is exactly the acceptance probability."""
    n, _, _ = orc.dyadic_digits(r)
    assert n <= 6
    pos = np.arange(64, dtype=np.uint64)
    draws = [int(np.bitwise_or.reduce(((pos >> np.uint64(i)) & np.uint64(1)) << pos)) for i in range(n)]
    w = orc.fold(r, draws)
    assert Fraction(bin(w).count("1"), 64) == Fraction(r)


def test_fold_one_is_all_ones(orc):
    assert orc.fold(1.0, []) == 2**64 - 1


def test_thresholds_golden_and_exact(orc):
    with open(os.path.join(HERE, "golden", "thresholds.txt")) as f:
        rows = [line.split() for line in f if line.strip() and not line.startswith("#")]
    for r_s, T_s in rows:
        r = float(r_s)
        exact = min(math.floor(Fraction(r) * 2**32), 2**32)
        assert orc.threshold(r) == exact == int(T_s)


@pytest.mark.parametrize("seed,t,parity", [(3, 0, 0), (3, 4999, 1), (2**40 + 17, 123, 0)])
def test_persite_words_follow_canonical_draws(orc, seed, t, parity):
    """Bit b of the per-site word is [u < T] with u lane b&3 of call b>>2 at
    counter (g, t, 2*(b>>2)+parity, 0)."""
    p, q = 0.93, 0.07
    g0, cnt = 1000, 4
    xp, xq = orc.acceptance_words(seed, t, parity, g0, cnt, p, q)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    Tp, Tq = orc.threshold(p), orc.threshold(q)
    for i in range(cnt):
        ep = eq = 0
        for b in range(64):
            u = int(orc.philox4x32_10([g0 + i, t, 2 * (b >> 2) + parity, 0], key)[b & 3])
            ep |= (u < Tp) << b
            eq |= (u < Tq) << b
        assert int(xp[i]) == ep and int(xq[i]) == eq


@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("p,q", [(0.75, 0.25), (0.9375, 0.0), (0.5, 0.5), (1.0, 0.25), (0.625, 0.0),
                                 (0.5, 0.0), (0.34375, 0.5)])
def test_mask_words_follow_canonical_draws(orc, p, q, parity):
    """Draw k of word g in half-step `parity` of MCS t is lanes 0|1 (k even)
    or 2|3 (k odd) of the call with counter (g, t, 2*(k>>1) + parity, 0); for
    an odd number n of draws the last one (k = n-1) is taken from the call
    (g, t, n-1, 0) in both half-steps, lanes 0|1 in the even one and 2|3 in
    the odd one, so that each call's 128 bits are all used."""
    seed, t, g0 = 7, 31, 12
    xp, xq = orc.acceptance_words(seed, t, parity, g0, 3, p, q)
    n = max(orc.dyadic_digits(p)[0], orc.dyadic_digits(q)[0])
    key = [seed, 0]
    for i in range(3):
        draws = []
        for k in range(n):
            if n % 2 == 1 and k == n - 1:
                o = orc.philox4x32_10([g0 + i, t, n - 1, 0], key)
                lo, hi = (o[0], o[1]) if parity == 0 else (o[2], o[3])
            else:
                o = orc.philox4x32_10([g0 + i, t, 2 * (k >> 1) + parity, 0], key)
                lo, hi = (o[0], o[1]) if k % 2 == 0 else (o[2], o[3])
            draws.append(int(lo) | (int(hi) << 32))
        assert int(xp[i]) == orc.fold(p, draws)
        assert int(xq[i]) == orc.fold(q, draws)


def test_half_draws_of_one_mcs_share_one_call(orc):
    """p = 1/2 (one draw): the even and the odd half-step of an MCS take the
    two halves of one Philox call, and no two half-steps or MCS share a word."""
    seed, t, g0, n = 5, 9, 0, 16
    e, _ = orc.acceptance_words(seed, t, 0, g0, n, 0.5, 0.0)
    o, _ = orc.acceptance_words(seed, t, 1, g0, n, 0.5, 0.0)
    e2, _ = orc.acceptance_words(seed, t + 1, 0, g0, n, 0.5, 0.0)
    for i in range(n):
        out = orc.philox4x32_10([g0 + i, t, 0, 0], [seed, 0])
        assert int(e[i]) == int(out[0]) | (int(out[1]) << 32)
        assert int(o[i]) == int(out[2]) | (int(out[3]) << 32)
    words = [int(x) for x in list(e) + list(o) + list(e2)]
    assert len(set(words)) == 3 * n


def test_forced_persite_at_dyadic_r(orc):
    xp, _ = orc.acceptance_words(1, 2, 0, 0, 2, 0.5, 0.0, force_persite=True)
    xm, _ = orc.acceptance_words(1, 2, 0, 0, 2, 0.5, 0.0, force_persite=False)
    assert not np.array_equal(xp, xm)  # different draws by design


@pytest.mark.parametrize("p,q,persite", [(0.5, 0.0, False), (0.75, 0.25, False), (0.9375, 0.0, False),
                                         (0.1875, 0.0, False), (0.93, 0.07, True), (0.5, 0.0, True)])
def test_bit_frequency_within_5_sigma(orc, p, q, persite):
    cnt = 4096
    xp, xq = orc.acceptance_words(99, 10, 1, 0, cnt, p, q, force_persite=persite)
    nbits = 64 * cnt
    for words, r in ((xp, p), (xq, q)):
        ones = int(np.unpackbits(words.view(np.uint8)).sum())
        sigma = math.sqrt(nbits * r * (1 - r)) or 1.0
        assert abs(ones - nbits * r) <= 5 * sigma, (r, ones / nbits)


def test_persite_threshold_is_strict(orc):
    """A site whose uniform u equals the threshold is rejected (u < T), and
    accepted once T = u + 1."""
    seed, t, parity, g, b = 11, 3, 1, 2, 37
    u = int(orc.philox4x32_10([g, t, 2 * (b >> 2) + parity, 0], [seed, 0])[b & 3])
    at = orc.acceptance_words(seed, t, parity, g, 1, u / 2**32, 0.0, force_persite=True)[0][0]
    above = orc.acceptance_words(seed, t, parity, g, 1, (u + 1) / 2**32, 0.0, force_persite=True)[0][0]
    assert (int(at) >> b) & 1 == 0
    assert (int(above) >> b) & 1 == 1
