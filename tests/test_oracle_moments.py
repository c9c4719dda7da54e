"""Pins of the oracle's height moments and two-time sums against plain
recomputation from heights (Python integers), and their identities."""
import numpy as np
import pytest


def _py_moments(h):
    v = [int(a) for a in h.ravel()]
    return len(v), sum(v), sum(a * a for a in v)


@pytest.mark.parametrize("X,Y,n", [(4, 4, 9), (16, 64, 40), (256, 32, 30)])
def test_moments_vs_python(orc, X, Y, n):
    st = orc.flat(X, Y)
    orc.run(st, n, 0.75, 0.25, seed=5)
    N, s1, s2, w2 = orc.moments(st)
    assert (N, s1, s2) == _py_moments(orc.heights(st))
    from fractions import Fraction
    assert w2 == pytest.approx(float(Fraction(N * s2 - s1 * s1, N * N)), rel=1e-15)


def test_series_matches_moments(orc):
    st = orc.flat(32, 32)
    ref = st.copy()
    ser, _ = orc.run(st, 12, 0.5, 0.0, seed=1, series=True)
    for i in range(12):
        orc.run(ref, 1, 0.5, 0.0, seed=1)
        assert tuple(ser[i]) == orc.moments(ref)[1:3]


def test_autocorr_vs_python_and_identities(orc):
    X, Y = 64, 32
    st = orc.flat(X, Y)
    orc.run(st, 20, 0.9375, 0.0, seed=3)
    snap = st.copy()
    orc.run(st, 15, 0.9375, 0.0, seed=3)
    N, sts, st_, ss, c = orc.autocorr(st, snap)
    ht, hs = orc.heights(st), orc.heights(snap)
    assert N == X * Y
    assert sts == sum(int(a) * int(b) for a, b in zip(ht.ravel(), hs.ravel()))
    assert st_ == int(ht.sum()) and ss == int(hs.sum())
    # C(t,t) = W^2(t)
    n2, s1, s2, w2 = orc.moments(st)
    a = orc.autocorr(st, st)
    assert a[1] == s2 and a[2] == s1 and a[4] == pytest.approx(w2, rel=1e-15)
    # shifting all heights by a constant leaves W^2 and C unchanged
    shifted = st.copy()
    shifted.h0 += 1000
    assert orc.moments(shifted)[3] == pytest.approx(w2, rel=1e-12)
    assert orc.autocorr(shifted, snap)[4] == pytest.approx(c, rel=1e-12)
