"""Closed-form evolutions from the flat surface (h = (x+y)&1, every even site
a minimum): deterministic growth for p = 1, q = 0; deterministic removal for
p = 0, q = 1; nothing for p = q = 0."""
import numpy as np
import pytest

SIZES = [(4, 4), (8, 16), (64, 8), (128, 128), (256, 4), (1024, 8)]


@pytest.mark.parametrize("X,Y", SIZES)
def test_p1_q0(orc, X, Y):
    st = orc.flat(X, Y)
    flat = (st.sx.copy(), st.sy.copy())
    par = np.add.outer(np.arange(Y), np.arange(X)) & 1
    N = X * Y
    for t in range(1, 6):
        ser, _ = orc.run(st, 1, 1.0, 0.0, seed=42, series=True)
        h = orc.heights(st)
        np.testing.assert_array_equal(h, 2 * t + par)
        assert st.h0 == 2 * t
        assert np.array_equal(st.sx, flat[0]) and np.array_equal(st.sy, flat[1])
        Nn, s1, s2, w2 = orc.moments(st)
        # sum h = N (2t + 1/2), sum h^2 = N (4t^2 + 2t + 1/2), W^2 = 1/4
        assert (Nn, 2 * s1, 2 * s2) == (N, N * (4 * t + 1), N * (8 * t * t + 4 * t + 1))
        assert w2 == 0.25
        assert tuple(ser[0]) == (s1, s2)


def test_p1_after_even_halfstep_all_slopes_inverted(orc):
    X, Y = 16, 8
    st = orc.flat(X, Y)
    W = 1
    ones = np.full(Y * W, 2**64 - 1, np.uint64)
    zero = np.zeros(Y * W, np.uint64)
    sx0, sy0 = st.sx.copy(), st.sy.copy()
    orc.halfstep_xi(st, 0, ones, zero)
    assert np.array_equal(st.sx, 1 - sx0) and np.array_equal(st.sy, 1 - sy0)
    assert st.h0 == 2


@pytest.mark.parametrize("X,Y", SIZES)
def test_p0_q1(orc, X, Y):
    st = orc.flat(X, Y)
    par = np.add.outer(np.arange(Y), np.arange(X)) & 1
    N = X * Y
    for t in range(1, 5):
        orc.run(st, 1, 0.0, 1.0, seed=1)
        h = orc.heights(st)
        # even sites are minima and never removed in the first half-step; the
        # odd maxima drop to -1, then everything alternates downwards
        np.testing.assert_array_equal(h, -2 * (t - 1) - par)
        assert st.h0 == -2 * (t - 1)
        Nn, s1, s2, w2 = orc.moments(st)
        assert 2 * s1 == -N * (4 * (t - 1) + 1)
        assert w2 == 0.25
    st1 = orc.flat(X, Y)
    orc.run(st1, 1, 0.0, 1.0, seed=1)
    assert orc.moments(st1)[1] == -N // 2


@pytest.mark.parametrize("X,Y", [(8, 8), (256, 16)])
def test_p0_q0_identity(orc, X, Y):
    st = orc.flat(X, Y)
    orc.run(st, 3, 0.5, 0.5, seed=2)
    before = st.copy()
    orc.run(st, 10, 0.0, 0.0, seed=2)
    assert np.array_equal(st.sx, before.sx) and np.array_equal(st.sy, before.sy)
    assert st.h0 == before.h0 and st.t == before.t + 10
