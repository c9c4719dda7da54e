"""Pins of the oracle by invariants the model fixes, for any state reached:
conserved up-slope counts per row and column under periodic boundaries,
height parity, explicit height bookkeeping and the packing round trip."""
import numpy as np
import pytest

import lattice_util as U

CASES = [  # X, Y, p, q, persite, n_mcs
    (4, 4, 0.5, 0.0, False, 50),
    (8, 32, 0.75, 0.25, False, 40),
    (64, 16, 0.93, 0.07, True, 30),
    (128, 64, 0.9375, 0.0, False, 25),
    (256, 32, 0.5, 0.5, False, 20),
    (512, 8, 0.3, 0.6, True, 20),
]


@pytest.mark.parametrize("X,Y,p,q,persite,n", CASES)
def test_conservation_and_bookkeeping(orc, X, Y, p, q, persite, n):
    st = orc.flat(X, Y)
    m0 = orc.moments(st)
    _, cnt = orc.run(st, n, p, q, seed=X + 7 * Y, force_persite=persite, counts=True)
    assert st.t == n
    # up-slopes per row (x) and per column (y) keep their flat values X/2, Y/2
    assert np.all(st.sx.sum(axis=1) == X // 2)
    assert np.all(st.sy.sum(axis=0) == Y // 2)
    h = orc.heights(st)
    # explicit heights tracked by +-2 per update equal the reconstruction
    np.testing.assert_array_equal(st.H, h)
    np.testing.assert_array_equal(U.heights_by_walk(st.sx, st.sy, st.h0), h)
    # every bond still has |dh| = 1 and h = x + y (mod 2)
    U.slopes_from_heights(h)
    assert np.all((h - np.add.outer(np.arange(Y), np.arange(X))) % 2 == 0)
    # sum h grows by 2 per deposition and drops by 2 per removal
    m1 = orc.moments(st)
    assert m1[1] - m0[1] == 2 * (int(cnt[0]) - int(cnt[1]))
    if q == 0.0:
        assert cnt[1] == 0


@pytest.mark.parametrize("X,Y", [(4, 4), (16, 8), (128, 4), (256, 16), (1024, 4)])
def test_pack_roundtrip_and_layout(orc, X, Y):
    st = orc.flat(X, Y)
    orc.run(st, 5, 0.6, 0.2, seed=3, force_persite=True)
    S = orc.pack(st)
    W = max(1, X // 128)
    assert S.shape == (2, 2, Y, W)
    back = orc.unpack(X, Y, S)
    assert np.array_equal(back.sx, st.sx) and np.array_equal(back.sy, st.sy)
    # bit k of word k>>6 of row y, parity array (x+y)&1, holds the site x with x>>1 == k
    rng = np.random.default_rng(0)
    for _ in range(50):
        x, y = int(rng.integers(X)), int(rng.integers(Y))
        pi, k = (x + y) & 1, x >> 1
        assert (int(S[0, pi, y, k >> 6]) >> (k & 63)) & 1 == st.sx[y, x]
        assert (int(S[1, pi, y, k >> 6]) >> (k & 63)) & 1 == st.sy[y, x]
    if X < 128:  # unused bits of a partial word stay zero
        assert np.all(S >> np.uint64(X // 2) == 0)


def test_flat_state_layout(orc):
    """Flat surface: parity-0 words all zero, parity-1 words all valid bits set."""
    for X in (4, 64, 128, 512):
        S = orc.pack(orc.flat(X, 8))
        valid = (1 << min(64, X // 2)) - 1
        assert np.all(S[:, 0] == 0)
        assert np.all(S[:, 1] == np.uint64(valid))


def test_heights_roundtrip_from_random_surface(orc):
    rng = np.random.default_rng(5)
    st = orc.flat(32, 16)
    orc.run(st, 30, 0.7, 0.4, seed=11, force_persite=True)
    h = orc.heights(st) + 2 * int(rng.integers(-50, 50))
    sx, sy = U.slopes_from_heights(h)
    again = orc.State(32, 16, sx, sy, h0=int(h[0, 0]))
    np.testing.assert_array_equal(orc.heights(again), h)
