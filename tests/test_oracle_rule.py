"""Pins of the oracle's half-step against the update rule stated on explicit
heights (Eq. (2)), independent of the slope encoding and of the packing."""
import numpy as np
import pytest

import lattice_util as U


@pytest.fixture(scope="module")
def surfaces_4x4():
    s = U.enumerate_torus_surfaces(4, 4)
    assert len(s) == 990  # zero-winding octahedron surfaces of the 4x4 torus with h(0,0) fixed
    return s


@pytest.mark.parametrize("parity", [0, 1])
def test_exhaustive_4x4(orc, surfaces_4x4, parity):
    """Every 4x4 surface x every acceptance pattern of the 8 sublattice sites:
    990 * 256 half-steps per parity, against the explicit height rule."""
    X = Y = 4
    S = surfaces_4x4
    B = len(S) * 256
    h = np.repeat(S, 256, axis=0)                          # [B, Y, X]
    pat = np.tile(np.arange(256), len(S))                  # acceptance pattern per item
    # sublattice site (y, k) -> pattern bit 2y + k; its x is 2k + (parity ^ (y&1))
    bits = np.zeros((B, Y, X // 2), bool)
    for y in range(Y):
        for k in range(X // 2):
            bits[:, y, k] = (pat >> (2 * y + k)) & 1
    acc = np.zeros((B, Y, X), bool)
    for y in range(Y):
        for k in range(X // 2):
            acc[:, y, 2 * k + (parity ^ (y & 1))] = bits[:, y, k]
    expect = U.height_rule_halfstep(h, parity, acc)

    sx = np.empty((B, Y, X), np.uint8)
    sy = np.empty((B, Y, X), np.uint8)
    for i in range(len(S)):
        a, b = U.slopes_from_heights(S[i])
        sx[i * 256:(i + 1) * 256] = a
        sy[i * 256:(i + 1) * 256] = b
    H = h.astype(np.int32).copy()
    h0 = np.zeros(B, np.int64)
    # canonical words: W = 1, word g = y, bit k
    xi = np.zeros((B, Y), np.uint64)
    for y in range(Y):
        for k in range(X // 2):
            xi[:, y] |= bits[:, y, k].astype(np.uint64) << np.uint64(k)
    orc.halfstep_xi_batch(X, Y, sx, sy, H, h0, parity, xi, xi)
    np.testing.assert_array_equal(H, expect)
    assert np.array_equal(h0, expect[:, 0, 0])
    # slopes still encode the new heights
    for i in range(0, B, 97):
        a, b = U.slopes_from_heights(expect[i])
        assert np.array_equal(sx[i], a) and np.array_equal(sy[i], b)


@pytest.mark.parametrize("X,Y", [(8, 4), (4, 16), (32, 32), (256, 8), (512, 16), (64, 128)])
@pytest.mark.parametrize("parity", [0, 1])
def test_random_states_vs_height_rule(orc, X, Y, parity):
    """Larger and non-square lattices (partial words, several words per
    row): random surfaces reached by random dynamics, random acceptance words,
    one half-step against the explicit rule applied through the canonical
    site -> (word, bit) map."""
    rng = np.random.default_rng(X * 1000 + Y + parity)
    st = orc.flat(X, Y)
    orc.run(st, 7, 0.6, 0.3, seed=int(rng.integers(1 << 30)), force_persite=True)
    h = orc.heights(st)
    W = max(1, X // 128)
    xp = rng.integers(0, 2**63, Y * W, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, Y * W, dtype=np.uint64)
    xq = rng.integers(0, 2**63, Y * W, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, Y * W, dtype=np.uint64)
    acc_p = U.acceptance_grid(X, Y, xp)
    acc_q = U.acceptance_grid(X, Y, xq)
    on = ((np.add.outer(np.arange(Y), np.arange(X))) & 1) == parity
    nb = [np.roll(h, s, axis=a) for s, a in ((1, 1), (-1, 1), (1, 0), (-1, 0))]
    is_min = np.all([n == h + 1 for n in nb], axis=0)
    is_max = np.all([n == h - 1 for n in nb], axis=0)
    expect = h + 2 * (on & is_min & acc_p) - 2 * (on & is_max & acc_q)
    orc.halfstep_xi(st, parity, xp, xq)
    np.testing.assert_array_equal(orc.heights(st), expect)
    np.testing.assert_array_equal(st.H, expect)
