"""The oracle's MCS loop draws the acceptance words of the even half-step of
MCS t from the counter (g, t, 2j+0, 0) and then those of the odd half-step
from (g, t, 2j+1, 0), except for the shared last draw of an odd number n of
draws, which both half-steps take from (g, t, n-1, 0) (Sec. I-A: one MCS is
the even, then the odd half-step; the counter layout is the documented
convention of the random stream).  One
MCS of ``run`` from an absolute time t0 != 0 must therefore equal two
half-steps with the words ``acceptance_words(seed, t0, 0)`` and
``acceptance_words(seed, t0, 1)`` injected, in that order.  A counter off by
one MCS, a swapped parity or a half-step order reversed fails here; the
closed forms (draw-free) and the conservation tests cannot see such a slip."""
import numpy as np
import pytest


def _random_state(orc, X, Y, t0):
    st = orc.flat(X, Y)
    orc.run(st, 5, 0.5, 0.5, seed=99)   # minima and maxima everywhere
    st.t = t0                           # the absolute MCS index the next MCS runs at
    return st


def _injected_mcs(orc, st, seed, p, q, persite):
    W = orc.words_per_row(st.X)
    for parity in (0, 1):
        xp, xq = orc.acceptance_words(seed, st.t, parity, 0, st.Y * W, p, q, force_persite=persite)
        orc.halfstep_xi(st, parity, xp, xq)
    st.t += 1


@pytest.mark.parametrize("p,q,persite", [(0.75, 0.25, False), (0.9375, 0.0, False), (0.93, 0.07, False),
                                         (0.5, 0.5, True), (0.5, 0.0, False), (0.625, 0.125, False)])
@pytest.mark.parametrize("X,Y,t0", [(256, 16, 37), (64, 32, 1), (512, 8, 4000000000)])
def test_one_mcs_equals_two_injected_halfsteps(orc, p, q, persite, X, Y, t0):
    seed = 0x1234_5678_9ABC_DEF1
    ref = _random_state(orc, X, Y, t0)
    got = ref.copy()
    orc.run(got, 1, p, q, seed=seed, force_persite=persite)
    for n in range(2):  # and a second MCS, at t0 + 1
        _injected_mcs(orc, ref, seed, p, q, persite)
        if n == 0:
            assert np.array_equal(got.sx, ref.sx) and np.array_equal(got.sy, ref.sy)
            assert np.array_equal(got.H, ref.H) and (got.h0, got.t) == (ref.h0, ref.t)
            orc.run(got, 1, p, q, seed=seed, force_persite=persite)
    assert np.array_equal(got.sx, ref.sx) and np.array_equal(got.sy, ref.sy)
    assert np.array_equal(got.H, ref.H) and (got.h0, got.t) == (ref.h0, ref.t)


def test_swapped_or_shifted_words_differ(orc):
    """The pin above can fail: the words of the other parity, or of the next
    MCS, give a different state on the same input."""
    X, Y, t0, seed, p, q = 256, 16, 37, 5, 0.75, 0.25
    W = orc.words_per_row(X)
    base = _random_state(orc, X, Y, t0)
    right = base.copy()
    orc.run(right, 1, p, q, seed=seed)
    for wrong in ((t0, 1, 0), (t0 + 1, 0, 1), (t0 - 1, 0, 1)):
        st = base.copy()
        for parity, src_par in zip((0, 1), wrong[1:]):
            xp, xq = orc.acceptance_words(seed, wrong[0], src_par, 0, Y * W, p, q)
            orc.halfstep_xi(st, parity, xp, xq)
        assert not np.array_equal(st.H, right.H), wrong


@pytest.mark.parametrize("p,q,persite", [(0.75, 0.25, False), (0.93, 0.07, False)])
def test_patch_from_late_time_uses_the_same_stream(orc, p, q, persite):
    """A light-cone patch started at t0 != 0 from a copy of the torus state
    follows the injected-word evolution of the whole torus in its interior."""
    X, Y, t0, T, seed = 128, 128, 1234, 3, 2024
    m = 2 * T + 1
    x0, y0, PX, PY = 100, 120, 30 + 2 * m, 26 + 2 * m   # straddles both seams
    full = _random_state(orc, X, Y, t0)
    ys = (y0 + np.arange(PY)) % Y
    xs = (x0 + np.arange(PX)) % X
    patch = orc.flat_patch(X, Y, x0, y0, PX, PY)
    patch.sx[:] = full.sx[np.ix_(ys, xs)]
    patch.sy[:] = full.sy[np.ix_(ys, xs)]
    patch.H[:] = full.H[np.ix_(ys, xs)]
    patch.t = t0
    orc.run(patch, T, p, q, seed=seed, force_persite=persite)
    for _ in range(T):
        _injected_mcs(orc, full, seed, p, q, persite)
    inner = (slice(m, PY - m), slice(m, PX - m))
    assert np.array_equal(patch.H[inner], full.H[np.ix_(ys, xs)][inner])
    assert np.array_equal(patch.sx[inner], full.sx[np.ix_(ys, xs)][inner])
    assert np.array_equal(patch.sy[inner], full.sy[np.ix_(ys, xs)][inner])
