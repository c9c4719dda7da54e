"""Light-cone patches: a patch with a frozen border reproduces the full-torus
evolution at every site farther than 2T from its border after T MCS."""
import numpy as np
import pytest


@pytest.mark.parametrize("x0,y0,p,q,persite", [
    (0, 0, 0.75, 0.25, False),      # holds the origin
    (100, 90, 0.9375, 0.0, False),  # straddles the periodic seam in x and y
    (30, 5, 0.93, 0.07, True),
])
def test_patch_matches_full_torus(orc, x0, y0, p, q, persite):
    X, Y, T = 128, 128, 6
    m = 2 * T + 1
    PX, PY = 40 + 2 * m, 36 + 2 * m
    full = orc.flat(X, Y)
    orc.run(full, T, p, q, seed=77, force_persite=persite)
    patch = orc.flat_patch(X, Y, x0, y0, PX, PY)
    orc.run(patch, T, p, q, seed=77, force_persite=persite)
    ys = (y0 + np.arange(PY)) % Y
    xs = (x0 + np.arange(PX)) % X
    inner = (slice(m, PY - m), slice(m, PX - m))
    ref_sx = full.sx[np.ix_(ys, xs)][inner]
    ref_sy = full.sy[np.ix_(ys, xs)][inner]
    ref_H = full.H[np.ix_(ys, xs)][inner]
    assert np.array_equal(patch.sx[inner], ref_sx)
    assert np.array_equal(patch.sy[inner], ref_sy)
    assert np.array_equal(patch.H[inner], ref_H)
    # and the frozen border really did make the outer ring differ
    assert not np.array_equal(patch.H, full.H[np.ix_(ys, xs)])
