"""The temporally blocked passes (all half-steps of `depth` MCS in one sweep,
out of place) against the two-launch form and the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_00310_amd as P

    P.lib()
    return P


PROBS = [(0.5, 0.0, False), (0.75, 0.25, False), (0.9375, 0.0, False), (1.0, 0.0, False), (0.0, 1.0, False),
         (0.93, 0.07, False), (0.5, 0.5, True)]


@pytest.mark.parametrize("X,Y", [(8192, 64), (16384, 128), (32768, 64), (65536, 64), (8192, 256), (131072, 32)])
@pytest.mark.parametrize("p,q,persite", PROBS)
@pytest.mark.parametrize("depth", [1, 2, 3, 4])
def test_fused_vs_oracle(orc, sca, X, Y, p, q, persite, depth):
    _say(f"[fused] X={X} Y={Y} p={p} q={q} depth={depth}")
    seed = 31 + X + Y
    n = 6
    lat = sca.Lattice(X, Y, seed=seed)
    lat.set_blocking(depth, 8)
    lat.step(n, p, q, force_persite=persite)
    st = orc.flat(X, Y, track_heights=False)
    orc.run(st, n, p, q, seed=seed, force_persite=persite)
    torch.cuda.synchronize()
    assert np.array_equal(lat.slopes.cpu().numpy().view(np.uint64), orc.pack(st))
    assert lat.meta() == (st.t, st.h0)
    assert lat.roughness()[:3] == orc.moments(st)[:3]


DRAW_FREE = [(1.0, 0.0), (0.0, 1.0), (1.0, 1.0)]


@pytest.mark.parametrize("X,Y", [(8192, 32), (16384, 64), (32768, 32), (65536, 32), (131072, 32)])
@pytest.mark.parametrize("p,q", DRAW_FREE + [(0.0, 0.0)])
@pytest.mark.parametrize("depth", [5, 6, 7, 8])
def test_deep_fused_vs_oracle(orc, sca, X, Y, p, q, depth):
    """Passes deeper than 4 MCS (draw-free p, q; lowered to 5 at X = 2^17)."""
    _say(f"[deep] X={X} Y={Y} p={p} q={q} depth={depth}")
    seed = 77 + X + Y
    n = 2 * depth + 3
    lat = sca.Lattice(X, Y, seed=seed)
    lat.set_blocking(depth, 16)
    lat.step(n, p, q)
    st = orc.flat(X, Y, track_heights=False)
    orc.run(st, n, p, q, seed=seed)
    torch.cuda.synchronize()
    assert np.array_equal(lat.slopes.cpu().numpy().view(np.uint64), orc.pack(st))
    assert lat.meta() == (st.t, st.h0)


@pytest.mark.parametrize("p,q", DRAW_FREE + [(0.0, 0.0)])
@pytest.mark.parametrize("depth,band,Y", [(9, 32, 64), (10, 32, 64), (11, 32, 64), (12, 32, 64), (12, 64, 128),
                                          (13, 32, 64), (13, 256, 512)])
def test_deeper_fused_vs_oracle(orc, sca, p, q, depth, band, Y):
    """Passes of 9..13 MCS, which only X = 2^16 runs (one word per lane of a
    512-thread workgroup); two whole passes and a 3-MCS remainder."""
    X = 65536
    _say(f"[deeper] Y={Y} p={p} q={q} depth={depth} band={band}")
    seed = 91 + depth + Y
    n = 2 * depth + 3
    lat = sca.Lattice(X, Y, seed=seed)
    lat.set_blocking(depth, band)
    lat.step(n, p, q)
    st = orc.flat(X, Y, track_heights=False)
    orc.run(st, n, p, q, seed=seed)
    torch.cuda.synchronize()
    assert np.array_equal(lat.slopes.cpu().numpy().view(np.uint64), orc.pack(st))
    assert lat.meta() == (st.t, st.h0)


@pytest.mark.parametrize("depth,band", [(5, 16), (6, 16), (7, 32), (8, 16), (8, 32), (8, 128)])
@pytest.mark.parametrize("n", [16, 17, 41])
def test_deep_fused_equals_unfused(sca, depth, band, n):
    X, Y = 16384, 256
    a = sca.Lattice(X, Y, seed=6)
    b = sca.Lattice(X, Y, seed=6)
    a.set_blocking(depth, band)
    for lat, fuse in ((a, True), (b, False)):
        lat.step(n, 1.0, 0.0, fuse=fuse)
        lat.step(n, 0.9375, 0.0, fuse=fuse)   # random words: the pass depth is lowered to 4
        lat.step(n, 1.0, 1.0, fuse=fuse)
        lat.step(n + 2, 0.0, 1.0, fuse=fuse)
    torch.cuda.synchronize()
    assert torch.equal(a.slopes, b.slopes) and a.meta() == b.meta()


@pytest.mark.parametrize("depth,band", [(1, 4), (1, 16), (1, 64), (2, 4), (2, 8), (2, 32), (3, 8), (3, 64), (4, 8),
                                        (4, 128)])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13])
def test_fused_equals_unfused(sca, depth, band, n):
    X, Y = 16384, 256
    a = sca.Lattice(X, Y, seed=5)
    b = sca.Lattice(X, Y, seed=5)
    a.set_blocking(depth, band)
    a.step(n, 0.9375, 0.0)
    a.step(n + 1, 0.75, 0.25)
    b.step(n, 0.9375, 0.0, fuse=False)
    b.step(n + 1, 0.75, 0.25, fuse=False)
    torch.cuda.synchronize()
    assert torch.equal(a.slopes, b.slopes) and a.meta() == b.meta()


def test_fused_graph_and_disable(sca):
    X, Y = 65536, 128
    a = sca.Lattice(X, Y, seed=9)
    b = sca.Lattice(X, Y, seed=9)
    c = sca.Lattice(X, Y, seed=9)
    a.step(10, 0.5, 0.0, graph=True)
    b.set_blocking(0)
    b.step(10, 0.5, 0.0)
    c.step(10, 0.5, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(a.slopes, b.slopes) and torch.equal(b.slopes, c.slopes)
    assert a.meta() == b.meta() == c.meta()
    for bad in [(1, 12), (14, 32), (-2, 0)]:
        with pytest.raises(sca.ScaError):
            a.set_blocking(*bad)
