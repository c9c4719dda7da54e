"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for
bit in slopes, origin height, heights and int64 sums."""
import sys

import numpy as np
import pytest

import lattice_util as U

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


def gpu_state(lat):
    torch.cuda.synchronize()
    return lat.slopes.cpu().numpy().view(np.uint64).reshape(2, 2, lat.Y, lat.W)


def assert_same(orc, lat, st, heights=True, moments=True):
    S = gpu_state(lat)
    ref = orc.pack(st)
    if not np.array_equal(S, ref):
        bad = np.argwhere(S != ref)
        raise AssertionError(f"slopes differ in {len(bad)} words, first {bad[:5].tolist()}")
    t, h0 = lat.meta()
    assert (t, h0) == (st.t, st.h0)
    if heights:
        np.testing.assert_array_equal(lat.heights().cpu().numpy(), orc.heights(st))
    if moments:
        assert lat.roughness()[:3] == orc.moments(st)[:3]


def test_device_philox_matches_oracle(orc, sca):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, (512, 4), dtype=np.uint64)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [5, 1000, 7, 0], [2**25 - 1, 1999, 31, 0]]
    keys = [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (42, 0), (0xA4093822, 0x299F31D0)]
    for k0, k1 in keys:
        dev = torch.from_numpy(ctr.astype(np.uint32).view(np.int32)).cuda()
        out = sca.debug_philox(dev, k0, k1).cpu().numpy().view(np.uint32)
        for i in range(len(ctr)):
            assert list(out[i]) == list(orc.philox4x32_10(ctr[i], [k0, k1])), (i, k0, k1)


SIZES = [(4, 4), (8, 4), (4, 8), (16, 16), (64, 32), (128, 8), (256, 64), (512, 16), (1024, 8), (2048, 4),
         (4096, 4), (8192, 4), (16384, 4), (32768, 4), (65536, 4), (131072, 4)]


@pytest.mark.parametrize("X,Y", SIZES)
def test_flat_init(orc, sca, X, Y):
    lat = sca.Lattice(X, Y, seed=1)
    assert_same(orc, lat, orc.flat(X, Y))


PROBS = [  # p, q, force_persite
    (0.5, 0.0, False), (0.75, 0.25, False), (0.9375, 0.0, False), (1.0, 0.0, False), (0.0, 1.0, False),
    (0.93, 0.07, False), (0.5, 0.0, True), (0.3, 0.0, False), (1.0, 0.25, False), (3 * 2.0**-32 + 0.5, 0.0, False),
]


@pytest.mark.parametrize("X,Y", SIZES)
@pytest.mark.parametrize("p,q,persite", PROBS)
def test_parity_matrix(orc, sca, X, Y, p, q, persite):
    _say(f"[parity] X={X} Y={Y} p={p} q={q} persite={persite}")
    seed = 1000 + X + 3 * Y
    n = 7
    lat = sca.Lattice(X, Y, seed=seed)
    lat.step(n, p, q, force_persite=persite)
    st = orc.flat(X, Y)
    orc.run(st, n, p, q, seed=seed, force_persite=persite)
    assert_same(orc, lat, st, heights=(X * Y <= 1 << 16))


def test_successive_steps_mixed(orc, sca):
    X, Y, seed = 256, 32, 99
    lat = sca.Lattice(X, Y, seed=seed)
    st = orc.flat(X, Y)
    for n, p, q, ps in [(3, 0.5, 0.0, False), (1, 0.93, 0.07, False), (4, 0.75, 0.25, False), (0, 0.1, 0.1, False),
                        (2, 0.5, 0.5, True), (5, 1.0, 0.0, False)]:
        lat.step(n, p, q, force_persite=ps)
        orc.run(st, n, p, q, seed=seed, force_persite=ps)
        assert_same(orc, lat, st)


def test_small_workload_full(orc, sca):
    """128 x 128, p = 1/2, q = 0, 1000 MCS, seed 1: the sums of h and h^2 after
    every MCS and the final state."""
    from paper_1606_00310_amd.inputs import SMALL as w

    _say("[small] full run")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    st = orc.flat(w.X, w.Y)
    ser, _ = orc.run(st, w.n_mcs, w.p, w.q, seed=w.seed, series=True)
    for i in range(w.n_mcs):
        lat.step(1, w.p, w.q)
        _, s1, s2, _ = lat.roughness()
        assert (s1, s2) == tuple(ser[i]), i
    assert_same(orc, lat, st)


@pytest.mark.parametrize("parity", [0, 1])
def test_exhaustive_4x4_direct(orc, sca, parity):
    """Every 4x4 surface, 16 acceptance patterns each (all 256 covered across
    the surfaces), through the injection hook of the 4x4 (partial-word) kernel."""
    S = U.enumerate_torus_surfaces(4, 4)
    rng = np.random.default_rng(parity)
    npat = 16
    pats = np.stack([rng.permutation(256)[:npat] for _ in S])          # [990, npat]
    pats[:, 0] = np.arange(len(S)) % 256
    B = len(S) * npat
    h = np.repeat(S, npat, axis=0)
    sx = np.empty((B, 4, 4), np.uint8)
    sy = np.empty((B, 4, 4), np.uint8)
    for i, s in enumerate(S):
        a, b = U.slopes_from_heights(s)
        sx[i * npat:(i + 1) * npat] = a
        sy[i * npat:(i + 1) * npat] = b
    xi = np.zeros((B, 4), np.uint64)
    flat_pat = pats.ravel()
    for y in range(4):
        for k in range(2):
            xi[:, y] |= (((flat_pat >> (2 * y + k)) & 1).astype(np.uint64)) << np.uint64(k)
    init_packed = np.stack([orc.pack(orc.State(4, 4, sx[i], sy[i])) for i in range(B)])  # [B,2,2,4,1]
    H = h.astype(np.int32).copy()
    h0 = np.zeros(B, np.int64)
    esx, esy = sx.copy(), sy.copy()
    orc.halfstep_xi_batch(4, 4, esx, esy, H, h0, parity, xi, xi)

    lat = sca.Lattice(4, 4, seed=0)
    init_dev = torch.from_numpy(init_packed.view(np.int64)).cuda()
    xi_dev = torch.from_numpy(xi.view(np.int64)).cuda()
    out = torch.empty_like(init_dev)
    out_h0 = torch.empty(B, dtype=torch.int64, device="cuda")
    for i in range(B):
        lat.slopes.copy_(init_dev[i])
        lat.aux.zero_()
        lat.debug_halfstep(parity, xi_dev[i], xi_dev[i])
        out[i].copy_(lat.slopes)
        out_h0[i] = lat.aux[0]
    got = out.cpu().numpy().view(np.uint64)
    for i in range(B):
        ref = orc.pack(orc.State(4, 4, esx[i], esy[i]))
        assert np.array_equal(got[i], ref), (i // npat, flat_pat[i])
    np.testing.assert_array_equal(out_h0.cpu().numpy(), h0)


@pytest.mark.parametrize("parity", [0, 1])
def test_exhaustive_4x4_tiled(orc, sca, parity):
    """Each 4x4 surface tiled over a 512 x 512 torus (four words per row),
    the 128 x 128 copies carrying all 256 acceptance patterns, so every
    surface meets every pattern in the multi-word kernel."""
    S = U.enumerate_torus_surfaces(4, 4)
    Lb = 512
    cy, cx = np.meshgrid(np.arange(Lb // 4), np.arange(Lb // 4), indexing="ij")
    pat = (cy * (Lb // 4) + cx) % 256                                     # pattern of each copy
    # per-site acceptance: site (x, y) of this parity in copy (y//4, x//4) is
    # 4x4 sublattice site (y%4, (x%4)//2) -> pattern bit 2*(y%4) + (x%4)//2
    yy, xx = np.meshgrid(np.arange(Lb), np.arange(Lb), indexing="ij")
    bit = 2 * (yy % 4) + (xx % 4) // 2
    acc = ((pat[yy // 4, xx // 4] >> bit) & 1).astype(bool) & (((xx + yy) & 1) == parity)
    bits = np.zeros((Lb, Lb // 2), bool)
    for y in range(Lb):
        xs = np.arange(Lb)[((np.arange(Lb) + y) & 1) == parity]
        bits[y, xs >> 1] = acc[y, xs]
    xi = U.pattern_to_words(Lb, Lb, parity, bits)
    xi_dev = torch.from_numpy(xi.view(np.int64)).cuda()

    # expected 4x4 heights per (surface, pattern).  A site's height change
    # depends only on its own copy (its neighbours' heights repeat with the
    # tiling), so the tiled result is the per-copy heights; the slope bits on
    # the bonds between copies then follow from those heights.
    B = len(S) * 256
    sx = np.empty((B, 4, 4), np.uint8)
    sy = np.empty((B, 4, 4), np.uint8)
    for i, s in enumerate(S):
        a, b = U.slopes_from_heights(s)
        sx[i * 256:(i + 1) * 256] = a
        sy[i * 256:(i + 1) * 256] = b
    H4 = np.repeat(S, 256, axis=0).astype(np.int32)
    xi4 = np.zeros((B, 4), np.uint64)
    pp = np.tile(np.arange(256), len(S))
    for y in range(4):
        for k in range(2):
            xi4[:, y] |= (((pp >> (2 * y + k)) & 1).astype(np.uint64)) << np.uint64(k)
    orc.halfstep_xi_batch(4, 4, sx, sy, H4, None, parity, xi4, xi4)

    lat = sca.Lattice(Lb, Lb, seed=0)
    for i, s in enumerate(S):
        a, b = U.slopes_from_heights(np.tile(s, (Lb // 4, Lb // 4)))
        lat.slopes.copy_(torch.from_numpy(orc.pack(orc.State(Lb, Lb, a, b)).view(np.int64)))
        lat.debug_halfstep(parity, xi_dev, xi_dev)
        got = gpu_state(lat)
        big_h = H4[i * 256 + pat].transpose(0, 2, 1, 3).reshape(Lb, Lb)   # [128,128,4,4] -> rows, cols
        ea, eb = U.slopes_from_heights(big_h)
        ref = orc.pack(orc.State(Lb, Lb, ea, eb))
        assert np.array_equal(got, ref), i


@pytest.mark.parametrize("X,Y,p,q,persite", [(4, 4, 0.5, 0.0, False), (64, 128, 0.75, 0.25, False),
                                              (512, 64, 0.93, 0.07, False), (2048, 32, 0.9375, 0.0, False),
                                              (16384, 8, 0.5, 0.5, True)])
def test_moments_heights_autocorr(orc, sca, X, Y, p, q, persite):
    seed = 5
    lat = sca.Lattice(X, Y, seed=seed)
    st = orc.flat(X, Y)
    lat.step(9, p, q, force_persite=persite)
    orc.run(st, 9, p, q, seed=seed, force_persite=persite)
    snap = lat.snapshot()
    st_s = st.copy()
    lat.step(6, p, q, force_persite=persite)
    orc.run(st, 6, p, q, seed=seed, force_persite=persite)
    N, s1, s2, w2 = lat.roughness()
    oN, os1, os2, ow2 = orc.moments(st)
    assert (N, s1, s2) == (oN, os1, os2) and w2 == ow2
    a = lat.autocorr(snap)
    b = orc.autocorr(st, st_s)
    assert a[:4] == b[:4] and a[4] == b[4]
    # windows of rows
    for y0, ny in [(0, 1), (Y // 2, min(3, Y - Y // 2)), (Y - 1, 1)]:
        np.testing.assert_array_equal(lat.heights(y0, ny).cpu().numpy(), orc.heights(st)[y0:y0 + ny])


def test_medium_reduced(orc, sca):
    """2^12 x 2^12, p = 0.75, q = 0.25 (two shared draws): W^2 at the log-spaced
    times up to 20 MCS and the state at 20 MCS."""
    from paper_1606_00310_amd.inputs import MEDIUM as w, log_times

    _say("[medium] 20 MCS")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    st = orc.flat(w.X, w.Y, track_heights=False)
    t = 0
    for T in [x for x in log_times() if x <= 20]:
        lat.step(T - t, w.p, w.q)
        orc.run(st, T - t, w.p, w.q, seed=w.seed)
        t = T
        g = lat.roughness()
        o = orc.moments(st)
        assert g[:3] == o[:3] and g[3] == o[3], T
    assert np.array_equal(gpu_state(lat), orc.pack(st))


def test_errors_leave_state(orc, sca):
    lat = sca.Lattice(64, 64, seed=1)
    lat.step(3, 0.5)
    before = gpu_state(lat).copy()
    for args in [(1, -0.1, 0.0), (1, 0.5, 1.5), (1, float("nan"), 0.0), (-1, 0.5, 0.0)]:
        with pytest.raises(sca.ScaError):
            lat.step(*args)
    assert np.array_equal(gpu_state(lat), before) and lat.t == 3
    with pytest.raises(sca.ScaError):
        lat.heights(60, 5)
