"""Parity at the full workload sizes, in the launch configuration bench.py
times: closed forms and invariants that hold at any size, light-cone windows
the oracle computes exactly, and moments recomputed by the oracle from the
GPU's own final state."""
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


def rows_wrapped(lat, y0, ny):
    """Heights of rows y0..y0+ny-1 modulo Y."""
    parts = []
    y = y0 % lat.Y
    left = ny
    while left > 0:
        k = min(left, lat.Y - y)
        parts.append(lat.heights(y, k).cpu().numpy())
        left -= k
        y = 0
    return np.concatenate(parts, axis=0)


def check_valid_rows(h, y0):
    """|dh| = 1 along rows (with the periodic wrap) and between consecutive
    rows, h = x + y (mod 2)."""
    dx = h - np.roll(h, 1, axis=1)
    assert np.all(np.abs(dx) == 1)
    assert np.all(np.abs(np.diff(h, axis=0)) == 1)
    X = h.shape[1]
    par = (np.arange(X)[None, :] + (y0 + np.arange(h.shape[0]))[:, None]) & 1
    assert np.all((h - par) % 2 == 0)


def check_windows(orc, lat, T, p, q, seed, windows, w=48, persite=False):
    m = 2 * T + 1
    for wx, wy in windows:
        _say(f"  window at x={wx} y={wy}")
        x0, y0 = (wx - m) % lat.X, (wy - m) % lat.Y
        patch = orc.flat_patch(lat.X, lat.Y, x0, y0, w + 2 * m, w + 2 * m)
        orc.run(patch, T, p, q, seed=seed, force_persite=persite)
        ref = patch.H[m:m + w, m:m + w]
        got = rows_wrapped(lat, wy, w)
        cols = (wx + np.arange(w)) % lat.X
        np.testing.assert_array_equal(got[:, cols], ref)


def test_headline_p1_full_length(sca):
    """2^16 x 2^16, p = 1, q = 0, all 2000 MCS: the closed form
    h = 2t + ((x+y)&1) after every MCS (slopes back to the flat ones)."""
    from paper_1606_00310_amd.inputs import HEADLINE as w

    _say("[fullsize] 65536^2 p=1 2000 MCS")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    lat.step(w.n_mcs, w.p, w.q)
    t = w.n_mcs
    assert lat.meta() == (t, 2 * t)
    S = lat.slopes
    assert bool((S[:, 0] == 0).all()) and bool((S[:, 1] == -1).all())
    N, s1, s2, w2 = lat.roughness()
    assert (N, 2 * s1, 2 * s2, w2) == (w.sites, w.sites * (4 * t + 1), w.sites * (8 * t * t + 4 * t + 1), 0.25)
    for y0 in (0, 32767, 65534):
        h = lat.heights(y0, 2).cpu().numpy()
        par = (np.arange(w.X)[None, :] + (y0 + np.arange(2))[:, None]) & 1
        np.testing.assert_array_equal(h, 2 * t + par)
    lat.close()


def test_headline_random_windows(orc, sca):
    """2^16 x 2^16 at p = 0.9375 (four-digit mask): 48 x 48 windows after 12 MCS
    against oracle light-cone patches, including the origin and the seams."""
    from paper_1606_00310_amd.inputs import HEADLINE_RANDOM as w

    T = 12
    _say("[fullsize] 65536^2 p=0.9375 windows")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    lat.step(T, w.p, w.q)
    check_windows(orc, lat, T, w.p, w.q, w.seed,
                  [(0, 0), (w.X - 24, w.Y - 24), (12345, 54321), (w.X - 48, 7), (64, 65535)])
    # the origin height agrees with the window holding (0, 0)
    assert lat.meta()[1] == int(lat.heights(0, 1)[0, 0])
    lat.close()


def test_headline_half_windows(orc, sca):
    """2^16 x 2^16 at p = 1/2, the paper's own throughput workload: windows
    after 13 MCS (blocked passes of 4 MCS and a remainder split in two)."""
    from paper_1606_00310_amd.inputs import HEADLINE_HALF as w

    T = 13
    _say("[fullsize] 65536^2 p=0.5 windows")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    lat.step(T, w.p, w.q)
    check_windows(orc, lat, T, w.p, w.q, w.seed, [(0, 0), (w.X - 30, 255), (40000, 65500)])
    assert lat.meta()[1] == int(lat.heights(0, 1)[0, 0])
    lat.close()


def run_sequence_windows(orc, lat, seq, seed, windows, w=40):
    """Runs the (n, p, q) phases of `seq` on the lattice, then checks w x w
    windows of heights against oracle light-cone patches that ran the same
    phases from the flat surface."""
    T = sum(n for n, _, _ in seq)
    for n, p, q in seq:
        plan = lat.plan(n, p, q)
        _say(f"  {n} MCS p={p} q={q}: {plan['n_pass']} x {plan['kernel']}, tails {plan['tail1']}+{plan['tail2']}")
        lat.step(n, p, q)
    m = 2 * T + 1
    for wx, wy in windows:
        _say(f"  window at x={wx} y={wy} (T={T})")
        x0, y0 = (wx - m) % lat.X, (wy - m) % lat.Y
        patch = orc.flat_patch(lat.X, lat.Y, x0, y0, w + 2 * m, w + 2 * m)
        for n, p, q in seq:
            orc.run(patch, n, p, q, seed=seed)
        got = rows_wrapped(lat, wy, w)
        np.testing.assert_array_equal(got[:, (wx + np.arange(w)) % lat.X], patch.H[m:m + w, m:m + w])
    assert lat.meta() == (T, int(lat.heights(0, 1)[0, 0]))


def test_headline_draw_free_passes_from_rough_state(orc, sca):
    """2^16 x 2^16 in the bench's launch configuration, from a rough state (4
    MCS at p = 3/4, q = 1/4): p = 1 for 52 MCS (four 13-MCS passes on 256-row
    bands) and 21 MCS (passes of 11 and 10), p = q = 1 for 26 MCS (the
    general-mask form of the 13-MCS kernel), then p = 1, q = 1/2 for 3 MCS;
    windows against oracle light-cone patches, the origin and both seams
    among them."""
    from paper_1606_00310_amd.inputs import HEADLINE as w

    _say("[fullsize] 65536^2 rough state, then draw-free passes")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    seq = [(4, 0.75, 0.25), (52, 1.0, 0.0), (21, 1.0, 0.0), (26, 1.0, 1.0), (3, 1.0, 0.5)]
    run_sequence_windows(orc, lat, seq, w.seed, [(0, 0), (w.X - 20, w.Y - 20), (31000, 255), (12345, 40000)])
    lat.close()


def test_wide_draw_free_passes_from_rough_state(orc, sca):
    """2^17 x 2^17 from a rough state: p = 1 for 12 MCS (two 6-MCS passes of
    the 1024-thread LDS-window kernel) and 7 MCS (passes of 4 and 3), then
    p = q = 1 for 12 MCS; windows against oracle patches."""
    from paper_1606_00310_amd.inputs import WIDE as w

    _say("[fullsize] 131072^2 rough state, then draw-free passes")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    seq = [(4, 0.75, 0.25), (12, 1.0, 0.0), (7, 1.0, 0.0), (12, 1.0, 1.0)]
    run_sequence_windows(orc, lat, seq, w.seed, [(0, 0), (w.X - 20, 70000), (65536, w.Y - 16)])
    lat.close()


def test_wide_p1_closed_form(sca):
    """2^17 x 2^17 (4 GiB of slopes), p = 1: 6-MCS passes of the LDS-window
    kernel with 1024-thread workgroups; the closed form after 120 MCS."""
    from paper_1606_00310_amd.inputs import WIDE as w

    _say("[fullsize] 131072^2 p=1 120 MCS")
    t = 120
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    lat.step(t, w.p, w.q)
    assert lat.meta() == (t, 2 * t)
    S = lat.slopes
    assert bool((S[:, 0] == 0).all()) and bool((S[:, 1] == -1).all())
    for y0 in (0, 65535, 131070):
        h = lat.heights(y0, 2).cpu().numpy()
        par = (np.arange(w.X)[None, :] + (y0 + np.arange(2))[:, None]) & 1
        np.testing.assert_array_equal(h, 2 * t + par)
    lat.close()


def test_headline_random_full_length_invariants(sca):
    """All 2000 MCS at p = 0.9375 on 2^16 x 2^16: sampled rows remain valid
    octahedron surfaces; moments agree with the sampled heights' bounds."""
    from paper_1606_00310_amd.inputs import HEADLINE_RANDOM as w

    _say("[fullsize] 65536^2 p=0.9375 2000 MCS")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    lat.step(w.n_mcs, w.p, w.q)
    for y0 in (0, 4097, 65533):
        h = rows_wrapped(lat, y0, 3)
        check_valid_rows(h, y0)
    t, h0 = lat.meta()
    assert t == w.n_mcs and h0 == int(lat.heights(0, 1)[0, 0])
    N, s1, s2, w2 = lat.roughness()
    assert N == w.sites and 0.0 < w2 < 1e4
    lat.close()


def test_persite_windows_and_moments(orc, sca):
    """2^14 x 2^14 with p = 0.93, q = 0.07 (per-site 32-bit compares): windows
    after 10 MCS, then moments and two-time sums recomputed by the oracle from
    the GPU's own states."""
    from paper_1606_00310_amd.inputs import PERSITE as w

    _say("[fullsize] 16384^2 persite")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    lat.step(4, w.p, w.q)
    snap = lat.snapshot()
    lat.step(6, w.p, w.q)
    check_windows(orc, lat, 10, w.p, w.q, w.seed, [(0, 0), (w.X - 30, 100), (8000, w.Y - 10)])
    torch.cuda.synchronize()
    words = 4 * w.Y * lat.W
    s_now = orc.unpack(w.X, w.Y, lat.slopes.cpu().numpy().view(np.uint64))
    s_now.h0 = lat.meta()[1]
    snap_np = snap.cpu().numpy()
    s_old = orc.unpack(w.X, w.Y, snap_np[:words].view(np.uint64))
    s_old.h0 = int(snap_np[words])
    assert lat.roughness()[:3] == orc.moments(s_now)[:3]
    assert lat.autocorr(snap)[:4] == orc.autocorr(s_now, s_old)[:4]
    lat.close()


def test_persite_full_length(orc, sca):
    """The whole 5000-MCS per-site run with snapshots at s = 100 and 1000 and
    C(t,s) at the log-spaced times; at the end the oracle recomputes the sums
    from the GPU's states, and C(t,t) equals W^2(t) throughout."""
    from paper_1606_00310_amd.inputs import PERSITE as w, PERSITE_SNAPSHOTS, autocorr_times

    _say("[fullsize] 16384^2 persite 5000 MCS")
    lat = sca.Lattice(w.X, w.Y, seed=w.seed)
    snaps = {}
    times = sorted(set(t for s in PERSITE_SNAPSHOTS for t in autocorr_times(s, w.n_mcs)))
    t = 0
    for T in times:
        lat.step(T - t, w.p, w.q)
        t = T
        if T in PERSITE_SNAPSHOTS:
            snaps[T] = lat.snapshot()
        w2 = lat.roughness()[3]
        for s, sn in snaps.items():
            c = lat.autocorr(sn)
            if s == T:
                assert c[4] == pytest.approx(w2, rel=1e-12, abs=1e-12)
    assert lat.t == w.n_mcs
    torch.cuda.synchronize()
    words = 4 * w.Y * lat.W
    s_now = orc.unpack(w.X, w.Y, lat.slopes.cpu().numpy().view(np.uint64))
    s_now.h0 = lat.meta()[1]
    assert np.all(s_now.sx.sum(axis=1) == w.X // 2) and np.all(s_now.sy.sum(axis=0) == w.Y // 2)
    for s, sn in snaps.items():
        arr = sn.cpu().numpy()
        s_old = orc.unpack(w.X, w.Y, arr[:words].view(np.uint64))
        s_old.h0 = int(arr[words])
        assert lat.autocorr(sn)[:4] == orc.autocorr(s_now, s_old)[:4]
    lat.close()
