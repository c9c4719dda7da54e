"""The draw-free temporally blocked passes (p, q in {0, 1}: the register- and
LDS-window kernels that produce the headline rate) against the oracle from
non-uniform states.

From the flat surface with draw-free p, q every site of the updating
sublattice is a minimum (or a maximum) at every half-step, so every bit flips
and a wrong x+ alignment of shifted rows (Fig. 3, Sec. II-B), a wrong y+ row
or a wrong band-halo row leaves the bits unchanged.  Here the state is first
made rough by the oracle (4 MCS at p = 3/4, q = 1/4, Eq. (2) with both
moves), restored into the GPU context with sca_restore, and then each of
(p, q) = (1, 0), (0, 1), (1, 1), (0, 0) runs for 2*depth + 3 MCS (two whole
passes and a remainder split into two shallower passes) on both sides, with
slopes, t, h(0,0) and the exact moments compared after each phase."""
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


def snapshot_of(orc, st, device):
    """An oracle state in the snapshot layout (packed S, then h(0,0))."""
    S = np.ascontiguousarray(orc.pack(st)).reshape(-1).view(np.int64)
    return torch.from_numpy(np.concatenate([S, np.array([st.h0], np.int64)])).to(device)


def rough_state(orc, X, Y, seed, n=4):
    st = orc.flat(X, Y, track_heights=False)
    orc.run(st, n, 0.75, 0.25, seed=seed)
    return st


PHASES = [(1.0, 0.0), (0.0, 1.0), (1.0, 1.0), (0.0, 0.0)]


def run_phases(orc, sca, X, Y, depth, band, seed, n, phases=PHASES, expect_depth=None, path=0):
    st = rough_state(orc, X, Y, seed)
    lat = sca.Lattice(X, Y, seed=seed)
    lat.restore(snapshot_of(orc, st, lat.device), st.t)
    lat.set_blocking(depth, band)
    for p, q in phases:
        plan = lat.plan(n, p, q)
        _say(f"  phase p={p} q={q} n={n}: {plan['n_pass']} x {plan['kernel']}, tails {plan['tail1']}+"
             f"{plan['tail2']} ({plan['tail_kernel']})")
        assert plan["path"] == path and plan["band"] == band
        if expect_depth is not None:
            assert plan["depth"] == (expect_depth if plan["n_pass"] else 0)
        lat.step(n, p, q)
        orc.run(st, n, p, q, seed=seed)
        torch.cuda.synchronize()
        got = lat.slopes.cpu().numpy().view(np.uint64)
        ref = orc.pack(st)
        if not np.array_equal(got, ref):
            bad = np.argwhere(got != ref)
            raise AssertionError(f"p={p} q={q}: {len(bad)} words differ, first at (d, pi, y, w) = {bad[0].tolist()}")
        assert lat.meta() == (st.t, st.h0)
        assert lat.roughness()[:3] == orc.moments(st)[:3]
    lat.close()


# X = 2^16: one word per lane of a 512-thread workgroup; 5 MCS runs the
# register-window kernel, 6 the LDS-window kernel, 7..13 mcs_fixed_kernel
# (DIST 3 up to 11, 1 at 12 and 13); the bench's 13-MCS passes on 256-row bands
WIDE16 = ([(65536, 64, d, 32) for d in range(5, 14)]
          + [(65536, 128, 12, 64), (65536, 128, 13, 64), (65536, 256, 10, 128), (65536, 512, 13, 256)])
# X = 2^13 .. 2^15: one, two and four waves per row, depths 1..8
NARROW = [(X, 32, d, 16) for X in (8192, 16384, 32768) for d in range(1, 9)]
# X = 2^17: two words per lane up to 5 MCS, the 1024-thread LDS window at 6
WIDE17 = [(131072, 32, d, 16) for d in range(1, 7)]


@pytest.mark.parametrize("X,Y,depth,band", WIDE16 + NARROW + WIDE17)
def test_draw_free_passes_from_rough_state(orc, sca, X, Y, depth, band):
    _say(f"[rough] X={X} Y={Y} depth={depth} band={band}")
    run_phases(orc, sca, X, Y, depth, band, seed=1000 + X // 1024 + 17 * depth + band, n=2 * depth + 3,
               expect_depth=depth)


@pytest.mark.parametrize("n", [21, 26, 47])
def test_bench_pass_plan_from_rough_state(orc, sca, n):
    """The bench's launch configuration (13-MCS passes on 256-row bands at
    X = 2^16): 21 MCS run as passes of 11 and 10 MCS, 26 as two whole
    passes, 47 as two whole passes and passes of 11 and 10 MCS."""
    _say(f"[rough bench plan] n={n}")
    run_phases(orc, sca, 65536, 512, 13, 256, seed=4242 + n, n=n)


@pytest.mark.parametrize("X,Y,p,q,k,n", [
    (65536, 512, 1.0, 0.0, 11, 47),      # split inside the 13-MCS pass plan
    (65536, 256, 0.5, 0.0, 5, 19),       # random words: 4-MCS passes
    (16384, 128, 0.75, 0.25, 3, 12),
    (16384, 64, 0.93, 0.07, 4, 9),       # per-site compares
    (512, 64, 0.9375, 0.0, 7, 15),       # half-step launches only
])
def test_resume_is_bit_exact(orc, sca, X, Y, p, q, k, n):
    """run(n) == run(k), snapshot, a fresh context, sca_restore, run(n - k)."""
    _say(f"[resume] X={X} Y={Y} p={p} q={q} k={k} n={n}")
    seed = 77 + X + k
    a = sca.Lattice(X, Y, seed=seed)
    a.step(n, p, q)
    b = sca.Lattice(X, Y, seed=seed)
    b.step(k, p, q)
    snap = b.snapshot()
    torch.cuda.synchronize()
    b.close()
    del b
    c = sca.Lattice(X, Y, seed=seed)
    c.step(3, 0.5, 0.5)  # overwritten by the restore
    c.restore(snap, k)
    assert c.t == k
    c.step(n - k, p, q)
    torch.cuda.synchronize()
    assert torch.equal(a.slopes, c.slopes)
    assert a.meta() == c.meta() == (n, c.meta()[1])
    st = orc.flat(X, Y, track_heights=False)
    orc.run(st, n, p, q, seed=seed)
    assert np.array_equal(c.slopes.cpu().numpy().view(np.uint64), orc.pack(st)) and c.meta()[1] == st.h0


def test_reset_and_plan(orc, sca):
    X, Y = 65536, 65536
    lat = sca.Lattice(X, Y, seed=42)
    plan = lat.plan(2000, 1.0, 0.0)
    assert (plan["path"], plan["depth"], plan["band"], plan["n_pass"], plan["tail1"], plan["tail2"],
            plan["n_unfused"]) == (0, 13, 256, 152, 12, 12, 0)
    assert plan["kernel"] == "mcs_fixed_kernel<8,13,1,false>"
    assert plan["tail_kernel"] == "mcs_fixed_kernel<8,12,1,false>"
    p20 = lat.plan(20, 1.0, 0.0)
    assert (p20["n_pass"], p20["depth"], p20["tail1"], p20["tail2"]) == (0, 0, 10, 10)
    half = lat.plan(200, 0.5, 0.0)
    assert (half["path"], half["depth"], half["band"]) == (1, 4, 128)
    # one draw (odd): the instantiation that keeps the shared draw between a row's half-steps
    assert half["kernel"] == "mcs_block_kernel<8,1,4,Mask,false,OddTail>"
    assert lat.plan(200, 0.9375, 0.0)["kernel"] == "mcs_block_kernel<8,1,4,Mask,false,Even>"
    assert lat.plan(200, 0.5, 0.5)["kernel"] == "mcs_block_kernel<8,1,4,Mask,true,OddTail>"
    assert lat.plan(200, 0.75, 0.25)["kernel"] == "mcs_block_kernel<8,1,4,Mask,true,Even>"
    ps = lat.plan(10, 0.93, 0.07)
    assert (ps["path"], ps["n_pass"], ps["n_unfused"]) == (2, 0, 10)
    assert ps["halfstep_kernel"] == "halfstep_kernel<64,8,PerSite,true>"
    lat.step(5, 1.0, 0.0)
    lat.reset()
    assert lat.meta() == (0, 0)
    small = orc.flat(256, 16, track_heights=False)
    s2 = sca.Lattice(256, 16, seed=1)
    s2.step(3, 0.5, 0.5)
    s2.reset()
    torch.cuda.synchronize()
    assert np.array_equal(s2.slopes.cpu().numpy().view(np.uint64), orc.pack(small)) and s2.meta() == (0, 0)
    lat.close()


def test_blocked_pass_needs_the_pass_buffer(sca):
    """Without a pass buffer a planned blocked pass is refused (nothing
    enqueued, t unchanged); depth 0 runs the two-launch form without one."""
    from paper_1606_00310_amd import _lib as L

    lat = sca.Lattice(16384, 64, seed=3)
    ref = sca.Lattice(16384, 64, seed=3)
    L.check(L.lib().sca_set_pass_buffer(lat._ctx, None, 0), "detach")
    with pytest.raises(sca.ScaError) as e:
        lat.step(8, 1.0, 0.0)
    assert e.value.code == L.SCA_ENOBUF and lat.t == 0
    lat.set_blocking(0)
    lat.step(8, 1.0, 0.0)
    ref.step(8, 1.0, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(lat.slopes, ref.slopes) and lat.meta() == ref.meta() == (8, 16)
    small = torch.empty(10, dtype=torch.int64, device=lat.device)
    assert L.lib().sca_set_pass_buffer(lat._ctx, small.data_ptr(), 80) == L.SCA_EINVAL
    assert L.lib().sca_set_pass_buffer(lat._ctx, lat.slopes.data_ptr(), lat.slopes.numel() * 8) == L.SCA_EINVAL


# Random-word passes with an odd number of draws (one Philox call per word and
# MCS, the even half-step keeps the shared draw for the odd one), with and
# without removals, from a rough state: 1..4 MCS per pass at one, two and
# eight waves per row, and at two words per lane (X = 2^17, where removals
# recompute the shared call).
ODD_DRAWS = [(0.5, 0.5), (0.625, 0.125), (0.5, 0.0), (0.34375, 0.0), (0.5, 0.25)]


@pytest.mark.parametrize("X,Y,depth,band", [(8192, 64, 4, 32), (16384, 32, 3, 16), (65536, 64, 4, 32),
                                            (65536, 32, 2, 16), (131072, 32, 4, 16), (65536, 128, 1, 32)])
def test_odd_draw_passes_from_rough_state(orc, sca, X, Y, depth, band):
    _say(f"[blocked] odd draw counts X={X} Y={Y} depth={depth} band={band}")
    run_phases(orc, sca, X, Y, depth, band, seed=7001 + depth, n=2 * depth + 3, phases=ODD_DRAWS,
               expect_depth=depth, path=1)
