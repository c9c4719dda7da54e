"""Randomized parity (hypothesis, derandomized): lattice shapes, probabilities
(dyadic of any length, arbitrary, 0 and 1), seeds, MCS counts and, on wide
lattices, the temporal-blocking depth and band, each against the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hyp = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402


@pytest.fixture(scope="module")
def sca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_00310_amd as P

    P.lib()
    return P


def _prob():
    return st.one_of(
        st.sampled_from([0.0, 1.0, 0.5, 0.25, 0.75, 0.9375]),
        st.integers(1, 2**12 - 1).map(lambda v: v / 2**12),          # dyadic, up to 12 digits
        st.integers(1, 2**32 - 1).map(lambda v: v / 2**32),          # dyadic, up to 32 digits
        st.floats(0.0, 1.0, allow_nan=False).filter(lambda r: r * 2**32 != int(r * 2**32)),  # per-site
    )


def _run_case(orc, sca, X, Y, p, q, seed, n, persite, blocking=None):
    print(f"[random] X={X} Y={Y} p={p!r} q={q!r} seed={seed} n={n} persite={persite} blocking={blocking}",
          flush=True)
    sys.stdout.flush()
    lat = sca.Lattice(X, Y, seed=seed)
    if blocking is not None:
        lat.set_blocking(*blocking)
    lat.step(n, p, q, force_persite=persite)
    st_ = orc.flat(X, Y, track_heights=False)
    orc.run(st_, n, p, q, seed=seed, force_persite=persite)
    torch.cuda.synchronize()
    assert np.array_equal(lat.slopes.cpu().numpy().view(np.uint64), orc.pack(st_))
    assert lat.meta() == (st_.t, st_.h0)
    assert lat.roughness()[:3] == orc.moments(st_)[:3]
    lat.close()


@settings(max_examples=60, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(lx=st.integers(2, 12), ly=st.integers(2, 9), p=_prob(), q=_prob(), seed=st.integers(0, 2**64 - 1),
       n=st.integers(0, 9), persite=st.booleans())
def test_random_small(orc, sca, lx, ly, p, q, seed, n, persite):
    _run_case(orc, sca, 2**lx, 2**ly, p, q, seed, n, persite)


@settings(max_examples=30, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(lx=st.integers(13, 17), ly=st.integers(4, 7), p=_prob(), q=_prob(), seed=st.integers(0, 2**64 - 1),
       n=st.integers(0, 27), depth=st.integers(0, 13), lband=st.integers(2, 6))
def test_random_blocked(orc, sca, lx, ly, p, q, seed, n, depth, lband):
    band = 2**lband
    Y = 2**ly
    if depth > 0 and (band < 2 * depth or Y < 2 * band):
        band = 0  # automatic band for this depth
    _run_case(orc, sca, 2**lx, Y, p, q, seed, n, False, (depth, band))
