"""The bit-vectorized CPU comparator (comparator/bitsweep.c: 64-bit words,
OpenMP over the rows of a half-step) against the published Philox vectors
and, word for word, against the oracle: from the flat surface and from rough
states, on partial-word (X < 128), one-word and many-word rows, for the
draw-free, dyadic-mask and per-site acceptance paths."""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def cmp_mod():
    import comparator

    comparator.build(force=not os.path.exists(comparator._SO))
    comparator.lib()
    return comparator


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(s, 16) for s in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_comparator_philox_known_answers(cmp_mod, ctr, key, expect):
    assert list(cmp_mod.philox(ctr, key)) == expect


SIZES = [(4, 4), (8, 16), (64, 8), (128, 8), (256, 4), (512, 16)]
PQ = [(1.0, 0.0), (0.0, 1.0), (1.0, 1.0), (0.5, 0.0), (0.75, 0.25), (0.9375, 0.0), (0.5, 0.5),
      (0.93, 0.07), (0.3, 1.0), (0.625, 0.125)]


@pytest.mark.parametrize("X,Y", SIZES)
@pytest.mark.parametrize("p,q", PQ)
def test_comparator_equals_oracle_from_flat(cmp_mod, orc, X, Y, p, q):
    seed = 900 + X + 7 * Y
    n = 9
    c = cmp_mod.Lattice(X, Y, seed)
    st = orc.flat(X, Y, track_heights=False)
    assert np.array_equal(c.S, orc.pack(st))
    c.step(4, p, q).step(n - 4, p, q)
    orc.run(st, n, p, q, seed=seed)
    assert np.array_equal(c.S, orc.pack(st)), (X, Y, p, q)
    assert (c.t, c.h0) == (st.t, st.h0)


@pytest.mark.parametrize("X,Y", [(16, 8), (128, 16), (1024, 32)])
@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.0, 1.0), (0.75, 0.25), (0.93, 0.07)])
def test_comparator_equals_oracle_from_rough_state(cmp_mod, orc, X, Y, p, q):
    """From a state the oracle made rough (5 MCS at p = 3/4, q = 1/4), where
    wrong alignment of the shifted x+ words or a wrong y+ row changes bits."""
    seed = 31 + X + Y
    st = orc.flat(X, Y, track_heights=False)
    orc.run(st, 5, 0.75, 0.25, seed=seed)
    c = cmp_mod.Lattice(X, Y, seed).set_state(orc.pack(st), st.h0, st.t)
    c.step(6, p, q)
    orc.run(st, 6, p, q, seed=seed)
    assert np.array_equal(c.S, orc.pack(st)), (X, Y, p, q)
    assert (c.t, c.h0) == (st.t, st.h0)


def test_comparator_thread_count_does_not_change_results(cmp_mod):
    prev = cmp_mod.num_threads()
    try:
        out = []
        for n in (1, max(2, prev)):
            cmp_mod.set_num_threads(n)
            out.append(cmp_mod.Lattice(256, 64, 5).step(7, 0.75, 0.25))
        assert np.array_equal(out[0].S, out[1].S) and out[0].h0 == out[1].h0
    finally:
        cmp_mod.set_num_threads(prev)


def test_comparator_rejects_invalid_arguments(cmp_mod):
    c = cmp_mod.Lattice(64, 64, 1)
    with pytest.raises(ValueError):
        c.step(1, 1.5, 0.0)
    with pytest.raises(ValueError):
        c.step(-1, 0.5, 0.0)
