"""sca_roughness_noalloc (the moments of a caller's state through the
library's static device scratch, no context, no allocation) against
sca_roughness on the same states: two calls in a row, the second on a smaller
lattice, so that the second call reads scratch words the first one left
behind wherever it does not overwrite them first."""
import ctypes
import sys

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


def _noalloc(L, lat):
    out = (ctypes.c_int64 * 3)()
    w2 = ctypes.c_double()
    rc = L.lib().sca_roughness_noalloc(lat.slopes.data_ptr(), lat.aux.data_ptr(), lat.X, lat.Y,
                                       lat.stream.cuda_stream, out, ctypes.byref(w2))
    L.check(rc, "sca_roughness_noalloc")
    return int(out[0]), int(out[1]), int(out[2]), float(w2.value)


@pytest.mark.parametrize("sizes", [((4096, 2048), (256, 64)), ((128, 1024), (64, 4))])
def test_noalloc_equals_roughness(sca, sizes):
    from paper_1606_00310_amd import _lib as L

    for k, (X, Y) in enumerate(sizes):
        _say(f"[noalloc] call {k + 1}: {X}x{Y}")
        lat = sca.Lattice(X, Y, seed=17 + k)
        lat.step(7, 0.75, 0.25)
        lat.step(3, 0.93, 0.07)
        ref = lat.roughness()
        got = _noalloc(L, lat)
        assert got[:3] == ref[:3], (X, Y, got, ref)
        assert got[3] == ref[3]
        assert got[0] == X * Y and got[3] > 0.0
        lat.close()


def test_noalloc_rejects_beyond_scratch(sca):
    from paper_1606_00310_amd import _lib as L

    out = (ctypes.c_int64 * 3)()
    w2 = ctypes.c_double()
    lat = sca.Lattice(64, 64, seed=1)
    rc = L.lib().sca_roughness_noalloc(lat.slopes.data_ptr(), lat.aux.data_ptr(), 64, 2 * L.SCA_NOALLOC_MAX_Y,
                                       lat.stream.cuda_stream, out, ctypes.byref(w2))
    assert rc == L.SCA_ESCRATCH
    lat.close()
