"""The C-ABI library loads on any machine and exports every function that
include/sca.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sca.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sca_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libsca():
    from paper_1606_00310_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1606_00310_amd import build

        build.build()
    return ctypes.CDLL(_lib.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("sca_init", "sca_step", "sca_heights", "sca_roughness", "sca_autocorr"):
        assert required in names


def test_every_declared_symbol_is_exported(libsca):
    missing = [n for n in _declared() if not hasattr(libsca, n)]
    assert not missing, missing


def test_host_only_calls(libsca):
    from paper_1606_00310_amd import _lib as L

    lib = L.lib()
    assert lib.sca_state_words(65536, 65536) == 4 * 65536 * 512
    assert lib.sca_state_words(4, 4) == 16
    assert lib.sca_state_words(100, 64) == 0
    assert lib.sca_state_words(1 << 18, 4) == 0
    assert lib.sca_strerror(L.SCA_EOVERFLOW).decode().startswith("exact result")
    # argument validation happens before any device work
    ctx = ctypes.c_void_p()
    assert lib.sca_init(ctypes.byref(ctx), 100, 64, 1, 1, 1, None) == L.SCA_EINVAL
    assert lib.sca_init(ctypes.byref(ctx), 64, 64, 1, None, 1, None) == L.SCA_EINVAL
    assert lib.sca_step(None, 1, 0.5, 0.0) == L.SCA_EINVAL
    # the allocation-free moments reject a lattice beyond their static scratch
    # and invalid arguments before touching the device
    out3 = (ctypes.c_int64 * 3)()
    w2 = ctypes.c_double()
    assert lib.sca_roughness_noalloc(1, 1, 64, 2 * L.SCA_NOALLOC_MAX_Y, None, out3, ctypes.byref(w2)) == L.SCA_ESCRATCH
    assert lib.sca_roughness_noalloc(None, 1, 64, 64, None, out3, ctypes.byref(w2)) == L.SCA_EINVAL
    assert lib.sca_roughness_noalloc(1, 1, 100, 64, None, out3, ctypes.byref(w2)) == L.SCA_EINVAL
    assert lib.sca_strerror(L.SCA_ESCRATCH).decode().startswith("lattice exceeds the static scratch")


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1606_00310_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b|liboracle|oracle\.c", src, re.M), f
