"""Pins of the oracle's Philox4x32-10 against things other than itself:
the published known-answer vectors and rocRAND's host-callable generator."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(s, 16) for s in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_known_answer_vectors(orc, ctr, key, expect):
    assert list(orc.philox4x32_10(ctr, key)) == expect


@pytest.fixture(scope="module")
def rocrand_helper(tmp_path_factory):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    exe = tmp_path_factory.mktemp("rr") / "rocrand_philox"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", os.path.join(HERE, "helpers", "rocrand_philox.cpp"),
                           "-o", str(exe)])
    return str(exe)


def test_matches_rocrand(orc, rocrand_helper):
    rng = np.random.default_rng(12345)
    cases = []
    for _ in range(300):
        k = rng.integers(0, 2**32, 2, dtype=np.uint64)
        c = rng.integers(0, 2**32, 4, dtype=np.uint64)
        c[1] &= np.uint64(2**30 - 1)  # rocRAND's offset argument covers c1 < 2^30
        cases.append((k, c))
    # the counters the SCA actually uses: (word, MCS, 2*call + parity, 0)
    for g, t, j, par in [(0, 0, 0, 0), (5, 1000, 3, 1), (2**25 - 1, 1999, 15, 1), (77, 2**29, 0, 0)]:
        cases.append((np.array([42, 0], np.uint64), np.array([g, t, 2 * j + par, 0], np.uint64)))
    text = "".join("%x %x %x %x %x %x\n" % (k[0], k[1], c[0], c[1], c[2], c[3]) for k, c in cases)
    out = subprocess.run([rocrand_helper], input=text, capture_output=True, text=True, check=True).stdout
    got = [[int(s, 16) for s in line.split()] for line in out.strip().splitlines()]
    assert len(got) == len(cases)
    for (k, c), ref in zip(cases, got):
        assert list(orc.philox4x32_10(c, k)) == ref, (k, c)
