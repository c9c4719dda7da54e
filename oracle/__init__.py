"""TEST INFRASTRUCTURE ONLY: numpy front end of the plain CPU oracle (oracle.c).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never imports it.

State convention (see oracle.c for the full statement): ``sx[y, x] = 1`` iff
h(x,y) - h(x-1,y) = +1 and ``sy[y, x] = 1`` iff h(x,y) - h(x,y-1) = +1, with
periodic indices; ``h0`` is the height of site (0, 0); ``t`` counts completed
Monte-Carlo steps.  Every function follows the octahedron-model SCA of
Kelling, Odor and Gemming (2016): Eq. (2) for the rule, Sec. I-A for the
checkerboard order and boundaries, Sec. II-A for the packed layout and
Sec. II-B / Sec. III for the acceptance words.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, EINVAL, ENOMEM, EOVERFLOW = 0, -1, -2, -4


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain C11 + OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
             _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None

_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_int = ctypes.c_int
_dbl = ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_dyadic_digits.argtypes = [_dbl, _vp, _vp]
        L.orc_dyadic_digits.restype = _int
        L.orc_threshold.argtypes = [_dbl]
        L.orc_threshold.restype = _u64
        L.orc_fold.argtypes = [_dbl, _u64p]
        L.orc_fold.restype = _u64
        L.orc_acceptance_words.argtypes = [_u64, ctypes.c_uint32, _int, _u64, _i64, _dbl, _dbl,
                                           _int, _u64p, _u64p]
        L.orc_acceptance_words.restype = _int
        L.orc_flat_patch.argtypes = [_i64] * 6 + [_u8p, _u8p, _vp]
        L.orc_flat_patch.restype = _int
        L.orc_halfstep_xi.argtypes = [_i64, _i64, _u8p, _u8p, _vp, _vp, _int, _u64p, _u64p]
        L.orc_halfstep_xi.restype = _int
        L.orc_halfstep_xi_batch.argtypes = [_i64, _i64, _i64, _u8p, _u8p, _vp, _vp, _int,
                                            _u64p, _u64p]
        L.orc_halfstep_xi_batch.restype = _int
        L.orc_heights.argtypes = [_i64, _i64, _u8p, _u8p, _i64, _i64p]
        L.orc_heights.restype = _int
        L.orc_moments.argtypes = [_i64, _i64, _u8p, _u8p, _i64, _i64p, _vp]
        L.orc_moments.restype = _int
        L.orc_autocorr.argtypes = [_i64, _i64, _u8p, _u8p, _i64, _u8p, _u8p, _i64, _i64p, _vp]
        L.orc_autocorr.restype = _int
        L.orc_run_patch.argtypes = [_i64] * 6 + [_u8p, _u8p, _vp, _vp, _u64, _i64, _i64, _dbl,
                                                 _dbl, _int, _vp, _vp]
        L.orc_run_patch.restype = _int
        L.orc_pack.argtypes = [_i64, _i64, _u8p, _u8p, _u64p]
        L.orc_pack.restype = _int
        L.orc_unpack.argtypes = [_i64, _i64, _u64p, _u8p, _u8p]
        L.orc_unpack.restype = _int
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = _int
        L.orc_set_num_threads.argtypes = [_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != OK:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# --------------------------------------------------------------------------
# Random stream
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function: counter (4 x u32), key (2 x u32)."""
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def dyadic_digits(r: float):
    """(n, [b_1..b_n], is_one), or None when r*2^32 is not an integer."""
    d = np.zeros(32, np.int32)
    one = np.zeros(1, np.int32)
    n = lib().orc_dyadic_digits(float(r), _ptr(d), _ptr(one))
    if n < 0:
        return None
    return n, [int(v) for v in d[:n]], bool(one[0])


def threshold(r: float) -> int:
    return int(lib().orc_threshold(float(r)))


def fold(r: float, draws) -> int:
    """The and/or fold of draws R_0..R_{n-1} (uint64) into a word of probability r."""
    d = np.zeros(32, np.uint64)
    draws = np.asarray(draws, np.uint64)
    d[: len(draws)] = draws
    return int(lib().orc_fold(float(r), d))


def acceptance_words(seed: int, t: int, parity: int, g0: int, count: int, p: float, q: float,
                     force_persite: bool = False):
    xp = np.zeros(count, np.uint64)
    xq = np.zeros(count, np.uint64)
    _check(lib().orc_acceptance_words(seed, t, parity, g0, count, p, q, int(force_persite), xp, xq),
           "acceptance_words")
    return xp, xq


# --------------------------------------------------------------------------
# Lattice state
# --------------------------------------------------------------------------
class State:
    """A lattice (or light-cone patch) in the oracle's one-byte-per-slope form."""

    def __init__(self, X, Y, sx, sy, h0=0, t=0, H=None, x0=0, y0=0):
        self.X, self.Y = int(X), int(Y)
        self.sx, self.sy = sx, sy
        self.h0 = int(h0)
        self.t = int(t)
        self.H = H
        self.x0, self.y0 = int(x0), int(y0)

    @property
    def PY(self):
        return self.sx.shape[0]

    @property
    def PX(self):
        return self.sx.shape[1]

    def copy(self):
        return State(self.X, self.Y, self.sx.copy(), self.sy.copy(), self.h0, self.t,
                     None if self.H is None else self.H.copy(), self.x0, self.y0)


def words_per_row(X: int) -> int:
    return max(1, X // 128)


def flat(X: int, Y: int, track_heights: bool = True) -> State:
    """Flat initial surface h(x,y) = (x+y)&1, h0 = 0, t = 0."""
    return flat_patch(X, Y, 0, 0, X, Y, track_heights)


def flat_patch(X, Y, x0, y0, PX, PY, track_heights: bool = True) -> State:
    sx = np.zeros((PY, PX), np.uint8)
    sy = np.zeros((PY, PX), np.uint8)
    H = np.zeros((PY, PX), np.int32) if track_heights else None
    _check(lib().orc_flat_patch(X, Y, x0, y0, PX, PY, sx, sy, _ptr(H)), "flat")
    return State(X, Y, sx, sy, 0, 0, H, x0, y0)


def run(st: State, n_mcs: int, p: float, q: float, seed: int, force_persite: bool = False,
        series: bool = False, counts: bool = False):
    """Advance st in place by n_mcs MCS.  Returns (series[n,2] or None, counts[2] or None)."""
    ser = np.zeros(2 * max(n_mcs, 1), np.int64) if series else None
    cnt = np.zeros(2, np.int64)
    h0 = np.array([st.h0], np.int64)
    _check(lib().orc_run_patch(st.X, st.Y, st.x0, st.y0, st.PX, st.PY, st.sx, st.sy, _ptr(st.H),
                               _ptr(h0), seed, st.t, n_mcs, p, q, int(force_persite),
                               _ptr(ser), _ptr(cnt)), "run")
    st.h0 = int(h0[0])
    st.t += n_mcs
    return (ser[: 2 * n_mcs].reshape(n_mcs, 2) if series else None), (cnt if counts else None)


def halfstep_xi(st: State, parity: int, xi_p, xi_q):
    """One half-step with injected acceptance words (whole torus only)."""
    h0 = np.array([st.h0], np.int64)
    _check(lib().orc_halfstep_xi(st.X, st.Y, st.sx, st.sy, _ptr(st.H), _ptr(h0), parity,
                                 np.ascontiguousarray(xi_p, np.uint64),
                                 np.ascontiguousarray(xi_q, np.uint64)), "halfstep_xi")
    st.h0 = int(h0[0])


def halfstep_xi_batch(X, Y, sx, sy, H, h0, parity, xi_p, xi_q):
    """Batched half-steps on [B, Y, X] arrays (modified in place)."""
    B = sx.shape[0]
    _check(lib().orc_halfstep_xi_batch(B, X, Y, sx, sy, _ptr(H), _ptr(h0), parity,
                                       np.ascontiguousarray(xi_p, np.uint64),
                                       np.ascontiguousarray(xi_q, np.uint64)), "halfstep_xi_batch")


def heights(st: State) -> np.ndarray:
    out = np.zeros((st.Y, st.X), np.int64)
    _check(lib().orc_heights(st.X, st.Y, st.sx, st.sy, st.h0, out), "heights")
    return out


def moments(st: State):
    """(N, sum h, sum h^2, W^2)."""
    out = np.zeros(3, np.int64)
    w2 = ctypes.c_double(0.0)
    _check(lib().orc_moments(st.X, st.Y, st.sx, st.sy, st.h0, out, ctypes.byref(w2)), "moments")
    return int(out[0]), int(out[1]), int(out[2]), float(w2.value)


def autocorr(st_t: State, st_s: State):
    """(N, sum h_t h_s, sum h_t, sum h_s, C(t,s))."""
    out = np.zeros(4, np.int64)
    c = ctypes.c_double(0.0)
    _check(lib().orc_autocorr(st_t.X, st_t.Y, st_t.sx, st_t.sy, st_t.h0, st_s.sx, st_s.sy,
                              st_s.h0, out, ctypes.byref(c)), "autocorr")
    return int(out[0]), int(out[1]), int(out[2]), int(out[3]), float(c.value)


def pack(st: State) -> np.ndarray:
    """Canonical role-grouped words S[2][2][Y][W] (uint64)."""
    W = words_per_row(st.X)
    S = np.zeros((2, 2, st.Y, W), np.uint64)
    _check(lib().orc_pack(st.X, st.Y, st.sx, st.sy, S), "pack")
    return S


def unpack(X: int, Y: int, S) -> State:
    S = np.ascontiguousarray(S).view(np.uint64).reshape(2, 2, Y, words_per_row(X))
    sx = np.zeros((Y, X), np.uint8)
    sy = np.zeros((Y, X), np.uint8)
    _check(lib().orc_unpack(X, Y, S, sx, sy), "unpack")
    return State(X, Y, sx, sy)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int):
    lib().orc_set_num_threads(int(n))
