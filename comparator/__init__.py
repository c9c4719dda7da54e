"""numpy front end of the bit-vectorized multithreaded CPU sweep (bitsweep.c),
the CPU side of a like-for-like GPU/CPU comparison: 64-bit words, the GPU
library's packed state layout and random stream, rows of a half-step split
over OpenMP threads (the paper's CPU code, Sec. II-B and Sec. III).

It is not the test oracle and not the GPU library, and shares no code with
either.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libbitsweep.so")
_SRC = os.path.join(_HERE, "bitsweep.c")

OK, EINVAL = 0, -1


def build(force: bool = True) -> str:
    """Compile bitsweep.c into libbitsweep.so (C11 + OpenMP, baseline x86-64
    code: the library also runs on hosts other than the one it was built on)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.bs_sweep.argtypes = [u64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]
        L.bs_sweep.restype = ctypes.c_int
        L.bs_philox.argtypes = [u32p, u32p, u32p]
        L.bs_philox.restype = None
        L.bs_num_threads.argtypes = []
        L.bs_num_threads.restype = ctypes.c_int
        L.bs_set_num_threads.argtypes = [ctypes.c_int]
        L.bs_set_num_threads.restype = None
        _lib = L
    return _lib


class Lattice:
    """An X x Y packed state S[2][2][Y][W] (uint64), its origin height and MCS
    count, advanced by the CPU sweep."""

    def __init__(self, X: int, Y: int, seed: int):
        self.X, self.Y, self.seed = int(X), int(Y), int(seed)
        self.W = max(1, self.X // 128)
        self.S = np.zeros((2, 2, self.Y, self.W), np.uint64)
        self.h0 = 0
        self.t = 0
        self.set_flat()

    def set_flat(self):
        """The flat surface h(x,y) = (x+y)&1: every odd site's slopes point up
        towards it, so the odd-parity arrays hold every used bit."""
        nb = 64 if self.X >= 128 else self.X // 2
        valid = np.uint64((1 << nb) - 1) if nb < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
        self.S[:, 0] = 0
        self.S[:, 1] = valid
        self.h0 = 0
        self.t = 0
        return self

    def set_state(self, S, h0: int, t: int):
        self.S[...] = np.asarray(S, np.uint64).reshape(self.S.shape)
        self.h0, self.t = int(h0), int(t)
        return self

    def step(self, n: int, p: float, q: float = 0.0):
        h0 = ctypes.c_int64(self.h0)
        rc = lib().bs_sweep(self.S.reshape(-1), self.X, self.Y, self.seed, self.t, int(n), float(p), float(q),
                            ctypes.byref(h0))
        if rc != OK:
            raise ValueError(f"bs_sweep({self.X}x{self.Y}, t={self.t}, n={n}, p={p}, q={q}): status {rc}")
        self.h0 = int(h0.value)
        self.t += int(n)
        return self


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().bs_philox(np.ascontiguousarray(ctr, np.uint32), np.ascontiguousarray(key, np.uint32), out)
    return out


def num_threads() -> int:
    return int(lib().bs_num_threads())


def set_num_threads(n: int) -> None:
    lib().bs_set_num_threads(int(n))
