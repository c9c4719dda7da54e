"""Bit-vectorized stochastic cellular automaton of the 2+1-dimensional
octahedron surface-growth model (Kelling, Odor, Gemming 2016) on AMD Instinct
MI355X: hand-written gfx950 HIP kernels behind the C ABI of include/sca.h,
with torch supplying device memory and streams."""
from ._lib import ScaError, lib  # noqa: F401
from .lattice import Lattice, debug_philox, philox_rate  # noqa: F401

__all__ = ["Lattice", "ScaError", "debug_philox", "lib", "philox_rate"]
