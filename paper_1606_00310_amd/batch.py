"""Ensembles of independent realizations advanced by one persistent,
graph-captured launch per epoch (sca_batch_* in include/sca.h).

The states live in one caller-owned device arena (a torch int64 tensor) whose
size is the HBM budget; admission fails with SCA_EBUSY when slots or arena
space run out.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L


@dataclass(frozen=True)
class Realization:
    """One independent lattice: X x Y, probabilities p and q, MCS budget, seed."""
    X: int
    Y: int
    p: float
    q: float
    n_mcs: int
    seed: int
    force_persite: bool = False

    def req(self) -> L.Req:
        return L.Req(self.X, self.Y, self.p, self.q, self.n_mcs, self.seed,
                     L.SCA_FORCE_PERSITE if self.force_persite else 0, 0)

    @property
    def sites(self) -> int:
        return self.X * self.Y


def state_bytes(X: int, Y: int) -> int:
    return int(L.lib().sca_batch_state_bytes(X, Y))


class Batch:
    def __init__(self, max_slots: int, arena_bytes: int, device="cuda", stream: torch.cuda.Stream | None = None,
                 config: dict | None = None):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        arena_bytes = (int(arena_bytes) + 7) // 8 * 8
        self.arena = torch.empty(arena_bytes // 8, dtype=torch.int64, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.max_slots = int(max_slots)
        b = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().sca_batch_create(ctypes.byref(b), self.max_slots, self.arena.data_ptr(), arena_bytes,
                                             self.stream.cuda_stream), "sca_batch_create")
        self._b = b
        if config:
            self.set_config(**config)

    # ------------------------------------------------------------ config
    def set_config(self, block_threads=None, blocks_per_cu=None, lds_bytes=None, order=None, words_per_lane=None,
                   depth=None, max_parts=None):
        c = self.get_config()
        for k, v in (("block_threads", block_threads), ("blocks_per_cu", blocks_per_cu), ("lds_bytes", lds_bytes),
                     ("order", order), ("words_per_lane", words_per_lane), ("depth", depth),
                     ("max_parts", max_parts)):
            if v is not None:
                setattr(c, k, int(v))
        L.check(L.lib().sca_batch_set_config(self._b, ctypes.byref(c)), "sca_batch_set_config")

    def get_config(self) -> L.BatchConfig:
        c = L.BatchConfig()
        L.check(L.lib().sca_batch_get_config(self._b, ctypes.byref(c)), "sca_batch_get_config")
        return c

    # ------------------------------------------------------------ slots
    def admit(self, reals) -> list[int]:
        """Admit realizations (all or none); returns their slots."""
        reals = list(reals)
        n = len(reals)
        arr = (L.Req * max(n, 1))(*[r.req() for r in reals])
        slots = (ctypes.c_int32 * max(n, 1))()
        L.check(L.lib().sca_batch_admit(self._b, arr, n, slots), "sca_batch_admit")
        return [int(slots[i]) for i in range(n)]

    def try_admit(self, reals):
        """As admit, but returns None instead of raising when over budget."""
        try:
            return self.admit(reals)
        except L.ScaError as e:
            if e.code == L.SCA_EBUSY:
                return None
            raise

    def run(self, mcs_epoch: int) -> int:
        """One epoch (asynchronous); returns how many realizations advanced."""
        active = ctypes.c_int32()
        L.check(L.lib().sca_batch_run(self._b, int(mcs_epoch), ctypes.byref(active)), "sca_batch_run")
        return int(active.value)

    def run_work(self, site_updates: int) -> int:
        """One epoch in which each realization advances max(1, site_updates /
        (X*Y)) MCS (asynchronous); returns how many advanced."""
        active = ctypes.c_int32()
        L.check(L.lib().sca_batch_run_work(self._b, int(site_updates), ctypes.byref(active)), "sca_batch_run_work")
        return int(active.value)

    def info(self, slot: int) -> L.SlotInfo:
        s = L.SlotInfo()
        L.check(L.lib().sca_batch_slot(self._b, int(slot), ctypes.byref(s)), "sca_batch_slot")
        return s

    def state(self, slot: int):
        """(slopes view (2, 2, Y, W) int64, h0 view (1,) int64) into the arena."""
        s = self.info(slot)
        W = max(1, s.X // 128)
        off = (s.slopes_dev - self.arena.data_ptr()) // 8
        n = 4 * s.Y * W
        return self.arena[off:off + n].view(2, 2, s.Y, W), self.arena[off + n:off + n + 1]

    def roughness(self, slot: int):
        out = (ctypes.c_int64 * 3)()
        w2 = ctypes.c_double()
        L.check(L.lib().sca_batch_roughness(self._b, int(slot), out, ctypes.byref(w2)), "sca_batch_roughness")
        return int(out[0]), int(out[1]), int(out[2]), float(w2.value)

    def release(self, slot: int):
        L.check(L.lib().sca_batch_release(self._b, int(slot)), "sca_batch_release")

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            L.lib().sca_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
