"""One octahedron-model lattice on the GPU: torch tensors for the device
memory and stream, every step of the computation in libsca.so."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L


class Lattice:
    """X x Y lattice with periodic boundaries, flat initial surface
    h(x,y) = (x+y)&1, slopes packed 64 sites per uint64 word in four
    role-grouped arrays (int64 tensor of shape (2, 2, Y, W), W = max(1, X/128)).
    """

    def __init__(self, X: int, Y: int, seed: int, device="cuda", stream: torch.cuda.Stream | None = None):
        self.X, self.Y, self.seed = int(X), int(Y), int(seed)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        n = L.lib().sca_state_words(self.X, self.Y)
        if n == 0:
            raise L.ScaError(L.SCA_EINVAL, f"lattice size {X}x{Y}")
        self.W = max(1, self.X // 128)
        self.slopes = torch.empty((2, 2, self.Y, self.W), dtype=torch.int64, device=self.device)
        self.aux = torch.zeros(L.SCA_AUX_LEN, dtype=torch.int64, device=self.device)
        # the temporally blocked passes (X >= 8192) run out of place into a
        # second buffer of the state's size
        self.pass_buffer = torch.empty_like(self.slopes) if self.X >= 8192 else None
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().sca_init(ctypes.byref(ctx), self.X, self.Y, self.seed, self.slopes.data_ptr(),
                                     self.aux.data_ptr(), self.stream.cuda_stream), "sca_init")
        self._ctx = ctx
        if self.pass_buffer is not None:
            L.check(L.lib().sca_set_pass_buffer(ctx, self.pass_buffer.data_ptr(),
                                                self.pass_buffer.numel() * 8), "sca_set_pass_buffer")

    # ------------------------------------------------------------------ steps
    def step(self, n_mcs: int, p: float, q: float = 0.0, force_persite: bool = False, graph: bool = False,
             fuse: bool = True):
        """Advance n_mcs MCS.  graph=True captures the launches into one
        hipGraph, launches it once and waits for it; fuse=False forces two
        half-step launches per MCS."""
        flags = ((L.SCA_FORCE_PERSITE if force_persite else 0) | (L.SCA_STEP_GRAPH if graph else 0)
                 | (0 if fuse else L.SCA_NO_FUSE))
        L.check(L.lib().sca_step_ex(self._ctx, int(n_mcs), float(p), float(q), flags), "sca_step")
        return self

    def plan(self, n_mcs: int, p: float, q: float = 0.0, force_persite: bool = False, fuse: bool = True) -> dict:
        """The launches step() would enqueue (sca_plan_step)."""
        flags = (L.SCA_FORCE_PERSITE if force_persite else 0) | (0 if fuse else L.SCA_NO_FUSE)
        out = L.StepPlan()
        L.check(L.lib().sca_plan_step(self._ctx, int(n_mcs), float(p), float(q), flags, ctypes.byref(out)),
                "sca_plan_step")
        return out.as_dict()

    def reset(self):
        """The flat initial surface again, t = 0."""
        L.check(L.lib().sca_reset(self._ctx), "sca_reset")

    def restore(self, snap: torch.Tensor, t: int):
        """State and h(0,0) from a snapshot-layout tensor (S words, then h(0,0)), MCS counter t."""
        if snap.numel() * 8 != L.lib().sca_snapshot_bytes(self._ctx) or snap.device != self.device \
                or not snap.is_contiguous():
            raise ValueError("snapshot of another lattice size or device")
        L.check(L.lib().sca_restore(self._ctx, snap.data_ptr(), int(t)), "sca_restore")

    def debug_halfstep(self, parity: int, xi_p: torch.Tensor, xi_q: torch.Tensor):
        """Half-step with injected acceptance words (int64 tensors of Y*W words)."""
        for xi in (xi_p, xi_q):
            if xi.dtype != torch.int64 or xi.numel() != self.Y * self.W or not xi.is_contiguous() \
                    or xi.device != self.device:
                raise ValueError("acceptance words must be contiguous int64 device tensors of Y*W words")
        L.check(L.lib().sca_debug_halfstep(self._ctx, int(parity), xi_p.data_ptr(), xi_q.data_ptr()),
                "sca_debug_halfstep")

    # ------------------------------------------------------------ measurement
    def heights(self, y0: int = 0, ny: int | None = None) -> torch.Tensor:
        ny = self.Y - y0 if ny is None else ny
        out = torch.empty((ny, self.X), dtype=torch.int32, device=self.device)
        L.check(L.lib().sca_heights(self._ctx, int(y0), int(ny), out.data_ptr()), "sca_heights")
        return out

    def roughness(self):
        """(N, sum h, sum h^2, W^2)."""
        out = (ctypes.c_int64 * 3)()
        w2 = ctypes.c_double()
        L.check(L.lib().sca_roughness(self._ctx, out, ctypes.byref(w2)), "sca_roughness")
        return int(out[0]), int(out[1]), int(out[2]), float(w2.value)

    def snapshot(self) -> torch.Tensor:
        nbytes = L.lib().sca_snapshot_bytes(self._ctx)
        snap = torch.empty(nbytes // 8, dtype=torch.int64, device=self.device)
        L.check(L.lib().sca_snapshot(self._ctx, snap.data_ptr()), "sca_snapshot")
        return snap

    def autocorr(self, snap: torch.Tensor):
        """(N, sum h_t h_s, sum h_t, sum h_s, C(t,s)) against a snapshot."""
        if snap.numel() * 8 != L.lib().sca_snapshot_bytes(self._ctx) or snap.device != self.device:
            raise ValueError("snapshot of another lattice size or device")
        out = (ctypes.c_int64 * 4)()
        c = ctypes.c_double()
        L.check(L.lib().sca_autocorr(self._ctx, snap.data_ptr(), out, ctypes.byref(c)), "sca_autocorr")
        return int(out[0]), int(out[1]), int(out[2]), int(out[3]), float(c.value)

    def meta(self):
        """(t, h0)."""
        t = ctypes.c_int64()
        h0 = ctypes.c_int64()
        L.check(L.lib().sca_get_meta(self._ctx, ctypes.byref(t), ctypes.byref(h0)), "sca_get_meta")
        return int(t.value), int(h0.value)

    @property
    def t(self) -> int:
        t = ctypes.c_int64()
        L.check(L.lib().sca_get_meta(self._ctx, ctypes.byref(t), None), "sca_get_meta")
        return int(t.value)

    def set_blocking(self, depth: int = -1, band: int = 0):
        """MCS per fused pass (1..13; 0 never fuses, -1 automatic) and rows per
        workgroup band (0 automatic)."""
        L.check(L.lib().sca_set_blocking(self._ctx, int(depth), int(band)), "sca_set_blocking")

    def set_time(self, t: int):
        L.check(L.lib().sca_set_time(self._ctx, int(t)), "sca_set_time")

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            L.lib().sca_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_philox(ctr: torch.Tensor, key0: int, key1: int) -> torch.Tensor:
    """Device Philox4x32-10 of counters ctr (int32/uint32-compatible tensor [n, 4])."""
    ctr = ctr.contiguous()
    n = ctr.shape[0]
    out = torch.empty_like(ctr)
    L.check(L.lib().sca_debug_philox(ctr.data_ptr(), key0 & 0xFFFFFFFF, key1 & 0xFFFFFFFF, n, out.data_ptr(),
                                     torch.cuda.current_stream(ctr.device).cuda_stream), "sca_debug_philox")
    return out


def philox_rate(threads: int = 1 << 20, calls: int = 256, device="cuda") -> float:
    """Philox4x32-10 blocks per second on this device (diagnostic kernel)."""
    sink = torch.zeros(256, dtype=torch.int32, device=device)
    stream = torch.cuda.current_stream(sink.device)
    L.check(L.lib().sca_debug_philox_rate(threads, calls, sink.data_ptr(), stream.cuda_stream), "philox_rate")
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    L.check(L.lib().sca_debug_philox_rate(threads, calls, sink.data_ptr(), stream.cuda_stream), "philox_rate")
    end.record(stream)
    end.synchronize()
    return threads * calls / (start.elapsed_time(end) / 1e3)
