"""Continuous batching of ensemble requests on one GPU.

A request is an ensemble run: a list of independent realizations (lattice
size, p, q, MCS budget, seed).  Requests queue in arrival order.  Before
every epoch the server admits queued requests, whole ones only, while the
batch has free slots and free arena bytes (the HBM budget).  It then advances
every admitted realization in one persistent launch -- by a fixed number of
MCS, or by a work quota of site updates so that small lattices finish in one
epoch while large ones advance a few MCS --
retires the finished ones (exact moments, final state, origin height) and
frees their slots and memory for the next arrivals.

Realizations that arrive while others are running share the same launches,
so their work overlaps on the device.  Each realization draws only from its
own seed's counters, so its result is bit-identical to running it alone.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    realizations: list            # batch.Realization
    arrival: float = 0.0          # seconds on the server clock
    admitted: float | None = None
    done: float | None = None
    slots: list = field(default_factory=list)
    results: list = field(default_factory=list)  # per realization: dict

    @property
    def work(self) -> int:
        return sum(r.sites * r.n_mcs for r in self.realizations)

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


class BatchBackend:
    """The GPU batch (batch.Batch) behind the server."""

    def __init__(self, batch, keep_states: bool = True):
        self.batch = batch
        self.keep_states = keep_states

    def try_admit(self, realizations):
        return self.batch.try_admit(realizations)

    def run(self, mcs_epoch):
        return self.batch.run(mcs_epoch)

    def run_work(self, site_updates):
        return self.batch.run_work(site_updates)

    def sync(self):
        import torch

        torch.cuda.current_stream(self.batch.device).synchronize()

    def finished(self, slot) -> bool:
        info = self.batch.info(slot)
        return info.t >= info.n_mcs

    def collect(self, slot):
        S, h0 = self.batch.state(slot)
        out = {"moments": self.batch.roughness(slot), "h0": int(h0[0])}
        if self.keep_states:
            out["slopes"] = S.clone()
        return out

    def release(self, slot):
        self.batch.release(slot)


class Server:
    def __init__(self, backend, mcs_epoch: int = 100, clock=time.perf_counter, work_quota: int | None = None):
        """mcs_epoch: MCS per epoch; or, if work_quota is given, site updates
        per realization per epoch (at least one MCS)."""
        self.backend = backend
        self.mcs_epoch = int(mcs_epoch)
        self.work_quota = None if work_quota is None else int(work_quota)
        self.clock = clock
        self.t0 = clock()
        self.queue: deque[Request] = deque()
        self.running: dict[int, Request] = {}   # rid -> request
        self.slot_owner: dict[int, tuple[int, int]] = {}  # slot -> (rid, index in request)
        self.completed: list[Request] = []
        self.epochs = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request):
        self.queue.append(req)

    def _admit(self):
        # arrival order; a request that does not fit blocks the ones behind it
        while self.queue:
            req = self.queue[0]
            slots = self.backend.try_admit(req.realizations)
            if slots is None:
                if not self.running:
                    raise RuntimeError(f"request {req.rid} can never fit the batch budget")
                return
            self.queue.popleft()
            req.slots = slots
            req.results = [None] * len(slots)
            req.admitted = self.now()
            self.running[req.rid] = req
            for i, s in enumerate(slots):
                self.slot_owner[s] = (req.rid, i)

    def _retire(self):
        for slot in list(self.slot_owner):
            if self.backend.finished(slot):
                rid, i = self.slot_owner.pop(slot)
                req = self.running[rid]
                req.results[i] = self.backend.collect(slot)
                self.backend.release(slot)
                if all(r is not None for r in req.results):
                    req.done = self.now()
                    self.completed.append(req)
                    del self.running[rid]

    def step(self) -> int:
        """Admit, run one epoch, retire.  Returns the realizations advanced."""
        self._admit()
        # zero-MCS realizations finish without running
        self._retire()
        self._admit()
        if not self.running:
            active = 0
        elif self.work_quota is not None:
            active = self.backend.run_work(self.work_quota)
        else:
            active = self.backend.run(self.mcs_epoch)
        if active:
            self.epochs += 1
            self.backend.sync()
        self._retire()
        return active

    def serve(self, arrivals, idle_sleep: float = 1e-4):
        """Feeds requests at their arrival times (seconds from now) and runs
        until all have completed.  arrivals: iterable of Request with .arrival
        set relative to the start."""
        pending = deque(sorted(arrivals, key=lambda r: r.arrival))
        self.t0 = self.clock()
        while pending or self.queue or self.running:
            now = self.now()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if not self.queue and not self.running:
                time.sleep(min(idle_sleep, max(0.0, pending[0].arrival - now)))
                continue
            self.step()
        return self.completed


def latency_stats(reqs):
    lat = np.array([r.latency for r in reqs if r.latency is not None], dtype=np.float64)
    if lat.size == 0:
        return {}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "n": int(lat.size)}
