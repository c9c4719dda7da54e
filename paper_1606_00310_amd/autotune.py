"""Autotuner for the persistent ensemble kernel.

It times each launch configuration (workgroup size, workgroups per compute
unit, LDS budget, word tile, processing order and the depth of the blocked
passes over large realizations) on a sample of the ensemble, checks that
every configuration leaves bit-identical states, and keeps the fastest.  The
sample should keep the ensemble's mix: with the MCS budgets scaled down
uniformly it has the same ratio of the longest realization (which one
workgroup runs alone) to the total work, so the ranking carries over.
The choice is cached in a JSON file keyed by the device name and the sample's
signature.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from .batch import Batch, state_bytes

LDS_PER_CU = 160 * 1024

# Blocked passes of 2 MCS for every shape, and of 3 or 4 MCS with one
# 512-thread workgroup per CU (the shape whose registers hold their window).
# 1-MCS passes are left out: on MI355X they ran 1.4-1.9x slower than 2-MCS
# passes of the same shape, since the launch streams every state from HBM.
CANDIDATES = [
    dict(block_threads=bt, blocks_per_cu=bpc, lds_bytes=65536, order=0, words_per_lane=wpl, depth=depth,
         max_parts=parts)
    for bt in (512, 1024)
    for bpc in (1, 2)
    for wpl in (1, 2)
    for depth in (2, 3, 4)
    for parts in (1, 2, 4)
    if bpc * 65536 <= LDS_PER_CU and bt * bpc <= 2048 and (depth <= 2 or (bt == 512 and bpc == 1))
]

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_batch.json")


def signature(reals) -> str:
    h = hashlib.sha256()
    for r in reals:
        h.update(f"{r.X},{r.Y},{r.p},{r.q},{r.n_mcs},{r.seed},{int(r.force_persite)};".encode())
    return h.hexdigest()[:16]


def _states(batch, slots):
    """The final states (slopes and origin height) of the whole sample as one
    device tensor, so that a configuration is checked with one comparison."""
    parts = []
    for s in slots:
        S, h0 = batch.state(s)
        parts += [S.reshape(-1), h0]
    return torch.cat(parts)


def time_config(reals, cfg, epoch=None, device="cuda"):
    """Seconds for one epoch over the sample with this configuration, and the
    final states."""
    b = Batch(max_slots=len(reals), arena_bytes=sum(state_bytes(r.X, r.Y) for r in reals), device=device,
              config=cfg)
    slots = b.admit(reals)
    torch.cuda.synchronize()
    epoch = epoch or max(r.n_mcs for r in reals)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    while b.run(epoch):
        pass
    end.record(b.stream)
    end.synchronize()
    secs = start.elapsed_time(end) / 1e3
    states = _states(b, slots)
    b.close()
    return secs, states


def autotune(reals, candidates=CANDIDATES, cache_path: str | None = DEFAULT_CACHE, force: bool = False,
             verbose: bool = False):
    """Returns (best config, table of (config, seconds)).  Raises if two
    configurations disagree on any bit of any final state."""
    dev = torch.cuda.get_device_name()
    key = f"{dev}|{signature(reals)}"
    if cache_path and not force and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"], cache[key]["table"]
    table = []
    ref = None
    for cfg in candidates:
        secs, states = time_config(reals, cfg)
        if ref is None:
            ref = states
        elif not torch.equal(states, ref):
            raise RuntimeError(f"configuration {cfg} changed the results")
        table.append((cfg, secs))
        if verbose:
            print(f"  {cfg} {secs * 1e3:.2f} ms", flush=True)
    best = min(table, key=lambda x: x[1])[0]
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {"best": best, "table": table}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, table
