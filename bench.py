"""Throughput of the bit-vectorized octahedron-model SCA sweep on one MI355X.

A step is one Monte-Carlo step (the even and the odd half-step) over the
2^16 x 2^16 lattice (1 GiB of packed slopes, resident in HBM), p = 1, q = 0,
seed 42, grown from the flat surface.  The metric is site updates per second
(X * Y * steps / time), timed with HIP events on the stream the kernels run
on.  The roofline object prices the half-step kernel against HBM bandwidth
with its algorithmic traffic: every packed slope word is read once and
written once per half-step, X*Y/4 bytes each way (1 byte per site update per
MCS, the paper's bandwidth model in Sec. III).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
COUNTERS = os.path.join(ROOT, "profiles", "halfstep_65536x65536_p1_counters.json")
SWEEP_SRC = os.path.join(ROOT, "paper_1606_00310_amd", "csrc", "sweep.hip")


def _ensure_built():
    from paper_1606_00310_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _traffic(bytes_per_launch_alg):
    """Counter-measured HBM bytes per half-step launch, if the counters were
    taken on the current kernel source."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("sweep_sha256") != _sha(SWEEP_SRC):
        return None
    return c.get("hbm_bytes_per_launch")


def time_path(torch, P, X, Y, p, q, seed, steps, warmup, force_persite=False):
    lat = P.Lattice(X, Y, seed=seed)
    lat.step(warmup, p, q, force_persite=force_persite)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.step(steps, p, q, force_persite=force_persite)
    end.record(lat.stream)
    end.synchronize()
    ms = start.elapsed_time(end)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return ms


def cpu_baseline(X, Y, p, q, seed, rows, budget_s, max_mcs=200):
    """The oracle, untuned, on a band of `rows` full-width rows of the same
    workload (a light-cone patch with a frozen border), one MCS at a time
    until about budget_s seconds of CPU work."""
    import oracle

    st = oracle.flat_patch(X, Y, 0, 0, X, rows, track_heights=False) if rows < Y else oracle.flat(X, Y, False)
    n, dt = 0, 0.0
    while dt < budget_s and n < max_mcs:
        t0 = time.perf_counter()
        oracle.run(st, 1, p, q, seed=seed)
        dt += time.perf_counter() - t0
        n += 1
    sites = X * rows
    return {"value": sites * n / dt, "unit": "site updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{X} x {rows} band of the {X}x{Y} p={p} q={q} workload (frozen border), {n} MCS "
                      f"in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-paths", action="store_true", help="skip the secondary paths")
    ap.add_argument("--cpu-rows", type=int, default=16384)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (torch copy_) three times, the known-size "
                         "reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the single-lattice sweep and the ensembles are measured per GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    _ensure_built()
    import paper_1606_00310_amd as P
    from paper_1606_00310_amd.inputs import HEADLINE, HEADLINE_RANDOM, PERSITE

    if args.copy_calibration:
        src = torch.ones(2**30 // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    w = HEADLINE
    K, Wm = args.steps, args.warmup
    torch.cuda.synchronize()
    ms = time_path(torch, P, w.X, w.Y, w.p, w.q, w.seed, K, Wm)
    value = w.sites * K / (ms / 1e3)
    launches = 2 * K
    avg_ms = ms / launches
    alg_bytes = w.sites // 2  # read X*Y/4 + write X*Y/4 bytes per half-step
    achieved = alg_bytes / (avg_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(alg_bytes),
                "kernel": "halfstep_kernel<64,8,Mask,false>", "alg_bytes_per_launch": alg_bytes,
                "avg_launch_ms": round(avg_ms, 5)}

    out = {
        "metric": "site updates/s (bit-vectorized sweep) vs HBM roofline",
        "value": value, "unit": "site updates/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (flat initial surface)",
        "config": {"workload": w.name, "X": w.X, "Y": w.Y, "p": w.p, "q": w.q, "seed": w.seed,
                   "mcs_per_step": 1},
        "roofline": roofline,
    }

    if not args.no_paths:
        paths = {}
        for wk, steps, ps in ((HEADLINE_RANDOM, 200, False), (PERSITE, 100, False)):
            pms = time_path(torch, P, wk.X, wk.Y, wk.p, wk.q, wk.seed, steps, 5, ps)
            rate = wk.sites * steps / (pms / 1e3)
            paths[wk.name] = {"value": rate, "unit": "site updates/s", "steps": steps,
                              "hbm_frac_1B_per_update": round(rate / (HBM_PEAK_GBS * 1e9), 4)}
        out["paths"] = paths

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w.X, w.Y, w.p, w.q, w.seed, args.cpu_rows, args.cpu_seconds)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
