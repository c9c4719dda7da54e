"""Throughput of the bit-vectorized octahedron-model SCA sweep on one MI355X.

A step is one run of the sweep-throughput workload: the flat surface on the
2^16 x 2^16 lattice (1 GiB of packed slopes, resident in HBM), 2000 MCS at
p = 1, q = 0 (seed 42), then the exact height moments.  The metric is site
updates per second (X * Y * 2000 * steps / time).  The sweep runs as the
temporally blocked passes sca_plan_step reports (152 passes of 13 MCS and two
of 12 for 2000 MCS); the warm-up steps run the same plan, so no kernel's first
launch is timed.  The roofline object prices the whole-pass kernel, whose
launches are timed with HIP events on the stream they run on: against HBM
with its algorithmic traffic (every packed slope word read once and written
once per pass, X*Y/4 bytes each way) and against the 32-bit VALU issue rate
with the instructions per launch that rocprofv3 counted; the roof the pass
comes closer to is the bound.  The paper's own bandwidth model (Sec. III: 1
byte per site update, one pass per half-step) is reported under a key of its
own.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: 32-bit VALU lane instructions/s
COUNTERS = os.path.join(ROOT, "profiles", "mcs_fixed_65536x65536_p1_counters.json")
VALU_COUNTERS = os.path.join(ROOT, "profiles", "valu_random_paths_counters.json")


def _ensure_built():
    from paper_1606_00310_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()


def _sha(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _pass_counters():
    """rocprofv3 counters of the blocked-pass kernel (HBM bytes and VALU
    instructions per launch), if they were taken on the current kernel
    sources."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return {}
    files = [os.path.join(ROOT, s) for s in c.get("sources", [])]
    if not files or c.get("sources_sha256") != _sha(files):
        return {}
    return c


def _valu_per_update(tag):
    """VALU lane instructions per site update that rocprofv3 counted for the
    path's kernel, if the kernel sources are unchanged since."""
    try:
        with open(VALU_COUNTERS) as f:
            c = json.load(f)[tag]
    except (OSError, ValueError, KeyError):
        return None
    files = [os.path.join(ROOT, s) for s in c["sources"]]
    if c.get("sources_sha256") != _sha(files):
        return None
    return c["valu_lane_instructions_per_site_update"]


def _hbm_per_update(tag):
    """Counted HBM bytes per site update of the path's kernel (FETCH_SIZE and
    WRITE_SIZE scaled by a device copy's counts), if they were taken and the
    kernel sources are unchanged since."""
    try:
        with open(VALU_COUNTERS) as f:
            c = json.load(f)[tag]
    except (OSError, ValueError, KeyError):
        return None
    files = [os.path.join(ROOT, s) for s in c["sources"]]
    if c.get("sources_sha256") != _sha(files) or "hbm_bytes_per_dispatch" not in c:
        return None
    return c["hbm_bytes_per_dispatch"] / c["site_updates_per_dispatch"]


def pass_roofline(alg_bytes, avg_ms, counters):
    """The pass kernel against HBM (algorithmic bytes per launch over the
    launch time) and, when rocprofv3 counted its VALU instructions per launch
    (`counters`, from _pass_counters), against the 32-bit VALU issue rate; the
    roof the pass comes closer to is `bound`, the other one sits beside it.
    `traffic` is the counted HBM bytes per launch, or None."""
    achieved = alg_bytes / (avg_ms / 1e3) / 1e9
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roofline = dict(hbm)
    valu = counters.get("valu", {}).get("sq_insts_valu_per_launch")
    if valu:
        # VALU lane instructions per launch (wave instructions x 64) over the launch time
        va = valu * 64 / (avg_ms / 1e3)
        alu = {"bound": "alu", "achieved": va, "peak": VALU_LANE_OPS, "unit": "VALU lane instructions/s",
               "frac": round(va / VALU_LANE_OPS, 4)}
        if alu["frac"] > hbm["frac"]:
            roofline = dict(alu, hbm=hbm)
        else:
            roofline["alu"] = alu
    roofline["traffic"] = counters.get("hbm_bytes_per_launch")
    return roofline


def time_path(torch, P, X, Y, p, q, seed, steps, warmup, force_persite=False, split=None, blocking=None):
    """Milliseconds for `steps` MCS after `warmup` MCS.  With split = m the
    timed region is recorded as two parts, the first m MCS (whole fused passes)
    and the rest; returns (total, first part).  blocking = (depth, band) for
    sca_set_blocking (default: the library's automatic choice)."""
    lat = P.Lattice(X, Y, seed=seed)
    if blocking is not None:
        lat.set_blocking(*blocking)
    lat.step(warmup, p, q, force_persite=force_persite)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    mid = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    if split:
        lat.step(split, p, q, force_persite=force_persite)
        mid.record(lat.stream)
        lat.step(steps - split, p, q, force_persite=force_persite)
    else:
        lat.step(steps, p, q, force_persite=force_persite)
    end.record(lat.stream)
    end.synchronize()
    ms = start.elapsed_time(end)
    first = start.elapsed_time(mid) if split else None
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return (ms, first) if split else ms


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(X, Y, p, q, seed, rows, budget_s, threads=None, max_mcs=200):
    """The oracle, untuned, on a band of `rows` full-width rows of the same
    workload (a light-cone patch with a frozen border), one MCS at a time
    until about budget_s seconds of CPU work, with `threads` OpenMP threads
    (default: all)."""
    import oracle

    prev = oracle.num_threads()
    if threads:
        oracle.set_num_threads(threads)
    try:
        used = oracle.num_threads()
        st = oracle.flat_patch(X, Y, 0, 0, X, rows, track_heights=False) if rows < Y else oracle.flat(X, Y, False)
        n, dt = 0, 0.0
        while dt < budget_s and n < max_mcs:
            t0 = time.perf_counter()
            oracle.run(st, 1, p, q, seed=seed)
            dt += time.perf_counter() - t0
            n += 1
    finally:
        oracle.set_num_threads(prev)
    return {"value": X * rows * n / dt, "unit": "site updates/s", "cores": used, "kind": "oracle",
            "sample": f"{X} x {rows} band of the {X}x{Y} p={p} q={q} workload (frozen border), {n} MCS "
                      f"in {dt:.1f} s on {used} thread(s)"}


def cpu_baseline(X, Y, p, q, seed, rows, budget_s):
    """The oracle on all host cores (the reported value) and on one core."""
    out = oracle_rate(X, Y, p, q, seed, rows, budget_s)
    one = oracle_rate(X, Y, p, q, seed, max(16, rows // 16), budget_s / 2, threads=1)
    out["one_core"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
    out["cpu_model"] = cpu_model()
    out["host_cpus"] = os.cpu_count()
    return out


def comparator_rate(X, Y, p, q, seed, budget_s, max_mcs=400):
    """The bit-vectorized CPU sweep (64-bit words, OpenMP over rows, the
    paper's kind of CPU code, Sec. II-B) from the flat surface, one MCS at a
    time until about budget_s seconds, on all host threads."""
    import comparator

    lat = comparator.Lattice(X, Y, seed)
    lat.step(1, p, q)  # first touch of the state
    n, dt = 0, 0.0
    while dt < budget_s and n < max_mcs:
        t0 = time.perf_counter()
        lat.step(1, p, q)
        dt += time.perf_counter() - t0
        n += 1
    return {"value": X * Y * n / dt, "unit": "site updates/s", "cores": comparator.num_threads(),
            "kind": "bit-vectorized CPU sweep (w=64)", "cpu_model": cpu_model(),
            "sample": f"{X}x{Y} p={p} q={q} from the flat surface, {n} MCS in {dt:.1f} s"}


def bench_headline(torch, P, w, steps, warmup):
    """`steps` timed runs of workload w after `warmup` untimed ones.  A run
    resets the lattice to the flat surface, advances w.n_mcs MCS and takes the
    exact moments; its whole blocked passes are bracketed by HIP events on the
    lattice's stream (the MCS after them, the remainder passes, run as a second
    call, which gives bit-identical results)."""
    lat = P.Lattice(w.X, w.Y, seed=w.seed)
    plan = lat.plan(w.n_mcs, w.p, w.q)
    n_main = plan["n_pass"] * plan["depth"]
    rest = lat.plan(w.n_mcs - n_main, w.p, w.q) if w.n_mcs > n_main else None
    stream = lat.stream

    def run(evs=None):
        lat.reset()
        if evs:
            evs[0].record(stream)
        if n_main:
            lat.step(n_main, w.p, w.q)
        if evs:
            evs[1].record(stream)
        if rest:
            lat.step(w.n_mcs - n_main, w.p, w.q)
        return lat.roughness()

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    moments = []
    start.record(stream)
    for k in range(steps):
        moments.append(run(evs[k]))
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    pass_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs)
    t, h0 = lat.meta()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    # p = 1, q = 0 from the flat surface: h = 2t + ((x+y)&1) after every MCS
    closed = None
    if (w.p, w.q) == (1.0, 0.0):
        N, T = w.sites, w.n_mcs
        closed = all(m[:3] == (N, N * (4 * T + 1) // 2, N * (8 * T * T + 4 * T + 1) // 2) for m in moments) \
            and (t, h0) == (T, 2 * T)
    return {"ms": ms, "pass_ms": pass_ms, "plan": plan, "rest_plan": rest, "n_main": n_main,
            "closed_form_holds": closed}


def device_copy_rate(torch, nbytes=2**30, reps=10):
    """HBM bytes per second of torch's plain device kernels on an nbytes
    buffer: a copy (read + written, the mixed rate a copy gets), a sum (read
    only) and a fill (written only) -- practical ceilings beside the
    published peak."""
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    ops = {"copy": (lambda: dst.copy_(src), 2 * nbytes), "read": (lambda: src.sum(), nbytes),
           "write": (lambda: dst.fill_(3), nbytes)}
    out = {}
    for name, (op, moved) in ops.items():
        for _ in range(3):
            op()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op()
        e1.record()
        e1.synchronize()
        out[name] = moved / (e0.elapsed_time(e1) / 1e3 / reps)
    del src, dst
    torch.cuda.empty_cache()
    return out


def bench_ensemble(torch, P, n=4096, solo_per_L=3, tune_scale=10, serving=True, solo=True):
    """The 4096-realization ensemble in one persistent launch vs one launch
    (graph-captured MCS loop) per realization, and a serving run."""
    from paper_1606_00310_amd import autotune, serve
    from paper_1606_00310_amd.batch import Batch, Realization, state_bytes
    from paper_1606_00310_amd.inputs import ensemble, poisson_arrivals

    members = ensemble(n)
    reals = [Realization(m.L, m.L, m.p, 0.0, m.n_mcs, m.seed) for m in members]
    work = sum(r.sites * r.n_mcs for r in reals)
    # The autotuner runs the whole ensemble with every MCS budget divided by
    # tune_scale: the same mix of sizes and the same ratio of the longest
    # realization (the critical path of one workgroup) to the total work.
    sample = [Realization(r.X, r.Y, r.p, r.q, max(1, r.n_mcs // tune_scale), r.seed) for r in reals]
    cfg, table = autotune.autotune(sample, cache_path=None)

    b = Batch(max_slots=len(reals), arena_bytes=sum(state_bytes(r.X, r.Y) for r in reals), config=cfg)
    b.admit(reals)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    launches = 0
    while b.run(max(r.n_mcs for r in reals)):
        launches += 1
    end.record(b.stream)
    end.synchronize()
    batched_s = start.elapsed_time(end) / 1e3
    b.close()
    del b
    torch.cuda.empty_cache()

    out = {"realizations": len(reals), "site_updates": work,
           "batched": {"seconds": batched_s, "value": work / batched_s, "unit": "site updates/s",
                       "launches": launches, "config": cfg},
           "autotune": [{"config": c, "ms": round(t * 1e3, 3)} for c, t in table]}
    if not solo:
        return out

    # one realization at a time through the single-lattice API, a stratified
    # sample of each lattice size, timed with the MCS loop graph-captured
    # (capture + instantiate + one launch) and with plain launches
    by_L = {}
    for r in reals:
        by_L.setdefault(r.X, []).append(r)
    est = {"graph": 0.0, "plain": 0.0}
    per_L = {}
    for L_, group in sorted(by_L.items()):
        pick = group[:solo_per_L]
        upd = sum(r.sites * r.n_mcs for r in pick)
        tot_upd = sum(r.sites * r.n_mcs for r in group)
        row = {}
        for mode in ("graph", "plain"):
            t_sum = 0.0
            for r in pick:
                lat = P.Lattice(r.X, r.Y, seed=r.seed)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lat.step(r.n_mcs, r.p, r.q, graph=(mode == "graph"))
                torch.cuda.synchronize()
                t_sum += time.perf_counter() - t0
                lat.close()
            rate = upd / t_sum
            est[mode] += tot_upd / rate
            row[mode] = rate
        per_L[str(L_)] = {"realizations": len(group), "sampled": len(pick),
                          "solo_graph_updates_per_s": row["graph"], "solo_plain_updates_per_s": row["plain"]}
    solo_s = min(est.values())
    out.update({"solo_estimate": {"seconds_graph": est["graph"], "seconds_plain": est["plain"],
                             "value": work / solo_s, "unit": "site updates/s", "per_L": per_L,
                             "method": f"{solo_per_L} realizations per lattice size timed one by one, "
                                       "scaled by each size's total work"},
           "speedup_vs_solo": solo_s / batched_s})
    if not serving:
        return out

    # serving: Poisson arrivals of small ensembles at 0.8x the measured capacity
    rng = np.random.default_rng(4242)
    n_req = 400
    reqs = []
    seed = 5_000_000
    for i in range(n_req):
        k = int(rng.integers(1, 5))
        rs = []
        for _ in range(k):
            m = members[int(rng.integers(len(members)))]
            rs.append(Realization(m.L, m.L, m.p, 0.0, m.n_mcs, seed))
            seed += 1
        reqs.append(serve.Request(i, rs))
    mean_work = sum(r.work for r in reqs) / n_req
    capacity_rps = (work / batched_s) / mean_work
    rate = 0.8 * capacity_rps
    arr = poisson_arrivals(n_req, rate, rng_seed=99)
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    budget = 16 << 30
    sb = Batch(max_slots=1024, arena_bytes=budget, config=cfg)
    quota = 100 * 2048 * 2048  # site updates per realization per epoch: 100 MCS of the largest lattice
    srv = serve.Server(serve.BatchBackend(sb, keep_states=False), work_quota=quota)
    t0 = time.perf_counter()
    done = srv.serve(reqs)
    wall = time.perf_counter() - t0
    sb.close()
    served = sum(r.work for r in done)
    out["serving"] = {"requests": n_req, "arrival_rate_per_s": rate, "capacity_requests_per_s": capacity_rps,
                      "hbm_budget_bytes": budget, "epoch_site_updates_per_realization": quota,
                      "epochs": srv.epochs,
                      "throughput": served / wall, "unit": "site updates/s", "wall_s": wall,
                      "latency": serve.latency_stats(done)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed runs of the 2000-MCS workload")
    ap.add_argument("--warmup", type=int, default=3, help="untimed runs before them")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-paths", action="store_true", help="skip the secondary paths")
    ap.add_argument("--cpu-rows", type=int, default=16384)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched ensemble and serving runs")
    ap.add_argument("--comparator-seconds", type=float, default=8.0,
                    help="time budget of the bit-vectorized CPU sweep (0: skip it)")
    ap.add_argument("--ensemble-only", action="store_true", help="only the batched ensemble (for profiling)")
    ap.add_argument("--only", choices=["random", "half", "persite", "wide"],
                    help="time one secondary path for --mcs MCS and print it (for profiling)")
    ap.add_argument("--mcs", type=int, default=200, help="MCS timed by --only (after 24 warm-up MCS)")
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
    from paper_1606_00310_amd.inputs import HEADLINE, HEADLINE_HALF, HEADLINE_RANDOM, PERSITE, WIDE

    if args.copy_calibration:
        src = torch.ones(2**30 // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    if args.only:
        wk = {"random": HEADLINE_RANDOM, "half": HEADLINE_HALF, "persite": PERSITE, "wide": WIDE}[args.only]
        pms = time_path(torch, P, wk.X, wk.Y, wk.p, wk.q, wk.seed, args.mcs, 24)
        print(json.dumps({"path": wk.name, "mcs": args.mcs, "ms": pms,
                          "value": wk.sites * args.mcs / (pms / 1e3)}), flush=True)
        return

    if args.ensemble_only:
        print(json.dumps({"ensemble": bench_ensemble(torch, P, serving=False, solo=False)}), flush=True)
        return

    w = HEADLINE
    K, Wm = args.steps, args.warmup
    hb = bench_headline(torch, P, w, K, Wm)
    ms = hb["ms"]
    plan = hb["plan"]
    value = w.sites * w.n_mcs * K / (ms / 1e3)
    # the dominant kernel: the whole blocked passes, state read once and
    # written once per launch (X*Y/4 bytes each way)
    alg_bytes = w.sites // 2
    launches = plan["n_pass"] * K
    avg_ms = hb["pass_ms"] / launches
    pc = _pass_counters()
    # counters taken on another kernel (or another instantiation) do not apply
    if pc and plan["kernel"] not in pc.get("kernel", "").replace(" ", ""):
        pc = {}
    roofline = pass_roofline(alg_bytes, avg_ms, pc)
    roofline.update({
        "kernel": plan["kernel"], "launches_timed": launches, "launches_per_step": plan["n_pass"],
        "mcs_per_launch": plan["depth"], "band_rows": plan["band"], "alg_bytes_per_launch": alg_bytes,
        "alg_bytes_per_site_update": alg_bytes / (w.sites * plan["depth"]), "avg_launch_ms": round(avg_ms, 5),
        "share_of_step_time": round(hb["pass_ms"] / ms, 4),
        "remainder": {"kernel": plan["tail_kernel"], "mcs": [plan["tail1"], plan["tail2"]]},
        # the paper's bandwidth model (Sec. III): 1 byte per site update, one
        # pass over the state per half-step; here a pass covers 2*depth half-steps
        "paper_model_1B_per_update": {"equivalent_GBps": round(value / 1e9, 1),
                                      "note": "site updates/s x 1 B; not HBM traffic"},
    })
    # the counted traffic of the pass against what a plain device copy of
    # 1 GiB moves per second on this GPU (reads and writes mixed, as in the pass)
    rates = device_copy_rate(torch)
    copy_gbs = rates["copy"] / 1e9
    roofline["device_copy"] = {"GBps": round(copy_gbs, 1), "bytes_per_copy": 2 * 2**30,
                               "note": "torch copy_ of 1 GiB, read + written",
                               "read_only_GBps": round(rates["read"] / 1e9, 1),
                               "write_only_GBps": round(rates["write"] / 1e9, 1)}
    if roofline.get("traffic"):
        counted = roofline["traffic"] / (avg_ms / 1e3) / 1e9
        roofline["device_copy"].update({"pass_counted_GBps": round(counted, 1),
                                        "pass_over_copy": round(counted / copy_gbs, 4)})

    out = {
        "metric": "site updates/s (bit-vectorized + arbitrary-p) vs HBM roofline; batched vs solo",
        "value": value, "unit": "site updates/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (flat initial surface)",
        "config": {"workload": w.name, "X": w.X, "Y": w.Y, "p": w.p, "q": w.q, "seed": w.seed,
                   "mcs_per_step": w.n_mcs, "step": "flat init + 2000 MCS + exact moments"},
        "roofline": roofline,
        "closed_form_holds": hb["closed_form_holds"],
    }

    if not args.no_paths:
        paths = {}
        # X = 2^17 runs 6-MCS passes (the LDS-window kernel with 1024-thread
        # workgroups) on 256-row bands, set explicitly so that its HBM roofline
        # below knows the pass depth.
        WIDE_DEPTH = 6
        for wk, steps, ps, blk in ((HEADLINE_HALF, 200, False, None), (HEADLINE_RANDOM, 200, False, None),
                                   (PERSITE, 100, False, None), (WIDE, 60, False, (WIDE_DEPTH, 256))):
            # 24 warm-up MCS: several whole passes over freshly allocated state
            # (the first passes over a new 8 GiB lattice pair run about 10 % slower)
            pms = time_path(torch, P, wk.X, wk.Y, wk.p, wk.q, wk.seed, steps, 24, ps, blocking=blk)
            rate = wk.sites * steps / (pms / 1e3)
            paths[wk.name] = {"value": rate, "unit": "site updates/s", "steps": steps,
                              "hbm_frac_1B_per_update": round(rate / (HBM_PEAK_GBS * 1e9), 4)}
        # the 2^17 pass is bandwidth-bound: its algorithmic traffic is the state
        # read and written once per pass, X*Y/4 bytes each way per WIDE_DEPTH MCS
        pw = paths[WIDE.name]
        wa = pw["value"] / (2 * WIDE_DEPTH) / 1e9  # passes/s x X*Y/2 bytes per pass
        pw["roofline"] = {"bound": "hbm", "achieved": round(wa, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(wa / HBM_PEAK_GBS, 4), "mcs_per_pass": WIDE_DEPTH,
                          "kernel": "mcs_block_lds_kernel<16,6,false>"}
        # The random-word paths are bound by the VALU (Philox4x32-10): priced
        # against 256 CUs x 64 lanes x 2.4 GHz of 32-bit VALU issue with the
        # VALU instructions per site update that rocprofv3's SQ_INSTS_VALU
        # counted for the same kernel build (profiles/valu_random_paths_*).
        for tag, wk in (("persite", PERSITE), ("random", HEADLINE_RANDOM), ("half", HEADLINE_HALF)):
            per_update = _valu_per_update(tag)
            pv = paths[wk.name]
            pv["roofline"] = None if per_update is None else {
                "bound": "alu", "achieved": pv["value"] * per_update, "peak": VALU_LANE_OPS,
                "unit": "VALU lane instructions/s", "frac": round(pv["value"] * per_update / VALU_LANE_OPS, 4),
                "valu_lane_instructions_per_site_update": per_update}
        # the p = 1/2 pass's counted HBM traffic beside its VALU roof
        bpu = _hbm_per_update("half")
        if bpu is not None and paths[HEADLINE_HALF.name]["roofline"] is not None:
            gbs = paths[HEADLINE_HALF.name]["value"] * bpu / 1e9
            paths[HEADLINE_HALF.name]["roofline"]["hbm"] = {
                "counted_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                "bytes_per_site_update": round(bpu, 5), "over_device_copy": round(gbs / copy_gbs, 4)}
        paths[PERSITE.name]["philox_only_blocks_per_s"] = P.philox_rate()
        out["paths"] = paths

    if not args.no_ensemble:
        out["ensemble"] = bench_ensemble(torch, P)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w.X, w.Y, w.p, w.q, w.seed, args.cpu_rows, args.cpu_seconds)
        if args.comparator_seconds > 0:
            # The paper's GPU/CPU comparison (Sec. III): the GPU at 2^16 x 2^16
            # against a bit-vectorized CPU code at 2^14 x 2^14, both at p = 1/2.
            cr = comparator_rate(16384, 16384, 0.5, 0.0, HEADLINE_HALF.seed, args.comparator_seconds)
            gpu_half = out.get("paths", {}).get(HEADLINE_HALF.name, {}).get("value")
            cr["gpu_p0.5_65536x65536_over_this"] = (gpu_half / cr["value"]) if gpu_half else None
            out["cpu_comparator"] = cr

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
