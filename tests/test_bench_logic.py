"""Host logic of bench.py: the roofline object of the pass kernel and the
check that ties stored counters to the kernel sources they were taken on."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_roofline_hbm_only_without_counters():
    r = bench.pass_roofline(2**31, 0.5, {})
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS
    assert r["achieved"] == round(2**31 / 0.5e-3 / 1e9, 1)
    assert r["frac"] == round(r["achieved"] / bench.HBM_PEAK_GBS, 4)
    assert r["traffic"] is None and "alu" not in r and "hbm" not in r


def test_roofline_picks_the_closer_roof():
    # 0.5 ms per launch: 4.29 TB/s algorithmic (0.54 of HBM); VALU lane
    # instructions of 0.7 and 0.3 of the 32-bit peak over the same time
    for frac, bound in ((0.7, "alu"), (0.3, "hbm")):
        waves = frac * bench.VALU_LANE_OPS * 0.5e-3 / 64
        c = {"valu": {"sq_insts_valu_per_launch": waves}, "hbm_bytes_per_launch": 123}
        r = bench.pass_roofline(2**31, 0.5, c)
        assert r["bound"] == bound and r["traffic"] == 123
        other = r["hbm"] if bound == "alu" else r["alu"]
        assert other["bound"] != bound
        alu = r if bound == "alu" else r["alu"]
        assert abs(alu["frac"] - frac) < 1e-4 and alu["peak"] == bench.VALU_LANE_OPS


def test_stored_counters_name_existing_sources():
    """Every counters file names the sources it was taken on, and they exist;
    bench.py reports its figures only while their sha256 is unchanged."""
    for name in ("mcs_fixed_65536x65536_p1_counters.json", "valu_random_paths_counters.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            c = json.load(f)
        entries = [c] if "sources" in c else list(c.values())
        for e in entries:
            assert e["sources"] and len(e["sources_sha256"]) == 64
            for src in e["sources"]:
                assert os.path.exists(os.path.join(ROOT, src)), src


def test_cpu_baseline_helpers():
    """The oracle timing reports the threads it used and the host's CPU model."""
    r = bench.oracle_rate(256, 256, 1.0, 0.0, 42, 64, 0.05, threads=1)
    assert r["cores"] == 1 and r["kind"] == "oracle" and r["value"] > 0 and "1 thread" in r["sample"]
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_counted_bytes_of_the_half_pass_match_its_pass_model():
    """The p = 1/2 pass's counted HBM bytes per site update lie between the
    algorithmic figure (the state read and written once per 4-MCS pass, 1/8
    byte per site update) and that figure with the whole band halo read
    twice (reads 1.25 x for 8 halo rows above and below a 128-row band)."""
    bpu = bench._hbm_per_update("half")
    if bpu is None:  # counters taken on other kernel sources: not reported
        return
    assert 0.125 <= bpu <= 0.125 * (1 + 0.25) / 2 + 0.125 / 2 + 1e-9
