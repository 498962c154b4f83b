"""bench.py's host side: the records behind `roofline.traffic` and
`roofline.valu` are computed from rocprofv3 counter files as documented,
keyed by the kernel source's code and ignored once that code changes; the
algorithmic FLOP count of the vehicle workload; and the one-GPU contract."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench
from paper_2504_06437_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORKLOAD = "ground vehicle K=4096 T=50 J=100 P=8"
ROLLOUT = "void dbas::(anonymous namespace)::k_rollout<2, 16, 8>(dbas::DevParams, dbas::StepArgs)"
FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _counter_csv(folder, rows):
    """A rocprofv3-style counter_collection.csv: (dispatch, kernel, counter, value)."""
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(FIELDS)
        for r in rows:
            w.writerow(r)


def test_digest_ignores_comments_and_whitespace_only():
    src = "int f(int a) {\n    return a + 1;   // one more\n}\n/* block\n comment */\n"
    same = "int f(int a) { return a + 1; }\n// another comment\n"
    other = "int f(int a) { return a + 2; }\n"
    assert bench._kernel_digest(src) == bench._kernel_digest(same)
    assert bench._kernel_digest(src) != bench._kernel_digest(other)
    assert len(bench._kernel_digest(src)) == 16


def test_traffic_summary_scales_counters_by_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "_kernel_digest", lambda text=None: "00000000000000aa")
    copy_bytes = 64 << 20
    # the copy reads half its bytes in FETCH_SIZE and all of them in WRITE_SIZE
    _counter_csv(tmp_path / "cf", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", copy_bytes / 2048)])
    _counter_csv(tmp_path / "cw", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", copy_bytes / 1024)])
    # two rollout dispatches, each FETCH_SIZE split over two counter instances;
    # one dispatch of another instantiation (an autotune candidate) is ignored
    _counter_csv(tmp_path / "f", [(5, ROLLOUT, "FETCH_SIZE", 100.0), (5, ROLLOUT, "FETCH_SIZE", 200.0),
                                  (6, ROLLOUT, "FETCH_SIZE", 150.0), (6, ROLLOUT, "FETCH_SIZE", 150.0),
                                  (7, ROLLOUT.replace("16, 8", "64, 8"), "FETCH_SIZE", 9999.0)])
    _counter_csv(tmp_path / "w", [(5, ROLLOUT, "WRITE_SIZE", 250.0), (6, ROLLOUT, "WRITE_SIZE", 260.0)])
    out = tmp_path / "traffic.json"
    r = bench.summarize_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                                str(tmp_path / "cw"), copy_bytes, WORKLOAD, str(out))
    assert r["fetch_scale"] == pytest.approx(2.0) and r["write_scale"] == pytest.approx(1.0)
    assert r["fetch_kib_raw"] == pytest.approx(300.0) and r["write_kib_raw"] == pytest.approx(255.0)
    assert r["dispatches"] == [2, 2] and r["kernels"] == [ROLLOUT]
    assert r["bytes_per_launch"] == pytest.approx(300.0 * 1024 * 2 + 255.0 * 1024)
    # the bench reads the record back only while the kernel source is unchanged
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    os.replace(out, tmp_path / "profiles" / "traffic.json")
    assert bench.load_traffic("rollout", WORKLOAD) == pytest.approx(r["bytes_per_launch"])
    assert bench.load_traffic("rollout", "another workload") is None
    monkeypatch.setattr(bench, "_kernel_digest", lambda text=None: "00000000000000bb")
    assert bench.load_traffic("rollout", WORKLOAD) is None


def test_counter_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "_kernel_digest", lambda text=None: "00000000000000aa")
    # one dispatch: 4 waves of 1000 cycles each, VALU active 600 (units of 4
    # cycles), 1200 VALU instructions, of which 60 transcendental
    _counter_csv(tmp_path / "sq1", [(3, ROLLOUT, "SQ_ACTIVE_INST_VALU", 600.0), (3, ROLLOUT, "SQ_WAVE_CYCLES", 4000.0),
                                    (3, ROLLOUT, "SQ_WAVES", 4.0), (3, ROLLOUT, "SQ_INSTS_VALU", 1200.0),
                                    (3, ROLLOUT, "SQ_WAIT_ANY", 2000.0)])
    # 500 FMA, 200 ADD and 100 MUL wave instructions: 64 * (1000 + 200 + 100) FLOPs
    _counter_csv(tmp_path / "sq2", [(4, ROLLOUT, "SQ_INSTS_VALU_TRANS_F32", 60.0),
                                    (4, ROLLOUT, "SQ_INSTS_VALU_FMA_F32", 500.0),
                                    (4, ROLLOUT, "SQ_INSTS_VALU_ADD_F32", 200.0),
                                    (4, ROLLOUT, "SQ_INSTS_VALU_MUL_F32", 100.0)])
    out = tmp_path / "counters.json"
    r = bench.summarize_counters(str(tmp_path / "sq1"), str(tmp_path / "sq2"), WORKLOAD, str(out))
    assert r["active_valu_ratio"] == pytest.approx(0.6)
    assert r["valu_insts_per_wave"] == pytest.approx(300.0)
    assert r["wait_frac"] == pytest.approx(0.5) and r["trans_share"] == pytest.approx(0.05)
    assert r["executed_flops_per_launch"] == pytest.approx(64 * 1300.0)
    # the third pass: GRBM_GUI_ACTIVE summed over the 8 XCDs, 2.0e6 cycles
    # each, over a 1 ms dispatch is a 2 GHz clock; 1200 VALU instructions
    # over 1024 SIMDs and those cycles; no matrix-core cycles
    sq3 = tmp_path / "sq3"
    os.makedirs(sq3)
    with open(sq3 / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(FIELDS + ["Start_Timestamp", "End_Timestamp"])
        w.writerow([5, ROLLOUT, "GRBM_GUI_ACTIVE", 8 * 2.0e6, 1_000_000, 2_000_000])
        w.writerow([5, ROLLOUT, "SQ_VALU_MFMA_BUSY_CYCLES", 0.0, 1_000_000, 2_000_000])
    r3 = bench.summarize_counters(str(tmp_path / "sq1"), str(tmp_path / "sq2"), WORKLOAD, str(out), str(sq3))
    assert r3["clock_ghz"] == pytest.approx(2.0) and r3["mfma_busy_cycles"] == 0.0
    assert r3["valu_insts_per_simd_cycle"] == pytest.approx(1200.0 / 1024 / 2.0e6)
    assert r3["executed_flops_per_launch"] == pytest.approx(64 * 1300.0)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    os.replace(out, tmp_path / "profiles" / "counters.json")
    assert bench.load_counters("rollout", WORKLOAD) == {"active_valu_ratio": pytest.approx(0.6),
                                                        "valu_insts_per_wave": pytest.approx(300.0),
                                                        "wait_frac": pytest.approx(0.5),
                                                        "executed_flops_per_launch": pytest.approx(64 * 1300.0)}


def test_committed_records_match_the_kernel_source():
    """The committed traffic and counter records carry the kernel digest they
    were taken on.  When the kernel source has changed since, the bench
    reports null for them until the counters are taken again: skipped, with
    the reason, rather than failed."""
    stale = []
    for name in ("traffic.json", "counters.json"):
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        for workload in (bench.workload_name(W.quad_large()), WORKLOAD):
            r = rec["rollout"][workload]
            assert set(r) >= {"kernel_source_sha256_16", "kernels", "dispatches"}, (name, workload)
            if r["kernel_source_sha256_16"] != bench._kernel_digest():
                stale.append(f"{name} [{workload}]")
    if stale:
        pytest.skip("records that predate the kernel source (the bench reports null for them until "
                    "re-profiled): " + ", ".join(stale))


def test_algorithmic_flops_follow_the_per_term_table():
    """7 FLOPs a (shape point, obstacle) pair, reciprocals apart; 2 FMAs a
    shape point on the quadrotor's axis, 4 on the vehicle's rectangle; 15
    FLOPs and a reciprocal a costmap point; dynamics 14 (quadrotor) or 10
    (vehicle); stage, control and barrier costs 27 or 21.  Per rollout step:
    559 (small quadrotor), 5 695 (vehicle), 19 774 (quadrotor at scale), and
    3.24e10 FLOPs with 4.6e9 reciprocals per launch at scale."""
    for wl, flops, rcp in ((W.quad_small(), 559, 70), (W.car(), 5695, 800),
                           (W.quad_large(cells=16), 19774, 2807)):
        p = wl["params"]
        m = wl.get("map") is not None
        assert bench.rollout_flops_per_step(p, len(wl["obstacles"]), m) == flops
        assert bench.rollout_rcp_per_step(p, len(wl["obstacles"]), m) == rcp
    p = W.quad_large(cells=16)["params"]
    assert p["K"] * p["T"] * 19774 == pytest.approx(3.24e10, rel=1e-3)
    r = bench.roofline(p, 400, True, kernel_ms=0.5, launches=10)
    assert r["achieved"] == pytest.approx(p["K"] * p["T"] * 19774 / 0.5e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["rcp_per_launch"] == p["K"] * p["T"] * 2807


def test_workload_names():
    assert bench.workload_name(W.car()) == WORKLOAD
    assert bench.workload_name(W.quad_large(cells=16)).startswith("quadrotor K=16384 T=100 J=400 P=7 + 16x16 costmap")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
