"""The traffic record that bench.py reads for `roofline.traffic`: written by
`bench.py --record-traffic` from rocprofv3 counter CSVs.  Synthetic counter
files with known values check the per-launch means, the copy-calibration
scaling, the selection of the record's own kernel among other dispatches and
the source hash the record is keyed on."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

CHUNK = "void paf::(anonymous namespace)::chunk_kernel<10, false, false, 1>(paf::FilterParams)"
LABEL = "void paf::(anonymous namespace)::chunk_kernel<31, false, false, 1>(paf::FilterParams)"
KEY = "void paf::(anonymous namespace)::key_kernel<10, true>(paf::(anonymous namespace)::KeyParams)"
COPY = "__amd_rocclr_copyBuffer"


def write_run(d, sub, dispatches):
    """dispatches: [(kernel name, {counter: [values, one row each]})]."""
    os.makedirs(os.path.join(d, sub, "host"), exist_ok=True)
    with open(os.path.join(d, sub, "host", "r_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, counters) in enumerate(dispatches, start=1):
            for cn, vals in counters.items():
                for v in vals:
                    w.writerow([i, name, cn, v])


def sq(valu, waves=100.0):
    return {"SQ_WAVES": [waves], "SQ_INSTS_VALU": [valu / 2, valu / 2], "SQ_ACTIVE_INST_VALU": [valu],
            "SQ_THREAD_CYCLES_VALU": [valu * 32], "SQ_INSTS_MFMA": [0.0], "SQ_WAIT_ANY": [10.0],
            "SQ_WAVE_CYCLES": [40.0], "GRBM_GUI_ACTIVE": [8000.0]}


def test_record_traffic_from_counter_csvs(tmp_path):
    d = str(tmp_path / "runs")
    gib2 = 2 << 30
    # The copy reads half its bytes in FETCH_SIZE and all of them in WRITE_SIZE (KiB).
    write_run(d, "cfetch", [(COPY, {"FETCH_SIZE": [gib2 / 2 / 1024 / 4] * 4})])
    write_run(d, "cwrite", [(COPY, {"WRITE_SIZE": [gib2 / 1024]})])
    for kind in ("plain", "keyed"):
        disp_f = [(LABEL, {"FETCH_SIZE": [1e9]})] + [(CHUNK, {"FETCH_SIZE": [1000.0 + 10 * i, 1000.0]})
                                                      for i in range(3)]
        disp_w = [(LABEL, {"WRITE_SIZE": [1e9]})] + [(CHUNK, {"WRITE_SIZE": [20.0]}) for _ in range(3)]
        disp_v = [(LABEL, sq(1e12))] + [(CHUNK, sq(3000.0)) for _ in range(3)]
        if kind == "keyed":
            disp_f += [(KEY, {"FETCH_SIZE": [500.0]})]
            disp_w += [(KEY, {"WRITE_SIZE": [7.0]})]
            disp_v += [(KEY, sq(900.0, waves=8.0))]
        write_run(d, f"{kind}_fetch", disp_f)
        write_run(d, f"{kind}_write", disp_w)
        write_run(d, f"{kind}_valu", disp_v)
    out = str(tmp_path / "hbm.json")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--record-traffic", d, "--record-out", out,
                        "--pairs", "1000"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rec = json.load(open(out))
    assert set(rec) == {"snake_chunk_plain_250bp_E10", "snake_chunk_keyed_250bp_E10", "key_levels_250bp_E10"}
    p = rec["snake_chunk_plain_250bp_E10"]
    assert p["dispatches"] == 3 and p["n_pairs"] == 1000
    assert abs(p["fetch_scale"] - 2.0) < 1e-12 and abs(p["write_scale"] - 1.0) < 1e-12
    # Mean over the chunk kernel's dispatches of the summed rows, KiB -> bytes, scaled.
    assert abs(p["fetch_bytes_per_launch"] - (2010.0 * 1024 * 2.0)) < 1e-6
    assert abs(p["write_bytes_per_launch"] - 20.0 * 1024) < 1e-6
    assert p["bytes_per_launch"] == p["fetch_bytes_per_launch"] + p["write_bytes_per_launch"]
    assert p["valu_insts_per_launch"] == 3000.0 and abs(p["valu_lane_util"] - 0.5) < 1e-12
    assert abs(p["wait_per_wave_cycle"] - 0.25) < 1e-12 and p["gui_active_cycles_per_xcd"] == 1000.0
    assert p["kernel_sha256_16"] == bench.kernel_source_hash("snake_chunk")
    k = rec["key_levels_250bp_E10"]
    assert k["dispatches"] == 1 and k["fetch_bytes_per_launch"] == 500.0 * 1024 * 2.0
    assert k["kernel_sha256_16"] == bench.kernel_source_hash("key_levels")
    assert k["kernel_sha256_16"] != p["kernel_sha256_16"]


def test_traffic_record_used_only_for_matching_sources(tmp_path):
    """bench.traffic_record returns a record only while its hash matches the
    current sources of the kernel the record's key names."""
    good = {"kernel_sha256_16": bench.kernel_source_hash("snake_chunk"), "n_pairs": 1, "bytes_per_launch": 1.0}
    stale = dict(good, kernel_sha256_16="0" * 16)
    path = tmp_path / "hbm_traffic.json"
    path.write_text(json.dumps({"a": good, "b": stale}))
    assert bench.traffic_record("a", str(path)) == good
    assert bench.traffic_record("b", str(path)) is None
    assert bench.traffic_record("c", str(path)) is None
    assert bench.traffic_record("a", str(tmp_path / "missing.json")) is None
    # A levels-kernel record is checked against the levels kernel's sources.
    lv = {"kernel_sha256_16": bench.kernel_source_hash("key_levels"), "n_pairs": 1, "bytes_per_launch": 2.0}
    path.write_text(json.dumps({"key_levels_250bp_E10": lv, "key_levels_250bp_E5": good,
                                "snake_chunk_plain_250bp_E10": lv}))
    assert bench.traffic_record("key_levels_250bp_E10", str(path)) == lv
    assert bench.traffic_record("key_levels_250bp_E5", str(path)) is None
    assert bench.traffic_record("snake_chunk_plain_250bp_E10", str(path)) is None


def test_layout_list_parsing():
    """--layout 'W,K,F,P;...' becomes forced paf_layout dicts in order."""
    lays = bench.parse_layouts("2,6,2,3;4,4,1,2")
    assert [bench.layout_tuple(l) for l in lays] == [[2, 6, 2, 3], [4, 4, 1, 2]]
    assert all(l["lanes_per_pair"] == 1 and l["blocks_per_cu"] == 0 and l["tiles_per_grab"] == 1 for l in lays)
    assert bench.layout_tuple(bench.parse_layouts(bench.LAYOUT_SWEEP)[0]) == [2, 6, 2, 3]


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus above 1, or a launch with several
    ranks, exits with status 2 and says so before touching a device."""
    env = dict(os.environ)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 2 and "one GPU only" in r.stderr
    env["WORLD_SIZE"] = "2"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")],
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 2 and "one GPU only" in r.stderr
