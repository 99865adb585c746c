"""Host-side checks of the benchmark's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The benchmark measures one GPU; --gpus above 1 exits with a message and no JSON line."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert "{" not in r.stdout


def test_source_hash_covers_the_kernel_sources():
    """The traffic records are used only while the kernel sources hash to their recorded value."""
    sys.path.insert(0, ROOT)
    import bench
    h = bench.source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    rec = bench.read_traffic("dst_cols", "2d_m255_n256", 6)
    assert rec is None or rec > 0


def _pmc_csv(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for i, (name, val) in enumerate(rows):
            f.write(f'"{i}","{name}","{counter}","{val}"\n')


def test_traffic_summary_scales_counters_by_the_reference_copy(tmp_path):
    """The committed converter from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) to bytes per launch: scaled by what the counters read for the 1 GiB reference copy,
    per kernel variant of the workload's transform lengths, other kernels ignored."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    cols = "void qbvm::k_dst_cols_p2<256, 1, true>(qbvm::DstArgs)"
    rows = "void qbvm::k_dst_rows_p2<256, 5>(qbvm::DstArgs)"
    inp = "void qbvm::k_dst_rows_p2<256, 2>(qbvm::DstArgs)"
    tim = "void qbvm::k_time_gt<3, 43, 1, true>(qbvm::TimeArgs)"
    other = "void qbvm::k_dst_cols_p2<512, 6, true>(qbvm::DstArgs)"  # 2D length: not this workload
    copy = "__amd_rocclr_copyBuffer"
    gib = 1 << 20
    _pmc_csv(str(tmp_path / "f" / "host" / "1_fetch_counter_collection.csv"), "FETCH_SIZE",
             [(copy, gib / 2), (copy, gib / 2), (copy, gib / 2), (cols, 1000.0), (cols, 1002.0), (cols, 1001.0), (rows, 500.0), (inp, 7.0),
              (tim, 3.0), (other, 9.0), (copy, 2 * gib)])
    _pmc_csv(str(tmp_path / "w" / "host" / "1_write_counter_collection.csv"), "WRITE_SIZE",
             [(copy, gib), (copy, gib), (copy, gib), (cols, 2000.0), (cols, 2000.0), (cols, 2000.0), (rows, 1000.0), (inp, 7.0),
              (tim, 4000.0), (other, 9.0), (copy, 4 * gib)])
    out = tmp_path / "out"
    out.mkdir()
    bench.write_traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), "3d_m127_n128", str(out))
    rec = json.load(open(out / "dst_cols_3d_m127_n128_traffic.json"))
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    e = rec["per_variant"]["1"]
    assert e["dispatches"] == 3 and e["fetch_kib_median"] == 1001.0
    assert e["hbm_bytes_per_launch"] == round((1001.0 * 2.0 + 2000.0) * 1024)
    assert json.load(open(out / "dst_rows_3d_m127_n128_traffic.json"))["per_variant"]["5"]["hbm_bytes_per_launch"] \
        == round((500.0 * 2 + 1000.0) * 1024)
    assert "2" in json.load(open(out / "dst_input_3d_m127_n128_traffic.json"))["per_variant"]
    assert "1" in json.load(open(out / "time_spectral_3d_m127_n128_traffic.json"))["per_variant"]
    md = open(out / "traffic_3d_m127_n128.md").read()
    assert "k_dst_cols_p2<512" not in md and "--traffic-summary" in md
