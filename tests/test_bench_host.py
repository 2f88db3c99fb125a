"""Host-side logic of bench.py: the single-GPU guard, the rocprofv3 CSV
summaries and the link between committed counters and the kernel source."""
import csv
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _counter_csv(path, rows, grids=None):
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size",
                                           "Counter_Value"])
        wr.writeheader()
        for i, (name, val) in enumerate(rows):
            g = 256 * (grids[i] if grids else 1)
            wr.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": g, "Workgroup_Size": 256,
                         "Counter_Value": val})


def test_summarize_counters_calibrates_on_the_256_mib_copy(tmp_path):
    # a 256 MiB copy whose counters read half the fetched and all written
    # bytes, a 1 GiB copy (not a calibration), and CG launches: two updating,
    # one that exits early
    names = ["__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer",
             "void sdc::k_cg_iter<7, false, 1, false>(...)", "void sdc::k_cg_iter<7, false, 1, false>(...)",
             "void sdc::k_cg_iter<7, false, 1, false>(...)", "void sdc::k_post<4>(...)"]
    fetch = [131072.0, 524288.0, 100.0, 300.0, 0.5, 7.0]
    write = [262144.0, 1048576.0, 50.0, 150.0, 0.2, 9.0]
    _counter_csv(tmp_path / "f.csv", zip(names, fetch))
    _counter_csv(tmp_path / "w.csv", zip(names, write))
    out = bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert out["fetch_factor"] == pytest.approx(2.0) and out["write_factor"] == pytest.approx(1.0)
    assert out["dispatches"] == 3 and out["updating"] == 2
    assert out["fetch_kib_per_launch"] == pytest.approx(200.0)
    assert out["write_kib_per_launch"] == pytest.approx(100.0)
    assert out["measured_bytes_per_launch"] == pytest.approx((2.0 * 200.0 + 100.0) * 1024.0)


def test_summarize_counters_filters_by_launch_size(tmp_path):
    names = ["__amd_rocclr_copyBuffer", "void sdc::k_cg_iter<7, false, 1, false>(...)",
             "void sdc::k_cg_iter2<19, false, true>(...)"]
    grids = [1, 200, 8192]
    _counter_csv(tmp_path / "f.csv", zip(names, [131072.0, 100.0, 1000.0]), grids)
    _counter_csv(tmp_path / "w.csv", zip(names, [262144.0, 50.0, 400.0]), grids)
    out = bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), min_blocks=2048)
    assert out["dispatches"] == 1 and out["fetch_kib_per_launch"] == pytest.approx(1000.0)
    out = bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert out["dispatches"] == 2


def test_summarize_counters_rejects_mismatched_runs(tmp_path):
    _counter_csv(tmp_path / "f.csv", [("a", 1.0), ("b", 2.0)])
    _counter_csv(tmp_path / "w.csv", [("a", 1.0)])
    with pytest.raises(AssertionError):
        bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))


def test_summarize_trace_bins_cg_launches_by_grid(tmp_path):
    # the two-rows-per-thread kernel has 128-thread blocks over the same 256-row entries
    path = tmp_path / "kt.csv"
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Workgroup_Size_X"]
    rows = [("void sdc::k_cg_iter<7, false, 1, false>(...)", 0, 5000, 200 * 256, 256),
            ("void sdc::k_cg_iter<7, false, 1, false>(...)", 0, 7000, 200 * 256, 256),
            ("void sdc::k_cg_iter2<7, false, false>(...)", 0, 11000, 1024 * 128, 128),
            ("void sdc::k_rhs<4, 7, false>(...)", 0, 6000, 1024 * 256, 256)]
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=fields)
        wr.writeheader()
        for r in rows:
            wr.writerow(dict(zip(fields, r)))
    text = bench.summarize_trace(str(path))
    assert "| k_cg_iter | 2 | 0.01 | 6.000 |" in text and "| k_cg_iter2 | 1 | 0.01 | 11.000 |" in text
    assert "CG iteration (k_cg_iter, k_cg_iter2): 3 dispatches, mean 7.667 us" in text
    assert "| k_rhs | 1 | 0.01 | 6.000 |" in text
    assert "| 128..255 | 2 | 6.00 | 6.00 |" in text
    assert "| 1024..1024 | 1 | 11.00 | 11.00 |" in text


def test_summarize_trace_window_starts_after_the_calibration_copies(tmp_path):
    # a setup copy longer than the calibration copies, then three calibration
    # copies back to back, then the window
    path = tmp_path / "kt.csv"
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Workgroup_Size_X"]
    # (rows listed out of time order, as rocprofv3 may write them)
    cp = "__amd_rocclr_copyBuffer"
    rows = [("void sdc::k_cg_iter<7, false, 1, false>(...)", 10 ** 7, 10 ** 7 + 5000, 200 * 256, 256),
            (cp, 0, 400000, 1, 1), ("void sdc::k_rhs<4, 7, false>(...)", 10 ** 6, 10 ** 6 + 9000, 256, 256),
            (cp, 2 * 10 ** 6, 2 * 10 ** 6 + 118000, 1, 1), (cp, 3 * 10 ** 6, 3 * 10 ** 6 + 101000, 1, 1),
            (cp, 4 * 10 ** 6, 4 * 10 ** 6 + 99500, 1, 1), (cp, 2 * 10 ** 7, 2 * 10 ** 7 + 3000, 1, 1)]
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=fields)
        wr.writeheader()
        for r in rows:
            wr.writerow(dict(zip(fields, r)))
    text = bench.summarize_trace(str(path))
    assert text.startswith("dispatches counted: 2 of 7 (after the calibration copies)")
    assert "k_rhs" not in text and "| k_cg_iter | 1 |" in text


def test_measured_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    src, hdr = tmp_path / "k.hip", tmp_path / "k.hpp"
    src.write_bytes(b"kernel source")
    hdr.write_bytes(b"launch constants")
    sha = hashlib.sha256(b"kernel source" + b"launch constants").hexdigest()
    md = tmp_path / "c.md"
    md.write_text(f"# x\n\n- kernel sources sha256: {sha}\n- measured bytes per launch: 90.5\n"
                  f"- measured bytes per listed launch: 40.0\n- measured bytes per all-rows launch: 120.0\n")
    monkeypatch.setattr(bench, "KERNEL_SRCS", [str(src), str(hdr)])
    assert bench.measured_traffic(str(md)) == {"all": 90.5, "listed": 40.0, "all_rows": 120.0}
    hdr.write_bytes(b"launch constants, edited")   # a header edit counts as a kernel change
    assert bench.measured_traffic(str(md)) is None
    hdr.write_bytes(b"launch constants")
    src.write_bytes(b"kernel source, edited")
    assert bench.measured_traffic(str(md)) is None


def test_committed_counters_name_the_current_kernel_source():
    """The profile summary bench.py reads carries the hash of the kernel
    sources; a kernel edit without new counters makes `traffic` null."""
    text = open(bench.COUNTERS).read()
    assert "kernel sources sha256:" in text and "measured bytes per launch:" in text


def test_cg_launch_classes_and_roofline_byte_models():
    assert bench.cg_launch_class("void sdc::k_cg_iter2<7, false, true>(...)") == "all_rows"
    assert bench.cg_launch_class("void sdc::k_cg_iter<7, false, 1, false>(...)") == "listed"
    assert bench.cg_launch_class("void sdc::k_cg_iter<0, true, 0, false>(...)") == "all_rows"
    assert bench.cg_launch_class("void sdc::k_post<4>(...)") is None
    # two launches: one over all 1000 rows (7000 entries), one over a list of 200 rows (1400 entries), 1 ms each
    prof = {"cg_launches": 2, "cg_ms": 2.0, "cg_rows": 1200.0, "cg_nnz": 8400.0, "cg_all_launches": 1,
            "cg_all_ms": 1.0, "cg_all_rows": 1000.0, "cg_all_nnz": 7000.0}
    r = bench.cg_roofline(prof, "dia", 7)
    assert r["bytes_per_launch_csr_count"] == pytest.approx((12 * 8400 + 116 * 1200 + 4 * 200) / 2)
    assert r["bytes_per_launch_storage_min"] == pytest.approx(((8 * 4 + 68) * 1200 + 4 * 200) / 2)
    assert r["achieved"] == pytest.approx(((8 * 4 + 68) * 1200 + 4 * 200) / 2e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["csr_count_GBps"] == pytest.approx((12 * 8400 + 116 * 1200 + 4 * 200) / 2e-3 / 1e9)
    assert r["listed"]["launches"] == 1 and r["all_rows"]["rows_per_launch"] == 1000.0
    c = bench.cg_roofline(prof, "csr", 0)
    assert c["bytes_per_launch_storage_min"] == pytest.approx((12 * 8400 + 72 * 1200 + 4 * 200) / 2)
    t = bench.add_traffic(dict(r), {"all": 50.0, "listed": 20.0, "all_rows": 100.0}, prof)
    assert t["traffic"] == pytest.approx(60.0) and t["listed"]["traffic"] == 20.0
    assert t["frac_measured"] == pytest.approx(120.0 / 2e-3 / 1e9 / 8000.0)


def test_front_shell_masks_are_nested_shells_around_the_level_crossing():
    import numpy as np
    from workloads import meshes
    coords, elems = meshes.square_tri_mesh(21, 21, 1.0, 1.0)
    N = coords.shape[0]
    v = (coords[:, 0] < 0.42).astype(float)
    dens = (1.0, 0.5, 0.1, 1e-3)
    masks = bench.front_shell_masks(coords, elems, v, dens)
    assert [m.size for m in masks] == [max(1, round(d * N)) for d in dens]
    for m in masks:
        assert m.dtype == np.int32 and np.all(np.diff(m) > 0)
    for big, small in zip(masks, masks[1:]):
        assert np.isin(small, big).all()
    # the edges v crosses 0.5 on join the columns x = 0.40 and x = 0.45 (spacing 0.05)
    seeds = np.nonzero(np.isclose(coords[:, 0], 0.40) | np.isclose(coords[:, 0], 0.45))[0]
    assert np.isin(seeds, masks[2]).all()
    x = coords[masks[2], 0]
    assert x.min() >= 0.35 - 1e-12 and x.max() <= 0.50 + 1e-12
    assert masks[3][0] == seeds.min()
    # no crossing: the shells grow from the node whose value is nearest the level
    flat = bench.front_shell_masks(coords, elems, np.zeros(N), (1e-3, 0.05))
    assert flat[0].tolist() == [0]
    d = np.linalg.norm(coords[flat[1]] - coords[0], axis=1)
    assert d.max() <= np.sort(np.linalg.norm(coords - coords[0], axis=1))[flat[1].size - 1] + 1e-12
