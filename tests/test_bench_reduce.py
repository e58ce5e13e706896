"""The reduction of rocprofv3 counter output into the traffic summaries (bench.py --reduce),
on synthetic counter files: bytes per dispatch scaled by a plain device copy of known size
in the same run, and the refusal of a calibration against a copy of another size."""
import json
import os

import pytest

import bench


def write_counters(path, counter, rows):
    """A counter_collection.csv with the columns the reduction reads; rows: (dispatch, kernel,
    grid, value)."""
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        for d, k, g, v in rows:
            f.write('%d,"%s",%d,%s,%r\n' % (d, k, g, counter, v))


def runs(tmp_path, copy_bytes, kernel_read, kernel_write):
    """FETCH_SIZE counts half the bytes a copy reads and WRITE_SIZE all it writes (KiB), as
    measured on MI355X; two dispatches of a kernel, one small copy and one of copy_bytes."""
    kib = copy_bytes / 1024.0
    fetch = [(1, "__amd_rocclr_copyBuffer", 512, 4.0), (2, "__amd_rocclr_copyBuffer", 512, kib / 2),
             (3, "void mfl::k<4, double>(double*)", 1024, kernel_read / 1024.0 / 2),
             (4, "void mfl::k<4, double>(double*)", 1024, kernel_read / 1024.0 / 2)]
    write = [(1, "__amd_rocclr_copyBuffer", 512, 8.0), (2, "__amd_rocclr_copyBuffer", 512, kib),
             (3, "void mfl::k<4, double>(double*)", 1024, kernel_write / 1024.0),
             (4, "void mfl::k<4, double>(double*)", 1024, kernel_write / 1024.0)]
    write_counters(str(tmp_path / "fetch"), "FETCH_SIZE", fetch)
    write_counters(str(tmp_path / "write"), "WRITE_SIZE", write)
    return str(tmp_path / "fetch"), str(tmp_path / "write")


def test_traffic_scaled_by_the_copy(tmp_path):
    f, w = runs(tmp_path, 1 << 30, kernel_read=3.0e8, kernel_write=1.0e8)
    out = str(tmp_path / "t.json")
    bench.reduce_traffic(f, w, 1 << 30, {"k": {"match": "k<4, double>", "algorithmic_bytes": 2.0e8}},
                         2.0e8, "synthetic", [], out)
    rec = json.load(open(out))
    assert rec["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["calibration"]["write_scale"] == pytest.approx(1.0)
    k = rec["kernels"]["k"]
    assert k["dispatches"] == [2, 2]
    assert k["hbm_read_bytes"] == pytest.approx(3.0e8)
    assert k["hbm_write_bytes"] == pytest.approx(1.0e8)
    assert k["hbm_over_algorithmic"] == pytest.approx(2.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(4.0e8)


def test_calibration_against_a_copy_of_another_size_refused(tmp_path):
    # the run's largest copy moved 1 GiB, the reduction is told 136 MB
    f, w = runs(tmp_path, 1 << 30, kernel_read=3.0e8, kernel_write=1.0e8)
    with pytest.raises(SystemExit):
        bench.reduce_traffic(f, w, 135796744, {"k": {"match": "k<4, double>"}}, None, "synthetic", [],
                             str(tmp_path / "t.json"))


def test_algorithmic_models():
    n, c, q = 257 ** 3, 64 ** 3, 125
    assert bench.apply_bytes(n, c, q, 8, "stored") == 1846554640
    assert bench.apply_bytes(n, c, q, 8, "otf") == 24 * n + 8 * c
    assert bench.apply_bytes(n, c, q, 8, "cartesian") == 16 * n + 8 * c
    # plain sum-factorization count per cell: 12 (stored) or 18 (on the fly) applications of
    # n^4 multiply-adds, plus the point work
    assert bench.apply_flops(5, 1, "stored") == 24 * 625 + 18 * 125
    assert bench.apply_flops(5, 1, "otf") == 36 * 625 + 49 * 125
