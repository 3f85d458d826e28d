"""Host logic of bench.py that needs no GPU: the kernel names it reports,
launch grids, the roofline byte model, and the attribution of profiled
dispatches to sweep runs."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_1405_1020_amd import binding as B  # noqa: E402


def test_lds_model_bytes():
    # 20 U + 8 L with U = 2(2r+1): the figures of the roofline model
    assert bench.lds_bytes_per_pixel(15, 20) == 1400
    assert bench.lds_bytes_per_pixel(5, 64) == 952
    assert bench.lds_bytes_per_pixel(0, 1) == 48


def test_kernel_names():
    assert bench.kernel_name(15, 20, B.Variant(0, 4, B.HIST_COLUMN, 64, 8)) == "k_plain_column15<7, 4>"
    assert bench.kernel_name(10, 32, B.Variant(0, 1, B.HIST_COLUMN, 64, 8)) == "k_plain_column15<11, 1>"
    assert bench.kernel_name(5, 8, B.Variant(0, 2, B.HIST_COLUMN, 64, 8)) == "k_plain_column15<3, 2>"
    assert bench.kernel_name(5, 64, B.Variant(0, 4, B.HIST_COLUMN, 64, 4)) == "k_plain_column15<22, 4>"
    assert bench.kernel_name(16, 20, B.Variant(0, 1, B.HIST_COLUMN, 64, 8)) == "k_plain_column<2>"
    assert bench.kernel_name(16, 20, B.Variant(0, 4, B.HIST_COLUMN, 64, 4)) == "k_plain_column31<10, 4>"
    assert bench.kernel_name(31, 64, B.Variant(0, 2, B.HIST_COLUMN, 64, 8)) == "k_plain_column31<32, 2>"
    assert bench.kernel_name(32, 20, B.Variant(0, 4, B.HIST_COLUMN, 64, 4)) == "k_plain_column<2>"
    assert bench.kernel_name(15, 100, B.Variant(0, 1, B.HIST_COLUMN, 64, 8)) == "k_plain_column<2>"
    assert bench.kernel_name(5, 64, B.Variant(0, 4, B.HIST_STREAM, 64, 4)) == "k_plain_split<5, 16>"
    assert bench.kernel_name(10, 20, B.Variant(0, 4, B.HIST_STREAM8, 64, 5)) == "k_plain_split8<10, 5>"


def test_launch_threads():
    # the streamed and column layouts: one run of `rows` per workgroup of
    # 64 x waves threads; the tile-staged layout: a run per wavefront
    assert bench.launch_threads(1920, 1080, [16, 4, 4, 64, 8]) == 30 * 68 * 256
    assert bench.launch_threads(1920, 1080, [26, 4, 1, 64, 5]) == 30 * 42 * 256
    assert bench.launch_threads(1920, 1080, [8, 2, 0, 64, 4]) == 30 * 68 * 128


def test_sweep_run_values_shared_kernel():
    # r10 and r15 launch the same kernel with the same grid: a step launches
    # every run once, then each run is timed alone in a block of equal length
    runs = [("a", "k1", 1), ("b", "k2", 2), ("c", "k2", 2), ("d", "k3", 3)]
    seq = []
    for step in range(3):
        seq += [("k1", 1, 10 + step), ("k2", 2, 20 + step), ("k2", 2, 30 + step), ("k3", 3, 40 + step)]
    seq += [("k1", 1, 11)] * 4 + [("k2", 2, 21)] * 4 + [("k2", 2, 31)] * 4 + [("k3", 3, 41)] * 4
    rows = [("f", i, k, g, v) for i, (k, g, v) in enumerate(seq)]
    out = bench.sweep_run_values(rows, runs)
    assert out["a"] == [10, 11, 12] + [11] * 4
    assert out["b"] == [20, 21, 22] + [21] * 4
    assert out["c"] == [30, 31, 32] + [31] * 4
    assert out["d"] == [40, 41, 42] + [41] * 4


def test_sweep_run_values_files_and_uneven_blocks():
    # dispatch ids restart per process file; a block that does not split
    # evenly among the runs sharing its key is left out; unknown kernels
    # are ignored
    runs = [("b", "k2", 2), ("c", "k2", 2)]
    rows = [("f1", 1, "k2", 2, 1.0), ("f1", 2, "k2", 2, 2.0), ("f1", 3, "kx", 9, 0.0),
            ("f1", 4, "k2", 2, 3.0),
            ("f2", 1, "k2", 2, 4.0), ("f2", 2, "k2", 2, 5.0)]
    out = bench.sweep_run_values(rows, runs)
    assert out["b"] == [1.0, 4.0]
    assert out["c"] == [2.0, 5.0]


def test_counter_metrics_per_xcd_and_sdk_precedence():
    # raw counters of two dispatches: GRBM_GUI_ACTIVE is the sum over the
    # XCDs, so per XCD it is 1/XCDS of it
    cus = 256
    gui = 1000.0 * bench.XCDS
    d = [{"kernel": "k", "grid": 1, "GRBM_GUI_ACTIVE": gui, "SQ_LDS_IDX_ACTIVE": 0.5 * 1000 * cus,
          "SQ_LDS_BANK_CONFLICT": 0.1 * 1000 * cus, "SQ_ACTIVE_INST_VALU": 0.25 * 1000 * cus,
          "SQ_INSTS_LDS": 64.0, "SQ_INSTS_VALU": 128.0}] * 2
    e = bench.counter_metrics(d, [1000.0, 3000.0], cus, 32)
    assert e["dispatches"] == 2 and e["trace_mean_us"] == 2.0
    assert e["lds_util"] == 0.5 and e["valu_busy"] == 0.25 and e["binding_unit"] == "lds"
    assert e["lds_bank_conflict_rate"] == round(0.1 / 0.4, 4)
    assert e["lds_insts_per_pixel"] == 2.0 and e["valu_insts_per_pixel"] == 4.0
    # rocprofiler-sdk's derived figures (per cent) take precedence
    d2 = [dict(d[0], LdsUtil=40.0, VALUBusy=60.0, LdsBankConflict=0.05)]
    e2 = bench.counter_metrics(d2, [], cus, 0)
    assert e2["lds_util"] == 0.4 and e2["lds_util_raw"] == 0.5 and e2["valu_busy"] == 0.6
    assert e2["lds_bank_conflict_rate"] == 0.05 and e2["binding_unit"] == "valu"
