"""Host logic of profile_summary.py on small hand-written rocprofv3 CSVs."""
import csv
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import profile_summary as PS  # noqa: E402


def test_short_name_strips_signature_and_anonymous_namespace():
    assert PS.short_name("void am::k_chain_f64_lds<8>(am::DevNet, unsigned long const*)") == "am::k_chain_f64_lds<8>"
    assert PS.short_name("am::(anonymous namespace)::k_edge_min(int const*, long long)") == "am::k_edge_min"
    assert PS.short_name("void rocprim::detail::scan_kernel<...>(...)") == "rocprim (scan / radix sort)"


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_dispatches_groups_by_workgroups(tmp_path):
    p = tmp_path / "trace.csv"
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Workgroup_Size_X"]
    rows = [["am::k(x)", 0, 10_000, 256 * 4, 256], ["am::k(x)", 0, 30_000, 256 * 4, 256],
            ["am::k(x)", 0, 20_000, 256 * 4, 256], ["am::k(x)", 0, 50_000, 256 * 8, 256],
            ["am::other(x)", 0, 99_000, 256, 256]]
    _write(p, hdr, rows)
    out = PS.dispatches(str(p), "am::k").splitlines()
    assert out[2] == "| 4 | 3 | 20.0 | 10.0 |"     # median of 10, 20, 30 us; fastest 10 us
    assert out[3] == "| 8 | 1 | 50.0 | 50.0 |"


def test_counter_scale_from_calibration_copies(tmp_path):
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    hdr = ["Kernel_Name", "Counter_Value", "Grid_Size"]
    mib = 256
    # copies read 2 x their size in FETCH_SIZE units (KiB), write 1 x
    _write(f, hdr, [["__amd_rocclr_copyBuffer", mib * 1024 / 2, 1]] * 3 + [["am::k(x)", 100.0, 1]])
    _write(w, hdr, [["__amd_rocclr_copyBuffer", mib * 1024, 1]] * 3 + [["am::k(x)", 50.0, 1]])
    fs = PS.calib_scale(PS.load_counter(str(f)), mib)
    ws = PS.calib_scale(PS.load_counter(str(w)), mib)
    assert fs == 2.0 and ws == 1.0
    table = PS.counters_table(str(f), str(w), mib, 4)
    # (100 x 2 + 50 x 1) KiB = 250 KiB = 0.256 MB
    assert "| `am::k` | 1 | 100.0 | 50.0 | 0.3 |" in table
