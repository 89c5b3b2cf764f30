"""The profile-summary helpers on synthetic rocprofv3 csv files (CPU)."""
import csv

from paper_1811_07325_amd import profsum

FIELDS = ["Kind", "Stream_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def write_trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for sid, s, e in rows:
            w.writerow({"Kind": "KERNEL_DISPATCH", "Stream_Id": sid, "Kernel_Name": "k", "Start_Timestamp": s,
                        "End_Timestamp": e})


def test_stream_overlap_counts_concurrent_streams(tmp_path):
    p = tmp_path / "trace.csv"
    # stream 1 busy [0, 100), stream 2 [50, 150), stream 3 [60, 70), stream 1 again [200, 300)
    write_trace(p, [(1, 0, 100), (2, 50, 150), (3, 60, 70), (1, 200, 300)])
    o = profsum.stream_overlap(str(p))
    assert o["dispatches"] == 4 and o["streams"] == 3
    assert abs(o["busy_ms"] - 250e-6) < 1e-12                 # [0, 150) and [200, 300)
    assert abs(o["frac_ge2_streams"] - 50 / 250) < 1e-12     # [50, 100)
    assert abs(o["frac_ge3_streams"] - 10 / 250) < 1e-12     # [60, 70)
    assert o["frac_ge4_streams"] == 0.0


def test_stream_overlap_back_to_back_kernels_of_one_stream(tmp_path):
    p = tmp_path / "trace.csv"
    write_trace(p, [(7, 0, 10), (7, 10, 20), (7, 20, 30)])
    o = profsum.stream_overlap(str(p))
    assert abs(o["busy_ms"] - 30e-6) < 1e-12 and o["frac_ge2_streams"] == 0.0
