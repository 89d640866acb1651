"""Host-side pieces of the measurement: roofline bookkeeping and the rocprofv3
summaries (no GPU needed)."""
import csv
import json
import os

import bench
from paper_2504_17615_amd import profiling as P


def test_short_names():
    assert P.short_name("void lmgp::(anonymous namespace)::k_rate_big<2>(lmgp::RateArgs)") == \
        "k_rate_big<2>"
    assert P.short_name("void lmgp::(anonymous namespace)::k_rate_group<64, 0>(lmgp::RateArgs)") \
        == "k_rate_group<64, 0>"
    assert P.short_name("lmgp::k_radix_hist(unsigned long const*, int)") == "k_radix_hist"
    assert P.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_roofline_picks_single_kernel_with_most_time():
    stats = {
        "cl:k_rate_big<2>": {"launches": 10, "total_ns": 1_000_000, "bytes": 2_000_000_000},
        "rf:k_rate_big<2>": {"launches": 10, "total_ns": 500_000, "bytes": 2_000_000_000},
        "cl:rate_hubs<2>": {"launches": 1, "total_ns": 9_000_000, "bytes": 1},
        "rf:k_rate_block<0>": {"launches": 4, "total_ns": 1_200_000, "bytes": 100},
    }
    r = bench.roofline(stats, steps=1, wall=1.0, workload="none")
    assert r["kernel"] == "k_rate_big<2>"  # 1.5 ms over both phases; hubs excluded
    assert r["launches"] == 20
    assert abs(r["achieved"] - 4e9 / 1.5e6) < 0.1  # bytes / ns = GB/s
    assert r["frac"] == round(r["achieved"] / 8000.0, 4)
    assert r["traffic"] is None


def _counter_csv(path, counter, rows):
    cols = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Kernel_Name": k,
                        "Counter_Name": counter, "Counter_Value": v})


def test_traffic_calibration(tmp_path):
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>(int)"
    kern = "void lmgp::(anonymous namespace)::k_rate_big<2>(lmgp::RateArgs)"
    # the copy of 64 MiB reads back as half its size on FETCH_SIZE: factor 2
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [(copy, 32768.0), (kern, 100.0), (kern, 300.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [(copy, 65536.0), (kern, 10.0), (kern, 10.0)])
    src = os.path.relpath(bench.__file__, P.ROOT)
    out = tmp_path / "t.json"
    P.write_traffic(str(out), str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 64, "x", src,
                    "cf", "cw")
    rec = json.load(open(out))
    assert rec["calibration"]["fetch_factor"] == 2.0
    assert rec["calibration"]["write_factor"] == 1.0
    k = rec["kernels"]["k_rate_big<2>"]
    assert k["dispatches"] == 2
    assert k["hbm_bytes_per_launch"] == (400 + 10) * 1024


def test_committed_traffic_record_is_well_formed():
    path = os.path.join(bench.ROOT, "profiles", "traffic_rmat22.json")
    if not os.path.exists(path):
        return
    rec = json.load(open(path))
    assert rec["workload"] == "rmat22"
    assert os.path.exists(os.path.join(bench.ROOT, rec["source"]))
    for k, v in rec["kernels"].items():
        assert v["hbm_bytes_per_launch"] >= 0 and v["dispatches"] > 0


def test_roofline_with_breakdown_from_a_separate_step():
    # timed region: only the dominant kernel's launches carry events
    timed = {"cl:k_rate_big<2>": {"launches": 30, "total_ns": 3_000_000, "bytes": 6_000_000_000}}
    warm = {
        "cl:k_rate_big<2>": {"launches": 10, "total_ns": 1_000_000, "bytes": 2_000_000_000},
        "rf:k_rate_block<0>": {"launches": 4, "total_ns": 500_000, "bytes": 100},
    }
    assert bench.dominant_kernel(warm) == "k_rate_big<2>"
    r = bench.roofline(timed, steps=3, wall=0.01, workload="none", breakdown=warm)
    assert r["kernel"] == "k_rate_big<2>" and r["launches"] == 30
    assert abs(r["achieved"] - 2000.0) < 0.1
    assert set(r["kernels"]) == {"k_rate_big<2>", "k_rate_block<0>"}
    assert r["kernels"]["k_rate_big<2>"]["ms_per_step"] == 1.0  # one warm-up step
    assert r["lp_rate_all"]["share_of_step"] == round(1.5e6 / 1e9 / 0.01, 3)
