"""The rocprofv3 summariser that writes profiles/ and profiles/traffic.json (host
logic only): on synthetic CSV files in rocprofv3's layout it must pick the full
launches, scale FETCH_SIZE / WRITE_SIZE by the copy kernel's readings and carry
the algorithmic work of each launch into the roofline table."""
import csv
import json
import os

from paper_2405_04253_amd import profile_summary as P

import bench

TRACE_COLS = ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"]
PMC_COLS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def write_csv(path, cols, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(cols, r)))


def test_summary_tables_and_traffic(tmp_path):
    k = "void (anonymous namespace)::aeq_pol_kernel<4, 1>(fnti::AeqItem const*, int)"
    d = str(tmp_path)
    # two full launches of 80 ms and 82 ms, one small launch (autotuning) that must be ignored
    write_csv(f"{d}/trace/run_kernel_trace.csv", TRACE_COLS,
              [(k, 131072, 0, 80_000_000), (k, 131072, 100_000_000, 182_000_000), (k, 4096, 0, 5_000_000)])
    # FETCH_SIZE split over two rows of one dispatch (summed), WRITE_SIZE in a separate run
    write_csv(f"{d}/fetch/run_counter_collection.csv", PMC_COLS,
              [(1, k, 131072, "FETCH_SIZE", 500.0), (1, k, 131072, "FETCH_SIZE", 500.0),
               (2, k, 131072, "FETCH_SIZE", 1000.0), (3, k, 4096, "FETCH_SIZE", 7.0)])
    write_csv(f"{d}/write/run_counter_collection.csv", PMC_COLS,
              [(1, k, 131072, "WRITE_SIZE", 3000.0), (2, k, 131072, "WRITE_SIZE", 3000.0)])
    # the copy kernel moves 1 MiB each way and reads 512 KiB FETCH, 1024 KiB WRITE
    c = "void at::native::copy_kernel(int)"
    write_csv(f"{d}/cf/run_counter_collection.csv", PMC_COLS, [(1, c, 1 << 20, "FETCH_SIZE", 512.0)])
    write_csv(f"{d}/cw/run_counter_collection.csv", PMC_COLS, [(1, c, 1 << 20, "WRITE_SIZE", 1024.0)])
    write_csv(f"{d}/sq/run_counter_collection.csv", PMC_COLS,
              [(1, k, 131072, "SQ_INSTS_VALU", 2e9), (1, k, 131072, "SQ_INSTS_LDS", 1e8)])
    blocks = 1000
    launches = {"batched": [{"kernel": "aeq_pol_kernel<4, 1>", "key": "aeq_pol_kernel<4, 1> (lead)",
                             "aeq_blocks": blocks, "cdc_blocks": 0,
                             "algorithmic_ops": bench.AEQ_OPS_PER_BLOCK * blocks,
                             "algorithmic_bytes": blocks * 16 * 12}]}
    with open(f"{d}/launches.json", "w") as f:
        json.dump(launches, f)
    md, tr = f"{d}/out.md", f"{d}/traffic.json"
    P.main(["--workload", "batched", "--launches", f"{d}/launches.json", "--trace", f"{d}/trace",
            "--fetch", f"{d}/fetch", "--write", f"{d}/write", "--calib-fetch", f"{d}/cf",
            "--calib-write", f"{d}/cw", "--calib-bytes", str(1 << 20), "--sq", f"{d}/sq",
            "--cmd", "rocprofv3 --kernel-trace -- python3 bench.py", "--md", md, "--traffic", tr])
    t = json.load(open(tr))
    assert abs(t["calibration"]["fetch_scale"] - 2.0) < 1e-12 and abs(t["calibration"]["write_scale"] - 1.0) < 1e-12
    e = t["batched"]["aeq_pol_kernel<4, 1> (lead)"]
    assert e["grid"] == 131072 and e["dispatches"] == 2 and abs(e["avg_ms"] - 81.0) < 1e-9
    assert e["fetch_kib_raw"] == 1000.0 and e["write_kib_raw"] == 3000.0
    assert e["bytes_per_launch"] == 1000 * 1024 * 2.0 + 3000 * 1024 * 1.0
    assert e["aeq_blocks"] == blocks and e["algorithmic_ops"] == bench.AEQ_OPS_PER_BLOCK * blocks
    assert e["source_hash"] == bench.kernel_source_hash()
    assert e["SQ_INSTS_VALU"] == 2e9
    text = open(md).read()
    gops = bench.AEQ_OPS_PER_BLOCK * blocks / 81.0 / 1e6
    assert f"{gops:.1f}" in text and "rocprofv3 --kernel-trace -- python3 bench.py" in text
    assert P.short_name(k) == "aeq_pol_kernel<4, 1>"
