"""Host-side tools: the profile summarizer's byte accounting on hand-made rocprofv3 CSVs, and
the benchmark's refusal of more than one GPU (no GPU needed)."""
import csv
import json
import os
import subprocess
import sys

from paper_2407_00829_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, prefix, entries):
    _write(os.path.join(d, f"{prefix}_counter_collection.csv"),
           ["Kernel_Name", "Counter_Name", "Counter_Value"], entries)


def test_profsum_traffic_two_kernel_product(tmp_path):
    """A product of two kernels (a gather pass and the fused kernel): per-dispatch counter
    means are added, scaled by the copy calibration (copy of 2 MiB: half read, half written),
    and the timed-region mean covers exactly the requested dispatches of each kernel."""
    t = str(tmp_path)
    ka, kb = "k_far_gather<float>(int const*)", "void k_spmv_stream<1, false>(PlanView)"
    # trace: 4 dispatches of each kernel, durations 10, 20, 30, 40 ns (a) and 100.. (b)
    trace = []
    for i in range(4):
        trace.append([ka, 1000 * i, 1000 * i + 10 * (i + 1)])
        trace.append([kb, 1000 * i + 500, 1000 * i + 500 + 100 * (i + 1)])
    _write(os.path.join(t, "tr", "run_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    _write(os.path.join(t, "tr", "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"],
           [[ka, 4, 100, 25, 10, 40], [kb, 4, 1000, 250, 100, 400]])
    # FETCH: a reads 10 KiB, b 90 KiB per dispatch; WRITE: 4 and 6 KiB
    _counters(os.path.join(t, "f"), "run", [[ka, "FETCH_SIZE", 10]] * 3 + [[kb, "FETCH_SIZE", 90]] * 3)
    _counters(os.path.join(t, "w"), "run", [[ka, "WRITE_SIZE", 4]] * 3 + [[kb, "WRITE_SIZE", 6]] * 3)
    # copy of 2 MiB: FETCH_SIZE reads 512 KiB of its 1024 KiB read (factor 2), WRITE exact
    _counters(os.path.join(t, "fc"), "copy", [["elementwise_kernel", "FETCH_SIZE", 512]])
    _counters(os.path.join(t, "wc"), "copy", [["elementwise_kernel", "WRITE_SIZE", 1024]])
    out = os.path.join(t, "out")
    profsum.main(["--name", "x", "--kernel", "k_far_gather + k_spmv_stream<1, false>",
                  "--trace", os.path.join(t, "tr"), "--fetch", os.path.join(t, "f"),
                  "--write", os.path.join(t, "w"), "--fetch-copy", os.path.join(t, "fc"),
                  "--write-copy", os.path.join(t, "wc"), "--copy-bytes", str(2 * 1024 ** 2),
                  "--cmd", "cmd", "--timed", "1,2", "--out", out])
    rec = json.load(open(os.path.join(out, "x_traffic.json")))
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["traffic_bytes"] == (100 * 2 + 10 * 1) * 1024
    assert rec["kernel_source_sha256"] == profsum.kernel_source_sha()
    # dispatches 1..2: a 20 and 30 ns, b 200 and 300 ns -> 25 + 250 ns = 0.275 us
    assert abs(profsum.timed_mean_us(os.path.join(t, "tr"), rec["kernel"], 1, 2) - 0.275) < 1e-12
    md = open(os.path.join(out, "x.md")).read()
    assert "Traffic per launch" in md and "Timed region" in md


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_profsum_dispatch_selection_and_append(tmp_path):
    """Counters and durations of the first N, the last N or all but the last N dispatches of a
    kernel (in dispatch order), the pmc summary over the same selection, and --append keeping
    one traffic record per kernel."""
    t = str(tmp_path)
    k = "void k_spmv_stream<1, false>(PlanView)"
    k2 = "void k_spmv_stream<1, true>(PlanView)"
    # 6 dispatches: FETCH 10, 20, ..., 60 KiB; durations 100, 200, ..., 600 ns
    _write(os.path.join(t, "tr", "run_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [[k, 1000 * i, 1000 * i + 100 * (i + 1)] for i in range(6)] +
           [[k2, 9000, 9400]])
    _write(os.path.join(t, "tr", "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"],
           [[k, 6, 2100, 350, 100, 600], [k2, 1, 400, 400, 400, 400]])
    rows = [[k, "FETCH_SIZE", 10 * (i + 1), i] for i in reversed(range(6))]  # out of order
    _write(os.path.join(t, "f", "run_counter_collection.csv"),
           ["Kernel_Name", "Counter_Name", "Counter_Value", "Dispatch_Id"],
           rows + [[k2, "FETCH_SIZE", 70, 7]])
    _write(os.path.join(t, "w", "run_counter_collection.csv"),
           ["Kernel_Name", "Counter_Name", "Counter_Value", "Dispatch_Id"],
           [[k, "WRITE_SIZE", 1, i] for i in range(6)] + [[k2, "WRITE_SIZE", 1, 7]])
    assert profsum.counter_mean_kib(os.path.join(t, "f"), "k_spmv_stream<1, false>", first=2) == (15.0, 2)
    assert profsum.counter_mean_kib(os.path.join(t, "f"), "k_spmv_stream<1, false>", last=2) == (55.0, 2)
    assert profsum.counter_mean_kib(os.path.join(t, "f"), "k_spmv_stream<1, false>", drop_last=2) == (25.0, 4)
    assert abs(profsum.last_mean_us(os.path.join(t, "tr"), "k_spmv_stream<1, false>", 2) - 0.55) < 1e-12
    _counters(os.path.join(t, "fc"), "copy", [["elementwise_kernel", "FETCH_SIZE", 512]])
    _counters(os.path.join(t, "wc"), "copy", [["elementwise_kernel", "WRITE_SIZE", 1024]])
    out = os.path.join(t, "out")
    common = ["--trace", os.path.join(t, "tr"), "--fetch", os.path.join(t, "f"),
              "--write", os.path.join(t, "w"), "--fetch-copy", os.path.join(t, "fc"),
              "--write-copy", os.path.join(t, "wc"), "--copy-bytes", str(2 * 1024 ** 2),
              "--cmd", "cmd", "--out", out]
    profsum.main(["--name", "c", "--kernel", "k_spmv_stream<1, false>", "--last", "2"] + common)
    profsum.main(["--name", "c", "--md-name", "c_nt", "--append", "--kernel",
                  "k_spmv_stream<1, true>"] + common)
    recs = json.load(open(os.path.join(out, "c_traffic.json")))
    assert [r["kernel"] for r in recs] == ["k_spmv_stream<1, false>", "k_spmv_stream<1, true>"]
    assert recs[0]["traffic_bytes"] == (55 * 2 + 1) * 1024 and recs[1]["traffic_bytes"] == (70 * 2 + 1) * 1024
    assert os.path.exists(os.path.join(out, "c.md")) and os.path.exists(os.path.join(out, "c_nt.md"))
    # pmc summary over the first 3 dispatches: mean FETCH 20, durations 100..300 ns
    profsum.main(["pmc", "--name", "p", "--kernel", "k_spmv_stream<1, false>",
                  "--dir", os.path.join(t, "f"), "--trace", os.path.join(t, "tr"), "--cmd", "cmd",
                  "--trace-cmd", "cmd", "--first", "3", "--note", "first three", "--out", out])
    md = open(os.path.join(out, "p.md")).read()
    assert "| FETCH_SIZE | 20 |" in md and "first three" in md
    assert "0.2 us over the counted ones (the first 3)" in md
