"""Summaries of rocprofv3 CSV output for profiles/: kernel durations and HBM bytes.

    python -m paper_2407_00829_amd.profsum --name spmv_c2 --kernel "k_spmv_stream<1, false>" \
        --trace DIR --fetch DIR --write DIR --fetch-copy DIR --write-copy DIR \
        --copy-bytes 1073741824 --cmd "<profiled command>"

Writes profiles/<name>.md (the figures and the commands) and profiles/<name>_traffic.json
(per-launch fetched / written bytes of the kernel, scaled by the copy calibration, and the
SHA-256 of the SpMV kernel source the counters were taken with).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("exec.h", "exec.hip", "plan.h", "spmm_tile.h", "spmm_panel.h")]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, f"*{suffix}"))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def kernel_stats(trace_dir):
    return _csv(trace_dir, "kernel_stats.csv")


def timed_mean_us(trace_dir, kernel, first, count):
    """Mean duration of dispatches [first, first + count) of each named kernel (in launch
    order), summed over the kernels of one product: the benchmark's timed region."""
    rows = _csv(trace_dir, "kernel_trace.csv")
    total = 0.0
    for k in kernel.split(" + "):
        d = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows
                   if k in r["Kernel_Name"])
        sel = d[first:first + count]
        if len(sel) < count:
            raise ValueError(f"only {len(d)} dispatches of {k!r}")
        total += sum(e - b for b, e in sel) / len(sel) / 1e3
    return total


def _dispatch_order(r):
    for k in ("Dispatch_Id", "Correlation_Id"):
        if k in r and r[k] not in ("", None):
            return int(r[k])
    return 0


def counter_mean_kib(d, kernel, last=0, drop_last=0, first=0):
    """Mean counter value per dispatch; kernel may name several kernels joined by ' + '
    (one product launching each once), whose means are added. last > 0: only the last
    `last` dispatches of each kernel (in dispatch order); drop_last > 0: all but the last
    `drop_last`; first > 0: the first `first`."""
    total, count = 0.0, None
    rows = _csv(d, "counter_collection.csv")
    for k in kernel.split(" + "):
        sel = sorted((r for r in rows if k in r["Kernel_Name"]), key=_dispatch_order)
        vals = [float(r["Counter_Value"]) for r in sel]
        if first:
            vals = vals[:first]
        elif last:
            vals = vals[-last:]
        elif drop_last:
            vals = vals[:-drop_last]
        if not vals:
            raise ValueError(f"kernel {k!r} not found under {d}")
        total += sum(vals) / len(vals)
        count = len(vals) if count is None else min(count, len(vals))
    return total, count


def last_mean_us(trace_dir, kernel, count):
    """Mean duration of the last `count` dispatches of each named kernel, summed over the
    kernels of one product (the benchmark's final cache-cold launches)."""
    rows = _csv(trace_dir, "kernel_trace.csv")
    total = 0.0
    for k in kernel.split(" + "):
        d = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows
                   if k in r["Kernel_Name"])
        sel = d[-count:]
        if len(sel) < count:
            raise ValueError(f"only {len(d)} dispatches of {k!r}")
        total += sum(e - b for b, e in sel) / len(sel) / 1e3
    return total


def pmc_summary(argv):
    """profsum pmc --name N --kernel K --dir DIR --trace DIR --cmd CMD --useful-flop F:
    per-dispatch means of every counter collected for kernel K, with the matrix-core busy
    fraction (sum of SQ_VALU_MFMA_BUSY_CYCLES over SIMDs / (GRBM_GUI_ACTIVE of one XCD x
    SIMDs)) and MFMA FLOP (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512) when present."""
    ap = argparse.ArgumentParser(prog="profsum pmc")
    ap.add_argument("--name", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--dir", required=True, action="append",
                    help="counter output directory (repeat for several counter passes)")
    ap.add_argument("--trace", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--trace-cmd", required=True)
    ap.add_argument("--simds", type=int, default=256 * 4)
    ap.add_argument("--xcds", type=int, default=8)
    ap.add_argument("--useful-flop", type=float, default=0.0,
                    help="algorithmic FLOP of one dispatch (2 nnz n x 3 products)")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--last", type=int, default=0,
                    help="only the last N dispatches of the kernel (the cache-cold launches)")
    ap.add_argument("--drop-last", type=int, default=0,
                    help="all but the last N dispatches of the kernel (the warm launches)")
    ap.add_argument("--first", type=int, default=0,
                    help="only the first N dispatches of the kernel (the benchmark's own plan)")
    ap.add_argument("--note", default="", help="a line describing which launches were counted")
    a = ap.parse_args(argv)
    by, passes = {}, []
    for d in a.dir:
        rows = [r for r in _csv(d, "counter_collection.csv") if a.kernel in r["Kernel_Name"]]
        if not rows:
            raise ValueError(f"kernel {a.kernel!r} not found under {d}")
        names = sorted({r["Counter_Name"] for r in rows})
        passes.append(names)
        for name in names:
            vals = [float(r["Counter_Value"]) for r in
                    sorted((r for r in rows if r["Counter_Name"] == name), key=_dispatch_order)]
            if a.first:
                vals = vals[:a.first]
            elif a.last:
                vals = vals[-a.last:]
            elif a.drop_last:
                vals = vals[:-a.drop_last]
            by.setdefault(name, []).extend(vals)
    mean = {k: sum(v) / len(v) for k, v in by.items()}
    st = [r for r in kernel_stats(a.trace) if a.kernel in r["Name"]]
    avg_us = float(st[0]["AverageNs"]) / 1e3 if st else 0.0
    sel_us, sel_what = avg_us, ""
    if st and (a.first or a.last or a.drop_last):  # durations of the counted dispatches only
        n_all = int(st[0]["Calls"])
        if a.first:
            sel_us, sel_what = timed_mean_us(a.trace, a.kernel, 0, a.first), f"the first {a.first}"
        elif a.last:
            sel_us, sel_what = last_mean_us(a.trace, a.kernel, a.last), f"the last {a.last}"
        else:
            sel_us = timed_mean_us(a.trace, a.kernel, 0, n_all - a.drop_last)
            sel_what = f"those before the last {a.drop_last}"
        avg_us = sel_us
    md = [f"# {a.name}: rocprofv3 counters of `{a.kernel}`", "",
          "Commands (run from /tmp with TMPDIR=/tmp; DIR is an output directory):", "",
          *[f"    rocprofv3 --pmc {' '.join(p)} --output-format csv -d DIR -o run -- {a.cmd}"
            for p in passes],
          f"    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o run -- {a.trace_cmd}", "",
          *([a.note, ""] if a.note else []),
          "| counter | mean per dispatch |", "|---|---|"]
    for k in sorted(mean):
        md.append(f"| {k} | {mean[k]:.6g} |")
    md.append("")
    if st:
        md.append(f"* Kernel-trace average duration: {float(st[0]['AverageNs']) / 1e3:.1f} us over "
                  f"{st[0]['Calls']} dispatches" + (f"; {sel_us:.1f} us over the counted ones "
                                                    f"({sel_what})." if sel_what else "."))
    if "SQ_WAIT_ANY" in mean and "SQ_WAVE_CYCLES" in mean:
        md.append(f"* Waves waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES): "
                  f"{100 * mean['SQ_WAIT_ANY'] / mean['SQ_WAVE_CYCLES']:.1f}% of their cycles.")
    if mean.get("SQ_ACTIVE_INST_VMEM") and "SQ_WAVE_CYCLES" in mean:  # 0 where not counted
        md.append(f"* Issuing vector memory instructions (SQ_ACTIVE_INST_VMEM / SQ_WAVE_CYCLES): "
                  f"{100 * mean['SQ_ACTIVE_INST_VMEM'] / mean['SQ_WAVE_CYCLES']:.1f}%.")
    if "TCC_HIT_sum" in mean and "TCC_MISS_sum" in mean:
        h, m = mean["TCC_HIT_sum"], mean["TCC_MISS_sum"]
        md.append(f"* L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)): {100 * h / max(h + m, 1):.1f}%.")
    if "SQ_VALU_MFMA_BUSY_CYCLES" in mean and "GRBM_GUI_ACTIVE" in mean:
        gui = mean["GRBM_GUI_ACTIVE"] / a.xcds  # one XCD's active cycles
        util = mean["SQ_VALU_MFMA_BUSY_CYCLES"] / (gui * a.simds)
        md.append(f"* Matrix-core busy fraction: {mean['SQ_VALU_MFMA_BUSY_CYCLES']:.4g} / "
                  f"({gui:.4g} x {a.simds}) = {100 * util:.2f}%.")
    if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in mean:
        fl = mean["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512
        md.append(f"* BF16 MFMA work issued: {fl / 1e9:.1f} GFLOP per dispatch"
                  + (f" ({fl / (avg_us * 1e-6) / 1e12:.1f} TFLOP/s at the traced duration)" if avg_us else "")
                  + ".")
        if a.useful_flop:
            md.append(f"* Algorithmic split-bf16 work {a.useful_flop / 1e9:.1f} GFLOP: "
                      f"{100 * a.useful_flop / fl:.1f}% of the issued MFMA work is useful "
                      "(the rest multiplies the zero fill of the operand tiles).")
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, f"{a.name}.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def trace_summary(argv):
    """profsum trace --name N --trace DIR --cmd CMD [--kernel K --flop F]: the kernel-trace
    stats table, and for kernel K its average duration and FLOP rate at F FLOP per dispatch."""
    ap = argparse.ArgumentParser(prog="profsum trace")
    ap.add_argument("--name", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--kernel", default="")
    ap.add_argument("--flop", type=float, default=0.0)
    ap.add_argument("--timed", default="",
                    help="'first,count': also the mean over these dispatches of the kernel")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args(argv)
    rows = kernel_stats(a.trace)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    md = [f"# {a.name}: rocprofv3 kernel trace", "",
          "Command (run from /tmp with TMPDIR=/tmp; DIR is an output directory):", "",
          f"    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o run -- {a.cmd}", "",
          "| kernel | calls | average us | min us | max us |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        md.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                  f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    sel = [r for r in rows if a.kernel and a.kernel in r["Name"]]
    if sel:
        avg = float(sel[0]["AverageNs"]) / 1e3
        md += ["", f"* `{a.kernel}`: average {avg:.1f} us over {sel[0]['Calls']} dispatches"
               + (f"; {a.flop / 1e9:.1f} GFLOP per dispatch -> {a.flop / (avg * 1e-6) / 1e12:.2f} TFLOP/s."
                  if a.flop else ".")]
        if a.timed:
            first, count = (int(v) for v in a.timed.split(","))
            tm = timed_mean_us(a.trace, a.kernel, first, count)
            md.append(f"* Dispatches {first}..{first + count - 1} of `{a.kernel}` (the benchmark's "
                      f"timed launches): mean {tm:.1f} us"
                      + (f" -> {a.flop / (tm * 1e-6) / 1e12:.2f} TFLOP/s." if a.flop else "."))
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, f"{a.name}.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def main(argv=None):
    import sys
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "pmc":
        return pmc_summary(argv[1:])
    if argv and argv[0] == "trace":
        return trace_summary(argv[1:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--copy-kernel", default="elementwise")
    ap.add_argument("--copy-bytes", type=float, default=2 * 1024 ** 3)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--fetch-copy", required=True)
    ap.add_argument("--write-copy", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--timed", default="",
                    help="'first,count': also report the mean over these dispatches of the "
                         "kernel (the benchmark's timed launches)")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--append", action="store_true",
                    help="add this kernel's traffic record to the existing file")
    ap.add_argument("--md-name", default="",
                    help="write the summary under this name instead of --name")
    ap.add_argument("--last", type=int, default=0,
                    help="counters and durations of the last N dispatches of the kernel only "
                         "(the benchmark's final cache-cold launches)")
    ap.add_argument("--drop-last", type=int, default=0,
                    help="counters of all but the last N dispatches of the kernel (the warm "
                         "launches before the cache-cold ones)")
    ap.add_argument("--first", type=int, default=0,
                    help="counters and durations of the first N dispatches of the kernel only "
                         "(the benchmark's own plan, before any baseline plan)")
    a = ap.parse_args(argv)
    rows = kernel_stats(a.trace)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    f_k, nf = counter_mean_kib(a.fetch, a.kernel, a.last, a.drop_last, a.first)
    w_k, nw = counter_mean_kib(a.write, a.kernel, a.last, a.drop_last, a.first)
    fc, _ = counter_mean_kib(a.fetch_copy, a.copy_kernel)
    wc, _ = counter_mean_kib(a.write_copy, a.copy_kernel)
    half = a.copy_bytes / 2  # the copy reads half and writes half of copy_bytes
    ff = half / (fc * 1024.0)
    wf = half / (wc * 1024.0)
    fetch_b = f_k * 1024.0 * ff
    write_b = w_k * 1024.0 * wf
    parts = a.kernel.split(" + ")
    sel = [[r for r in rows if k in r["Name"]] for k in parts]
    md = [f"# {a.name}: rocprofv3 kernel trace and HBM counters", "",
          "Commands (run from /tmp with TMPDIR=/tmp; DIR is an output directory):", "",
          f"    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o run -- {a.cmd}",
          f"    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR -o run -- {a.cmd}",
          f"    rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR -o run -- {a.cmd}",
          "    rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE --output-format csv -d DIR -o copy -- "
          "python3 bench.py --workload copy --steps 10 --warmup 2", "",
          "## Kernel durations (kernel-trace stats, top 12 by total time)", "",
          "| kernel | calls | average us | min us | max us |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        md.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                  f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    md += ["", f"## HBM bytes of `{a.kernel}`" + (f" (last {a.last} dispatches)" if a.last else "")
           + (f" (all but the last {a.drop_last} dispatches)" if a.drop_last else "")
           + (f" (first {a.first} dispatches)" if a.first else ""), "",
           f"* FETCH_SIZE mean {f_k:.1f} KiB per dispatch over {nf} dispatches; WRITE_SIZE "
           f"{w_k:.1f} KiB over {nw}.",
           f"* Calibration with a plain device copy of {a.copy_bytes / 2 ** 30:.2f} GiB "
           f"(half read, half written): FETCH_SIZE reads {fc:.0f} KiB -> factor {ff:.3f}; "
           f"WRITE_SIZE reads {wc:.0f} KiB -> factor {wf:.3f}.",
           f"* Traffic per launch: fetched {fetch_b / 1e6:.1f} MB + written {write_b / 1e6:.1f} MB "
           f"= {(fetch_b + write_b) / 1e6:.1f} MB."]
    if all(sel):
        avgs = [float(r[0]["AverageNs"]) / 1e3 for r in sel]
        avg = sum(avgs)
        if len(avgs) > 1:
            md.append("* Average durations " + " + ".join(f"{v:.2f}" for v in avgs) +
                      f" = {avg:.2f} us per product.")
        md.append(f"* Average duration {avg:.2f} us -> {(fetch_b + write_b) / (avg * 1e-6) / 1e12:.2f} "
                  "TB/s of counted traffic.")
        if a.timed:
            first, count = (int(v) for v in a.timed.split(","))
            tm = timed_mean_us(a.trace, a.kernel, first, count)
            md.append(f"* Timed region (dispatches {first}..{first + count - 1} of the kernel, "
                      f"after the warm-up and before the cache-cold launches): mean {tm:.2f} us -> "
                      f"{(fetch_b + write_b) / (tm * 1e-6) / 1e12:.2f} TB/s of counted traffic.")
        if a.first:
            tm = timed_mean_us(a.trace, a.kernel, 0, a.first)
            md.append(f"* First {a.first} dispatches of the kernel: mean {tm:.2f} us -> "
                      f"{(fetch_b + write_b) / (tm * 1e-6) / 1e12:.2f} TB/s of counted traffic.")
        if a.last:
            tm = last_mean_us(a.trace, a.kernel, a.last)
            md.append(f"* Last {a.last} dispatches of the kernel (the cache-cold launches): mean "
                      f"{tm:.2f} us -> {(fetch_b + write_b) / (tm * 1e-6) / 1e12:.2f} TB/s of "
                      "counted traffic.")
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, f"{a.md_name or a.name}.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    rec = {"kernel": a.kernel, "fetch_kib": f_k, "write_kib": w_k, "fetch_factor": ff,
           "write_factor": wf, "traffic_bytes": fetch_b + write_b,
           "kernel_source_sha256": kernel_source_sha(), "command": a.cmd}
    path = os.path.join(a.out, f"{a.name}_traffic.json")
    recs = []
    if a.append and os.path.exists(path):  # keep the records of other kernels
        with open(path) as f:
            old = json.load(f)
        recs = [r for r in (old if isinstance(old, list) else [old]) if r.get("kernel") != a.kernel]
    recs.append(rec)
    with open(path, "w") as f:
        json.dump(recs if len(recs) > 1 else rec, f, indent=1)
    print("\n".join(md))


if __name__ == "__main__":
    main()
