"""Benchmark: hybrid VDIA + VBR + CSR SpMV on one MI355X against plain GPU CSR.

Default workload (one step = one fused hybrid SpMV launch over the planned matrix, the
executor of the inspector-executor scheme; planning is done once before timing and
reported separately as plan_ms):
  PDE-like matrix, 2,097,152 rows: 7-point stencil on a 128^3 grid with 20% of the
  off-diagonal chunks truncated, 64 dense 128x128 blocks at unaligned positions, one
  scattered entry per row, values and x ~ N(0,1); plan [VDIA, VBR(tiled), CSR] with
  delta_band = 0.75, delta_block = 0.5.

Prints ONE JSON line with value = hybrid GFLOP/s (2 * nnz / t), the roofline of the fused
kernel (algorithmic bytes per launch / event-timed launch duration vs 8 TB/s), the plain
CSR baseline (this library's autotuned CSR kernels, and ROCm's rocsparse_scsrmv with its
analysis step as an outside reference; speedup_vs_best_plain_csr uses the faster of them), the normwise error against an FP64 reference (scipy.sparse) and the CPU oracle's own rate.

Other workloads (--workload): c1 (4096^2 mixed, SpMV), c3 (FEM-like SpMM, n=128),
copy (a plain device copy used to calibrate HBM byte counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / steps  # ms per launch (device events)


class ColdCache:
    """Cache-cold conditions before a timed launch: a 1 GiB write, then a 1 GiB read of a
    second buffer. The write alone leaves up to the Infinity Cache's 256 MB of dirty lines,
    whose write-back would then land in the timed launch (a plain device copy of 132 MB takes
    38 us after the write alone, 27 us after write + read, 19 us warm); after the read the
    caches hold clean lines of an unrelated buffer, so the launch reads everything from HBM
    and pays for nothing else."""

    def __init__(self, torch, write_only=False):
        self.torch = torch
        self.write_only = write_only
        n = 256 * 1024 * 1024
        self.w = torch.empty(n, device="cuda")
        self.r = None if write_only else torch.ones(n, device="cuda")

    def __call__(self):
        self.w.fill_(1.0)
        if self.r is not None:
            self.r.sum()


def cold_launch_ms(fn, reps, torch, flush):
    """Per-launch event time with `flush` (cache-cold conditions) before every launch;
    decile-filtered mean, as in the paper's protocol."""
    times = []
    for _ in range(reps):
        flush()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    t = np.sort(np.array(times))
    lo, hi = int(0.1 * t.size), int(np.ceil(0.9 * t.size))
    return float(np.mean(t[lo:hi]))


def cold_tune(sable, p, op, cands, fn, reps, torch, flush):
    """Choose among kernel variants by their cache-cold time: cands are tuples of
    (op, variant) settings applied with sable_plan_set_variant; returns (best settings,
    its time, every candidate's time). Candidates within 2% of the fastest resolve to the
    first in list order."""
    times = []
    for c in cands:
        for o, v in c:
            sable.sable_plan_set_variant(p, o, v)
        times.append(cold_launch_ms(fn, reps, torch, flush))
    best = min(times)
    log("cold candidates: " + ", ".join(f"{c}: {t * 1e3:.1f} us" for c, t in zip(cands, times)))
    k = next(i for i, t in enumerate(times) if t <= 1.02 * best)
    for o, v in cands[k]:
        sable.sable_plan_set_variant(p, o, v)
    return cands[k], times[k], times


# ---- FP64 references for the reported errors (scipy.sparse in float64; the CPU oracle is
# used only for the timed CPU baseline) ----------------------------------------------------

def _sp64(A):
    import scipy.sparse as sp
    return sp.csr_matrix((A.values.astype(np.float64), A.indices, A.indptr),
                         shape=(A.nrows, A.ncols))


def ref_spmv(A, x):
    return _sp64(A) @ x.astype(np.float64)


def ref_spmm_rows(A, X, rows):
    return np.asarray(_sp64(A)[rows] @ X.astype(np.float64))


def rel_err(y, ref):
    d = np.linalg.norm(y.astype(np.float64) - ref)
    n = np.linalg.norm(ref)
    return float(d / n) if n > 0 else float(d)


def graph_ms(make, reps, torch):
    """Per-launch time of `reps` launches captured in one graph and replayed: the GPU's own
    time for kernels of a few microseconds, without the host's per-launch cost. `make()`
    returns the launch callable; it is built inside the capture so that it launches on the
    capturing stream."""
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        make()()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        f = make()
        for _ in range(reps):
            f()
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(3):
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        best = ms if best is None else min(best, ms)
    del g
    return best


def rocsparse_csrmv_ms(A, ip, ix, vv, xd, y, steps, warmup, torch):
    """Reference point: ROCm's own CSR SpMV (rocsparse_scsrmv with its analysis step) on the
    same matrix and stream; event-timed per launch. Returns (ms, y) or (None, None) when the
    library is not available."""
    import ctypes
    try:
        L = ctypes.CDLL("librocsparse.so")
    except OSError:
        return None, None
    P, i32 = ctypes.c_void_p, ctypes.c_int32

    def ok(rc, fn):
        if rc != 0:
            raise RuntimeError(f"{fn} failed: {rc}")

    h, d, info = P(), P(), P()
    ok(L.rocsparse_create_handle(ctypes.byref(h)), "create_handle")
    ok(L.rocsparse_set_stream(h, P(torch.cuda.current_stream().cuda_stream)), "set_stream")
    ok(L.rocsparse_create_mat_descr(ctypes.byref(d)), "create_mat_descr")
    ok(L.rocsparse_create_mat_info(ctypes.byref(info)), "create_mat_info")
    m, n, nnz = i32(A.nrows), i32(A.ncols), i32(A.nnz)
    op = i32(111)  # rocsparse_operation_none
    ok(L.rocsparse_scsrmv_analysis(h, op, m, n, nnz, d, P(vv.data_ptr()), P(ip.data_ptr()),
                                   P(ix.data_ptr()), info), "scsrmv_analysis")
    one, zero = ctypes.c_float(1.0), ctypes.c_float(0.0)

    cargs = (h, op, m, n, nnz, ctypes.byref(one), d, P(vv.data_ptr()), P(ip.data_ptr()),
             P(ix.data_ptr()), info, P(xd.data_ptr()), ctypes.byref(zero), P(y.data_ptr()))
    fn = L.rocsparse_scsrmv

    def f():  # arguments marshalled once, as for the library's own launches
        rc = fn(*cargs)
        if rc != 0:
            ok(rc, "scsrmv")
    _, ms = timed_steps(f, steps, warmup, torch)
    L.rocsparse_destroy_mat_info(info)
    L.rocsparse_destroy_mat_descr(d)
    L.rocsparse_destroy_handle(h)
    return ms, y


def rocsparse_csrmm_ms(A, ip, ix, vv, Xd, n, steps, warmup, torch):
    """Reference point: ROCm's CSR SpMM (rocsparse_scsrmm) on the same matrix and row-major X
    (passed as the transpose of a column-major n x ncols matrix); its output is column-major.
    Event-timed per launch. Returns (ms, C as an nrows x n view) or (None, None)."""
    import ctypes
    try:
        L = ctypes.CDLL("librocsparse.so")
    except OSError:
        return None, None
    P, i32 = ctypes.c_void_p, ctypes.c_int32

    def ok(rc, fn):
        if rc != 0:
            raise RuntimeError(f"{fn} failed: {rc}")

    h, d = P(), P()
    ok(L.rocsparse_create_handle(ctypes.byref(h)), "create_handle")
    ok(L.rocsparse_set_stream(h, P(torch.cuda.current_stream().cuda_stream)), "set_stream")
    ok(L.rocsparse_create_mat_descr(ctypes.byref(d)), "create_mat_descr")
    C = torch.empty(n, A.nrows, device="cuda")  # column-major nrows x n
    one, zero = ctypes.c_float(1.0), ctypes.c_float(0.0)
    cargs = (h, i32(111), i32(112), i32(A.nrows), i32(n), i32(A.ncols), i32(A.nnz),
             ctypes.byref(one), d, P(vv.data_ptr()), P(ip.data_ptr()), P(ix.data_ptr()),
             P(Xd.data_ptr()), i32(n), ctypes.byref(zero), P(C.data_ptr()), i32(A.nrows))
    fn = L.rocsparse_scsrmm

    def f():
        rc = fn(*cargs)
        if rc != 0:
            ok(rc, "scsrmm")
    try:
        _, ms = timed_steps(f, steps, warmup, torch)
    except RuntimeError:
        ms = None
    L.rocsparse_destroy_mat_descr(d)
    L.rocsparse_destroy_handle(h)
    return ms, (C.t() if ms else None)


def host_cpu_record():
    """What the host CPU is: model, logical CPUs, threads per core, sockets (from lscpu),
    and the CPUs this process may run on."""
    import subprocess
    rec = {"nproc": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return rec
    keep = {"Model name": "model", "CPU(s)": "cpus", "Thread(s) per core": "threads_per_core",
            "Core(s) per socket": "cores_per_socket", "Socket(s)": "sockets",
            "CPU max MHz": "max_mhz", "L3": "l3"}
    for line in out.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keep:
            rec[keep[k.strip()]] = v.strip()
    return rec


def _oracle_rate(run, flop_per_pass, target_s):
    run()
    t0 = time.perf_counter()
    passes = 0
    while time.perf_counter() - t0 < target_s:
        run()
        passes += 1
    dt = time.perf_counter() - t0
    return flop_per_pass * passes / dt / 1e9, passes, dt


def cpu_baseline_spmv(A, x, target_s=10.0):
    """The oracle's FP64 SpMV timed on the host: on every available thread (the reported
    value) and on one thread, with the host's lscpu record."""
    import oracle
    threads = oracle.max_threads()
    run = lambda: oracle.spmv(A, x)  # noqa: E731
    g, passes, dt = _oracle_rate(run, 2.0 * A.nnz, 0.6 * target_s)
    oracle.set_threads(1)
    try:
        g1, passes1, dt1 = _oracle_rate(run, 2.0 * A.nnz, 0.4 * target_s)
    finally:
        oracle.set_threads(threads)
    return {"value": round(g, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 COO SpMV over the full matrix, {passes} passes ({dt:.1f} s)",
            "single_thread": {"value": round(g1, 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": f"{passes1} passes ({dt1:.1f} s)"},
            "host": host_cpu_record()}


def cpu_baseline_spmm(A, X, rows=20000, target_s=10.0):
    """The oracle's FP64 SpMM on the first `rows` rows, timed as cpu_baseline_spmv."""
    import oracle
    threads = oracle.max_threads()
    sel = np.arange(min(rows, A.nrows), dtype=np.int64)
    nnz_sel = int(A.indptr[sel[-1] + 1] - A.indptr[0])
    n = X.shape[1]
    run = lambda: oracle.spmm_rows(A, X, sel)  # noqa: E731
    g, passes, dt = _oracle_rate(run, 2.0 * nnz_sel * n, 0.6 * target_s)
    oracle.set_threads(1)
    try:
        g1, passes1, dt1 = _oracle_rate(run, 2.0 * nnz_sel * n, 0.4 * target_s)
    finally:
        oracle.set_threads(threads)
    return {"value": round(g, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 SpMM (n={n}) of the first {sel.size} rows, {passes} passes ({dt:.1f} s)",
            "single_thread": {"value": round(g1, 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": f"{passes1} passes ({dt1:.1f} s)"},
            "host": host_cpu_record()}


def variant_kernel(v: int, far: int = 0) -> str:
    """Kernel(s) one hybrid SpMV launches for variant v ('A + B' when the far-column gather
    pass runs first)."""
    if v >= 15:
        k = f"k_spmv_persist<{'true' if v == 16 else 'false'}>"
        return f"k_far_gather + {k}" if far else k
    if v >= 12:
        return "k_spmv_binned"
    if v == 11:
        return "sable_spec_spmv"
    if v <= 2:
        k = f"k_spmv_stream<{1 << v}, false>"
    elif v >= 8:
        k = f"k_spmv_stream<{1 << (v - 8)}, true>"
    else:
        return f"k_spmv_fused<{1 << (v - 3)}>"
    return f"k_far_gather + {k}" if far else k


def plain_kernel(v: int) -> str:
    """Kernel the plain CSR baseline launches for its variant v."""
    if v >= 16:
        return f"k_csr_persist<{'true' if v == 17 else 'false'}>"
    if v >= 13:
        return "k_csr_binned"
    if v <= 2:
        return f"k_csr_stream<{1 << v}, false>"
    if v >= 10:
        return f"k_csr_stream<{1 << (v - 10)}, true>"
    return f"k_spmv_plain<{1 << (v - 3)}>"


def measured_traffic(name: str, kernel: str):
    """Counter-based bytes per launch from profiles/<name>_traffic.json, only if they were
    taken for this kernel with the current kernel source (else None)."""
    from paper_2407_00829_amd import profsum
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    recs = rec if isinstance(rec, list) else [rec]  # one record per profiled kernel
    for r in recs:
        if r.get("kernel") == kernel and r.get("kernel_source_sha256") == profsum.kernel_source_sha():
            return r["traffic_bytes"]
    return None


def run_spmv(args, torch, sable, synth):
    if args.workload == "c2":
        log("[bench] generating PDE-like matrix (2,097,152 rows)")
        A, x = synth.gen_c2(args.seed)
        th = sable.Thresholds(delta_band_pm=750, delta_block_pm=500)
        kinds = [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR]
        mode = sable.SABLE_VBR_TILED
        wl = ("PDE-like SpMV: 7-point stencil on 128^3 grid (20% off-diagonal chunks truncated) + "
              "64 dense 128x128 unaligned blocks + 1 scattered nnz/row; N(0,1)")
    else:
        log("[bench] generating 4096^2 mixed matrix")
        A, x = synth.gen_c1(args.seed)
        th = sable.Thresholds(amin_band=256, amin_block=256)
        kinds = [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR]
        mode = sable.SABLE_VBR_PAPER
        wl = "4096^2 mixed SpMV: bands {0,-1,+1,+37}, 12 aligned blocks, 0.05% scatter; U(-1,1)"
    log(f"[bench] nnz={A.nnz}; planning")
    t0 = time.perf_counter()
    p = sable.plan_host(A, kinds, mode, th)
    torch.cuda.synchronize()
    plan_wall = time.perf_counter() - t0
    info = sable.sable_plan_info(p)
    log(f"[bench] plan: {info}")
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, device="cuda")
    yp = torch.empty(A.nrows, device="cuda")
    if args.variants:  # fixed kernels (profiling runs name the kernels the bench line chose)
        hv, fs, pv = (int(v) for v in args.variants.split(","))
        sable.sable_plan_set_variant(p, 0, hv)
        sable.sable_plan_set_variant(p, 3, fs)
        sable.sable_plan_set_variant(p, 2, pv)
    elif args.autotune:
        sable.sable_autotune(p, 0, 1, xd, y)
    info = sable.sable_plan_info(p)
    warm_var = (info["spmv_variant"], info["far_split"], info["plain_variant"])
    f_h = sable.launcher("sable_spmv", p, xd, y)
    f_p = sable.launcher("sable_csr_spmv", p, xd, yp)
    wall, ev_ms = timed_steps(f_h, args.steps, args.warmup, torch)
    wall_p, ev_ms_p = timed_steps(f_p, args.steps, args.warmup, torch)
    ref = ref_spmv(A, x)
    ref_d = torch.from_numpy(ref).cuda()
    err = sable.sable_error_norm_f64(y, ref_d)
    err_p = sable.sable_error_norm_f64(yp, ref_d)
    ip_, ix_, vv_ = p._src
    yr = torch.empty(A.nrows, device="cuda")
    rs_ms, yr = rocsparse_csrmv_ms(A, ip_, ix_, vv_, xd, yr, args.steps, args.warmup, torch)
    rs_err = sable.sable_error_norm_f64(yr, ref_d) if rs_ms else None
    single = None
    if warm_var[1] and not args.variants:
        # the same streamed tile without the far-column pass: one launch instead of two
        # (skipped in profiling runs, whose fixed variants keep each kernel's dispatches apart)
        sable.sable_plan_set_variant(p, 3, 0)
        _, ev_1 = timed_steps(f_h, args.steps, args.warmup, torch)
        sable.sable_plan_set_variant(p, 3, 1)
        single = {"kernel": variant_kernel(warm_var[0], 0), "launch_ms": round(ev_1, 5)}
    # cache-cold: the variants are chosen again by their cold times (the hybrid's and the
    # plain CSR's), then the chosen ones are timed last, 30 launches each
    bytes_h = info["bytes_matrix"] + 4 * (A.nrows + A.ncols)
    flush = ColdCache(torch)
    if args.cold_variants:
        ch, cf, cp = (int(v) for v in args.cold_variants.split(","))
        sable.sable_plan_set_variant(p, 0, ch)
        sable.sable_plan_set_variant(p, 3, cf)
        sable.sable_plan_set_variant(p, 2, cp)
    elif args.autotune:
        hc = [((3, 0), (0, v)) for v in (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 13, 14, 15, 16)]
        if info["far_nnz"]:
            hc += [((3, 1), (0, v)) for v in (0, 1, 2, 8, 9, 10, 15, 16)]
        cold_tune(sable, p, 0, hc, f_h, 8, torch, flush)
        cold_tune(sable, p, 2, [((2, v),) for v in range(18)], f_p, 8, torch, flush)
    cinfo = sable.sable_plan_info(p)
    sable.sable_spmv(p, xd, y)
    err_c = sable.sable_error_norm_f64(y, ref_d)
    flush_w = ColdCache(torch, write_only=True)
    cold_w = cold_launch_ms(f_h, 30, torch, flush_w)
    # the same number of bytes through a plain device copy (half read, half written), under
    # the three conditions: what streaming these bytes costs on this GPU
    src = torch.empty(bytes_h // 8, device="cuda")
    dst = torch.empty_like(src)
    f_c = lambda: dst.copy_(src)  # noqa: E731
    _, copy_warm = timed_steps(f_c, 50, 5, torch)
    copy_ref = {"bytes": 2 * src.numel() * 4, "warm_launch_ms": round(copy_warm, 5),
                "cold_launch_ms": round(cold_launch_ms(f_c, 30, torch, flush), 5),
                "cold_write_flush_only_launch_ms": round(cold_launch_ms(f_c, 30, torch, flush_w), 5)}
    del src, dst, flush_w
    # last: the chosen kernels' cache-cold launches (a profile's last 30 dispatches of each)
    cold = cold_launch_ms(f_h, 30, torch, flush)
    cold_p = cold_launch_ms(f_p, 30, torch, flush)
    del flush
    nnz = A.nnz
    kern = variant_kernel(warm_var[0], warm_var[1])
    ckern = variant_kernel(cinfo["spmv_variant"], cinfo["far_split"])
    bytes_p = 8 * nnz + 4 * (A.nrows + 1) + 4 * (A.nrows + A.ncols)
    ms = wall / args.steps * 1e3
    gflops = 2.0 * nnz / (ms * 1e-3) / 1e9
    achieved = bytes_h / (ev_ms * 1e-3) / 1e9
    achieved_c = bytes_h / (cold * 1e-3) / 1e9
    out = {
        "metric": "hybrid SpMV/SpMM GFLOP/s & %HBM peak vs plain GPU CSR; rel err vs FP64",
        "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl, "rows": A.nrows, "nnz": nnz, "op": "SpMV",
                   "plan": "VDIA+VBR+CSR", "vbr_mode": info["vbr_mode_used"],
                   "vbr_tile": info["vbr_tile"], "seed": args.seed},
        # cache-cold (the condition the HBM target is defined for): every launch reads the
        # matrix, x and y from HBM
        "roofline": {"bound": "hbm", "achieved": round(achieved_c, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved_c / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(f"spmv_{args.workload}_cold", ckern),
                     "kernel": ckern, "bytes_per_launch": bytes_h,
                     "launch_ms": round(cold, 5),
                     "condition": "cold: 1 GiB write + 1 GiB read of other buffers before each "
                                  "launch; decile-filtered mean of 30 launches"},
        # back-to-back launches (the timed steps): the working set stays in the Infinity Cache
        "roofline_warm": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                          "traffic": measured_traffic(f"spmv_{args.workload}", kern),
                          "kernel": kern, "bytes_per_launch": bytes_h,
                          "launch_ms": round(ev_ms, 5), "one_launch_without_far_pass": single},
        "rel_err_fp64": err,
        "rel_err_fp64_cold_variant": err_c,
        "plain_csr": {"kernel": plain_kernel(warm_var[2]),
                      "traffic": measured_traffic(f"spmv_{args.workload}_plain_csr",
                                                  plain_kernel(warm_var[2])),
                      "gflops": round(2.0 * nnz / (wall_p / args.steps) / 1e9, 2),
                      "launch_ms": round(ev_ms_p, 5), "rel_err_fp64": err_p,
                      "gbs": round(bytes_p / (ev_ms_p * 1e-3) / 1e9, 1)},
        "speedup_vs_plain_csr": round(ev_ms_p / ev_ms, 4),
        "speedup_vs_best_plain_csr": round(min(ev_ms_p, rs_ms or ev_ms_p) / ev_ms, 4),
        "rocsparse_csrmv": None if rs_ms is None else {
            "launch_ms": round(rs_ms, 5), "gflops": round(2.0 * nnz / (rs_ms * 1e-3) / 1e9, 2),
            "rel_err_fp64": rs_err, "speedup_hybrid_vs_rocsparse": round(rs_ms / ev_ms, 4)},
        "cold": {"hybrid_launch_ms": round(cold, 5), "plain_launch_ms": round(cold_p, 5),
                 "hybrid_kernel": ckern, "plain_kernel": plain_kernel(cinfo["plain_variant"]),
                 "speedup_vs_plain_csr": round(cold_p / cold, 4),
                 "plain_gbs": round(bytes_p / (cold_p * 1e-3) / 1e9, 1),
                 "hybrid_launch_ms_write_flush_only": round(cold_w, 5)},
        "copy_reference": copy_ref,
        "plan_ms": round(info["plan_ms"], 1), "plan_wall_s": round(plan_wall, 2),
        "partition": {k: info[k] for k in ("nseg", "vdia_nnz", "nblk", "vbr_nnz", "csr_nnz")},
        "variants": {"hybrid": warm_var[0], "far_split": warm_var[1], "far_nnz": info["far_nnz"],
                     "plain": warm_var[2], "cold_hybrid": cinfo["spmv_variant"],
                     "cold_far_split": cinfo["far_split"], "cold_plain": cinfo["plain_variant"]},
    }
    if not args.no_cpu:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline_spmv(A, x, args.cpu_seconds)
    return out


def run_spmv_f64(args, torch, sable, synth):
    """FP64 executor on the C2 matrix: the fp32 plan's formats with fp64 value copies."""
    log("[bench] generating PDE-like matrix (2,097,152 rows), FP64 executor")
    A, x32 = synth.gen_c2(args.seed)
    th = sable.Thresholds(delta_band_pm=750, delta_block_pm=500)
    p = sable.plan_host(A, [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR],
                        sable.SABLE_VBR_TILED, th)
    v64 = A.values.astype(np.float64)
    x = x32.astype(np.float64)
    sable.sable_update_values_f64(p, torch.from_numpy(v64).cuda())
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    best = None
    for fs in (1, 0):  # far-column split on / off
        for v in (0, 1, 2):  # streamed tile sizes
            sable.sable_plan_set_variant(p, 3, fs)
            sable.sable_plan_set_variant(p, 0, v)
            _, t = timed_steps(sable.launcher("sable_spmv_f64", p, xd, y), 20, 5, torch)
            if best is None or t < 0.98 * best[2]:
                best = (v, fs, t)
    sable.sable_plan_set_variant(p, 0, best[0])
    sable.sable_plan_set_variant(p, 3, best[1])
    info = sable.sable_plan_info(p)
    kern = f"k_spmv_stream_f64<{1 << best[0]}>"
    if info["far_split"]:
        kern = "k_far_gather<double> + " + kern
    f_h = sable.launcher("sable_spmv_f64", p, xd, y)
    wall, ev_ms = timed_steps(f_h, args.steps, args.warmup, torch)
    err = rel_err(y.cpu().numpy(), ref_spmv(A, x))  # values and x are fp32-representable
    bytes_h = (8 * info["vdia_cells"] + 20 * info["nseg"] + 8 * info["vbr_cells"]
               + 12 * info["csr_nnz"] + 4 * (A.nrows + 1) + 8 * (A.nrows + A.ncols))
    ms = wall / args.steps * 1e3
    achieved = bytes_h / (ev_ms * 1e-3) / 1e9
    return {
        "metric": "hybrid SpMV/SpMM GFLOP/s & %HBM peak vs plain GPU CSR; rel err vs FP64",
        "value": round(2.0 * A.nnz / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "PDE-like SpMV, FP64 executor: 7-point stencil on 128^3 grid "
                               "(20% off-diagonal chunks truncated) + 64 dense 128x128 blocks + "
                               "1 scattered nnz/row", "rows": A.nrows, "nnz": A.nnz},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": kern, "bytes_per_launch": bytes_h, "launch_ms": round(ev_ms, 5)},
        "rel_err_fp64": err,
        "variants": {"tile": best[0], "far_split": info["far_split"], "far_nnz": info["far_nnz"]},
    }


def run_spmm(args, torch, sable, synth):
    log("[bench] generating FEM-like matrix (500,000 rows)")
    if args.plan == "vbr":  # diagnostic: blocks only (no scatter), [VBR, CSR]
        A, X = synth.gen_c3(args.seed, scatter_density=0.0)
        kinds = [sable.SABLE_X_VBR, sable.SABLE_X_CSR]
    else:
        A, X = synth.gen_c3(args.seed)
        kinds = [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR]
    n = X.shape[1]
    th = sable.Thresholds(delta_band_pm=900, delta_block_pm=900, amin_block=36)
    log(f"[bench] nnz={A.nnz}; planning")
    p = sable.plan_host(A, kinds, sable.SABLE_VBR_TILED, th)
    info = sable.sable_plan_info(p)
    log(f"[bench] plan: {info}")
    Xd = torch.from_numpy(X).cuda()
    Y = torch.empty(A.nrows, n, device="cuda")
    if args.spmm_variant >= 0:  # fixed kernel (profiling runs name the kernel the bench chose)
        sable.sable_plan_set_variant(p, 1, args.spmm_variant)
        info = sable.sable_plan_info(p)
    elif args.autotune:
        sable.sable_autotune(p, 1, n, Xd, Y)
        info = sable.sable_plan_info(p)
    f_h = sable.launcher("sable_spmm", p, Xd, Y, n)
    wall, ev_ms = timed_steps(f_h, args.steps, args.warmup, torch)
    rows = np.random.default_rng(0).choice(A.nrows, 4096, replace=False)
    rows_d = torch.from_numpy(rows).cuda()
    ref = ref_spmm_rows(A, X, rows)
    err = rel_err(Y[rows_d].cpu().numpy(), ref)
    # plain CSR SpMM: the whole input as CSR through the fused SpMM kernel (autotuned)
    q = sable.plan_host(A, [sable.SABLE_X_CSR], sable.SABLE_VBR_TILED, sable.Thresholds())
    Yq = torch.empty_like(Y)
    if args.autotune:
        sable.sable_autotune(q, 1, n, Xd, Yq)
    _, ev_q = timed_steps(sable.launcher("sable_spmm", q, Xd, Yq, n), args.steps, args.warmup, torch)
    err_q = rel_err(Yq[rows_d].cpu().numpy(), ref)
    del Yq
    q.destroy()
    ip_, ix_, vv_ = p._src
    rs_ms, C = rocsparse_csrmm_ms(A, ip_, ix_, vv_, Xd, n, args.steps, args.warmup, torch)
    rs_err = rel_err(C[rows_d].cpu().numpy(), ref) if rs_ms else None
    del C
    ms = wall / args.steps * 1e3
    gflops = 2.0 * A.nnz * n / (ms * 1e-3) / 1e9
    bytes_h = info["bytes_matrix"] + 4 * (A.nrows + A.ncols) * n
    achieved = bytes_h / (ev_ms * 1e-3) / 1e9
    mm_kernel = {0: "k_spmm_tile", 1: "k_spmm_tile_valu", 2: "k_spmm_fused_valu", 3: "k_spmm_tile",
                 4: "k_spmm_panel"}[info["spmm_variant"]]
    out = {
        "metric": "hybrid SpMV/SpMM GFLOP/s & %HBM peak vs plain GPU CSR; rel err vs FP64",
        "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16x3" if info["spmm_variant"] in (0, 3, 4) and info["nblk"] else "f32",
        "data": "synthetic",
        "config": {"workload": "FEM-like SpMM n=128: 500,000 rows, 6x6 node blocks on a periodic "
                               "27-point block stencil, 2 bands, 0.01% scatter; U(-1,1)",
                   "rows": A.nrows, "nnz": A.nnz, "n": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("spmm_c3", mm_kernel),
                     "kernel": mm_kernel, "bytes_per_launch": bytes_h,
                     "launch_ms": round(ev_ms, 4)},
        "rel_err_fp64_sampled": err,
        "plain_csr": {"launch_ms": round(ev_q, 4),
                      "gflops": round(2.0 * A.nnz * n / (ev_q * 1e-3) / 1e9, 2),
                      "rel_err_fp64_sampled": err_q},
        "speedup_vs_plain_csr": round(ev_q / ev_ms, 4),
        "rocsparse_csrmm": None if rs_ms is None else {
            "launch_ms": round(rs_ms, 4), "gflops": round(2.0 * A.nnz * n / (rs_ms * 1e-3) / 1e9, 2),
            "rel_err_fp64_sampled": rs_err, "speedup_hybrid_vs_rocsparse": round(rs_ms / ev_ms, 4)},
        "partition": {k: info[k] for k in ("nseg", "vdia_nnz", "nblk", "vbr_nnz", "csr_nnz",
                                           "mm_panels", "mm_units")},
        "spmm_mode": info["spmm_variant"],
        "plan_ms": round(info["plan_ms"], 1),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_spmm(A, X, target_s=args.cpu_seconds)
    return out


def run_spmm_f64(args, torch, sable, synth):
    """FEM SpMM (C3, n = 128) on the FP64 executor: the fp32 plan's formats with fp64 value
    copies, fp64 X and Y, blocks on the fp64 VALU."""
    log("[bench] generating FEM-like matrix (500,000 rows), FP64 executor")
    A, X32 = synth.gen_c3(args.seed)
    n = X32.shape[1]
    th = sable.Thresholds(delta_band_pm=900, delta_block_pm=900, amin_block=36)
    p = sable.plan_host(A, [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR],
                        sable.SABLE_VBR_TILED, th)
    sable.sable_update_values_f64(p, torch.from_numpy(A.values.astype(np.float64)).cuda())
    info = sable.sable_plan_info(p)
    X = X32.astype(np.float64)
    Xd = torch.from_numpy(X).cuda()
    Y = torch.empty(A.nrows, n, dtype=torch.float64, device="cuda")
    f_h = sable.launcher("sable_spmm_f64", p, Xd, Y, n)
    wall, ev_ms = timed_steps(f_h, args.steps, args.warmup, torch)
    rows = np.random.default_rng(0).choice(A.nrows, 4096, replace=False)
    err = rel_err(Y[torch.from_numpy(rows).cuda()].cpu().numpy(), ref_spmm_rows(A, X32, rows))
    ms = wall / args.steps * 1e3
    bytes_h = (8 * info["vdia_cells"] + 20 * info["nseg"] + 8 * info["vbr_cells"]
               + 12 * info["csr_nnz"] + 4 * (A.nrows + 1) + 8 * (A.nrows + A.ncols) * n)
    achieved = bytes_h / (ev_ms * 1e-3) / 1e9
    return {
        "metric": "hybrid SpMV/SpMM GFLOP/s & %HBM peak vs plain GPU CSR; rel err vs FP64",
        "value": round(2.0 * A.nnz * n / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FEM-like SpMM n=128, FP64 executor: 500,000 rows, 6x6 node "
                               "blocks on a periodic 27-point block stencil, 2 bands, 0.01% "
                               "scatter", "rows": A.nrows, "nnz": A.nnz, "n": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_spmm_tile_f64", "bytes_per_launch": bytes_h,
                     "launch_ms": round(ev_ms, 4)},
        "rel_err_fp64_sampled": err,
    }


def run_batch(args, torch, sable, synth):
    """Serving batch: 256 matrices of uneven size, planner-chosen plans, one persistent
    hipGraph launch vs one launch per matrix on a stream; latency = completion time of each
    matrix measured from the batch submission."""
    import numpy as np

    from paper_2407_00829_amd import planner
    params, mean, std, tau = planner.load_weights(planner.WEIGHTS)
    Pd = torch.from_numpy(params).cuda()
    import concurrent.futures as cf
    plans, items, flops, classes, fallbacks = [], [], 0.0, [], 0
    t0 = time.perf_counter()
    seeds = [args.seed * 100000 + i for i in range(args.count)]
    with cf.ProcessPoolExecutor(8) as ex:
        mats = list(ex.map(synth.gen_c5_matrix, seeds))
    log(f"[bench] generated {len(mats)} matrices in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    for i, (A, kind, op) in enumerate(mats):
        ip, ix, vv = sable.device_csr(A)
        x = torch.from_numpy(synth.gen_dense_vector(i, A.ncols)).cuda()
        y = torch.empty(A.nrows, device="cuda")
        p, c, conf, fb = sable.sable_plan_auto(A.nrows, A.ncols, ip, ix, vv, Pd, mean, std, tau, x, y)
        p._src = (ip, ix, vv)
        classes.append(c)
        fallbacks += int(fb)
        if op == 0:
            sable.sable_autotune(p, 0, 1, x, y)
            items.append((0, 1, x, y))
            flops += 2.0 * A.nnz
        else:
            X = torch.from_numpy(synth.gen_dense_matrix(i, A.ncols, 16)).cuda()
            Y = torch.empty(A.nrows, 16, device="cuda")
            sable.sable_autotune(p, 1, 16, X, Y)
            items.append((1, 16, X, Y))
            flops += 2.0 * A.nnz * 16
        plans.append(p)
    plan_s = time.perf_counter() - t0
    log(f"[bench] planned {args.count} matrices in {plan_s:.1f} s ({fallbacks} fallbacks)")
    b = sable.sable_batch_create(plans, items)

    def run_batch_once():
        sable.sable_batch_run(b)

    seq = [sable.launcher("sable_spmv", p, x, y) if op == 0 else
           sable.launcher("sable_spmm", p, x, y, n) for p, (op, n, x, y) in zip(plans, items)]

    def run_sequential():
        for f in seq:
            f()

    wall_b, ev_b = timed_steps(run_batch_once, args.steps, args.warmup, torch)
    run_batch_once()
    torch.cuda.synchronize()
    ticks, hz = sable.sable_batch_latencies(b)
    lat_b = ticks.astype(np.float64) / hz * 1e6
    wall_s, ev_s = timed_steps(run_sequential, args.steps, args.warmup, torch)
    # per-matrix completion times of the sequential launches, from the first launch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(plans) + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for k, f in enumerate(seq):
        f()
        evs[k + 1].record()
    torch.cuda.synchronize()
    lat_s = np.array([evs[0].elapsed_time(e) * 1e3 for e in evs[1:]])
    # every item's batched result against an FP64 reference
    run_batch_once()
    torch.cuda.synchronize()
    errs = []
    for i, ((A, kind, op), (_, n, x, y)) in enumerate(zip(mats, items)):
        if op == 0:
            ref = ref_spmv(A, synth.gen_dense_vector(i, A.ncols))
        else:
            ref = ref_spmm_rows(A, synth.gen_dense_matrix(i, A.ncols, 16), np.arange(A.nrows))
        errs.append(rel_err(y.cpu().numpy(), ref))
    ms = wall_b / args.steps * 1e3
    return {
        "metric": "hybrid SpMV/SpMM GFLOP/s & %HBM peak vs plain GPU CSR; rel err vs FP64",
        "value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16x3",
        "data": "synthetic",
        "config": {"workload": f"serving batch: {args.count} matrices n~logU[1e3,2e5], mixed "
                               "generators, SpMV or SpMM n=16, planner-chosen plans, one "
                               "persistent hipGraph launch"},
        "matrices_per_s": round(args.count / (ms * 1e-3), 1),
        "batch": {"ms": round(ev_b, 4), "p50_us": round(float(np.percentile(lat_b, 50)), 2),
                  "p99_us": round(float(np.percentile(lat_b, 99)), 2)},
        "per_matrix_launches": {"ms": round(ev_s, 4),
                                "p50_us": round(float(np.percentile(lat_s, 50)), 2),
                                "p99_us": round(float(np.percentile(lat_s, 99)), 2)},
        "speedup_vs_per_matrix_launches": round(ev_s / ev_b, 3),
        "rel_err_fp64_max": float(np.max(errs)), "rel_err_fp64_median": float(np.median(errs)),
        "planner": {"fallbacks": fallbacks, "class_hist": np.bincount(classes, minlength=15).tolist(),
                    "plan_s": round(plan_s, 1)},
    }


def run_spec(args, torch, sable, synth):
    """Run-time specialization vs the generic fused kernels on small matrices: for each of
    --count C5-style matrices (SpMV), the autotuned generic variant and the hipRTC-specialized
    kernel, per-launch event time; geomean speedup and compile time."""
    import concurrent.futures as cf
    seeds = [args.seed * 100000 + i for i in range(args.count)]
    with cf.ProcessPoolExecutor(8) as ex:
        mats = list(ex.map(synth.gen_c5_matrix, seeds))
    th = sable.Thresholds()
    ratios, comp, skipped = [], [], 0
    for i, (A, kind, op) in enumerate(mats):
        p = sable.plan_host(A, [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR],
                            sable.SABLE_VBR_TILED, th)
        x = torch.from_numpy(synth.gen_dense_vector(i, A.ncols)).cuda()
        y = torch.empty(A.nrows, device="cuda")
        sable.sable_autotune(p, 0, 1, x, y)
        _, t_gen = timed_steps(sable.launcher("sable_spmv", p, x, y), 50, 10, torch)
        try:
            sable.sable_plan_specialize(p)
        except sable.SableError:
            skipped += 1
            continue
        comp.append(sable.sable_plan_info(p)["spec_ms"])
        sable.sable_plan_set_variant(p, 0, 11)
        _, t_spec = timed_steps(sable.launcher("sable_spmv", p, x, y), 50, 10, torch)
        ratios.append(t_gen / t_spec)
        p.destroy()
    r = np.array(ratios)
    return {"workload": "spec", "matrices": len(r), "too_large": skipped,
            "geomean_speedup_spec_vs_generic": float(np.exp(np.mean(np.log(r)))),
            "spec_faster_fraction": float(np.mean(r > 1.0)),
            "speedup_p10_p50_p90": [float(v) for v in np.percentile(r, [10, 50, 90])],
            "compile_ms_median": float(np.median(comp))}


def _small_matrix(seed):
    """The planner's generator at n ~ logU[1e3, 3e3] (mean row length U[4, 64]): sizes where
    the literal block search is within its budget."""
    from paper_2407_00829_amd import planner, synth
    n, rowlen, pi = planner.matrix_params(seed, nmin=1e3, nmax=3e3)
    A, x = synth.gen_mixed(seed, n=n, rowlen=rowlen, pi=pi)
    return seed, A, x


def run_coverage(args, torch, sable, synth):
    """Block-coverage cutoff sweep, the paper's coverage-threshold table (Appendix, Tab.
    threshold) on generated matrices: --count matrices from the planner's generator (band /
    block / scatter mixes), each planned as [VBR, CSR] (tiled search, paper defaults delta
    0.5, A_min 2500) without a coverage cutoff; coverage = VBR nnz / nnz. SpMV: the autotuned
    plan against this library's autotuned plain CSR kernel; SpMM (n = 128): against the
    autotuned CSR-only plan. These kernels take microseconds, so each is timed as a captured
    graph of --steps launches (GPU time without the host's per-launch cost); rocSPARSE csrmv,
    which is not captured, is reported per matrix with ordinary back-to-back event timing.
    For each cutoff t the matrices with coverage >= t are included, with the count of
    speedups > 1 and <= 1 and their geometric mean."""
    import concurrent.futures as cf

    import numpy as np

    from paper_2407_00829_amd import planner
    seeds = [300000 + args.seed * 100000 + i for i in range(args.count)]
    literal = args.vbr_mode == "paper"
    with cf.ProcessPoolExecutor(8) as ex:
        if literal:  # sizes where the literal block search of Alg. 1 / Alg. 2 is allowed
            mats = list(ex.map(_small_matrix, seeds))
        else:
            mats = list(ex.map(planner.make_matrix, seeds))
    log(f"[bench] generated {len(mats)} matrices")
    n_rhs = 128
    mode = sable.SABLE_VBR_PAPER if literal else sable.SABLE_VBR_TILED
    cov, sv, sm, times = [], [], [], []
    for i, (_, A, x) in enumerate(mats):
        p = sable.plan_host(A, [sable.SABLE_X_VBR, sable.SABLE_X_CSR], mode,
                            sable.Thresholds(coverage_pm=0))
        q = sable.plan_host(A, [sable.SABLE_X_CSR], sable.SABLE_VBR_TILED, sable.Thresholds())
        cov.append(sable.sable_plan_info(p)["vbr_nnz"] / max(A.nnz, 1))
        xd = torch.from_numpy(x).cuda()
        y = torch.empty(A.nrows, device="cuda")
        sable.sable_autotune(p, 0, 1, xd, y)
        t_h = graph_ms(lambda: sable.launcher("sable_spmv", p, xd, y), args.steps, torch)
        t_p = graph_ms(lambda: sable.launcher("sable_csr_spmv", p, xd, y), args.steps, torch)
        ip, ix, vv = p._src
        t_r, _ = rocsparse_csrmv_ms(A, ip, ix, vv, xd, torch.empty_like(y), args.steps,
                                    args.warmup, torch)
        sv.append(t_p / t_h)
        times.append([t_h, t_p, t_r])
        X = torch.from_numpy(synth.gen_dense_matrix(i, A.ncols, n_rhs)).cuda()
        Y = torch.empty(A.nrows, n_rhs, device="cuda")
        sable.sable_autotune(p, 1, n_rhs, X, Y)
        sable.sable_autotune(q, 1, n_rhs, X, Y)
        t_hm = graph_ms(lambda: sable.launcher("sable_spmm", p, X, Y, n_rhs), args.steps, torch)
        t_qm = graph_ms(lambda: sable.launcher("sable_spmm", q, X, Y, n_rhs), args.steps, torch)
        sm.append(t_qm / t_hm)
        p.destroy()
        q.destroy()
        if (i + 1) % 20 == 0:
            log(f"[bench] {i + 1} matrices timed")
    cov, sv, sm = np.array(cov), np.array(sv), np.array(sm)
    table = []
    for t in list(range(0, 16)) + [20]:
        m = cov >= t / 100.0
        row = {"threshold_pct": t, "matrices": int(m.sum())}
        for name, r in (("spmv", sv[m]), ("spmm", sm[m])):
            row[name] = {"faster": int((r > 1.0).sum()), "not_faster": int((r <= 1.0).sum()),
                         "geomean": float(np.exp(np.mean(np.log(r)))) if r.size else None}
        table.append(row)
    return {"workload": "coverage", "block_search": "literal" if literal else "tiled",
            "matrices": len(cov), "spmm_n": n_rhs,
            "coverage_p10_p50_p90": [float(v) for v in np.percentile(cov, [10, 50, 90])],
            "table": table,
            "per_matrix": [[round(float(c), 4), round(float(a), 4), round(float(b), 4)]
                           for c, a, b in zip(cov, sv, sm)],
            "spmv_ms_hybrid_plain_rocsparse": [[round(v, 5) if v else None for v in t]
                                               for t in times]}


def run_copy(args, torch):
    """Plain elementwise device copy (1 GiB read, 1 GiB written): the reference for scaling
    HBM byte counters."""
    a = torch.empty(256 * 1024 * 1024, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    f = lambda: torch.mul(a, 1.0, out=b)  # noqa: E731
    wall, ev_ms = timed_steps(f, args.steps, args.warmup, torch)
    nbytes = 2 * a.numel() * 4
    return {"workload": "copy", "bytes_per_launch": nbytes, "launch_ms": ev_ms,
            "gbs": nbytes / (ev_ms * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=["c2", "c1", "c3", "batch", "spec", "coverage", "copy"])
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--plan", default="hybrid", choices=["hybrid", "vbr"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--variants", default="",
                    help="SpMV: 'hybrid,far_split,plain' kernel variants instead of autotuning")
    ap.add_argument("--vbr-mode", default="tiled", choices=["tiled", "paper"],
                    help="coverage: the block search (paper = literal Alg. 1 / Alg. 2 on "
                         "matrices of 1e3 - 3e3 rows)")
    ap.add_argument("--spmm-variant", type=int, default=-1,
                    help="SpMM (c3): this kernel variant instead of autotuning")
    ap.add_argument("--cold-variants", default="",
                    help="SpMV,far-split,plain variants for the cache-cold launches (skips their tuning)")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"],
                    help="c2 / c3: f64 runs the FP64 executor")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch

    from paper_2407_00829_amd import sable, synth
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "c2" and args.dtype == "f64":
        out = run_spmv_f64(args, torch, sable, synth)
    elif args.workload in ("c2", "c1"):
        out = run_spmv(args, torch, sable, synth)
    elif args.workload == "c3" and args.dtype == "f64":
        out = run_spmm_f64(args, torch, sable, synth)
    elif args.workload == "c3":
        out = run_spmm(args, torch, sable, synth)
    elif args.workload == "batch":
        out = run_batch(args, torch, sable, synth)
    elif args.workload == "spec":
        out = run_spec(args, torch, sable, synth)
    elif args.workload == "coverage":
        out = run_coverage(args, torch, sable, synth)
    else:
        out = run_copy(args, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
