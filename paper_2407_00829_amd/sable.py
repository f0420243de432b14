"""Thin Python binding of libsable (argument marshalling only).

Every function here calls the C entry point of the same name in libsable.so; all work runs in
the library's HIP kernels. PyTorch tensors provide device memory and streams only. If the
library is missing the first call raises ``RuntimeError`` (there is no fallback).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsable.so")

SABLE_X_VDIA, SABLE_X_VBR, SABLE_X_CSR = 1, 2, 3
SABLE_VBR_AUTO, SABLE_VBR_PAPER, SABLE_VBR_TILED = 0, 1, 2
SABLE_F_SPLIT_BF16 = 1
SABLE_F_SPARSE_SEARCH = 2
SABLE_NFEAT = 140
SABLE_NCLASS = 15
SABLE_MLP_NPARAM = 128 * 140 + 128 + 128 * 128 + 128 + 15 * 128 + 15

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "INVALID_CSR", 3: "INCOMPLETE", 4: "TOO_LARGE",
          5: "OOM", 6: "HIP", 7: "INTERNAL"}

EXPORTED = [
    "sable_thresholds_default", "sable_plan", "sable_plan_destroy", "sable_plan_info",
    "sable_plan_export", "sable_spmv", "sable_spmm", "sable_csr_spmv", "sable_error_norm_f64",
    "sable_update_values", "sable_autotune", "sable_plan_set_variant", "sable_features", "sable_class_plan",
    "sable_mlp_forward", "sable_mlp_train_step", "sable_plan_exhaustive", "sable_plan_auto", "sable_batch_create", "sable_batch_run",
    "sable_batch_latencies", "sable_batch_destroy", "sable_last_error",
    "sable_update_values_f64", "sable_spmv_f64", "sable_spmm_f64", "sable_plan_specialize",
    "sable_error_norm_f64_noalloc", "sable_autotune_cache_clear",
]


class SableError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn}: {STATUS.get(code, code)}: {msg}")
        self.code = code


class sable_extractor(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("vbr_mode", ctypes.c_int32)]


class sable_csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int32), ("ncols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("values", ctypes.c_void_p)]


class sable_thresholds(ctypes.Structure):
    _fields_ = [("delta_band_pm", ctypes.c_int32), ("delta_block_pm", ctypes.c_int32),
                ("amin_band", ctypes.c_int64), ("amin_block", ctypes.c_int64),
                ("lseg", ctypes.c_int32), ("wmax", ctypes.c_int32), ("dmax", ctypes.c_int32),
                ("coverage_pm", ctypes.c_int32), ("tile_set_mask", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class sable_plan_stats(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int32), ("ncols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("nseg", ctypes.c_int32), ("nidiag", ctypes.c_int64),
                ("vdia_cells", ctypes.c_int64), ("vdia_nnz", ctypes.c_int64),
                ("nblk", ctypes.c_int32), ("vbr_mode_used", ctypes.c_int32),
                ("vbr_tile", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("vbr_cells", ctypes.c_int64), ("vbr_nnz", ctypes.c_int64),
                ("csr_nnz", ctypes.c_int64), ("bytes_matrix", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("plan_ms", ctypes.c_double),
                ("spmv_variant", ctypes.c_int32), ("spmm_variant", ctypes.c_int32),
                ("plain_variant", ctypes.c_int32), ("far_split", ctypes.c_int32),
                ("far_nnz", ctypes.c_int64), ("spec_ms", ctypes.c_double),
                ("structure_hash", ctypes.c_uint64), ("partition_hash", ctypes.c_uint64),
                ("mm_panels", ctypes.c_int64), ("mm_units", ctypes.c_int64)]


class sable_partition_host(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in (
        "vdia_val", "idiag", "seg_row_start", "seg_nrows", "seg_ndiags", "seg_val_ptr",
        "seg_idiag_ptr", "blk", "blk_val_ptr", "vbr_val", "csr_ptr", "csr_col", "csr_val",
        "owner", "slot", "vbr_bf16")]


class sable_batch_item(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("n", ctypes.c_int32), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libsable.so (raises if it has not been built: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2407_00829_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "sable_thresholds_default": [P],
        "sable_plan": [P, P, i32, P, P, P],
        "sable_plan_destroy": [P],
        "sable_plan_info": [P, P],
        "sable_plan_export": [P, P],
        "sable_spmv": [P, P, P, P],
        "sable_spmm": [P, P, P, i32, P],
        "sable_csr_spmv": [P, P, P, P],
        "sable_error_norm_f64": [P, P, i64, P, P],
        "sable_error_norm_f64_noalloc": [P, P, i64, P, P],
        "sable_update_values": [P, P, P],
        "sable_autotune": [P, i32, i32, P, P, P],
        "sable_autotune_cache_clear": [],
        "sable_plan_set_variant": [P, i32, i32],
        "sable_features": [P, P, P],
        "sable_class_plan": [i32, P, P, P],
        "sable_mlp_forward": [P, P, i32, P, P],
        "sable_mlp_train_step": [P, P, P, P, P, P, i32, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, i32, P, P],
        "sable_plan_exhaustive": [P, P, P, i32, P, P, P, P, P],
        "sable_plan_auto": [P, P, P, P, ctypes.c_float, P, P, P, P, P, P, P],
        "sable_batch_create": [P, P, i32, P, P],
        "sable_batch_run": [P, P],
        "sable_batch_latencies": [P, P, P],
        "sable_batch_destroy": [P],
        "sable_update_values_f64": [P, P, P],
        "sable_spmv_f64": [P, P, P, P],
        "sable_spmm_f64": [P, P, P, i32, P],
        "sable_plan_specialize": [P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.sable_last_error.restype = ctypes.c_char_p
    L.sable_last_error.argtypes = []
    _lib = L
    return L


def sable_last_error() -> str:
    return lib().sable_last_error().decode()


def _check(fn, rc):
    if rc != 0:
        raise SableError(fn, rc, sable_last_error())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclasses.dataclass
class Thresholds:
    """Mirror of sable_thresholds (per-mille densities; see include/sable.h)."""
    delta_band_pm: int = 750
    delta_block_pm: int = 500
    amin_band: int = 2500
    amin_block: int = 2500
    lseg: int = 64
    wmax: int = 32
    dmax: int = -1
    coverage_pm: int = 80
    tile_set_mask: int = 0
    flags: int = SABLE_F_SPLIT_BF16

    def c(self):
        return sable_thresholds(self.delta_band_pm, self.delta_block_pm, self.amin_band,
                                self.amin_block, self.lseg, self.wmax, self.dmax,
                                self.coverage_pm, self.tile_set_mask, self.flags)


def sable_thresholds_default() -> Thresholds:
    t = sable_thresholds()
    _check("sable_thresholds_default", lib().sable_thresholds_default(ctypes.byref(t)))
    return Thresholds(t.delta_band_pm, t.delta_block_pm, t.amin_band, t.amin_block, t.lseg,
                      t.wmax, t.dmax, t.coverage_pm, t.tile_set_mask, t.flags)


def csr_struct(nrows, ncols, indptr, indices, values) -> sable_csr:
    """sable_csr over device tensors (int32 indptr / indices, fp32 values)."""
    return sable_csr(int(nrows), int(ncols), int(indices.numel()), _ptr(indptr), _ptr(indices),
                     _ptr(values))


class Plan:
    """Owner of a sable_plan_t handle."""

    def __init__(self, handle, nrows, ncols, nnz):
        self.h = handle
        self.nrows, self.ncols, self.nnz = nrows, ncols, nnz

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def destroy(self):
        if self.h:
            lib().sable_plan_destroy(self.h)
            self.h = None


def sable_plan(nrows, ncols, indptr, indices, values, kinds, vbr_mode=SABLE_VBR_AUTO,
               th: Thresholds | None = None, stream=None) -> Plan:
    """Plan over device CSR tensors. kinds: extractor kinds, CSR last."""
    lst = (sable_extractor * len(kinds))(*[sable_extractor(int(k), int(vbr_mode)) for k in kinds])
    A = csr_struct(nrows, ncols, indptr, indices, values)
    th = th or Thresholds()
    cth = th.c()
    h = ctypes.c_void_p()
    _check("sable_plan", lib().sable_plan(ctypes.byref(A), lst, len(kinds), ctypes.byref(cth),
                                          _stream(stream), ctypes.byref(h)))
    return Plan(h, int(nrows), int(ncols), int(indices.numel()))


def sable_plan_info(p: Plan) -> dict:
    s = sable_plan_stats()
    _check("sable_plan_info", lib().sable_plan_info(p.h, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in s._fields_ if k != "pad0"}


def sable_plan_export(p: Plan) -> dict:
    """Host copies of every format array (layout in include/sable.h)."""
    st = sable_plan_info(p)
    nseg, nblk = st["nseg"], st["nblk"]
    out = dict(
        vdia_val=np.zeros(st["vdia_cells"], np.float32), idiag=np.zeros(st["nidiag"], np.int32),
        seg_row_start=np.zeros(nseg, np.int32), seg_nrows=np.zeros(nseg, np.int32),
        seg_ndiags=np.zeros(nseg, np.int32), seg_val_ptr=np.zeros(nseg, np.int64),
        seg_idiag_ptr=np.zeros(nseg, np.int32), blk=np.zeros(4 * nblk, np.int32),
        blk_val_ptr=np.zeros(nblk, np.int64), vbr_val=np.zeros(st["vbr_cells"], np.float32),
        csr_ptr=np.zeros(st["nrows"] + 1, np.int64), csr_col=np.zeros(st["csr_nnz"], np.int32),
        csr_val=np.zeros(st["csr_nnz"], np.float32), owner=np.zeros(st["nnz"], np.int8),
        slot=np.zeros(st["nnz"], np.int64), vbr_bf16=np.zeros(st["vbr_cells"], np.uint32))
    ph = sable_partition_host(*[out[k].ctypes.data_as(ctypes.c_void_p) for k, _ in
                                sable_partition_host._fields_])
    _check("sable_plan_export", lib().sable_plan_export(p.h, ctypes.byref(ph)))
    out["blk"] = out["blk"].reshape(nblk, 4)
    out["vbr_tile"] = st["vbr_tile"]
    out["vbr_mode"] = st["vbr_mode_used"]
    out["nrows"] = st["nrows"]
    out["ncols"] = st["ncols"]
    return out


def sable_spmv(p: Plan, x, y, stream=None) -> None:
    _check("sable_spmv", lib().sable_spmv(p.h, _ptr(x), _ptr(y), _stream(stream)))


def sable_csr_spmv(p: Plan, x, y, stream=None) -> None:
    _check("sable_csr_spmv", lib().sable_csr_spmv(p.h, _ptr(x), _ptr(y), _stream(stream)))


def sable_spmm(p: Plan, X, Y, n: int, stream=None) -> None:
    _check("sable_spmm", lib().sable_spmm(p.h, _ptr(X), _ptr(Y), int(n), _stream(stream)))


def launcher(fn: str, p: Plan, *args, stream=None):
    """A zero-argument callable for repeated calls of one product entry point (sable_spmv,
    sable_csr_spmv, sable_spmm, their _f64 forms) with its arguments marshalled once, so that
    a loop of launches of kernels that take a few microseconds is bound by the GPU rather
    than by per-call argument conversion. args: tensors (device pointers) and ints (n). The
    tensors' addresses are taken once: they must stay alive (and unmoved) while the callable
    is used; the stream is the current one at construction unless given."""
    f = getattr(lib(), fn)
    cargs = [p.h] + [ctypes.c_int32(a) if isinstance(a, int) else _ptr(a) for a in args]
    cargs.append(_stream(stream))

    def call():
        rc = f(*cargs)
        if rc:
            _check(fn, rc)
    return call


def sable_update_values(p: Plan, values, stream=None) -> None:
    _check("sable_update_values", lib().sable_update_values(p.h, _ptr(values), _stream(stream)))


def sable_plan_specialize(p: Plan, stream=None) -> None:
    _check("sable_plan_specialize", lib().sable_plan_specialize(p.h, _stream(stream)))


def sable_update_values_f64(p: Plan, values, stream=None) -> None:
    _check("sable_update_values_f64", lib().sable_update_values_f64(p.h, _ptr(values), _stream(stream)))


def sable_spmv_f64(p: Plan, x, y, stream=None) -> None:
    _check("sable_spmv_f64", lib().sable_spmv_f64(p.h, _ptr(x), _ptr(y), _stream(stream)))


def sable_spmm_f64(p: Plan, X, Y, n: int, stream=None) -> None:
    _check("sable_spmm_f64", lib().sable_spmm_f64(p.h, _ptr(X), _ptr(Y), int(n), _stream(stream)))


def sable_error_norm_f64(y, yref, stream=None) -> float:
    out = ctypes.c_double()
    _check("sable_error_norm_f64", lib().sable_error_norm_f64(
        _ptr(y), _ptr(yref), int(y.numel()), _stream(stream), ctypes.byref(out)))
    return out.value


def sable_error_norm_f64_noalloc(y, yref, out, stream=None) -> None:
    """out: a device float64 tensor of at least one element that receives the error."""
    _check("sable_error_norm_f64_noalloc", lib().sable_error_norm_f64_noalloc(
        _ptr(y), _ptr(yref), int(y.numel()), _stream(stream), _ptr(out)))


def sable_autotune(p: Plan, op: int, n: int, x, y, stream=None) -> None:
    _check("sable_autotune", lib().sable_autotune(p.h, int(op), int(n), _ptr(x), _ptr(y),
                                                  _stream(stream)))


def sable_autotune_cache_clear() -> None:
    _check("sable_autotune_cache_clear", lib().sable_autotune_cache_clear())


def sable_plan_set_variant(p: Plan, op: int, variant: int) -> None:
    _check("sable_plan_set_variant", lib().sable_plan_set_variant(p.h, int(op), int(variant)))


def sable_features(nrows, ncols, indptr, indices, values, stream=None) -> np.ndarray:
    A = csr_struct(nrows, ncols, indptr, indices, values)
    out = np.zeros(SABLE_NFEAT, np.float32)
    _check("sable_features", lib().sable_features(ctypes.byref(A), _stream(stream),
                                                  out.ctypes.data_as(ctypes.c_void_p)))
    return out


def sable_class_plan(c: int):
    lst = (sable_extractor * 3)()
    n = ctypes.c_int32()
    th = sable_thresholds()
    _check("sable_class_plan", lib().sable_class_plan(int(c), lst, ctypes.byref(n), ctypes.byref(th)))
    kinds = [lst[i].kind for i in range(n.value)]
    mode = lst[0].vbr_mode if n.value else 0
    t = Thresholds(th.delta_band_pm, th.delta_block_pm, th.amin_band, th.amin_block, th.lseg,
                   th.wmax, th.dmax, th.coverage_pm, th.tile_set_mask, th.flags)
    return kinds, mode, t


def sable_mlp_forward(params, feats, logits, stream=None) -> None:
    _check("sable_mlp_forward", lib().sable_mlp_forward(_ptr(params), _ptr(feats),
                                                        int(feats.shape[0]), _ptr(logits),
                                                        _stream(stream)))


def sable_mlp_train_step(params, grads, m, v, feats, labels, lr, beta1, beta2, eps, t,
                         stream=None) -> float:
    loss = ctypes.c_float()
    _check("sable_mlp_train_step", lib().sable_mlp_train_step(
        _ptr(params), _ptr(grads), _ptr(m), _ptr(v), _ptr(feats), _ptr(labels),
        int(feats.shape[0]), float(lr), float(beta1), float(beta2), float(eps), int(t),
        _stream(stream), ctypes.byref(loss)))
    return loss.value


def sable_plan_exhaustive(nrows, ncols, indptr, indices, values, x, y, reps=10, stream=None,
                          with_refs=False):
    """Returns (Plan, best_class, times_ms[15]), and with_refs the same-path times of the
    plain CSR baseline and the default list (ref_ms[2]) as a fourth element."""
    A = csr_struct(nrows, ncols, indptr, indices, values)
    h = ctypes.c_void_p()
    bc = ctypes.c_int32()
    times = np.zeros(SABLE_NCLASS, np.float32)
    ref = np.zeros(2, np.float32)
    _check("sable_plan_exhaustive", lib().sable_plan_exhaustive(
        ctypes.byref(A), _ptr(x), _ptr(y), int(reps), _stream(stream), ctypes.byref(h),
        ctypes.byref(bc), times.ctypes.data_as(ctypes.c_void_p),
        ref.ctypes.data_as(ctypes.c_void_p) if with_refs else None))
    plan = Plan(h, int(nrows), int(ncols), int(indices.numel()))
    return (plan, bc.value, times, ref) if with_refs else (plan, bc.value, times)


def sable_plan_auto(nrows, ncols, indptr, indices, values, params, feat_mean, feat_std,
                    tau_conf, x, y, stream=None):
    """Returns (Plan, chosen_class, confidence, fell_back)."""
    A = csr_struct(nrows, ncols, indptr, indices, values)
    fm = np.ascontiguousarray(feat_mean, np.float32)
    fs = np.ascontiguousarray(feat_std, np.float32)
    h = ctypes.c_void_p()
    c = ctypes.c_int32()
    conf = ctypes.c_float()
    fb = ctypes.c_int32()
    _check("sable_plan_auto", lib().sable_plan_auto(
        ctypes.byref(A), _ptr(params), fm.ctypes.data_as(ctypes.c_void_p),
        fs.ctypes.data_as(ctypes.c_void_p), float(tau_conf), _ptr(x), _ptr(y), _stream(stream),
        ctypes.byref(h), ctypes.byref(c), ctypes.byref(conf), ctypes.byref(fb)))
    return Plan(h, int(nrows), int(ncols), int(indices.numel())), c.value, conf.value, bool(fb.value)


class Batch:
    def __init__(self, h, count, keep):
        self.h, self.count, self._keep = h, count, keep

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def destroy(self):
        if self.h:
            lib().sable_batch_destroy(self.h)
            self.h = None


def sable_batch_create(plans, items, stream=None) -> Batch:
    """items: list of (op, n, x_tensor, y_tensor)."""
    n = len(plans)
    ph = (ctypes.c_void_p * n)(*[p.h for p in plans])
    it = (sable_batch_item * n)(*[sable_batch_item(int(o), int(k), _ptr(x), _ptr(y))
                                  for (o, k, x, y) in items])
    h = ctypes.c_void_p()
    _check("sable_batch_create", lib().sable_batch_create(ph, it, n, _stream(stream),
                                                          ctypes.byref(h)))
    return Batch(h, n, (plans, items))


def sable_batch_run(b: Batch, stream=None) -> None:
    _check("sable_batch_run", lib().sable_batch_run(b.h, _stream(stream)))


def sable_batch_latencies(b: Batch):
    ticks = np.zeros(b.count, np.uint64)
    hz = ctypes.c_double()
    _check("sable_batch_latencies", lib().sable_batch_latencies(
        b.h, ticks.ctypes.data_as(ctypes.c_void_p), ctypes.byref(hz)))
    return ticks, hz.value


# ---- convenience wrappers used by tests and the benchmark -------------------------------

def device_csr(A, device="cuda"):
    """Copy a host CSR (synth.CSR) to device tensors (int32 indptr/indices, fp32 values)."""
    import torch
    if A.nnz >= 2 ** 31:
        raise ValueError("nnz >= 2^31")
    ip = torch.from_numpy(np.ascontiguousarray(A.indptr, np.int32)).to(device)
    ix = torch.from_numpy(np.ascontiguousarray(A.indices, np.int32)).to(device)
    vv = torch.from_numpy(np.ascontiguousarray(A.values, np.float32)).to(device)
    return ip, ix, vv


def plan_host(A, kinds, vbr_mode=SABLE_VBR_AUTO, th: Thresholds | None = None, stream=None):
    """Plan for a host CSR: copies it to the GPU, plans, keeps the device copy alive."""
    ip, ix, vv = device_csr(A)
    p = sable_plan(A.nrows, A.ncols, ip, ix, vv, kinds, vbr_mode, th, stream)
    p._src = (ip, ix, vv)
    return p
