"""CPU oracle for the hybrid VDIA + VBR + CSR method (test infrastructure).

Plain FP64 / exact-integer reference implementation written from the paper, used only by
tests/, the smoke check and the benchmark's CPU-baseline leg. It shares no code with the
GPU library (paper_2407_00829_amd) and never imports it.

Functions (each follows the passage cited in oracle/sor.cpp):
  plan(A, kinds, vbr_mode, th)   extractors in list order (Sec. 3, Alg. 1-4) -> dict of arrays
  spmv(A, x), spmm(A, X)         FP64 products over A's entries (Sec. 5 "Kernels")
  spmv_rows / spmm_rows          the same for selected rows (sampled checks at full size)
  spmv64(A, v, x), spmm64(A, v, X)  FP64 products with fp64 values and operands (the
                                 paper's precision, Sec. 5 / App. A), entries in CSR order
  partition_spmv(A, kinds, vbr_mode, th, x)  FP64 product over the formats of the plan the
                                 oracle builds for A (fill included, Sec. 3.4 shared output)
  find_block(A, region, by_rows, th, sparse)  one pass of the block search (Alg. 2) on a
                                 region; sparse = the window rule over non-empty inner
                                 indices only (same result, pinned against the dense scan)
  best_window(H, s, th, sparse)  the window scan of Alg. 2 for one span's inner counts
  paper_fits(A, th)              the literal search's budget test and work count
  bf16_split(a)                  round-to-nearest-even hi/lo split of fp32 values
  rel_err(y, yref)               normwise relative error ||y - yref||_2 / ||yref||_2
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsor.so")
_lib = None

VDIA, VBR, CSR = 1, 2, 3
MODE_AUTO, MODE_PAPER, MODE_TILED = 0, 1, 2
TILES = (4, 6, 8, 16, 32)

ERRORS = {1: "invalid argument", 2: "invalid CSR", 3: "incomplete plan (CSR must be last)",
          4: "too large for the literal block search", 5: "out of memory"}


def build(force: bool = True) -> str:
    """Compile oracle/sor.cpp with g++ (OpenMP for the parallel-for of Alg. 2 and the
    row-parallel products)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           os.path.join(_HERE, "sor.cpp"), "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Thr(ctypes.Structure):
    _fields_ = [("delta_band_pm", ctypes.c_int32), ("delta_block_pm", ctypes.c_int32),
                ("amin_band", ctypes.c_int64), ("amin_block", ctypes.c_int64),
                ("lseg", ctypes.c_int32), ("wmax", ctypes.c_int32), ("dmax", ctypes.c_int32),
                ("coverage_pm", ctypes.c_int32), ("tile_set_mask", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


@dataclasses.dataclass
class Thresholds:
    """Extraction thresholds. Densities are per-mille integers (delta = p / 1000).

    Defaults: delta = 0.5 for blocks and A_min = 2500 (Sec. 4.1), delta = 0.75 for bands
    (the value used for the band evaluation, Sec. 5 "Implementation"), coverage cutoff 8%
    (Alg. 1). l_seg, W_max and d_max have no value in the paper (readings: 64, 32, all).
    """
    delta_band_pm: int = 750
    delta_block_pm: int = 500
    amin_band: int = 2500
    amin_block: int = 2500
    lseg: int = 64
    wmax: int = 32
    dmax: int = -1
    coverage_pm: int = 80
    tile_set_mask: int = 0

    def _c(self):
        return _Thr(self.delta_band_pm, self.delta_block_pm, self.amin_band, self.amin_block,
                    self.lseg, self.wmax, self.dmax, self.coverage_pm, self.tile_set_mask, 0)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.sor_validate.argtypes = [i64, i64, i64, P, P]
    lib.sor_validate.restype = ctypes.c_int
    lib.sor_plan.argtypes = [i64, i64, i64, P, P, P, P, P, ctypes.c_int32,
                             ctypes.POINTER(_Thr), ctypes.POINTER(ctypes.c_void_p)]
    lib.sor_plan.restype = ctypes.c_int
    lib.sor_counts.argtypes = [P, P]
    lib.sor_export.argtypes = [P] * 16
    lib.sor_free.argtypes = [P]
    lib.sor_set_threads.argtypes = [ctypes.c_int32]
    lib.sor_max_threads.restype = ctypes.c_int32
    lib.sor_spmv_f64.argtypes = [i64, P, P, P, P, P]
    lib.sor_spmv_rows_f64.argtypes = [i64, P, P, P, P, P, P]
    lib.sor_spmm_f64.argtypes = [i64, P, P, P, P, i64, P]
    lib.sor_spmm_rows_f64.argtypes = [i64, P, P, P, P, P, i64, P]
    lib.sor_partition_spmv_f64.argtypes = [P, P, P]
    lib.sor_find_block.argtypes = [i64, i64, i64, P, P, i64, i64, i64, i64, ctypes.c_int32,
                                   ctypes.POINTER(_Thr), P]
    lib.sor_find_block.restype = ctypes.c_int
    lib.sor_find_block_sparse.argtypes = lib.sor_find_block.argtypes
    lib.sor_find_block_sparse.restype = ctypes.c_int
    lib.sor_best_window.argtypes = [i64, P, i64, ctypes.POINTER(_Thr), ctypes.c_int32, P]
    lib.sor_paper_fits.argtypes = [i64, i64, i64, P, P, ctypes.POINTER(_Thr), P]
    lib.sor_paper_fits.restype = ctypes.c_int32
    lib.sor_bf16_split.argtypes = [i64, P, P, P]
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _csr_arrays(A):
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    values = np.ascontiguousarray(A.values, dtype=np.float32)
    return indptr, indices, values


def set_threads(n: int) -> None:
    _load().sor_set_threads(int(n))


def max_threads() -> int:
    return int(_load().sor_max_threads())


def validate(A) -> int:
    lib = _load()
    ip, ix, _ = _csr_arrays(A)
    return int(lib.sor_validate(A.nrows, A.ncols, int(ip[-1]), _p(ip), _p(ix)))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}: {ERRORS.get(code, 'error')}")
        self.code = code


def plan(A, kinds, vbr_mode=MODE_AUTO, th: Thresholds | None = None) -> dict:
    """Run the extractors `kinds` (e.g. [VDIA, VBR, CSR]) on A; return the formats.

    Returned keys: vdia_val, idiag, seg_row_start, seg_nrows, seg_ndiags, seg_val_ptr,
    seg_idiag_ptr (VDIA, Fig. "vdia"); blk (nblk x 4: r0, r1, c0, c1), blk_val_ptr, vbr_val
    (column-major per block), vbr_tile, vbr_mode (VBR); csr_ptr, csr_col, csr_val (CSR);
    owner (0 VDIA / 1 VBR / 2 CSR per input entry) and slot (index in that format's values).
    """
    lib = _load()
    th = th or Thresholds()
    ip, ix, vv = _csr_arrays(A)
    kinds = np.asarray(kinds, dtype=np.int32)
    modes = np.full(kinds.size, vbr_mode, dtype=np.int32)
    h = ctypes.c_void_p()
    cth = th._c()
    rc = lib.sor_plan(A.nrows, A.ncols, int(ip[-1]), _p(ip), _p(ix), _p(vv), _p(kinds),
                      _p(modes), int(kinds.size), ctypes.byref(cth), ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    try:
        c = np.zeros(8, dtype=np.int64)
        lib.sor_counts(h, _p(c))
        nseg, nval, nid, nblk, nbv, ncsr = (int(t) for t in c[:6])
        out = dict(
            vdia_val=np.zeros(nval, np.float32), idiag=np.zeros(nid, np.int32),
            seg_row_start=np.zeros(nseg, np.int32), seg_nrows=np.zeros(nseg, np.int32),
            seg_ndiags=np.zeros(nseg, np.int32), seg_val_ptr=np.zeros(nseg, np.int64),
            seg_idiag_ptr=np.zeros(nseg, np.int32), blk=np.zeros(4 * nblk, np.int32),
            blk_val_ptr=np.zeros(nblk, np.int64), vbr_val=np.zeros(nbv, np.float32),
            csr_ptr=np.zeros(A.nrows + 1, np.int64), csr_col=np.zeros(ncsr, np.int32),
            csr_val=np.zeros(ncsr, np.float32), owner=np.zeros(int(ip[-1]), np.int8),
            slot=np.zeros(int(ip[-1]), np.int64))
        keys = ["vdia_val", "idiag", "seg_row_start", "seg_nrows", "seg_ndiags", "seg_val_ptr",
                "seg_idiag_ptr", "blk", "blk_val_ptr", "vbr_val", "csr_ptr", "csr_col",
                "csr_val", "owner", "slot"]
        lib.sor_export(h, *[_p(out[k]) for k in keys])
        out["blk"] = out["blk"].reshape(nblk, 4)
        out["vbr_tile"] = int(c[6])
        out["vbr_mode"] = int(c[7])
        out["nrows"] = A.nrows
        out["ncols"] = A.ncols
        return out
    finally:
        lib.sor_free(h)


def partition_spmv(A, kinds, vbr_mode=MODE_AUTO, th: Thresholds | None = None,
                   x: np.ndarray | None = None) -> np.ndarray:
    """FP64 y = (VDIA part + VBR part + CSR part) x over the formats of the plan the oracle
    builds for A (stored fill cells included, out-of-range band cells skipped). Equals
    spmv(A, x) up to FP64 rounding order (Sec. 3.4: regions accumulate into one output)."""
    lib = _load()
    th = th or Thresholds()
    ip, ix, vv = _csr_arrays(A)
    kinds = np.asarray(kinds, dtype=np.int32)
    modes = np.full(kinds.size, vbr_mode, dtype=np.int32)
    h = ctypes.c_void_p()
    cth = th._c()
    rc = lib.sor_plan(A.nrows, A.ncols, int(ip[-1]), _p(ip), _p(ix), _p(vv), _p(kinds),
                      _p(modes), int(kinds.size), ctypes.byref(cth), ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    try:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros(A.nrows, np.float64)
        lib.sor_partition_spmv_f64(h, _p(x), _p(y))
        return y
    finally:
        lib.sor_free(h)


def find_block(A, region, by_rows: bool, th: Thresholds | None = None, sparse: bool = False):
    """One FindBlock pass (Alg. 2) over region (r0, r1, c0, c1) of A: by_rows = the CSR pass
    (outer = rows), else the CSC pass. Returns (nnz, area, o0, o1, i0, i1), region-relative,
    with nnz = -1 when no window qualifies. sparse: evaluate the window rule over the
    non-empty inner indices only (the same result; pinned against the dense scan)."""
    lib = _load()
    th = th or Thresholds()
    ip, ix, _ = _csr_arrays(A)
    out = np.zeros(6, np.int64)
    cth = th._c()
    r0, r1, c0, c1 = (int(t) for t in region)
    fn = lib.sor_find_block_sparse if sparse else lib.sor_find_block
    rc = fn(A.nrows, A.ncols, int(ip[-1]), _p(ip), _p(ix), r0, r1, c0, c1,
            1 if by_rows else 0, ctypes.byref(cth), _p(out))
    if rc:
        raise OracleError(rc)
    return tuple(int(t) for t in out)


def best_window(H, s: int, th: Thresholds | None = None, sparse: bool = False):
    """The window scan of Alg. 2 for one span of s slices with inner counts H: (nnz, area,
    i0, i1), nnz = -1 when no window qualifies."""
    lib = _load()
    th = th or Thresholds()
    H = np.ascontiguousarray(H, dtype=np.int64)
    out = np.zeros(4, np.int64)
    cth = th._c()
    lib.sor_best_window(H.size, _p(H), int(s), ctypes.byref(cth), 1 if sparse else 0, _p(out))
    return tuple(int(t) for t in out)


def paper_fits(A, th: Thresholds | None = None):
    """The literal block search's budget test on A: (allowed, work count). Allowed when
    nrows * ncols * max(nrows, ncols) <= 2^37, or when the sparse scan's work, one step per
    outer span of both passes plus min(inner length, the span's entries), is <= 2^37."""
    lib = _load()
    th = th or Thresholds()
    ip, ix, _ = _csr_arrays(A)
    cost = np.zeros(1, np.int64)
    cth = th._c()
    ok = lib.sor_paper_fits(A.nrows, A.ncols, int(ip[-1]), _p(ip), _p(ix), ctypes.byref(cth),
                            _p(cost))
    return bool(ok), int(cost[0])


def partition_spmv_from_export(P: dict, x: np.ndarray) -> np.ndarray:
    """FP64 y from exported formats (pure numpy; used to cross-check exports)."""
    n, m = P["nrows"], P["ncols"]
    y = np.zeros(n, np.float64)
    xd = x.astype(np.float64)
    for s in range(P["seg_row_start"].size):
        r0, nr, nd = int(P["seg_row_start"][s]), int(P["seg_nrows"][s]), int(P["seg_ndiags"][s])
        vp, ipp = int(P["seg_val_ptr"][s]), int(P["seg_idiag_ptr"][s])
        rows = np.arange(r0, r0 + nr)
        for t in range(nd):
            o = int(P["idiag"][ipp + t])
            c = rows + o
            ok = (c >= 0) & (c < m)
            vals = P["vdia_val"][vp + t * nr: vp + (t + 1) * nr].astype(np.float64)
            y[rows[ok]] += vals[ok] * xd[c[ok]]
    for b in range(P["blk"].shape[0]):
        r0, r1, c0, c1 = (int(t) for t in P["blk"][b])
        h, w = r1 - r0, c1 - c0
        vp = int(P["blk_val_ptr"][b])
        blk = P["vbr_val"][vp: vp + h * w].astype(np.float64).reshape(w, h).T
        y[r0:r1] += blk @ xd[c0:c1]
    ptr, col, val = P["csr_ptr"], P["csr_col"], P["csr_val"]
    rows = np.repeat(np.arange(n), np.diff(ptr))
    np.add.at(y, rows, val.astype(np.float64) * xd[col])
    return y


def spmv(A, x: np.ndarray) -> np.ndarray:
    lib = _load()
    ip, ix, vv = _csr_arrays(A)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.zeros(A.nrows, np.float64)
    lib.sor_spmv_f64(A.nrows, _p(ip), _p(ix), _p(vv), _p(x), _p(y))
    return y


def spmv_rows(A, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    lib = _load()
    ip, ix, vv = _csr_arrays(A)
    x = np.ascontiguousarray(x, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.zeros(rows.size, np.float64)
    lib.sor_spmv_rows_f64(rows.size, _p(rows), _p(ip), _p(ix), _p(vv), _p(x), _p(y))
    return y


def spmm(A, X: np.ndarray) -> np.ndarray:
    lib = _load()
    ip, ix, vv = _csr_arrays(A)
    X = np.ascontiguousarray(X, dtype=np.float32)
    n = X.shape[1]
    Y = np.zeros((A.nrows, n), np.float64)
    lib.sor_spmm_f64(A.nrows, _p(ip), _p(ix), _p(vv), _p(X), n, _p(Y))
    return Y


def spmv64(A, values: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y[i] = sum over A's stored entries (i, j) of values[k] * x[j], all in FP64; values are
    given in A's CSR order (the plan's input order) and replace A.values. Entries are added
    in CSR order."""
    rows = np.repeat(np.arange(A.nrows, dtype=np.int64), np.diff(np.asarray(A.indptr, np.int64)))
    v = np.asarray(values, np.float64)
    xd = np.asarray(x, np.float64)
    y = np.zeros(A.nrows, np.float64)
    np.add.at(y, rows, v * xd[np.asarray(A.indices, np.int64)])
    return y


def spmm64(A, values: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Y = A X in FP64 with fp64 values (CSR order) and a row-major fp64 X."""
    rows = np.repeat(np.arange(A.nrows, dtype=np.int64), np.diff(np.asarray(A.indptr, np.int64)))
    v = np.asarray(values, np.float64)
    Xd = np.asarray(X, np.float64)
    Y = np.zeros((A.nrows, Xd.shape[1]), np.float64)
    np.add.at(Y, rows, v[:, None] * Xd[np.asarray(A.indices, np.int64)])
    return Y


def spmm_rows(A, X: np.ndarray, rows: np.ndarray) -> np.ndarray:
    lib = _load()
    ip, ix, vv = _csr_arrays(A)
    X = np.ascontiguousarray(X, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n = X.shape[1]
    Y = np.zeros((rows.size, n), np.float64)
    lib.sor_spmm_rows_f64(rows.size, _p(rows), _p(ip), _p(ix), _p(vv), _p(X), n, _p(Y))
    return Y


def bf16_split(a: np.ndarray):
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float32).ravel()
    hi = np.zeros(a.size, np.uint16)
    lo = np.zeros(a.size, np.uint16)
    lib.sor_bf16_split(a.size, _p(a), _p(hi), _p(lo))
    return hi, lo


def bf16_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, np.uint32) << 16).view(np.float32)


def rel_err(y, yref) -> float:
    """Normwise relative error ||y - yref||_2 / ||yref||_2 (||y - yref||_2 if yref = 0)."""
    y = np.asarray(y, np.float64).ravel()
    yref = np.asarray(yref, np.float64).ravel()
    num = float(np.sqrt(np.sum((y - yref) ** 2)))
    den = float(np.sqrt(np.sum(yref ** 2)))
    return num / den if den > 0 else num


# ---------------------------------------------------------------------------------------
# SPARSKIT VBR view (App. B, Fig. "vbr"): Val holds each dense block column-major, Indx the
# start of every block in Val (plus the total), Bindx the block-column index of every block,
# Bpntrb the CSR-style pointer of block rows into Bindx, Rpntr / Cpntr the block boundaries.

def vbr_from_dense(D: np.ndarray, rpntr, cpntr):
    """SPARSKIT arrays for dense matrix D on the partition (rpntr, cpntr): every block that
    holds a nonzero is stored, block rows in order, block columns ascending."""
    Val, Indx, Bindx, Bpntrb = [], [0], [], [0]
    for I in range(len(rpntr) - 1):
        for J in range(len(cpntr) - 1):
            blk = D[rpntr[I]:rpntr[I + 1], cpntr[J]:cpntr[J + 1]]
            if np.any(blk != 0):
                Val.extend(blk.T.ravel().tolist())  # column-major
                Indx.append(len(Val))
                Bindx.append(J)
        Bpntrb.append(len(Bindx))
    return (np.array(Val, np.float64), np.array(Indx, np.int64), np.array(Bindx, np.int64),
            np.array(Bpntrb, np.int64))


def sparskit_spmv(Val, Indx, Bindx, Rpntr, Cpntr, Bpntrb, x) -> np.ndarray:
    """y = A x for a SPARSKIT VBR matrix, FP64, block by block."""
    y = np.zeros(Rpntr[-1], np.float64)
    for I in range(len(Rpntr) - 1):
        r0, r1 = Rpntr[I], Rpntr[I + 1]
        for q in range(Bpntrb[I], Bpntrb[I + 1]):
            J = Bindx[q]
            c0, c1 = Cpntr[J], Cpntr[J + 1]
            h, w = r1 - r0, c1 - c0
            blk = np.asarray(Val[Indx[q]:Indx[q + 1]], np.float64).reshape(w, h).T
            y[r0:r1] += blk @ np.asarray(x[c0:c1], np.float64)
    return y


def export_to_sparskit(P: dict):
    """SPARSKIT view of exported VBR blocks whose row and column ranges never straddle another
    block's boundary (always true for the literal search, whose blocks are row- and
    column-disjoint). Grid cells without a block are absent."""
    blk = P["blk"]
    rb = sorted(set([0, P["nrows"]] + blk[:, 0].tolist() + blk[:, 1].tolist()))
    cb = sorted(set([0, P["ncols"]] + blk[:, 2].tolist() + blk[:, 3].tolist()))
    rid = {v: i for i, v in enumerate(rb)}
    cid = {v: i for i, v in enumerate(cb)}
    cells = {}
    for b in range(blk.shape[0]):
        r0, r1, c0, c1 = (int(t) for t in blk[b])
        I, J = rid[r0], cid[c0]
        if rid[r1] != I + 1 or cid[c1] != J + 1:
            raise ValueError("blocks do not form a grid")
        vp = int(P["blk_val_ptr"][b])
        cells[(I, J)] = P["vbr_val"][vp: vp + (r1 - r0) * (c1 - c0)]
    Val, Indx, Bindx, Bpntrb = [], [0], [], [0]
    for I in range(len(rb) - 1):
        for J in range(len(cb) - 1):
            if (I, J) in cells:
                Val.extend(cells[(I, J)].tolist())
                Indx.append(len(Val))
                Bindx.append(J)
        Bpntrb.append(len(Bindx))
    return (np.array(Val, np.float64), np.array(Indx, np.int64), np.array(Bindx, np.int64),
            np.array(rb, np.int64), np.array(cb, np.int64), np.array(Bpntrb, np.int64))


def check_partition(A, P: dict, th: Thresholds, kinds) -> None:
    """Exact-cover and threshold invariants of an exported partition (raises AssertionError).

    * every input entry is stored exactly once, in the format named by owner[], at slot[],
      with a bitwise-equal value; every other stored VDIA/VBR cell is 0 (fill) ;
    * band segments are row-disjoint, at least l_seg rows; blocks are element-disjoint,
      width >= 2, delta-dense and >= A_min (Alg. 1, Alg. 3, Alg. 4).
    """
    n, m = A.nrows, A.ncols
    rows = A.rows()
    cols = A.indices.astype(np.int64)
    vals = A.values
    owner, slot = P["owner"], P["slot"]
    assert owner.size == A.nnz and np.all((owner >= 0) & (owner <= 2))
    vd_used = np.zeros(P["vdia_val"].size, bool)
    vb_used = np.zeros(P["vbr_val"].size, bool)
    # VDIA cells
    segs = []
    for s in range(P["seg_row_start"].size):
        r0, nr, nd = int(P["seg_row_start"][s]), int(P["seg_nrows"][s]), int(P["seg_ndiags"][s])
        segs.append((r0, r0 + nr))
        assert nr >= th.lseg
        idg = P["idiag"][P["seg_idiag_ptr"][s]: P["seg_idiag_ptr"][s] + nd]
        assert np.all(np.diff(idg) == 1)
    segs.sort()
    for a, b in zip(segs, segs[1:]):
        assert a[1] <= b[0], "segments overlap in rows"
    sel = owner == 0
    if np.any(sel):
        vd = P["vdia_val"][slot[sel]]
        assert np.array_equal(vd.view(np.uint32), vals[sel].view(np.uint32))
        vd_used[slot[sel]] = True
    assert not np.any(P["vdia_val"][~vd_used] != 0)
    # VBR cells
    occ = {}
    for b in range(P["blk"].shape[0]):
        r0, r1, c0, c1 = (int(t) for t in P["blk"][b])
        assert c1 - c0 >= 2 and r1 > r0
        for r in range(r0, r1):
            occ.setdefault(r, []).append((c0, c1))
    for r, iv in occ.items():
        iv.sort()
        for a, b in zip(iv, iv[1:]):
            assert a[1] <= b[0], "blocks overlap"
    sel = owner == 1
    if np.any(sel):
        vb = P["vbr_val"][slot[sel]]
        assert np.array_equal(vb.view(np.uint32), vals[sel].view(np.uint32))
        vb_used[slot[sel]] = True
    assert not np.any(P["vbr_val"][~vb_used] != 0)
    # CSR
    sel = owner == 2
    assert int(sel.sum()) == P["csr_col"].size
    if np.any(sel):
        cv = P["csr_val"][slot[sel]]
        assert np.array_equal(cv.view(np.uint32), vals[sel].view(np.uint32))
        assert np.array_equal(P["csr_col"][slot[sel]].astype(np.int64), cols[sel])
    # slots of one format are distinct
    for o in (0, 1, 2):
        s = slot[owner == o]
        assert np.unique(s).size == s.size
    # entry positions agree with the format geometry
    for t in np.nonzero(owner == 0)[0][:2000]:
        i, j = int(rows[t]), int(cols[t])
        s = int(np.searchsorted(P["seg_row_start"], i, side="right") - 1)
        r0, nr = int(P["seg_row_start"][s]), int(P["seg_nrows"][s])
        assert r0 <= i < r0 + nr
        o0 = int(P["idiag"][P["seg_idiag_ptr"][s]])
        tt = (j - i) - o0
        assert int(slot[t]) == int(P["seg_val_ptr"][s]) + tt * nr + (i - r0)
