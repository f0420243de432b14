"""Planner oracle (test infrastructure): matrix features and an FP64 MLP.

Independent NumPy implementations of what the GPU planner computes, used only by tests:
  features(A)          the 140 structure features (definitions below, exact integer counts)
  mlp_forward / mlp_loss_grad   FP64 forward pass and softmax cross-entropy gradients of the
                       140-128-128-15 ReLU network (parameters in the same flat layout)
  init_params(seed)    a deterministic initialisation shared by GPU tests

Feature definitions (n rows, m columns, nnz entries):
  [0, 64)   diagonal run lengths: maximal runs of consecutive rows carrying an entry on the
            same diagonal d = j - i; a run of length L falls in bin 4e + floor(4L / 2^e) - 4
            with e = floor(log2 L) (four bins per octave; L >= 2^16 -> bin 63); the bin
            receives weight L; weights are divided by nnz.
  [64, 128) 16 x 16 tile densities: for every non-empty tile (edge tiles clipped) with c
            entries over area a, bin min(63, floor(64 c / a)) receives weight c / nnz.
  128..130  log1p(mean row length), log1p(std of row length), log1p(max row length)
  131..133  ln n, ln m, ln nnz
  134, 135  fraction of nnz with d = 0, with |d| <= 32
  136       largest diagonal count / n
  137       number of occupied diagonals / (n + m - 1)
  138       fraction of nnz in tiles with 2c >= a
  139       fraction of empty rows
"""
from __future__ import annotations

import numpy as np

NFEAT, NH, NOUT = 140, 128, 15
SHAPES = [("W1", (NH, NFEAT)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def _log_bin(L: np.ndarray) -> np.ndarray:
    L = np.asarray(L, np.int64)
    e = np.floor(np.log2(L)).astype(np.int64)
    # guard float log2 at exact powers of two
    e = np.where((1 << (e + 1)) <= L, e + 1, e)
    e = np.where((1 << e) > L, e - 1, e)
    b = 4 * e + ((L << 2) >> e) - 4
    return np.where(e >= 16, 63, np.minimum(b, 63))


def features(A) -> np.ndarray:
    n, m, nnz = A.nrows, A.ncols, A.nnz
    out = np.zeros(NFEAT, np.float64)
    rowlen = np.diff(A.indptr).astype(np.int64)
    if nnz:
        rows = A.rows()
        cols = A.indices.astype(np.int64)
        d = cols - rows
        order = np.lexsort((rows, d))
        ds, rs = d[order], rows[order]
        start = np.ones(nnz, bool)
        start[1:] = (ds[1:] != ds[:-1]) | (rs[1:] != rs[:-1] + 1)
        rid = np.cumsum(start) - 1
        lens = np.bincount(rid)
        out[0:64] = np.bincount(_log_bin(lens), weights=lens, minlength=64)[:64] / nnz
        T = 16
        ntc = (m + T - 1) // T
        key = (rows // T) * ntc + cols // T
        uk, cnt = np.unique(key, return_counts=True)
        I, J = uk // ntc, uk % ntc
        h = np.minimum((I + 1) * T, n) - I * T
        w = np.minimum((J + 1) * T, m) - J * T
        b = np.minimum((64 * cnt) // (h * w), 63)
        out[64:128] = np.bincount(b, weights=cnt, minlength=64)[:64] / nnz
        out[138] = cnt[2 * cnt >= h * w].sum() / nnz
        ud, dc = np.unique(d, return_counts=True)
        out[134] = dc[ud == 0].sum() / nnz
        out[135] = dc[np.abs(ud) <= 32].sum() / nnz
        out[136] = dc.max() / max(n, 1)
        out[137] = ud.size / max(n + m - 1, 1)
    mean = nnz / max(n, 1)
    var = max(0.0, float((rowlen.astype(np.float64) ** 2).sum()) / max(n, 1) - mean * mean)
    out[128] = np.log1p(mean)
    out[129] = np.log1p(np.sqrt(var))
    out[130] = np.log1p(rowlen.max() if n else 0)
    out[131] = np.log(max(n, 1))
    out[132] = np.log(max(m, 1))
    out[133] = np.log(max(nnz, 1))
    out[139] = (rowlen == 0).sum() / max(n, 1)
    return out.astype(np.float32)


def unflatten(p: np.ndarray) -> dict:
    out, o = {}, 0
    for k, s in SHAPES:
        size = int(np.prod(s))
        out[k] = np.asarray(p[o:o + size], np.float64).reshape(s)
        o += size
    return out


def flatten(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[k], np.float64).ravel() for k, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (fp32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, s in SHAPES:
        if k.startswith("W"):
            lim = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def mlp_forward(p: np.ndarray, X: np.ndarray) -> np.ndarray:
    P = unflatten(p)
    X = np.asarray(X, np.float64)
    H1 = np.maximum(X @ P["W1"].T + P["b1"], 0.0)
    H2 = np.maximum(H1 @ P["W2"].T + P["b2"], 0.0)
    return H2 @ P["W3"].T + P["b3"]


def mlp_loss_grad(p: np.ndarray, X: np.ndarray, y: np.ndarray):
    """Mean softmax cross-entropy and its gradient (flat, same layout), FP64."""
    P = unflatten(p)
    X = np.asarray(X, np.float64)
    B = X.shape[0]
    Z1 = X @ P["W1"].T + P["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.maximum(Z2, 0.0)
    Z3 = H2 @ P["W3"].T + P["b3"]
    Z3s = Z3 - Z3.max(axis=1, keepdims=True)
    lse = np.log(np.exp(Z3s).sum(axis=1))
    loss = float(np.mean(lse - Z3s[np.arange(B), y]))
    S = np.exp(Z3s - lse[:, None])
    G3 = S.copy()
    G3[np.arange(B), y] -= 1.0
    G3 /= B
    g = {"W3": G3.T @ H2, "b3": G3.sum(axis=0)}
    G2 = (G3 @ P["W3"]) * (H2 > 0)
    g["W2"] = G2.T @ H1
    g["b2"] = G2.sum(axis=0)
    G1 = (G2 @ P["W2"]) * (H1 > 0)
    g["W1"] = G1.T @ X
    g["b1"] = G1.sum(axis=0)
    return loss, flatten(g)
