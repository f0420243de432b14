"""Seeded synthetic sparse matrices with the structure the hybrid-format method targets.

This module only draws random numbers and assembles coordinate lists. It holds none of
the method's arithmetic (no extraction, no multiply), so both the GPU library's tests and
the CPU oracle's tests can take their inputs from here without sharing any logic.

Every generator uses NumPy's PCG64 (`numpy.random.default_rng(seed)`), draws in a fixed
documented order, concatenates the parts in the order listed, stable-sorts entries by
(row, column) and keeps the first occurrence of a duplicated coordinate. Values are fp32.

Structures (the paper evaluates on matrices that mix dense blocks, diagonal bands of
non-uniform length and scattered entries; Sec. 1 and Sec. 4):
  gen_c1    4096^2: bands {0,-1,+1,+37} of random length, 12 block-aligned dense blocks,
            0.05% scatter (density of n^2); values and x ~ U(-1,1).
  gen_c2    7-point stencil on a 128^3 grid with 20% of the off-diagonal chunks truncated,
            64 unaligned dense 128x128 blocks, one scattered entry per row; N(0,1).
  gen_c3    FEM-like: 6x6 dense node blocks on a periodic 27-point block stencil, two long
            bands, 0.01% scatter (density of n^2); U(-1,1). Dense X is n x ncol.
  gen_mixed Dirichlet mixture of band / block / scatter parts (planner and batch inputs).
  gen_random_small  tiny matrices for brute-force and property tests.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "CSR", "from_coo", "gen_c1", "gen_c2", "gen_c3", "gen_mixed", "gen_random_small",
    "gen_dense_vector", "gen_dense_matrix", "c4_params", "c5_params",
]


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: int64 indptr, int32 sorted unique column indices, fp32 values."""
    nrows: int
    ncols: int
    indptr: np.ndarray
    indices: np.ndarray
    values: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (COO row array)."""
        return np.repeat(np.arange(self.nrows, dtype=np.int64), np.diff(self.indptr))


def from_coo(nrows: int, ncols: int, r, c, v) -> CSR:
    """Build CSR from coordinate lists: stable sort by (row, col), keep first duplicate."""
    r = np.asarray(r, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    v = np.asarray(v, dtype=np.float32)
    if r.size:
        if r.min() < 0 or r.max() >= nrows or c.min() < 0 or c.max() >= ncols:
            raise ValueError("coordinate out of range")
    key = r * np.int64(ncols) + c
    order = np.argsort(key, kind="stable")
    key = key[order]
    keep = np.ones(key.size, dtype=bool)
    if key.size:
        keep[1:] = key[1:] != key[:-1]
    order = order[keep]
    r, c, v = r[order], c[order], v[order]
    indptr = np.zeros(nrows + 1, dtype=np.int64)
    indptr[1:] = np.bincount(r, minlength=nrows)
    indptr = np.cumsum(indptr, dtype=np.int64)
    return CSR(nrows, ncols, indptr, c.astype(np.int32), v)


def _diag_cells(n_rows: int, n_cols: int, d: int, start: int, length: int):
    """Cells start..start+length-1 along diagonal d (cell t at (t+max(0,-d), t+max(0,d)))."""
    t = np.arange(start, start + length, dtype=np.int64)
    return t + max(0, -d), t + max(0, d)


def gen_c1(seed: int, n: int = 4096, scatter_count: int | None = None):
    """4096 x 4096 mixed matrix and x (both U(-1,1)).

    Draw order: for d in (0,-1,+1,+37): L ~ U{512..4096} clipped to n-|d|, start ~
    U{0..n-|d|-L}; then 12 blocks: h, w ~ {16,32,64}, r0 = h*U{0..n/h-1}, c0 =
    w*U{0..n/w-1}; then round(0.0005 n^2) scatter rows, then columns; then one value per
    generated entry; then x.
    """
    rng = np.random.default_rng(seed)
    rs, cs = [], []
    for d in (0, -1, 1, 37):
        ncell = n - abs(d)
        L = min(int(rng.integers(512, 4097)), ncell)
        start = int(rng.integers(0, ncell - L + 1))
        r, c = _diag_cells(n, n, d, start, L)
        rs.append(r)
        cs.append(c)
    sides = np.array([16, 32, 64])
    for _ in range(12):
        h = int(sides[rng.integers(0, 3)])
        w = int(sides[rng.integers(0, 3)])
        r0 = h * int(rng.integers(0, n // h))
        c0 = w * int(rng.integers(0, n // w))
        rr, cc = np.meshgrid(np.arange(r0, r0 + h), np.arange(c0, c0 + w), indexing="ij")
        rs.append(rr.ravel())
        cs.append(cc.ravel())
    k = int(round(0.0005 * n * n)) if scatter_count is None else int(scatter_count)
    rs.append(rng.integers(0, n, k))
    cs.append(rng.integers(0, n, k))
    r = np.concatenate(rs)
    c = np.concatenate(cs)
    v = rng.uniform(-1.0, 1.0, r.size).astype(np.float32)
    x = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    return from_coo(n, n, r, c, v), x


def gen_c2(seed: int, g: int = 128, nblocks: int = 64, bs: int = 128, trunc_frac: float = 0.2):
    """PDE-like: 7-point stencil on a g^3 grid (row i = x + g*y + g*g*z) with boundary
    exclusion. Each of the 6 off-diagonals is cut into g chunks of g*g rows; a seeded
    trunc_frac of the 6*g chunks keep only a prefix of length U{0..g*g-1}. Plus nblocks
    dense bs x bs blocks at unaligned r0, c0 ~ U{0..n-bs} and one scattered entry per row
    at a uniform column. Values and x ~ N(0,1).

    Draw order: chunk choice (permutation of 6*g), prefix lengths, block positions
    (r0 then c0 per block), scatter columns, values, x.
    """
    rng = np.random.default_rng(seed)
    n = g * g * g
    chunk = g * g
    i = np.arange(n, dtype=np.int64)
    xx = i % g
    yy = (i // g) % g
    zz = i // chunk
    nchunks = 6 * g
    ntr = int(round(trunc_frac * nchunks))
    chosen = rng.permutation(nchunks)[:ntr]
    lens = rng.integers(0, chunk, ntr)
    keep_len = np.full(nchunks, chunk, dtype=np.int64)
    keep_len[chosen] = lens
    rs, cs = [i], [i]
    offs = [(-1, xx > 0), (1, xx < g - 1), (-g, yy > 0), (g, yy < g - 1),
            (-chunk, zz > 0), (chunk, zz < g - 1)]
    for q, (o, ok) in enumerate(offs):
        within = i - (i // chunk) * chunk
        klen = keep_len[q * g + (i // chunk)]
        m = ok & (within < klen)
        rs.append(i[m])
        cs.append(i[m] + o)
    pos = rng.integers(0, n - bs + 1, size=(nblocks, 2))
    bb = np.arange(bs, dtype=np.int64)
    for b in range(nblocks):
        rr, cc = np.meshgrid(pos[b, 0] + bb, pos[b, 1] + bb, indexing="ij")
        rs.append(rr.ravel())
        cs.append(cc.ravel())
    rs.append(i.copy())
    cs.append(rng.integers(0, n, n))
    r = np.concatenate(rs)
    c = np.concatenate(cs)
    v = rng.standard_normal(r.size, dtype=np.float32)
    x = rng.standard_normal(n, dtype=np.float32)
    return from_coo(n, n, r, c, v), x


def gen_c3(seed: int, n: int = 500_000, bsz: int = 6, ystride: int = 44, zstride: int = 1936,
           scatter_density: float = 1e-4, ncol_x: int = 128, with_x: bool = True):
    """FEM-like: N = ceil(n/bsz) node blocks; block row k couples to block columns
    (k + dx + ystride*dy + zstride*dz) mod N for dx, dy, dz in {-1,0,1}; every bsz x bsz
    block is dense (clipped at the last rows/columns). Two bands: L ~ U{0.3n..n},
    d ~ U{-(n-L)..n-L}, start ~ U{0..n-|d|-L}. Scatter: round(scatter_density*n^2)
    uniform pairs. Values ~ U(-1,1); X is n x ncol_x ~ U(-1,1).
    """
    rng = np.random.default_rng(seed)
    N = -(-n // bsz)
    k = np.arange(N, dtype=np.int64)
    rs, cs = [], []
    loc_r, loc_c = np.meshgrid(np.arange(bsz), np.arange(bsz), indexing="ij")
    loc_r = loc_r.ravel()
    loc_c = loc_c.ravel()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                kc = (k + dx + ystride * dy + zstride * dz) % N
                rr = (k[:, None] * bsz + loc_r[None, :]).ravel()
                cc = (kc[:, None] * bsz + loc_c[None, :]).ravel()
                m = (rr < n) & (cc < n)
                rs.append(rr[m])
                cs.append(cc[m])
    for _ in range(2):
        L = int(rng.integers(int(0.3 * n), n + 1))
        d = int(rng.integers(-(n - L), n - L + 1))
        ncell = n - abs(d)
        start = int(rng.integers(0, ncell - L + 1))
        r, c = _diag_cells(n, n, d, start, L)
        rs.append(r)
        cs.append(c)
    ks = int(round(scatter_density * n * n))
    rs.append(rng.integers(0, n, ks))
    cs.append(rng.integers(0, n, ks))
    r = np.concatenate(rs)
    c = np.concatenate(cs)
    v = rng.uniform(-1.0, 1.0, r.size).astype(np.float32)
    A = from_coo(n, n, r, c, v)
    X = rng.uniform(-1.0, 1.0, (n, ncol_x)).astype(np.float32) if with_x else None
    return A, X


def _band_part(rng, n, nnz_target, maxd_frac=0.25):
    rs, cs = [], []
    got = 0
    while got < nnz_target:
        maxd = max(1, int(maxd_frac * n))
        d = int(rng.integers(-maxd, maxd + 1))
        ncell = n - abs(d)
        L = int(rng.integers(max(1, int(0.1 * ncell)), ncell + 1))
        start = int(rng.integers(0, ncell - L + 1))
        w = int(rng.integers(1, 4))  # ribbon of w adjacent diagonals
        for q in range(w):
            dd = d + q
            if abs(dd) >= n:
                continue
            nc = n - abs(dd)
            s = min(start, nc - 1)
            LL = min(L, nc - s)
            r, c = _diag_cells(n, n, dd, s, LL)
            rs.append(r)
            cs.append(c)
            got += LL
    return rs, cs


def _block_part(rng, n, nnz_target, sides=(6, 16, 32, 64, 128)):
    rs, cs = [], []
    got = 0
    while got < nnz_target:
        h = int(sides[rng.integers(0, len(sides))])
        w = int(sides[rng.integers(0, len(sides))])
        h = min(h, n)
        w = min(w, n)
        r0 = int(rng.integers(0, n - h + 1))
        c0 = int(rng.integers(0, n - w + 1))
        rr, cc = np.meshgrid(np.arange(r0, r0 + h), np.arange(c0, c0 + w), indexing="ij")
        rs.append(rr.ravel())
        cs.append(cc.ravel())
        got += h * w
    return rs, cs


def c4_params(seed: int):
    """Size and mix for one planner-training matrix: n = round(exp U[ln 1e4, ln 1e6]),
    mean row length ~ U[4,64], proportions ~ Dirichlet(1,1,1) over band/block/scatter."""
    rng = np.random.default_rng(seed)
    n = int(round(np.exp(rng.uniform(np.log(1e4), np.log(1e6)))))
    rowlen = float(rng.uniform(4, 64))
    pi = rng.dirichlet([1.0, 1.0, 1.0])
    return n, rowlen, pi


def c5_params(seed: int, count: int = 256):
    """Sizes, generator kinds and operations for a batch of matrices: n ~ logU[1e3, 2e5],
    kind ~ U{0..3} (C1-, C2-, C3-, mixed-style), op ~ Bernoulli(0.5) (0 SpMV, 1 SpMM n=16)."""
    rng = np.random.default_rng(seed)
    ns = np.round(np.exp(rng.uniform(np.log(1e3), np.log(2e5), count))).astype(np.int64)
    kinds = rng.integers(0, 4, count)
    ops = rng.integers(0, 2, count)
    seeds = rng.integers(0, 2**31 - 1, count)
    return ns, kinds, ops, seeds


def gen_mixed(seed: int, n: int | None = None, rowlen: float | None = None, pi=None,
              max_nnz: int | None = None):
    """Dirichlet mixture of band, block and scatter parts (values U(-1,1))."""
    rng = np.random.default_rng(seed)
    if n is None or rowlen is None or pi is None:
        n0, r0, p0 = c4_params(seed)
        n = n0 if n is None else n
        rowlen = r0 if rowlen is None else rowlen
        pi = p0 if pi is None else pi
    total = int(rowlen * n)
    if max_nnz is not None:
        total = min(total, max_nnz)
    rs, cs = [], []
    b_r, b_c = _band_part(rng, n, int(pi[0] * total))
    k_r, k_c = _block_part(rng, n, int(pi[1] * total))
    rs += b_r + k_r
    cs += b_c + k_c
    ks = int(pi[2] * total)
    rs.append(rng.integers(0, n, ks))
    cs.append(rng.integers(0, n, ks))
    r = np.concatenate(rs) if rs else np.zeros(0, np.int64)
    c = np.concatenate(cs) if cs else np.zeros(0, np.int64)
    v = rng.uniform(-1.0, 1.0, r.size).astype(np.float32)
    x = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    return from_coo(n, n, r, c, v), x


def gen_grid_stencil(seed: int, g: int, nblocks: int = 4, bs: int = 32):
    """Small C2-style matrix (grid g^3) for batches and quick tests."""
    return gen_c2(seed, g=g, nblocks=nblocks, bs=min(bs, g * g * g), trunc_frac=0.2)


def gen_random_small(seed: int, nrows: int, ncols: int, density: float,
                     nbands: int = 0, nblocks: int = 0, block_max: int = 8):
    """Tiny matrix: uniform scatter of the given density plus optional full bands and dense
    blocks (sizes 1..block_max). Values ~ U(-1,1); some values are exactly 0.0 to exercise
    explicitly stored zeros."""
    rng = np.random.default_rng(seed)
    k = int(round(density * nrows * ncols))
    rs = [rng.integers(0, nrows, k)]
    cs = [rng.integers(0, ncols, k)]
    for _ in range(nbands):
        d = int(rng.integers(-(nrows - 1), ncols))
        r = np.arange(max(0, -d), min(nrows, ncols - d), dtype=np.int64)
        if r.size:
            a = int(rng.integers(0, r.size))
            b = int(rng.integers(a, r.size + 1))
            r = r[a:b]
        rs.append(r)
        cs.append(r + d)
    for _ in range(nblocks):
        h = int(rng.integers(1, min(block_max, nrows) + 1))
        w = int(rng.integers(1, min(block_max, ncols) + 1))
        r0 = int(rng.integers(0, nrows - h + 1))
        c0 = int(rng.integers(0, ncols - w + 1))
        rr, cc = np.meshgrid(np.arange(r0, r0 + h), np.arange(c0, c0 + w), indexing="ij")
        rs.append(rr.ravel())
        cs.append(cc.ravel())
    r = np.concatenate(rs)
    c = np.concatenate(cs)
    v = rng.uniform(-1.0, 1.0, r.size).astype(np.float32)
    if v.size:
        v[rng.random(v.size) < 0.02] = 0.0
    return from_coo(nrows, ncols, r, c, v)


def gen_c5_matrix(seed: int):
    """One matrix of a serving batch: n ~ logU[1e3, 2e5]; generator kind uniform over
    {C1-style, C2-style (grid g = round(n^(1/3))), C3-style, mixed}; op ~ Bernoulli(0.5)
    (0 = SpMV, 1 = SpMM with 16 right-hand sides). Returns (A, kind, op)."""
    rng = np.random.default_rng(7_000_003 + seed)
    n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
    kind = int(rng.integers(0, 4))
    op = int(rng.integers(0, 2))
    sub = int(rng.integers(0, 2 ** 31 - 1))
    if kind == 0:
        m = max(n, 256)  # 0.05% of m^2 scattered entries, at most 4 per row
        A, _ = gen_c1(sub, n=m, scatter_count=min(int(round(0.0005 * m * m)), 4 * m))
    elif kind == 1:
        g = max(8, int(round(n ** (1.0 / 3.0))))
        bs = min(128, g * g)
        A, _ = gen_c2(sub, g=g, nblocks=max(1, g * g * g // 32768), bs=bs)
    elif kind == 2:
        N = -(-n // 6)
        ys = max(2, int(round(N ** (1.0 / 3.0))))
        A, _ = gen_c3(sub, n=n, ystride=ys, zstride=ys * ys, scatter_density=min(1e-4, 20.0 / n),
                      with_x=False)
    else:
        A, _ = gen_mixed(sub, n=n, rowlen=float(rng.uniform(4, 32)), pi=rng.dirichlet([1, 1, 1]))
    return A, kind, op


def gen_dense_vector(seed: int, n: int, normal: bool = False) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if normal:
        return rng.standard_normal(n, dtype=np.float32)
    return rng.uniform(-1.0, 1.0, n).astype(np.float32)


def gen_dense_matrix(seed: int, rows: int, cols: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (rows, cols)).astype(np.float32)
