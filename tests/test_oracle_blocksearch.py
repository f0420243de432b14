"""Pins of the oracle's block search (Alg. 2) and partition product against independent
formulations (no GPU).

* The window rule of Sec. 4.1, restated declaratively over a summed-area table: for an outer
  span of s slices and each right end i1 of the inner range, the left end is the smallest
  index j >= the previous right end's left end such that the window [j, i1] is either too
  small (s * width < A_min) or delta-dense; the window is a candidate when it is large
  enough. The best candidate has the highest score area * (density - 0.5)^1.5, compared as
  the exact rational (2n - a)^3 / a, ties to the smallest (o0, o1, i1). This is computed
  here by enumeration with Python integers and must equal the oracle's FindBlock exactly.
* The objective the heuristic approximates: over EVERY delta-dense rectangle of the region
  with outer span >= ceil(sqrt(A_min)) and area >= A_min, the best score is at least the
  found block's; a single fully dense planted block in an empty region is the optimum, every
  pass's window contains it and the full Partition (with Trim) returns exactly it.
* The partition product (formats of the oracle's plan, fill included) equals the COO product
  up to FP64 rounding, and the numpy product over the exported arrays.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2407_00829_amd import synth


def _dense(A):
    D = np.zeros((A.nrows, A.ncols), np.int64)
    D[A.rows(), A.indices.astype(np.int64)] = 1
    return D


def _score(n, a):
    return Fraction((2 * n - a) ** 3, a)  # score^2 * 8, order-preserving for density >= 0.5


def _isqrt_ceil(a):
    s = 0
    while s * s < a:
        s += 1
    return s


def window_rule(D, region, by_rows, th):
    """Sec. 4.1's window rule over a summed-area table (region-relative result)."""
    r0, r1, c0, c1 = region
    M = D[r0:r1, c0:c1]
    if not by_rows:
        M = M.T
    Lout, Lin = M.shape
    S = np.zeros((Lout + 1, Lin + 1), np.int64)  # S[a, b] = entries in outer < a, inner < b
    S[1:, 1:] = np.cumsum(np.cumsum(M, axis=0), axis=1)
    p, amin = th.delta_block_pm, th.amin_block
    smin = _isqrt_ceil(amin)

    def cnt(o0, o1, i0, i1):
        return int(S[o1 + 1, i1 + 1] - S[o0, i1 + 1] - S[o1 + 1, i0] + S[o0, i0])

    best = None  # (score, o0, o1, i0, i1, n, a)
    for o0 in range(Lout):
        for o1 in range(o0 + smin - 1, Lout):
            s = o1 - o0 + 1
            left = 0
            for i1 in range(Lin):
                j = left
                while j <= i1:
                    a = s * (i1 - j + 1)
                    if a < amin or 1000 * cnt(o0, o1, j, i1) >= p * a:
                        break
                    j += 1
                left = j
                if j > i1 or s * (i1 - j + 1) < amin:
                    continue
                a = s * (i1 - j + 1)
                n = cnt(o0, o1, j, i1)
                key = _score(n, a)
                if best is None or key > best[0]:  # loop order is (o0, o1, i1) ascending
                    best = (key, o0, o1, j, i1, n, a)
    if best is None:
        return None
    _, o0, o1, i0, i1, n, a = best
    return (n, a, o0, o1, i0, i1)


def global_best(D, region, th):
    """Best score over every delta-dense rectangle with both passes' constraints (outer span
    >= s_min for the rows or for the columns, area >= A_min)."""
    r0, r1, c0, c1 = region
    M = D[r0:r1, c0:c1]
    h, w = M.shape
    S = np.zeros((h + 1, w + 1), np.int64)
    S[1:, 1:] = np.cumsum(np.cumsum(M, axis=0), axis=1)
    p, amin = th.delta_block_pm, th.amin_block
    smin = _isqrt_ceil(amin)
    best = None
    for a0 in range(h):
        for a1 in range(a0, h):
            for b0 in range(w):
                for b1 in range(b0, w):
                    hh, ww = a1 - a0 + 1, b1 - b0 + 1
                    if max(hh, ww) < smin or hh * ww < amin:
                        continue
                    n = int(S[a1 + 1, b1 + 1] - S[a0, b1 + 1] - S[a1 + 1, b0] + S[a0, b0])
                    if 1000 * n < p * hh * ww:
                        continue
                    k = _score(n, hh * ww)
                    if best is None or k > best:
                        best = k
    return best


def _random_case(seed):
    rng = np.random.default_rng(seed)
    nr, nc = int(rng.integers(6, 22)), int(rng.integers(6, 22))
    dens = float(rng.choice([0.15, 0.35, 0.55, 0.75]))
    A = synth.gen_random_small(seed, nr, nc, dens, nbands=int(rng.integers(0, 2)),
                               nblocks=int(rng.integers(0, 3)), block_max=10)
    r0 = int(rng.integers(0, nr // 3 + 1))
    c0 = int(rng.integers(0, nc // 3 + 1))
    r1 = int(rng.integers(max(r0 + 1, 2 * nr // 3), nr + 1))
    c1 = int(rng.integers(max(c0 + 1, 2 * nc // 3), nc + 1))
    th = oracle.Thresholds(delta_block_pm=int(rng.choice([500, 600, 750, 900])),
                           amin_block=int(rng.choice([4, 6, 9, 16, 20])))
    return A, (r0, r1, c0, c1), th


@pytest.mark.parametrize("seed", range(40))
def test_find_block_equals_window_rule(seed):
    A, reg, th = _random_case(seed)
    D = _dense(A)
    for by_rows in (True, False):
        got = oracle.find_block(A, reg, by_rows, th)
        want = window_rule(D, reg, by_rows, th)
        if want is None:
            assert got[0] == -1, (got, reg, by_rows)
        else:
            assert got == want, (got, want, reg, by_rows)


@pytest.mark.parametrize("seed", range(12))
def test_find_block_within_global_optimum(seed):
    A, reg, th = _random_case(1000 + seed)
    D = _dense(A)
    opt = global_best(D, reg, th)
    for by_rows in (True, False):
        got = oracle.find_block(A, reg, by_rows, th)
        if got[0] < 0:
            continue
        assert opt is not None and _score(got[0], got[1]) <= opt
        # the found window really is what it claims: count, area, density, span
        n, a, o0, o1, i0, i1 = got
        r0, r1, c0, c1 = reg
        rect = (r0 + o0, r0 + o1 + 1, c0 + i0, c0 + i1 + 1) if by_rows else \
               (r0 + i0, r0 + i1 + 1, c0 + o0, c0 + o1 + 1)
        sub = D[rect[0]:rect[1], rect[2]:rect[3]]
        assert sub.sum() == n and sub.size == a and 1000 * n >= th.delta_block_pm * a
        assert o1 - o0 + 1 >= _isqrt_ceil(th.amin_block) and a >= th.amin_block


@pytest.mark.parametrize("h,w,r,c", [(5, 7, 3, 2), (9, 4, 0, 10), (6, 6, 8, 8), (4, 12, 1, 1)])
def test_planted_dense_block_is_the_global_optimum(h, w, r, c):
    """One fully dense h x w block in an empty 20 x 20 matrix. Density-1 rectangles score by
    area, so the global optimum is the planted block. The window scan may stop at a window
    that also holds empty slices next to it (its left end only moves while the window is
    sparse), so each pass returns a window containing the block, and the full Partition
    (Alg. 1: FindBlock, then Trim) returns exactly the block."""
    rr, cc = np.meshgrid(np.arange(r, r + h), np.arange(c, c + w), indexing="ij")
    A = synth.from_coo(20, 20, rr.ravel(), cc.ravel(), np.ones(h * w))
    th = oracle.Thresholds(delta_block_pm=500, amin_block=9)
    reg = (0, 20, 0, 20)
    assert global_best(_dense(A), reg, th) == _score(h * w, h * w)
    for by_rows in (True, False):
        n, a, o0, o1, i0, i1 = oracle.find_block(A, reg, by_rows, th)
        (ro0, ro1), (ri0, ri1) = ((r, r + h - 1), (c, c + w - 1)) if by_rows else \
            ((c, c + w - 1), (r, r + h - 1))
        assert n == h * w and o0 <= ro0 and o1 >= ro1 and i0 <= ri0 and i1 >= ri1
        assert (n, a, o0, o1, i0, i1) == window_rule(_dense(A), reg, by_rows, th)
    P = oracle.plan(A, [oracle.VBR, oracle.CSR], oracle.MODE_PAPER,
                    oracle.Thresholds(amin_block=9, coverage_pm=0))
    assert P["blk"].tolist() == [[r, r + h, c, c + w]]


@pytest.mark.parametrize("kinds", [[3], [1, 3], [2, 3], [1, 2, 3], [2, 1, 3]])
@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_TILED])
def test_partition_product_equals_coo_product(kinds, mode):
    A = synth.gen_random_small(11, 150, 130, 0.04, nbands=3, nblocks=4, block_max=30)
    x = synth.gen_dense_vector(5, A.ncols)
    th = oracle.Thresholds(lseg=8, amin_band=16, amin_block=36)
    y = oracle.partition_spmv(A, kinds, mode, th, x)
    ref = oracle.spmv(A, x)
    assert oracle.rel_err(y, ref) <= 1e-14
    P = oracle.plan(A, kinds, mode, th)
    assert oracle.rel_err(oracle.partition_spmv_from_export(P, x), y) <= 1e-14
    if 2 in kinds and P["blk"].shape[0]:
        assert P["vbr_val"].size > 0  # the plan really has blocks, so fill is exercised


# ---- the sparse window scan (empty inner indices crossed in O(1) per run) -------------------

def _wide_sparse_case(seed):
    """Wide or tall sparse matrices with long runs of empty columns and rows, a few dense
    clusters (some narrower than A_min allows, so windows must take in empty columns), and
    thresholds from delta = 0.5 to 1."""
    rng = np.random.default_rng(seed)
    nr, nc = int(rng.integers(8, 70)), int(rng.integers(8, 400))
    if rng.random() < 0.5:
        nr, nc = nc, nr
    rows, cols = [], []
    nsc = int(rng.integers(0, max(1, nr * nc // 40)))
    rows.append(rng.integers(0, nr, nsc))
    cols.append(rng.integers(0, nc, nsc))
    for _ in range(int(rng.integers(0, 4))):
        h, w = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        r, c = int(rng.integers(0, nr - h + 1)), int(rng.integers(0, nc - w + 1))
        rr, cc = np.meshgrid(np.arange(r, r + h), np.arange(c, c + w), indexing="ij")
        keep = rng.random(rr.size) < float(rng.choice([0.6, 0.9, 1.0]))
        rows.append(rr.ravel()[keep])
        cols.append(cc.ravel()[keep])
    r, c = np.concatenate(rows), np.concatenate(cols)
    A = synth.from_coo(nr, nc, r, c, np.ones(r.size, np.float32))
    reg = (int(rng.integers(0, nr // 4 + 1)), nr, int(rng.integers(0, nc // 4 + 1)), nc)
    th = oracle.Thresholds(delta_block_pm=int(rng.choice([500, 501, 667, 750, 900, 1000])),
                           amin_block=int(rng.choice([1, 2, 4, 9, 16, 30, 64])))
    return A, reg, th


@pytest.mark.parametrize("seed", range(60))
def test_sparse_scan_equals_dense_scan(seed):
    A, reg, th = _wide_sparse_case(seed)
    for by_rows in (True, False):
        dense = oracle.find_block(A, reg, by_rows, th)
        assert oracle.find_block(A, reg, by_rows, th, sparse=True) == dense, (reg, by_rows)


@pytest.mark.parametrize("seed", range(40))
def test_sparse_scan_equals_window_rule(seed):
    A, reg, th = _random_case(seed)
    D = _dense(A)
    for by_rows in (True, False):
        got = oracle.find_block(A, reg, by_rows, th, sparse=True)
        want = window_rule(D, reg, by_rows, th)
        if want is None:
            assert got[0] == -1, got
        else:
            assert got == want, (got, want)


@pytest.mark.parametrize("h,w,r,c", [(5, 7, 3, 2), (9, 4, 0, 10), (6, 6, 8, 8), (4, 12, 1, 1)])
def test_sparse_scan_planted_block(h, w, r, c):
    """The closed-form case: a fully dense block in an empty matrix, found by the sparse
    scan exactly as by the dense one, and returned by the full Partition."""
    rr, cc = np.meshgrid(np.arange(r, r + h), np.arange(c, c + w), indexing="ij")
    A = synth.from_coo(20, 20, rr.ravel(), cc.ravel(), np.ones(h * w))
    th = oracle.Thresholds(delta_block_pm=500, amin_block=9)
    for by_rows in (True, False):
        got = oracle.find_block(A, (0, 20, 0, 20), by_rows, th, sparse=True)
        assert got == oracle.find_block(A, (0, 20, 0, 20), by_rows, th)
        assert got[0] == h * w


@pytest.mark.parametrize("by_rows", [True, False])
def test_sparse_scan_cluster_at_the_inner_edge(by_rows):
    """A 3 x 3 dense cluster touching the first inner index of the region, A_min = 16 and
    delta = 0.5: with a span of 4 slices the window first becomes large enough (4 x 4) at
    the empty inner index just past the cluster, where it is also dense (9 / 16), and no
    later window of that span qualifies. The sparse scan must test that candidate in the
    middle of an empty run."""
    r, c = (10, 0) if by_rows else (0, 10)
    rr, cc = np.meshgrid(np.arange(r, r + 3), np.arange(c, c + 3), indexing="ij")
    A = synth.from_coo(30, 30, rr.ravel(), cc.ravel(), np.ones(9))
    th = oracle.Thresholds(delta_block_pm=500, amin_block=16)
    dense = oracle.find_block(A, (0, 30, 0, 30), by_rows, th)
    n, a, o0, o1, i0, i1 = dense
    assert (n, a, i0, i1) == (9, 16, 0, 3)  # the window ends on the empty index 3
    assert oracle.find_block(A, (0, 30, 0, 30), by_rows, th, sparse=True) == dense


@pytest.mark.parametrize("chunk", range(8))
def test_sparse_scan_equals_dense_scan_many(chunk):
    """Many small random cases per chunk (both passes): every branch of the sparse scan,
    including the first candidate after a non-empty column leaves the window at the left
    while the right end crosses empty columns."""
    for seed in range(10_000 + 150 * chunk, 10_000 + 150 * (chunk + 1)):
        A, reg, th = _wide_sparse_case(seed)
        for by_rows in (True, False):
            dense = oracle.find_block(A, reg, by_rows, th)
            assert oracle.find_block(A, reg, by_rows, th, sparse=True) == dense, (seed, by_rows)


def _window_rule_counts(H, s, th):
    """Sec. 4.1's window rule over one span's inner counts (Python integers)."""
    p, amin = th.delta_block_pm, th.amin_block
    pre = np.concatenate([[0], np.cumsum(H)]).astype(object)
    best, left = None, 0
    for i1 in range(len(H)):
        j = left
        while j <= i1:
            a = s * (i1 - j + 1)
            if a < amin or 1000 * (pre[i1 + 1] - pre[j]) >= p * a:
                break
            j += 1
        left = j
        if j > i1 or s * (i1 - j + 1) < amin:
            continue
        n, a = int(pre[i1 + 1] - pre[j]), s * (i1 - j + 1)
        if best is None or _score(n, a) > _score(best[0], best[1]):
            best = (n, a, j, i1)
    return best


def test_window_scan_hand_case_after_left_removal():
    """Counts 0 1 0 2 2 2 2 2 0 over a span of 2 slices, A_min = 12, delta = 0.75: the best
    window [3, 8] (10 entries, area 12) is found at the last, empty, index, right after the
    non-empty index 1 left the window; the first candidate after a left removal must be
    tested."""
    th = oracle.Thresholds(delta_block_pm=750, amin_block=12)
    H = [0, 1, 0, 2, 2, 2, 2, 2, 0]
    assert _window_rule_counts(H, 2, th) == (10, 12, 3, 8)
    assert oracle.best_window(H, 2, th) == (10, 12, 3, 8)
    assert oracle.best_window(H, 2, th, sparse=True) == (10, 12, 3, 8)


@pytest.mark.parametrize("chunk", range(6))
def test_window_scan_sparse_equals_rule_random(chunk):
    """Random span counts (mostly empty), every threshold pair: the dense and the sparse scans
    both equal the declarative rule."""
    rng = np.random.default_rng(500 + chunk)
    for _ in range(2000):
        L, s = int(rng.integers(1, 15)), int(rng.integers(1, 7))
        H = np.where(rng.random(L) < 0.6, rng.integers(0, s + 1, L), 0)
        th = oracle.Thresholds(delta_block_pm=int(rng.choice([500, 501, 550, 600, 667, 750, 900, 1000])),
                               amin_block=int(rng.choice([1, 2, 3, 4, 6, 8, 9, 12, 16, 20])))
        want = _window_rule_counts(H.tolist(), s, th)
        want = want if want is not None else (-1,)
        for sparse in (False, True):
            got = oracle.best_window(H, s, th, sparse=sparse)
            assert got[:len(want)] == want, (H.tolist(), s, th, sparse, got, want)
