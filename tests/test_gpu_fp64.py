"""GPU parity of the FP64 executor (fp64 values, operands and arithmetic) against the oracle's
FP64-input products, through the C ABI.

A plan is built from the structure (fp32 values), fp64 values are then stored with
sable_update_values_f64; products must match oracle.spmv64 / spmm64 to FP64 rounding
(normwise 1e-13; the summation orders differ) and be bitwise reproducible.
"""
import numpy as np
import pytest

import oracle
from paper_2407_00829_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_00829_amd import sable  # noqa: E402

V, B, C = sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR
TOL = 1e-13


def fp64_values(A, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(A.nnz) * (1.0 + 1e-9 * rng.standard_normal(A.nnz))


def plan64(A, kinds, mode, th, seed):
    print(f"[plan] {A.nrows}x{A.ncols} nnz={A.nnz} kinds={kinds}", flush=True)
    p = sable.plan_host(A, kinds, mode, th)
    v = fp64_values(A, seed)
    sable.sable_update_values_f64(p, torch.from_numpy(v).cuda())
    return p, v


def check_spmv64(p, A, v, seed):
    x = np.random.default_rng(seed + 1).standard_normal(A.ncols)
    xd = torch.from_numpy(x).cuda()
    y = torch.full((A.nrows,), float("nan"), dtype=torch.float64, device="cuda")
    sable.sable_spmv_f64(p, xd, y)
    torch.cuda.synchronize()
    ref = oracle.spmv64(A, v, x)
    err = oracle.rel_err(y.cpu().numpy(), ref)
    print(f"  spmv64 rel_err={err:.3e}", flush=True)
    assert err <= TOL
    y2 = torch.empty_like(y)
    sable.sable_spmv_f64(p, xd, y2)
    torch.cuda.synchronize()
    assert torch.equal(y, y2), "FP64 SpMV not bitwise reproducible"
    return err


def check_spmm64(p, A, v, n, seed):
    X = np.random.default_rng(seed + 2).standard_normal((A.ncols, n))
    Xd = torch.from_numpy(X).cuda()
    Y = torch.full((A.nrows, n), float("nan"), dtype=torch.float64, device="cuda")
    sable.sable_spmm_f64(p, Xd, Y, n)
    torch.cuda.synchronize()
    err = oracle.rel_err(Y.cpu().numpy(), oracle.spmm64(A, v, X))
    print(f"  spmm64 n={n} rel_err={err:.3e}", flush=True)
    assert err <= TOL
    return err


@pytest.mark.parametrize("seed", range(4))
def test_random_small_fp64(seed):
    A = synth.gen_random_small(seed, 300 + 37 * seed, 280 + 11 * seed, 0.02, nbands=2, nblocks=3)
    th = sable.Thresholds(amin_band=64, amin_block=64)
    for kinds in ([C], [V, C], [B, C], [V, B, C], [B, V, C]):
        p, v = plan64(A, kinds, sable.SABLE_VBR_TILED, th, seed)
        check_spmv64(p, A, v, seed)
        check_spmm64(p, A, v, 5, seed)


def test_c1_every_streamed_variant_fp64():
    """C1-style mixed matrix with bands, blocks and scatter: every streamed tile size."""
    A, _ = synth.gen_c1(3, n=3000)
    th = sable.Thresholds(amin_band=256, amin_block=256)
    p, v = plan64(A, [V, B, C], sable.SABLE_VBR_TILED, th, 7)
    info = sable.sable_plan_info(p)
    assert info["nseg"] > 0 and info["nblk"] > 0 and info["csr_nnz"] > 0
    for var in (0, 1, 2, 8, 9, 10, 3):
        sable.sable_plan_set_variant(p, 0, var)
        check_spmv64(p, A, v, var)


@pytest.mark.parametrize("n", [1, 16, 130])
def test_spmm_fp64_widths(n):
    A, _ = synth.gen_c1(4, n=1536)
    th = sable.Thresholds(amin_band=256, amin_block=256)
    p, v = plan64(A, [V, B, C], sable.SABLE_VBR_TILED, th, n)
    check_spmm64(p, A, v, n, n)


def test_fem_blocks_fp64():
    """C3-like FEM blocks (6x6 node blocks, 27-point block stencil) scaled down."""
    A, _ = synth.gen_c3(0, n=6000, ystride=10, zstride=100, scatter_density=1e-4, with_x=False)
    th = sable.Thresholds(delta_band_pm=900, delta_block_pm=900, amin_block=36)
    p, v = plan64(A, [V, B, C], sable.SABLE_VBR_TILED, th, 3)
    assert sable.sable_plan_info(p)["nblk"] > 0
    check_spmv64(p, A, v, 3)
    check_spmm64(p, A, v, 32, 3)


def test_fp64_requires_values_and_refreshes():
    A, _ = synth.gen_c1(5, n=1024)
    p = sable.plan_host(A, [V, B, C], sable.SABLE_VBR_TILED, sable.Thresholds(amin_band=256, amin_block=256))
    x = torch.zeros(A.ncols, dtype=torch.float64, device="cuda")
    y = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    with pytest.raises(sable.SableError):
        sable.sable_spmv_f64(p, x, y)
    for seed in (1, 2):  # a second call replaces the values
        v = fp64_values(A, seed)
        sable.sable_update_values_f64(p, torch.from_numpy(v).cuda())
        check_spmv64(p, A, v, seed)
    # fp32 products are untouched by the fp64 copies
    x32 = synth.gen_dense_vector(0, A.ncols)
    y32 = torch.empty(A.nrows, device="cuda")
    sable.sable_spmv(p, torch.from_numpy(x32).cuda(), y32)
    torch.cuda.synchronize()
    assert oracle.rel_err(y32.cpu().numpy(), oracle.spmv(A, x32)) <= 1e-5


def test_c2_full_size_fp64_sampled():
    """PDE-like 2,097,152-row matrix: FP64 executor on sampled rows."""
    A, _ = synth.gen_c2(0)
    th = sable.Thresholds(delta_band_pm=750, delta_block_pm=500)
    p, v = plan64(A, [V, B, C], sable.SABLE_VBR_TILED, th, 11)
    x = np.random.default_rng(12).standard_normal(A.ncols)
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    sable.sable_spmv_f64(p, torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(13).choice(A.nrows, 20000, replace=False))
    sub_ptr = np.concatenate([[0], np.cumsum(np.diff(A.indptr)[rows])])
    idx = np.concatenate([np.arange(A.indptr[r], A.indptr[r + 1]) for r in rows])
    S = synth.CSR(rows.size, A.ncols, sub_ptr.astype(A.indptr.dtype), A.indices[idx], A.values[idx])
    ref = oracle.spmv64(S, v[idx], x)
    err = oracle.rel_err(y.cpu().numpy()[rows], ref)
    print(f"  sampled rel_err={err:.3e}")
    assert err <= TOL


def wide_scatter(nr, nc, seed):
    """Main diagonal plus ~0.15 uniform-random entries per row and 70,000 more: a CSR part
    with well over 2^16 entries more than 2^17 columns from their row."""
    rng = np.random.default_rng(seed)
    d = np.arange(min(nr, nc))
    ns = int(0.15 * nr) + 70000
    rows = np.concatenate([d, rng.integers(0, nr, ns)])
    cols = np.concatenate([d, rng.integers(0, nc, ns)])
    vals = rng.uniform(-1, 1, rows.size).astype(np.float32)
    return synth.from_coo(nr, nc, rows, cols, vals)


@pytest.mark.parametrize("shape", [(1_300_001, 1_300_001), (200_003, 3_000_000)])
def test_far_column_split_fp64(shape):
    """FP64 executor with the far-column split: every streamed variant matches the oracle
    with the split on and off, the two agree bit for bit, and a second value update reaches
    the far entries' fp64 copies."""
    A = wide_scatter(*shape, seed=shape[0] % 89)
    p, v = plan64(A, [V, B, C], sable.SABLE_VBR_TILED, sable.Thresholds(), 21)
    assert sable.sable_plan_info(p)["far_split"] == 1
    for var in (0, 1, 2):
        sable.sable_plan_set_variant(p, 0, var)
        ys = []
        for fs in (1, 0):
            sable.sable_plan_set_variant(p, 3, fs)
            x = np.random.default_rng(22).standard_normal(A.ncols)
            y = torch.full((A.nrows,), float("nan"), dtype=torch.float64, device="cuda")
            sable.sable_spmv_f64(p, torch.from_numpy(x).cuda(), y)
            torch.cuda.synchronize()
            err = oracle.rel_err(y.cpu().numpy(), oracle.spmv64(A, v, x))
            print(f"  variant {var} far_split {fs}: rel_err={err:.3e}", flush=True)
            assert err <= TOL
            ys.append(y)
        assert torch.equal(ys[0].view(torch.int64), ys[1].view(torch.int64)), var
    sable.sable_plan_set_variant(p, 3, 1)
    v2 = fp64_values(A, 23)
    sable.sable_update_values_f64(p, torch.from_numpy(v2).cuda())
    check_spmv64(p, A, v2, 24)


def test_c3_full_size_fp64_sampled():
    """FEM-like 500,000-row matrix, FP64 SpMM with n = 128 on sampled rows (plus the first and
    last) against the oracle's FP64-input product of those rows."""
    A, X32 = synth.gen_c3(0)
    th = sable.Thresholds(delta_band_pm=900, delta_block_pm=900, amin_block=36)
    p, v = plan64(A, [V, B, C], sable.SABLE_VBR_TILED, th, 31)
    n = X32.shape[1]
    X = np.random.default_rng(32).standard_normal((A.ncols, n))
    Y = torch.full((A.nrows, n), float("nan"), dtype=torch.float64, device="cuda")
    sable.sable_spmm_f64(p, torch.from_numpy(X).cuda(), Y, n)
    torch.cuda.synchronize()
    rows = np.concatenate([np.random.default_rng(33).choice(A.nrows, 1024, replace=False),
                           [0, A.nrows - 1]])
    sub_ptr = np.concatenate([[0], np.cumsum(np.diff(A.indptr)[rows])])
    idx = np.concatenate([np.arange(A.indptr[r], A.indptr[r + 1]) for r in rows])
    S = synth.CSR(rows.size, A.ncols, sub_ptr.astype(A.indptr.dtype), A.indices[idx], A.values[idx])
    err = oracle.rel_err(Y.cpu().numpy()[rows], oracle.spmm64(S, v[idx], X))
    print(f"  sampled rel_err={err:.3e}")
    assert err <= TOL
