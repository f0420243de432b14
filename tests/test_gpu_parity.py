"""GPU parity: libsable (through its C ABI) against the CPU oracle.

* the partition export is bit-exact: every VDIA / VBR / CSR array, the owner/slot map;
* SpMV results within normwise relative error 1e-5 of the FP64 oracle, SpMM with split-bf16
  blocks within 1e-4, every result reports its error;
* results are bitwise reproducible run to run.
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

V, B, C = oracle.VDIA, oracle.VBR, oracle.CSR
KIND = {V: sable.SABLE_X_VDIA, B: sable.SABLE_X_VBR, C: sable.SABLE_X_CSR}
EXPORT_KEYS = ("vdia_val", "idiag", "seg_row_start", "seg_nrows", "seg_ndiags", "seg_val_ptr",
               "seg_idiag_ptr", "blk", "blk_val_ptr", "vbr_val", "csr_ptr", "csr_col", "csr_val",
               "owner", "slot")


def to_sable_th(th: oracle.Thresholds) -> sable.Thresholds:
    return sable.Thresholds(th.delta_band_pm, th.delta_block_pm, th.amin_band, th.amin_block,
                            th.lseg, th.wmax, th.dmax, th.coverage_pm, th.tile_set_mask)


def gpu_plan(A, kinds, mode, th):
    print(f"[plan] {A.nrows}x{A.ncols} nnz={A.nnz} kinds={kinds} mode={mode}", flush=True)
    return sable.plan_host(A, [KIND[k] for k in kinds], mode, to_sable_th(th))


def assert_same_partition(got, ref):
    for k in EXPORT_KEYS:
        a, b = np.asarray(got[k]), np.asarray(ref[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        if a.dtype == np.float32:
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), k
        else:
            assert np.array_equal(a, b), k
    if ref["vbr_mode"]:
        assert got["vbr_mode"] == ref["vbr_mode"]
        assert got["vbr_tile"] == ref["vbr_tile"]


def run_spmv(p, A, x):
    xd = torch.from_numpy(x).cuda()
    y = torch.full((A.nrows,), float("nan"), device="cuda")
    sable.sable_spmv(p, xd, y)
    torch.cuda.synchronize()
    return y


def check_spmv(p, A, x, tol=1e-5):
    y = run_spmv(p, A, x)
    ref = oracle.spmv(A, x)
    err = oracle.rel_err(y.cpu().numpy(), ref)
    # the GPU FP64 error-norm reduction reports the same number
    gerr = sable.sable_error_norm_f64(y, torch.from_numpy(ref).cuda())
    print(f"  spmv rel_err={err:.3e} (gpu norm {gerr:.3e})", flush=True)
    assert err <= tol
    assert abs(gerr - err) <= 1e-9 + 1e-6 * err
    y2 = run_spmv(p, A, x)
    assert torch.equal(y, y2), "SpMV not bitwise reproducible"
    return err


def check_spmm(p, A, n, seed=0, tol=1e-4):
    X = synth.gen_dense_matrix(seed, A.ncols, n)
    Xd = torch.from_numpy(X).cuda()
    Y = torch.full((A.nrows, n), float("nan"), device="cuda")
    sable.sable_spmm(p, Xd, Y, n)
    torch.cuda.synchronize()
    ref = oracle.spmm(A, X)
    err = oracle.rel_err(Y.cpu().numpy(), ref)
    print(f"  spmm n={n} rel_err={err:.3e}", flush=True)
    assert err <= tol
    Y2 = torch.empty_like(Y)
    sable.sable_spmm(p, Xd, Y2, n)
    torch.cuda.synchronize()
    assert torch.equal(Y, Y2), "SpMM not bitwise reproducible"
    return err


# ---- worked example ---------------------------------------------------------------------

def test_fig_vdia_on_gpu():
    D = np.zeros((10, 10), np.float32)
    D[1, 0:3] = [4, 7, 2]; D[2, 1:4] = [1, 5, 3]; D[3, 2:5] = [2, 8, 1]; D[4, 3:6] = [3, 6, 4]
    D[6, 0:4] = [3, 2, 5, 1]; D[7, 1:5] = [4, 3, 7, 2]; D[8, 2:6] = [1, 6, 2, 8]
    r, c = np.nonzero(D)
    A = synth.from_coo(10, 10, r, c, D[r, c])
    th = oracle.Thresholds(lseg=3, amin_band=12)
    p = gpu_plan(A, [V, C], 0, th)
    got = sable.sable_plan_export(p)
    assert got["vdia_val"].tolist() == [4, 1, 2, 3, 7, 5, 8, 6, 2, 3, 1, 4, 3, 4, 1, 2, 3, 6, 5, 7, 2, 1, 2, 8]
    assert got["idiag"].tolist() == [-1, 0, 1, -6, -5, -4, -3]
    assert_same_partition(got, oracle.plan(A, [V, C], 0, th))
    check_spmv(p, A, np.arange(10, dtype=np.float32))


# ---- random small matrices: every plan shape, both block-search modes ---------------------

PLANS = [[C], [V, C], [B, C], [V, B, C], [B, V, C]]


@pytest.mark.parametrize("seed", range(8))
def test_random_small_bit_exact(seed):
    rng = np.random.default_rng(100 + seed)
    nr, nc = int(rng.integers(40, 300)), int(rng.integers(40, 300))
    A = synth.gen_random_small(seed, nr, nc, 0.03, nbands=4, nblocks=4, block_max=40)
    th = oracle.Thresholds(lseg=8, amin_band=32, amin_block=64, coverage_pm=40 * (seed % 3),
                           delta_band_pm=[500, 700, 900][seed % 3],
                           delta_block_pm=[500, 700, 900][(seed + 1) % 3])
    x = synth.gen_dense_vector(seed, A.ncols)
    for kinds in PLANS:
        for mode in (oracle.MODE_PAPER, oracle.MODE_TILED):
            if B not in kinds and mode == oracle.MODE_TILED:
                continue
            p = gpu_plan(A, kinds, mode, th)
            assert_same_partition(sable.sable_plan_export(p), oracle.plan(A, kinds, mode, th))
            check_spmv(p, A, x)
            check_spmm(p, A, 5 + seed)


@pytest.mark.parametrize("seed", range(3))
def test_c1_small_paper_mode_bit_exact(seed):
    """C1-style structure at n = 1024 (bands, 12 block-aligned blocks, 0.05% scatter)."""
    A, x = synth.gen_c1(seed, n=1024)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    kinds = [V, B, C]
    p = gpu_plan(A, kinds, oracle.MODE_PAPER, th)
    assert_same_partition(sable.sable_plan_export(p), oracle.plan(A, kinds, oracle.MODE_PAPER, th))
    check_spmv(p, A, x)
    check_spmm(p, A, 16)


def test_c1_full_tiled_bit_exact():
    A, x = synth.gen_c1(0)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    for kinds in ([V, B, C], [B, V, C]):
        p = gpu_plan(A, kinds, oracle.MODE_TILED, th)
        assert_same_partition(sable.sable_plan_export(p), oracle.plan(A, kinds, oracle.MODE_TILED, th))
        check_spmv(p, A, x)


# ---- edge cases ------------------------------------------------------------------------------

def test_empty_and_degenerate():
    th = oracle.Thresholds(lseg=2, amin_band=2, amin_block=4)
    for (nr, nc, dens) in [(1, 1, 1.0), (1, 50, 0.5), (50, 1, 0.5), (300, 7, 0.0), (257, 513, 0.01)]:
        A = synth.gen_random_small(nr * 7 + nc, nr, nc, dens)
        x = synth.gen_dense_vector(1, nc)
        for kinds in PLANS:
            p = gpu_plan(A, kinds, oracle.MODE_PAPER, th)
            assert_same_partition(sable.sable_plan_export(p), oracle.plan(A, kinds, 1, th))
            y = run_spmv(p, A, x)
            assert np.allclose(y.cpu().numpy(), oracle.spmv(A, x), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("shape", [(0, 5), (5, 0), (0, 0), (9, 9)])
def test_no_rows_columns_or_entries(shape):
    """Empty shapes: the partition export matches the oracle's (all formats empty), every
    product entry point (hybrid, plain CSR, SpMM, FP64, autotuned) writes y = 0 or nothing,
    and the planner features are finite."""
    nr, nc = shape
    A = synth.from_coo(nr, nc, [], [], [])
    th = oracle.Thresholds(lseg=2, amin_band=2, amin_block=4)
    for kinds in PLANS:
        for mode in (oracle.MODE_PAPER, oracle.MODE_TILED):
            p = gpu_plan(A, kinds, mode, th)
            assert_same_partition(sable.sable_plan_export(p), oracle.plan(A, kinds, mode, th))
            x = torch.zeros(nc, device="cuda")
            y = torch.full((nr,), float("nan"), device="cuda")
            sable.sable_spmv(p, x, y)
            yp = torch.full((nr,), float("nan"), device="cuda")
            sable.sable_csr_spmv(p, x, yp)
            X = torch.zeros((nc, 3), device="cuda")
            Y = torch.full((nr, 3), float("nan"), device="cuda")
            sable.sable_spmm(p, X, Y, 3)
            sable.sable_update_values_f64(p, torch.zeros(0, dtype=torch.float64, device="cuda"))
            y64 = torch.full((nr,), float("nan"), dtype=torch.float64, device="cuda")
            sable.sable_spmv_f64(p, x.double(), y64)
            sable.sable_autotune(p, 0, 1, x, y)
            sable.sable_spmv(p, x, y)
            torch.cuda.synchronize()
            for t in (y, yp, Y, y64):
                assert bool((t == 0).all())
    ip, ix, vv = sable.device_csr(A)
    assert np.isfinite(sable.sable_features(nr, nc, ip, ix, vv)).all()


def test_invalid_csr_rejected():
    A = synth.from_coo(4, 4, [0, 1], [0, 1], [1.0, 2.0])
    ip, ix, vv = sable.device_csr(A)
    ix[1] = 7  # column out of range
    with pytest.raises(sable.SableError) as e:
        sable.sable_plan(4, 4, ip, ix, vv, [sable.SABLE_X_CSR])
    assert e.value.code == 2


def test_update_values_matches_replan():
    """New values through sable_update_values give the same formats (fp32 values and the
    split-bf16 words), the same SpMV and the same SpMM under every SpMM variant, bit for bit,
    as planning again with those values."""
    A, x = synth.gen_c1(1, n=768)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    kinds = [V, B, C]
    p = gpu_plan(A, kinds, oracle.MODE_PAPER, th)
    A2 = synth.CSR(A.nrows, A.ncols, A.indptr, A.indices,
                   synth.gen_dense_vector(9, A.nnz, normal=True))
    p.nnz = A2.nnz
    sable.sable_update_values(p, torch.from_numpy(A2.values).cuda())
    torch.cuda.synchronize()
    q = gpu_plan(A2, kinds, oracle.MODE_PAPER, th)
    ep, eq = sable.sable_plan_export(p), sable.sable_plan_export(q)
    assert_same_partition(ep, eq)
    assert ep["vbr_bf16"].size > 0
    assert np.array_equal(ep["vbr_bf16"], eq["vbr_bf16"])
    y1, y2 = run_spmv(p, A2, x), run_spmv(q, A2, x)
    assert torch.equal(y1, y2)
    n = 24
    Xd = torch.from_numpy(synth.gen_dense_matrix(5, A.ncols, n)).cuda()
    for mode in range(5):
        sable.sable_plan_set_variant(p, 1, mode)
        sable.sable_plan_set_variant(q, 1, mode)
        Y1 = torch.full((A.nrows, n), float("nan"), device="cuda")
        Y2 = torch.full((A.nrows, n), float("nan"), device="cuda")
        sable.sable_spmm(p, Xd, Y1, n)
        sable.sable_spmm(q, Xd, Y2, n)
        torch.cuda.synchronize()
        assert torch.equal(Y1, Y2), mode


def bf16_words(vals):
    hi, lo = oracle.bf16_split(vals)
    return hi.astype(np.uint32) | (lo.astype(np.uint32) << 16)


@pytest.mark.parametrize("case", ["c1_tiled", "fem", "odd_shapes"])
def test_bf16_split_words_bit_exact(case):
    """The plan's split-bf16 copy of every block cell (the words the matrix-core SpMM
    multiplies) equals the oracle's round-to-nearest-even split of the fp32 value bit for
    bit, fill cells included (zero words)."""
    if case == "c1_tiled":
        A, _ = synth.gen_c1(5, n=2048)
        th = oracle.Thresholds(amin_band=256, amin_block=256)
        p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    elif case == "fem":
        A, _ = synth.gen_c3(2, n=6000, ystride=8, zstride=64, scatter_density=2e-4,
                            with_x=False)
        th = oracle.Thresholds(delta_band_pm=900, delta_block_pm=900, amin_block=36)
        p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    else:  # blocks of widths not a multiple of 4, values with long mantissas and signs
        rng = np.random.default_rng(11)
        rows, cols = [], []
        for (r0, h, c0, w) in [(0, 7, 3, 9), (20, 13, 40, 5), (50, 3, 0, 31), (70, 17, 60, 2)]:
            rr, cc = np.meshgrid(np.arange(r0, r0 + h), np.arange(c0, c0 + w), indexing="ij")
            keep = rng.random(rr.size) < 0.8
            rows.append(rr.ravel()[keep])
            cols.append(cc.ravel()[keep])
        r, c = np.concatenate(rows), np.concatenate(cols)
        v = (rng.standard_normal(r.size) * 10.0 ** rng.integers(-30, 30, r.size)).astype(np.float32)
        A = synth.from_coo(100, 100, r, c, v)
        p = gpu_plan(A, [B, C], oracle.MODE_TILED, oracle.Thresholds(delta_block_pm=500, amin_block=4))
    got = sable.sable_plan_export(p)
    assert got["vbr_val"].size > 0
    want = bf16_words(got["vbr_val"])
    assert np.array_equal(got["vbr_bf16"], want)
    # the words really split: hi + lo reproduces the value to 2^-16 relative
    hi = oracle.bf16_to_f32((got["vbr_bf16"] & 0xFFFF).astype(np.uint16)).astype(np.float64)
    lo = oracle.bf16_to_f32((got["vbr_bf16"] >> 16).astype(np.uint16)).astype(np.float64)
    a = got["vbr_val"].astype(np.float64)
    assert np.all(np.abs(hi + lo - a) <= 2.0 ** -16 * np.abs(a))


def test_plain_csr_baseline():
    A, x = synth.gen_c1(2, n=2048)
    p = gpu_plan(A, [C], 0, oracle.Thresholds())
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, device="cuda")
    sable.sable_csr_spmv(p, xd, y)
    torch.cuda.synchronize()
    assert oracle.rel_err(y.cpu().numpy(), oracle.spmv(A, x)) <= 1e-5


# ---- every kernel variant --------------------------------------------------------------------

def test_every_spmv_variant_and_baseline():
    A, x = synth.gen_c1(3, n=3000)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    ref = oracle.spmv(A, x)
    xd = torch.from_numpy(x).cuda()
    for v in [*range(11), 12, 13, 14, 15, 16]:
        sable.sable_plan_set_variant(p, 0, v)
        err = check_spmv(p, A, x)
        print(f"  variant {v}: {err:.2e}")
    y = torch.empty(A.nrows, device="cuda")
    for v in range(18):
        sable.sable_plan_set_variant(p, 2, v)
        sable.sable_csr_spmv(p, xd, y)
        torch.cuda.synchronize()
        assert oracle.rel_err(y.cpu().numpy(), ref) <= 1e-5, v


@pytest.mark.parametrize("shape", [(1, 1), (5, 300), (300, 5), (17, 17), (257, 129)])
def test_every_variant_on_tiny_and_ragged_shapes(shape):
    """Every SpMV variant, plain CSR variant and SpMM mode on shapes smaller than or ragged
    against every tile height (256 RPT rows, 256 / W rows, 64-row SpMM tiles)."""
    nr, nc = shape
    A = synth.gen_random_small(7 * nr + nc, nr, nc, 0.3, nbands=1, nblocks=1)
    th = oracle.Thresholds(lseg=2, amin_band=2, amin_block=4)
    x = synth.gen_dense_vector(2, nc)
    ref = oracle.spmv(A, x)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(nr, device="cuda")
    for v in [*range(11), 12, 13, 14, 15, 16]:
        sable.sable_plan_set_variant(p, 0, v)
        check_spmv(p, A, x)
    for v in range(18):
        sable.sable_plan_set_variant(p, 2, v)
        sable.sable_csr_spmv(p, xd, y)
        torch.cuda.synchronize()
        assert oracle.rel_err(y.cpu().numpy(), ref) <= 1e-5, v
    X = synth.gen_dense_matrix(3, nc, 5)
    for m in range(5):
        sable.sable_plan_set_variant(p, 1, m)
        Y = torch.full((nr, 5), float("nan"), device="cuda")
        sable.sable_spmm(p, torch.from_numpy(X).cuda(), Y, 5)
        torch.cuda.synchronize()
        assert oracle.rel_err(Y.cpu().numpy(), oracle.spmm(A, X)) <= 1e-4, m


@pytest.mark.parametrize("n", [1, 3, 16, 64, 128, 130, 200])
def test_spmm_modes_and_widths(n):
    A, _ = synth.gen_c1(4, n=1536)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    for mode in range(5):
        sable.sable_plan_set_variant(p, 1, mode)
        check_spmm(p, A, n, seed=n)


def test_spmm_panel_unit_counts():
    """The SpMM operand panels store only occupied units (one row x 8 columns): every block cell
    falls in exactly one unit and a panel has 256 units, so 8 units >= cells and units <= 256
    panels; a plan without blocks has no panels."""
    A, _ = synth.gen_c1(4, n=1536)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    st = sable.sable_plan_info(p)
    assert st["nblk"] > 0 and st["mm_panels"] > 0
    assert 8 * st["mm_units"] >= st["vbr_cells"] and st["mm_units"] <= 256 * st["mm_panels"]
    q = gpu_plan(A, [V, C], oracle.MODE_TILED, th)
    sq = sable.sable_plan_info(q)
    assert sq["nblk"] == 0 and sq["mm_panels"] == 0 and sq["mm_units"] == 0
    check_spmm(q, A, 128, seed=3)


def test_csr_only_plan_runs_the_plain_kernels():
    """A plan whose partition is CSR alone runs its SpMV through the plain CSR kernels: after
    autotuning, sable_spmv equals sable_csr_spmv bit for bit, for a [CSR] plan and for a
    [VDIA, VBR, CSR] plan whose extractors find nothing."""
    A = synth.gen_random_small(11, 3000, 2500, 0.004)
    x = synth.gen_dense_vector(4, A.ncols)
    xd = torch.from_numpy(x).cuda()
    for kinds in ([C], [V, B, C]):
        p = gpu_plan(A, kinds, oracle.MODE_TILED, oracle.Thresholds())
        st = sable.sable_plan_info(p)
        assert st["nseg"] == 0 and st["nblk"] == 0
        y1 = torch.full((A.nrows,), float("nan"), device="cuda")
        y2 = torch.full((A.nrows,), float("nan"), device="cuda")
        sable.sable_autotune(p, 0, 1, xd, y1)
        sable.sable_spmv(p, xd, y1)
        sable.sable_csr_spmv(p, xd, y2)
        torch.cuda.synchronize()
        assert torch.equal(y1.view(torch.int32), y2.view(torch.int32))
        assert oracle.rel_err(y1.cpu().numpy(), oracle.spmv(A, x)) <= 1e-5
        for v in (0, 3, 8, 12, 15):  # every hybrid variant setting gives the plain result
            sable.sable_plan_set_variant(p, 0, v)
            sable.sable_spmv(p, xd, y1)
            torch.cuda.synchronize()
            assert torch.equal(y1.view(torch.int32), y2.view(torch.int32)), v


def test_spmm_autotune_kept_per_width():
    """The SpMM variant tuned for one n stays in use for that n after tuning another n, and
    an explicit variant applies to every n."""
    A, _ = synth.gen_c1(8, n=2048)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, oracle.Thresholds(amin_band=256, amin_block=256))
    X16 = torch.from_numpy(synth.gen_dense_matrix(1, A.ncols, 16)).cuda()
    X130 = torch.from_numpy(synth.gen_dense_matrix(2, A.ncols, 130)).cuda()
    Y16 = torch.empty(A.nrows, 16, device="cuda")
    Y130 = torch.empty(A.nrows, 130, device="cuda")
    sable.sable_autotune(p, 1, 16, X16, Y16)
    m16 = sable.sable_plan_info(p)["spmm_variant"]
    sable.sable_autotune(p, 1, 130, X130, Y130)
    m130 = sable.sable_plan_info(p)["spmm_variant"]
    print(f"  tuned modes: n=16 -> {m16}, n=130 -> {m130}")
    sable.sable_spmm(p, X16, Y16, 16)
    ref = torch.empty_like(Y16)
    q = gpu_plan(A, [V, B, C], oracle.MODE_TILED, oracle.Thresholds(amin_band=256, amin_block=256))
    sable.sable_plan_set_variant(q, 1, m16)
    sable.sable_spmm(q, X16, ref, 16)
    torch.cuda.synchronize()
    assert torch.equal(Y16, ref)
    for m in range(5):  # an explicit choice reaches every width
        sable.sable_plan_set_variant(p, 1, m)
        sable.sable_plan_set_variant(q, 1, m)
        sable.sable_spmm(p, X16, Y16, 16)
        sable.sable_spmm(q, X16, ref, 16)
        torch.cuda.synchronize()
        assert torch.equal(Y16, ref), m


def test_spmm_split_bf16_block_accuracy():
    """One dense 300x200 block (all regions VBR): the split-bf16 matrix-core path keeps the
    normwise error near 2^-16 relative, far below plain bf16 (~2^-9)."""
    rng = np.random.default_rng(7)
    D = rng.uniform(-1, 1, (300, 200)).astype(np.float32)
    r, c = np.nonzero(np.ones_like(D))
    A = synth.from_coo(300, 200, r, c, D[r, c])
    p = gpu_plan(A, [B, C], oracle.MODE_PAPER, oracle.Thresholds(amin_block=64))
    got = sable.sable_plan_export(p)
    assert got["blk"].tolist() == [[0, 300, 0, 200]]
    for mode in (0, 4):
        sable.sable_plan_set_variant(p, 1, mode)
        err = check_spmm(p, A, 48, tol=2e-5)
        assert err > 1e-8  # the matrix-core path really ran in reduced precision


def test_c1_full_paper_mode_against_stored_oracle():
    """Full 4096^2 C1 under the literal block search: structure equal to the oracle's stored
    result (tests/golden/c1_seed0_paper.txt, written by make_c1_paper.py from oracle/ only),
    values checked entry by entry by the exact-cover invariants, product within 1e-5."""
    from tests.conftest import read_golden
    g = read_golden("c1_seed0_paper.txt")
    A, x = synth.gen_c1(0)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    p = gpu_plan(A, [V, B, C], oracle.MODE_PAPER, th)
    got = sable.sable_plan_export(p)
    assert got["seg_row_start"].tolist() == g["seg_row_start"]
    assert got["seg_nrows"].tolist() == g["seg_nrows"]
    assert got["idiag"].tolist() == g["idiag"]
    assert got["blk"].ravel().tolist() == g["blk"]
    assert got["csr_col"].size == g["csr_nnz"][0]
    oracle.check_partition(A, got, th, [V, B, C])
    check_spmv(p, A, x)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c2_full_size(seed):
    """PDE-like 2,097,152-row matrix in the benchmark's configuration (autotuned kernel):
    exact cover of every input entry, and the whole product vector against the FP64
    oracle (every row), for the autotuned variant and for the plain CSR baseline."""
    A, x = synth.gen_c2(seed)
    th = oracle.Thresholds(delta_band_pm=750, delta_block_pm=500)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, device="cuda")
    sable.sable_autotune(p, 0, 1, xd, y)
    got = sable.sable_plan_export(p)
    oracle.check_partition(A, got, th, [V, B, C])
    ref = oracle.spmv(A, x)
    y.fill_(float("nan"))
    sable.sable_spmv(p, xd, y)
    torch.cuda.synchronize()
    err = oracle.rel_err(y.cpu().numpy(), ref)
    info = sable.sable_plan_info(p)
    print(f"  full rel_err={err:.3e} (variant {info['spmv_variant']}, far split {info['far_split']})")
    assert err <= 1e-5
    yp = torch.full((A.nrows,), float("nan"), device="cuda")
    sable.sable_csr_spmv(p, xd, yp)
    torch.cuda.synchronize()
    errp = oracle.rel_err(yp.cpu().numpy(), ref)
    print(f"  plain CSR full rel_err={errp:.3e}")
    assert errp <= 1e-5


@pytest.fixture(scope="module")
def c3_case():
    """The FEM-like 500,000-row matrix (n = 128), its plan and the oracle's FP64 product."""
    A, X = synth.gen_c3(0)
    th = oracle.Thresholds(delta_band_pm=900, delta_block_pm=900, amin_block=36)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, th)
    print("  oracle FP64 SpMM (n = 128)", flush=True)
    ref = oracle.spmm(A, X)
    return A, X, th, p, ref


def _c3_product(p, X):
    n = X.shape[1]
    Xd = torch.from_numpy(X).cuda()
    Y = torch.full((X.shape[0], n), float("nan"), device="cuda")
    sable.sable_spmm(p, Xd, Y, n)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def test_c3_full_size(c3_case):
    """FEM-like matrix, SpMM with n = 128, in the benchmark's configuration (autotuned):
    exact cover of every input entry, and the whole 500,000 x 128 product against the
    FP64 oracle."""
    A, X, th, p, ref = c3_case
    n = X.shape[1]
    Xd = torch.from_numpy(X).cuda()
    Y = torch.empty(A.nrows, n, device="cuda")
    sable.sable_autotune(p, 1, n, Xd, Y)
    del Xd, Y
    oracle.check_partition(A, sable.sable_plan_export(p), th, [V, B, C])
    err = oracle.rel_err(_c3_product(p, X), ref)
    print(f"  full rel_err={err:.3e} (spmm variant {sable.sable_plan_info(p)['spmm_variant']})")
    assert err <= 1e-4


@pytest.mark.parametrize("mode", [0, 3, 4])
def test_c3_full_size_matrix_cores(c3_case, mode):
    """The same product with the VBR blocks forced onto the split-bf16 matrix-core paths
    (SpMM variants 0, 3 and 4): the whole product within 1e-4 of the FP64 oracle, and above
    plain fp32 rounding (the reduced-precision path really ran)."""
    A, X, th, p, ref = c3_case
    sable.sable_plan_set_variant(p, 1, mode)
    err = oracle.rel_err(_c3_product(p, X), ref)
    print(f"  full rel_err={err:.3e} (spmm variant {mode})")
    assert err <= 1e-4
    assert err > 5e-7  # fp32 blocks give ~1e-7 here; split bf16 drops the lo * lo term


# ---- far-column split of the CSR part (streamed SpMV) ------------------------------------

FAR_WINDOW = 1 << 17  # entries more than this many columns from their row are far


def wide_scatter(nr, nc, seed):
    """Main diagonal (a VDIA band) plus ~0.15 uniform-random entries per row and 70,000
    more, so that the CSR part has well over 2^16 far entries and rows of uneven length."""
    rng = np.random.default_rng(seed)
    d = np.arange(min(nr, nc))
    ns = int(0.15 * nr) + 70000
    rows = np.concatenate([d, rng.integers(0, nr, ns)])
    cols = np.concatenate([d, rng.integers(0, nc, ns)])
    vals = rng.uniform(-1, 1, rows.size).astype(np.float32)
    return synth.from_coo(nr, nc, rows, cols, vals)


@pytest.mark.parametrize("shape", [(1_300_001, 1_300_001), (200_003, 3_000_000),
                                   (2_000_000, 1_100_000)])
def test_far_column_split(shape):
    """Square, wide and tall matrices: the plan reports the far-entry count the CSR export
    implies; every streamed variant matches the oracle with the split on and off, and the
    two agree bit for bit (the split keeps each row's summation order); a value refresh
    reaches the gathered copies."""
    nr, nc = shape
    A = wide_scatter(nr, nc, seed=nr % 97)
    x = synth.gen_dense_vector(1, nc)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, oracle.Thresholds())
    info = sable.sable_plan_info(p)
    got = sable.sable_plan_export(p)
    ptr = np.asarray(got["csr_ptr"], np.int64)
    erow = np.repeat(np.arange(nr, dtype=np.int64), np.diff(ptr))
    nfar = int(np.count_nonzero(np.abs(got["csr_col"].astype(np.int64) - erow) > FAR_WINDOW))
    print(f"  far entries {nfar} of {got['csr_col'].size}", flush=True)
    assert nfar >= 1 << 16
    assert info["far_split"] == 1 and info["far_nnz"] == nfar
    for v in (0, 1, 2, 8, 9, 10):
        sable.sable_plan_set_variant(p, 0, v)
        ys = []
        for fs in (1, 0):
            sable.sable_plan_set_variant(p, 3, fs)
            print(f"  variant {v} far_split {fs}", flush=True)
            check_spmv(p, A, x)
            ys.append(run_spmv(p, A, x))
        assert torch.equal(ys[0].view(torch.int32), ys[1].view(torch.int32)), v
    sable.sable_plan_set_variant(p, 0, 1)
    sable.sable_plan_set_variant(p, 3, 1)
    A2 = synth.CSR(A.nrows, A.ncols, A.indptr, A.indices,
                   synth.gen_dense_vector(5, A.nnz, normal=True))
    sable.sable_update_values(p, torch.from_numpy(A2.values).cuda())
    torch.cuda.synchronize()
    check_spmv(p, A2, x)


def test_far_split_absent_below_thresholds():
    """Narrow matrices (x within a few MB) and CSR parts with few far entries keep the
    single fused launch."""
    A = wide_scatter(500_000, 500_000, seed=3)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, oracle.Thresholds())
    assert sable.sable_plan_info(p)["far_split"] == 0
    check_spmv(p, A, synth.gen_dense_vector(2, A.ncols))


def test_prebound_launcher_matches_direct_calls():
    """sable.launcher marshals once and calls the same entry points: identical results."""
    A, x = synth.gen_c1(6, n=1024)
    p = gpu_plan(A, [V, B, C], oracle.MODE_TILED, oracle.Thresholds(amin_band=256, amin_block=256))
    xd = torch.from_numpy(x).cuda()
    y1, y2 = torch.empty(A.nrows, device="cuda"), torch.empty(A.nrows, device="cuda")
    sable.sable_spmv(p, xd, y1)
    sable.launcher("sable_spmv", p, xd, y2)()
    X = torch.from_numpy(synth.gen_dense_matrix(2, A.ncols, 8)).cuda()
    Y1, Y2 = torch.empty(A.nrows, 8, device="cuda"), torch.empty(A.nrows, 8, device="cuda")
    sable.sable_spmm(p, X, Y1, 8)
    sable.launcher("sable_spmm", p, X, Y2, 8)()
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(Y1, Y2)
    with pytest.raises(sable.SableError):
        sable.launcher("sable_spmm", p, X, Y2, 0)()  # n < 1 is rejected by the entry point


# ---- autotuning cache ----------------------------------------------------------------------

def test_structure_hash_and_autotune_cache():
    """Plans of one pattern (any values) share a structure hash and an autotuning result: the
    second plan's sable_autotune takes the cached choice without timing; another pattern or
    other thresholds give another hash; clearing the cache makes the next call time again."""
    import time
    A, x = synth.gen_c1(6, n=2048)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    kinds = [V, B, C]
    A2 = synth.CSR(A.nrows, A.ncols, A.indptr, A.indices,
                   synth.gen_dense_vector(3, A.nnz, normal=True))
    p, q = gpu_plan(A, kinds, oracle.MODE_TILED, th), gpu_plan(A2, kinds, oracle.MODE_TILED, th)
    hp, hq = sable.sable_plan_info(p)["structure_hash"], sable.sable_plan_info(q)["structure_hash"]
    assert hp == hq and hp != 0
    A3, _ = synth.gen_c1(7, n=2048)
    assert sable.sable_plan_info(gpu_plan(A3, kinds, oracle.MODE_TILED, th))["structure_hash"] != hp
    th2 = oracle.Thresholds(amin_band=256, amin_block=512)
    assert sable.sable_plan_info(gpu_plan(A, kinds, oracle.MODE_TILED, th2))["structure_hash"] != hp
    sable.sable_autotune_cache_clear()
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, device="cuda")
    t0 = time.perf_counter()
    sable.sable_autotune(p, 0, 1, xd, y)
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    sable.sable_autotune(q, 0, 1, xd, y)
    t_cached = time.perf_counter() - t0
    ip, iq = sable.sable_plan_info(p), sable.sable_plan_info(q)
    for k in ("spmv_variant", "far_split", "plain_variant"):
        assert ip[k] == iq[k], k
    print(f"  first {t_first * 1e3:.1f} ms, cached {t_cached * 1e3:.2f} ms")
    assert t_cached < 0.2 * t_first
    check_spmv(q, A2, x)
    sable.sable_autotune_cache_clear()
    t0 = time.perf_counter()
    sable.sable_autotune(q, 0, 1, xd, y)
    assert time.perf_counter() - t0 > 5 * t_cached


@pytest.mark.parametrize("far", [0, 1])
def test_persistent_tiles_equal_one_tile_per_workgroup(far):
    """The persistent streamed SpMV (variants 15, 16; plain 16, 17) runs the streamed tile body
    on every tile in turn: its results equal the one-tile-per-workgroup launch (variants 0, 8;
    plain 0, 10) bit for bit, with and without the far-column pass, on a matrix with many
    more tiles than resident workgroups."""
    A = wide_scatter(1_300_001, 1_300_001, 5)
    x = synth.gen_dense_vector(3, A.ncols)
    p = gpu_plan(A, [V, C], 0, oracle.Thresholds())
    sable.sable_plan_set_variant(p, 3, far)
    xd = torch.from_numpy(x).cuda()
    out = {}
    for v in (0, 15, 8, 16):
        sable.sable_plan_set_variant(p, 0, v)
        out[v] = run_spmv(p, A, x)
    assert torch.equal(out[0], out[15]) and torch.equal(out[8], out[16])
    assert oracle.rel_err(out[15].cpu().numpy(), oracle.spmv(A, x)) <= 1e-5
    y = {}
    for v in (0, 16, 10, 17):
        sable.sable_plan_set_variant(p, 2, v)
        y[v] = torch.full((A.nrows,), float("nan"), device="cuda")
        sable.sable_csr_spmv(p, xd, y[v])
    torch.cuda.synchronize()
    assert torch.equal(y[0], y[16]) and torch.equal(y[10], y[17])
