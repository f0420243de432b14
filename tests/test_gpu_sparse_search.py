"""The literal block search (Alg. 1 / Alg. 2) with the sparse window scan on the GPU, through
the C ABI, against the CPU oracle: the same blocks bit for bit whether the scan visits every
inner index or only the non-empty ones, and the same budget decisions past the dense scan's
bound."""
import numpy as np
import pytest

import oracle
from paper_2407_00829_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_00829_amd import sable  # noqa: E402
from tests.test_gpu_parity import (KIND, assert_same_partition, check_spmv,  # noqa: E402
                                   to_sable_th)

V, B, C = oracle.VDIA, oracle.VBR, oracle.CSR


def sparse_plan(A, kinds, mode, th):
    t = to_sable_th(th)
    t.flags = sable.SABLE_F_SPLIT_BF16 | sable.SABLE_F_SPARSE_SEARCH
    print(f"[plan sparse search] {A.nrows}x{A.ncols} nnz={A.nnz} kinds={kinds} mode={mode}", flush=True)
    return sable.plan_host(A, [KIND[k] for k in kinds], mode, t)


@pytest.mark.parametrize("seed", range(8))
def test_random_small_sparse_scan_bit_exact(seed):
    rng = np.random.default_rng(300 + seed)
    nr, nc = int(rng.integers(40, 300)), int(rng.integers(40, 300))
    A = synth.gen_random_small(seed, nr, nc, float(rng.choice([0.005, 0.03, 0.1])), nbands=3,
                               nblocks=4, block_max=40)
    th = oracle.Thresholds(lseg=8, amin_band=32, amin_block=int(rng.choice([16, 64, 100])),
                           coverage_pm=40 * (seed % 3), delta_block_pm=[500, 700, 900][seed % 3])
    for kinds in ([B, C], [V, B, C], [B, V, C]):
        p = sparse_plan(A, kinds, oracle.MODE_PAPER, th)
        assert_same_partition(sable.sable_plan_export(p), oracle.plan(A, kinds, oracle.MODE_PAPER, th))
    check_spmv(p, A, synth.gen_dense_vector(seed, A.ncols))


def test_c1_full_sparse_scan_against_stored_oracle():
    """Full 4096^2 C1 through the sparse scan: the blocks of the stored oracle result."""
    from tests.conftest import read_golden
    g = read_golden("c1_seed0_paper.txt")
    A, x = synth.gen_c1(0)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    p = sparse_plan(A, [V, B, C], oracle.MODE_PAPER, th)
    got = sable.sable_plan_export(p)
    assert got["blk"].ravel().tolist() == g["blk"]
    assert got["csr_col"].size == g["csr_nnz"][0]
    oracle.check_partition(A, got, th, [V, B, C])
    check_spmv(p, A, x)


def _planted(n, seed):
    """n x n with three dense blocks and a few scattered entries."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for (r0, h, c0, w) in [(100, 64, 4000, 64), (3000, 48, 200, 80), (4700, 70, 4500, 60)]:
        rr, cc = np.meshgrid(np.arange(r0, r0 + h), np.arange(c0, c0 + w), indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
    rows.append(rng.integers(0, n, 300))
    cols.append(rng.integers(0, n, 300))
    r, c = np.concatenate(rows), np.concatenate(cols)
    return synth.from_coo(n, n, r, c, rng.uniform(-1, 1, r.size).astype(np.float32))


def test_literal_search_past_the_dense_bound():
    """5200^2 is past nrows * ncols * max <= 2^37, but with few entries the sparse scan's work
    is within the budget: the literal search runs (auto picks it too) and gives the oracle's
    blocks bit for bit."""
    A = _planted(5200, 1)
    th = oracle.Thresholds(amin_block=1024)
    ok, cost = oracle.paper_fits(A, th)
    assert ok and cost < 1 << 37
    ref = oracle.plan(A, [B, C], oracle.MODE_PAPER, th)
    assert ref["blk"].shape[0] == 3
    p = sable.plan_host(A, [sable.SABLE_X_VBR, sable.SABLE_X_CSR], sable.SABLE_VBR_PAPER, to_sable_th(th))
    assert_same_partition(sable.sable_plan_export(p), ref)
    q = sable.plan_host(A, [sable.SABLE_X_VBR, sable.SABLE_X_CSR], sable.SABLE_VBR_AUTO, to_sable_th(th))
    assert sable.sable_plan_info(q)["vbr_mode_used"] == sable.SABLE_VBR_PAPER
    check_spmv(p, A, synth.gen_dense_vector(2, A.ncols))


def test_literal_search_over_budget():
    """6000^2 with eight entries per row: the sparse scan's work is about 2e11 > 2^37, so a
    literal request fails with SABLE_ERR_TOO_LARGE and auto takes the tiled search, as in the
    oracle."""
    rng = np.random.default_rng(0)
    r = np.repeat(np.arange(6000), 8)
    A = synth.from_coo(6000, 6000, r, rng.integers(0, 6000, r.size),
                       rng.uniform(-1, 1, r.size).astype(np.float32))
    assert not oracle.paper_fits(A)[0]
    with pytest.raises(sable.SableError) as e:
        sable.plan_host(A, [sable.SABLE_X_VBR, sable.SABLE_X_CSR], sable.SABLE_VBR_PAPER,
                        sable.Thresholds())
    assert e.value.code == 4
    p = sable.plan_host(A, [sable.SABLE_X_VBR, sable.SABLE_X_CSR], sable.SABLE_VBR_AUTO,
                        sable.Thresholds())
    ref = oracle.plan(A, [B, C], oracle.MODE_AUTO)
    assert sable.sable_plan_info(p)["vbr_mode_used"] == sable.SABLE_VBR_TILED == ref["vbr_mode"]
    assert_same_partition(sable.sable_plan_export(p), ref)
