"""Run-time specialized SpMV (hipRTC, SpMV variant 11) against the oracle through the C ABI."""
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


def spmv(p, A, x):
    y = torch.full((A.nrows,), float("nan"), device="cuda")
    sable.sable_spmv(p, torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    return y


def check_spec(A, kinds, mode, th, seed):
    print(f"[plan] {A.nrows}x{A.ncols} nnz={A.nnz} kinds={kinds}", flush=True)
    p = sable.plan_host(A, kinds, mode, th)
    sable.sable_plan_specialize(p)
    info = sable.sable_plan_info(p)
    assert info["spec_ms"] > 0
    sable.sable_plan_set_variant(p, 0, 11)
    x = synth.gen_dense_vector(seed, A.ncols)
    y = spmv(p, A, x)
    err = oracle.rel_err(y.cpu().numpy(), oracle.spmv(A, x))
    print(f"  specialized rel_err={err:.3e} (nseg={info['nseg']} nblk={info['nblk']}, "
          f"compiled in {info['spec_ms']:.0f} ms)", flush=True)
    assert err <= 1e-5
    assert torch.equal(y, spmv(p, A, x)), "not bitwise reproducible"
    return p


@pytest.mark.parametrize("seed", range(3))
def test_random_mixed(seed):
    A = synth.gen_random_small(seed, 900 + 131 * seed, 700 + 97 * seed, 0.01, nbands=3, nblocks=4)
    check_spec(A, [V, B, C], sable.SABLE_VBR_TILED, sable.Thresholds(amin_band=64, amin_block=64), seed)


def test_c1_paper_mode():
    A, _ = synth.gen_c1(2, n=3000)
    check_spec(A, [V, B, C], sable.SABLE_VBR_PAPER, sable.Thresholds(amin_band=256, amin_block=256), 2)


def test_bands_leaving_the_matrix_and_csr_only():
    """Offsets that run past both edges (bound checks in the generated code) and a plan with
    no bands or blocks at all (the switch is empty)."""
    n = 5000
    rows, cols = [], []
    for off in (-2000, -1, 0, 1, 4500):
        r = np.arange(max(0, -off), min(n, n - off))
        rows.append(r)
        cols.append(r + off)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    A = synth.from_coo(n, n, r, c, synth.gen_dense_vector(1, r.size))
    check_spec(A, [V, C], 0, sable.Thresholds(amin_band=64), 1)
    check_spec(A, [C], 0, sable.Thresholds(), 3)


def test_too_large_and_not_specialized():
    A, _ = synth.gen_c2(0, g=48)  # 110,592 rows: 432 tiles, fine
    p = sable.plan_host(A, [V, B, C], sable.SABLE_VBR_TILED, sable.Thresholds())
    with pytest.raises(sable.SableError):
        sable.sable_plan_set_variant(p, 0, 11)  # not specialized yet
    big, _ = synth.gen_c2(0, g=128)  # 8192 tiles
    q = sable.plan_host(big, [V, B, C], sable.SABLE_VBR_TILED, sable.Thresholds())
    with pytest.raises(sable.SableError) as e:
        sable.sable_plan_specialize(q)
    assert e.value.code == 4  # SABLE_ERR_TOO_LARGE


def test_autotune_with_specialized_variant():
    A, x = synth.gen_c1(6, n=4096)
    p = check_spec(A, [V, B, C], sable.SABLE_VBR_TILED, sable.Thresholds(amin_band=256, amin_block=256), 6)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, device="cuda")
    sable.sable_autotune(p, 0, 1, xd, y)
    info = sable.sable_plan_info(p)
    print(f"  autotuned variant {info['spmv_variant']}")
    y = spmv(p, A, x)
    assert oracle.rel_err(y.cpu().numpy(), oracle.spmv(A, x)) <= 1e-5
