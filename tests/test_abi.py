"""The C-ABI library loads and exports every symbol include/sable.h declares; argument checks
that precede any GPU work return the documented status codes (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2407_00829_amd import sable

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sable.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sable_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = sable.lib()
    names = declared_functions()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(names) == sorted(sable.EXPORTED)


def _fake_csr(nrows=10, ncols=10, nnz=5):
    return sable.sable_csr(nrows, ncols, nnz, 0x1000, 0x2000, 0x3000)


def _plan_rc(A, kinds, mode=0, th=None):
    L = sable.lib()
    lst = (sable.sable_extractor * len(kinds))(*[sable.sable_extractor(k, mode) for k in kinds])
    h = ctypes.c_void_p(1234)
    cth = th.c() if th else None
    rc = L.sable_plan(ctypes.byref(A), lst, len(kinds), ctypes.byref(cth) if cth else None,
                      None, ctypes.byref(h))
    return rc, h.value


def test_incomplete_plan_rejected_before_gpu_work():
    rc, h = _plan_rc(_fake_csr(), [sable.SABLE_X_VDIA, sable.SABLE_X_VBR])
    assert rc == 3 and h is None
    assert "CSR" in sable.sable_last_error()


def test_bad_lists_and_sizes():
    assert _plan_rc(_fake_csr(), [sable.SABLE_X_CSR, sable.SABLE_X_VDIA, sable.SABLE_X_CSR])[0] == 1
    assert _plan_rc(_fake_csr(), [sable.SABLE_X_VDIA, sable.SABLE_X_VDIA, sable.SABLE_X_CSR])[0] == 1
    assert _plan_rc(_fake_csr(), [7, sable.SABLE_X_CSR])[0] == 1
    assert _plan_rc(_fake_csr(nnz=2 ** 31), [sable.SABLE_X_CSR])[0] == 4
    assert _plan_rc(_fake_csr(nrows=-1), [sable.SABLE_X_CSR])[0] == 1
    # literal block search over budget before any GPU work: 400,000^2 has about 1.6e11
    # spans of at least ceil(sqrt(2500)) rows or columns, one step each is past 2^37
    A = _fake_csr(400000, 400000, 5)
    assert _plan_rc(A, [sable.SABLE_X_VBR, sable.SABLE_X_CSR], sable.SABLE_VBR_PAPER)[0] == 4
    th = sable.Thresholds(delta_block_pm=400)
    assert _plan_rc(_fake_csr(), [sable.SABLE_X_VBR, sable.SABLE_X_CSR], 0, th)[0] == 1


def test_null_arguments():
    L = sable.lib()
    assert L.sable_spmv(None, None, None, None) == 1
    assert L.sable_plan_info(None, None) == 1
    assert L.sable_plan_destroy(None) == 0
    assert L.sable_thresholds_default(None) == 1


def test_defaults_match_documentation():
    t = sable.sable_thresholds_default()
    assert (t.delta_band_pm, t.delta_block_pm, t.amin_band, t.amin_block) == (750, 500, 2500, 2500)
    assert (t.lseg, t.wmax, t.dmax, t.coverage_pm, t.flags) == (64, 32, -1, 80, 1)
