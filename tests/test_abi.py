"""The C-ABI library loads, exports every symbol include/ens.h declares, and
rejects bad arguments before touching a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "ens.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ens_status|const char \*)\s*(ens_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2506_23712_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.lib()


def test_header_declares_the_expected_calls():
    syms = header_symbols()
    from paper_2506_23712_amd import _lib
    assert syms == sorted(_lib.EXPORTS)
    for name in ("ens_member_init", "ens_step", "ens_accumulate_stats", "ens_mix"):
        assert name in syms


def test_every_declared_symbol_is_exported(L):
    for name in header_symbols():
        assert hasattr(L, name), name


def test_argument_validation_without_a_gpu(L):
    from paper_2506_23712_amd import _lib
    # null context
    b = ctypes.c_size_t()
    d = _lib.MemberDesc(32, 0, 6.283185307179586, 0.02, 0.1, 0.0, 0.0, 2.0, 0.01, 0.5, 1, 2.0, 0.5, 0, 0)
    assert L.ens_member_workspace_bytes(None, ctypes.byref(d), ctypes.byref(b)) == _lib.ENS_E_INVALID
    assert b"null context" in L.ens_last_error()
    # unsupported transform length, bad sign and empty batch are decided on the host
    assert L.ens_fft_pencils(48, 0, -1, 10, None, None, None) == _lib.ENS_E_UNSUPPORTED
    assert L.ens_fft_pencils(64, 0, 2, 10, None, None, None) == _lib.ENS_E_INVALID
    assert L.ens_fft_pencils(64, 0, -1, 0, None, None, None) == _lib.ENS_OK
    assert L.ens_step(None, None, 0, 1, None) == _lib.ENS_E_INVALID
    assert L.ens_spectrum(None, 0, 8, None, None) == _lib.ENS_E_INVALID
    assert L.ens_lambda_pdf_from_cf(None, 64, 0.0, 0.1, None, None) == _lib.ENS_E_INVALID
    assert L.ens_mix_table(None, None, 0, None, 64, 0.0, 0.1, None, None) == _lib.ENS_E_INVALID
    assert L.ens_mix_noalloc(None, None, 0, 0.023, 1.0, 0, 1.0, None, None) == _lib.ENS_E_INVALID
    assert L.ens_scale_gap(None, None, 0, 100.0, None, None, None) == _lib.ENS_E_INVALID
    assert L.ens_member_refine(None, 0, 1, None) == _lib.ENS_E_INVALID
    assert L.ens_member_set_diag(None, 0, None, None) == _lib.ENS_E_INVALID
    assert L.ens_set_stats(None, 0, None, None, None) == _lib.ENS_E_INVALID
    ctx = ctypes.c_void_p()
    bad = _lib.HistDesc(0, -1, 1, -1, 1, 8, -1, 1, 8, -1, 1, 1.0, 1.0)
    assert L.ens_create(ctypes.byref(ctx), 0, ctypes.byref(bad)) == _lib.ENS_E_INVALID
    # ranges and reference scales must be finite (checked before any device call)
    inf = float("inf")
    for i, v in ((2, inf), (1, -inf), (7, inf), (10, inf), (11, inf), (12, inf), (4, float("nan"))):
        fields = [8, -1.0, 1.0, -1.0, 1.0, 8, -1.0, 1.0, 8, -1.0, 1.0, 1.0, 1.0]
        fields[i] = v
        bad = _lib.HistDesc(*fields)
        assert L.ens_create(ctypes.byref(ctx), 0, ctypes.byref(bad)) == _lib.ENS_E_INVALID, i


def test_no_gpu_means_a_clean_error(L):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    from paper_2506_23712_amd import _lib
    ctx = ctypes.c_void_p()
    assert L.ens_create(ctypes.byref(ctx), 0, None) == _lib.ENS_E_HIP
    assert L.ens_last_error()


def test_package_refuses_to_run_without_the_library(tmp_path, monkeypatch):
    from paper_2506_23712_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()
