"""The C-ABI library loads on a host without a GPU, exports every function
include/ddm.h declares, and validates problems in host code (no compute)."""
import ctypes

import pytest

import paper_1807_04180_amd as ddm
from paper_1807_04180_amd import _ffi


def test_library_exports_every_declared_function():
    L = ddm.lib()
    names = ddm.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert L.ddm_version().startswith(b"libddm")


def _prob(**kw):
    base = dict(dim=2, M=(80, 80), h=1 / 80, n_pml=10, sigma0=3.3, N=(2, 2), n_ov=4)
    base.update(kw)
    return ddm.Problem(**base)


def test_memory_required_grows_with_rhs_and_precision():
    p64 = _prob()
    b1 = p64.memory_required(1)
    b4 = p64.memory_required(4)
    assert b4 > b1 > 0
    pm = _prob(mixed=True)
    assert pm.memory_required(4) < b4  # complex64 factors and workspaces


def test_memory_required_counts_factor_bytes():
    # 2x2 of 62/63-node boxes: sum over boxes of nb * bs^2 complex128 entries
    p = _prob()
    sizes = [(62, 62), (63, 62), (62, 63), (63, 63)]
    fbytes = sum(ny * nx * nx * 16 for nx, ny in sizes)
    assert p.memory_required(1) > fbytes


@pytest.mark.parametrize("bad", [
    dict(dim=4),
    dict(M=(81, 80)),          # not divisible
    dict(n_ov=1),
    dict(n_pml=1),
    dict(N=(20, 20)),          # core 4 < n_ov + 2
    dict(sigma0=float("nan")),
    dict(h=0.0),
])
def test_invalid_problems_rejected(bad):
    p = _prob(**bad)
    with pytest.raises(ddm.DDMError) as e:
        p.memory_required(1)
    assert e.value.code == _ffi.DDM_EINVAL
    assert ddm.lib().ddm_last_error(None)


def test_product_path_has_no_cpu_fallback(monkeypatch, tmp_path):
    monkeypatch.setattr(_ffi, "_lib", None)
    monkeypatch.setattr(_ffi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _ffi.lib()
