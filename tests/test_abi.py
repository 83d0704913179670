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


# ---- ddm_setup's host-side refusals (no device memory is touched) ----------

def _setup_host_k2(prob, k2):
    """ddm_setup with k2 in host memory; returns (status, message)."""
    import numpy as np
    L = ddm.lib()
    k2 = np.ascontiguousarray(k2, dtype=np.float64)
    p = prob.to_c(k2_on_host=True)
    h = ctypes.c_void_p()
    st = L.ddm_setup(ctypes.byref(p), k2.ctypes.data_as(ctypes.c_void_p), 1, None, ctypes.byref(h))
    if st == 0:
        L.ddm_destroy(h)
    return st, L.ddm_last_error(None).decode()


def _k2(prob, value=2500.0):
    import numpy as np
    G = [m + 2 * prob.n_pml - 1 for m in prob.M]
    return np.full(int(np.prod(G)), value)


def test_setup_rejects_non_finite_k2():
    import numpy as np
    p = _prob()
    for bad in (float("nan"), float("inf")):
        k2 = _k2(p)
        k2[1234] = bad
        st, msg = _setup_host_k2(p, k2)
        assert st == _ffi.DDM_EINVAL and "non-finite" in msg


@pytest.mark.parametrize("kw,value,needle", [
    (dict(sigma0=3.3, reflection=1e-6), 2500.0, "not both"),
    (dict(sigma0=0.0, reflection=1.0), 2500.0, "reflection"),
    (dict(sigma0=0.0, reflection=-0.5), 2500.0, "reflection"),
    (dict(sigma0=0.0, reflection=1e-6), 0.0, "k2 > 0"),
])
def test_setup_rejects_bad_pml_request(kw, value, needle):
    p = _prob(**kw)
    st, msg = _setup_host_k2(p, _k2(p, value))
    assert st == _ffi.DDM_EINVAL and needle in msg


def test_setup_refuses_plan_beyond_budget():
    """SURVEY failure mode (iv): a plan larger than hbm_budget_bytes is refused
    with DDM_ENOMEM before any device allocation."""
    p = _prob()
    need = p.memory_required(1)
    p.hbm_budget_bytes = need - 1
    st, msg = _setup_host_k2(p, _k2(p))
    assert st == _ffi.DDM_ENOMEM and "budget" in msg
