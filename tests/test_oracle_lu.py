"""Pins of the oracle's banded LU (global and subdomain direct solves, the
MUMPS role of Sec. 4) against a dense library solve (numpy.linalg.solve) of
the matrix probed column by column from the oracle's operator, and against the
residual of that operator on larger grids."""
import numpy as np
import pytest

import ddm_inputs as di
from oracle import Oracle


def _dense_global(o):
    n = o.nglob
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        A[:, j] = o.apply(e).reshape(-1)
    return A


@pytest.mark.parametrize("dim", [2, 3])
def test_global_banded_lu_vs_dense_solve(dim):
    M, n_pml = (12, 4) if dim == 2 else (6, 2)
    h = 1.0 / M
    G = M + 2 * n_pml - 1
    rng = np.random.default_rng(21 + dim)
    k2 = rng.uniform(30, 200, size=(G,) * dim)
    o = Oracle(dim, (M,) * dim, h, n_pml, 3.0, (1,) * dim, 2, k2)
    f = di.random_field((2, o.nglob), seed=dim)
    u = o.global_solve(f)
    A = _dense_global(o)
    uref = np.linalg.solve(A, f.T).T
    np.testing.assert_allclose(u, uref, rtol=0, atol=1e-12 * np.abs(uref).max())


def test_local_banded_lu_vs_dense_solve():
    w = di.small_2d(M=20, N=(2, 2), n_pml=3, n_ov=2, layered=True, seed=2)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    g = di.random_field((1, o.etot), seed=9)
    x = o.local_solve(g)
    for a in range(o.nsub):
        sd = o.subdomain(a)
        sl = slice(sd["off"], sd["off"] + sd["n"])
        n = sd["n"]
        A = np.empty((n, n), dtype=np.complex128)
        e = np.zeros(n, dtype=np.complex128)
        for j in range(n):
            e[:] = 0
            e[j] = 1
            A[:, j] = o.apply_local(a, e)
        xr = np.linalg.solve(A, g[0, sl])
        np.testing.assert_allclose(x[0, sl], xr, rtol=0, atol=1e-12 * np.abs(xr).max())


def test_global_solve_residual_medium_size():
    w = di.small_2d(M=96, N=(1, 1), n_pml=8, n_ov=2, layered=True, seed=4, nrhs=2)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    u = o.global_solve(w.f)
    assert np.all(o.relres(w.f, u) < 1e-12)


def test_relres_definition():
    """relres = ||f - L u|| / ||f|| (the stopping test of Sec. 4.2)."""
    w = di.small_2d(M=16, N=(1, 1), n_pml=3, n_ov=2)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    u = di.random_field((1, o.nglob), seed=1)
    r = w.f.reshape(1, -1) - o.apply(u)
    assert o.relres(w.f, u)[0] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(w.f), rel=1e-13)
