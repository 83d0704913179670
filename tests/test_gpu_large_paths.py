"""GPU parity on the code paths the largest workloads take, against the CPU
oracle through the C-ABI:

* the one-directional factor layout (every subdomain eliminated from its
  first block on, as with more subdomains than the twisted layout can keep
  co-resident, e.g. 16 x 16) with 16 and 20 right-hand sides: the 16-RHS
  substitution tiles (and a ragged second tile of 4) of the vector chain
  kernel and of the matrix-core kernel, in FP64 and complex64, local solves
  and six DDM steps (Algorithm 3.1);
* FGMRES(30) preconditioned by K DDM steps (Sec. 4.2.2) in 3D and with
  K = 1 and K = 2, FP64 and mixed, against the oracle's global solve, with
  n_Local_Solve = K n_GMRES_Iter (the identity of Tables 5 and 6).

Tolerances: FP64 local solves and iterates 1e-10; complex64 local solves
and iterates 5e-5 (c64 roundoff times the local condition number); FGMRES
solutions 1e-8 (FP64) and 1e-7 (mixed: the FP64 outer iteration corrects
the complex64 preconditioner) after relres 1e-10.
"""
import numpy as np
import pytest
import torch

import ddm_inputs as di
from oracle import Oracle
import paper_1807_04180_amd as ddm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _n(t):
    return t.detach().cpu().numpy()


def relerr(a, b, axis=None):
    a = np.asarray(a).reshape(b.shape)
    return np.max(np.linalg.norm(a - b, axis=axis) / np.maximum(np.linalg.norm(b, axis=axis), 1e-300))


def _pair(w, nrhs_max, mixed=False):
    print("case", w.name, w.N, "nrhs_max", nrhs_max, "mixed", mixed, flush=True)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), _t(w.k2.reshape(-1)), nrhs_max)
    return o, g


# blocks of 75-98 (3x3 layered: two 64-row tiles, ragged) and 146 unknowns
# (2x2: three tiles); odd and even block sizes
ONEDIR = {
    "3x3-layered": lambda n: di.small_2d(M=192, N=(3, 3), n_pml=7, n_ov=5, nrhs=n, layered=True, seed=4),
    "2x2-146": lambda n: di.small_2d(M=256, N=(2, 2), n_pml=8, n_ov=4, nrhs=n, seed=6),
}


@pytest.mark.parametrize("variant", ["chain", "mma"])
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("case", sorted(ONEDIR))
def test_onedir_16_and_20_rhs(case, mixed, variant):
    w = ONEDIR[case](20)
    o, g = _pair(w, 20, mixed=mixed)
    tol = 5e-5 if mixed else 1e-10
    try:
        g.set_factor_layout(False)
        assert g.solve_variant() == "mma", g.solve_variant()   # the default from 8 RHS on
        g.set_solve_variant(variant)
        for nrhs in (16, 20):
            gin = di.random_field((nrhs, o.etot), seed=300 + nrhs)
            xg = _n(g.local_solve(_t(gin)))
            assert relerr(xg, o.local_solve(gin), axis=1) < tol, nrhs
            # repeatable, and a RHS gives the same bits in either batch
            assert np.array_equal(_n(g.local_solve(_t(gin))), xg)
            if nrhs == 20:
                x16 = _n(g.local_solve(_t(gin[4:20])))
                assert np.array_equal(x16, xg[4:20])
        for nrhs in (16, 20):
            f = w.f[:nrhs]
            uo, _ = o.ddm_run(f, 6)
            ug, _ = g.iterate(_t(f.reshape(nrhs, -1)), 6)
            assert relerr(_n(ug), uo.reshape(nrhs, -1), axis=1) < tol, nrhs
    finally:
        g.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_fgmres_3d_matches_global_solve(mixed):
    w = di.small_3d(M=16, N=(2, 2, 2), n_pml=3, n_ov=2, nrhs=2, seed=1)
    o, g = _pair(w, w.nrhs, mixed=mixed)
    try:
        f = _t(w.f.reshape(w.nrhs, -1))
        u, info, st = g.solve(f, method="fgmres", tol=1e-10, maxiter=100, restart=30)
        assert st == 0, info
        uref = o.global_solve(w.f).reshape(w.nrhs, -1)
        assert relerr(_n(u), uref, axis=1) < (1e-7 if mixed else 1e-8)
        K = sum(w.N)
        assert all(i["local_solves"] == K * i["iters"] for i in info), info
    finally:
        g.close()


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("K", [1, 2, 3])
def test_fgmres_small_K(K, mixed):
    w = di.small_2d(M=192, N=(3, 3), n_pml=7, n_ov=5, nrhs=3, layered=True, seed=4)
    o, g = _pair(w, w.nrhs, mixed=mixed)
    try:
        f = _t(w.f.reshape(w.nrhs, -1))
        u, info, st = g.solve(f, method="fgmres", tol=1e-10, maxiter=300, restart=30, K=K)
        assert st == 0, info
        uref = o.global_solve(w.f).reshape(w.nrhs, -1)
        assert relerr(_n(u), uref, axis=1) < (1e-7 if mixed else 1e-8)
        assert all(i["local_solves"] == K * i["iters"] for i in info), info
        # fewer DDM steps per application need more Arnoldi steps
        assert all(i["iters"] > 2 for i in info), info
    finally:
        g.close()


# the matrix-core substitution: block sizes 1-3 row tiles of 16 with ragged
# last tiles and odd and even widths (column groups of 8 / 4 with padding);
# 3D planes of 49-100 unknowns; both layouts
MMA_CASES = {
    "2d-3x3-layered": lambda n: di.small_2d(M=192, N=(3, 3), n_pml=7, n_ov=5, nrhs=n, layered=True, seed=4),
    "2d-2x2-small": lambda n: di.small_2d(M=40, N=(2, 2), n_pml=3, n_ov=2, nrhs=n, seed=7),
    "3d-2x2x2": lambda n: di.small_3d(M=16, N=(2, 2, 2), n_pml=3, n_ov=2, nrhs=n, seed=1),
}


@pytest.mark.parametrize("twisted", [True, False])
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("case", sorted(MMA_CASES))
def test_mma_substitution(case, mixed, twisted):
    w = MMA_CASES[case](20)
    o, g = _pair(w, 20, mixed=mixed)
    tol = 5e-5 if mixed else 1e-10
    try:
        g.set_factor_layout(twisted)
        g.set_solve_variant("mma")
        for nrhs in (1, 5, 16, 20):
            gin = di.random_field((nrhs, o.etot), seed=400 + nrhs)
            xg = _n(g.local_solve(_t(gin)))
            assert relerr(xg, o.local_solve(gin), axis=1) < tol, nrhs
            assert np.array_equal(_n(g.local_solve(_t(gin))), xg), nrhs
            # a right-hand side gives the same bits alone and in any position
            assert np.array_equal(_n(g.local_solve(_t(gin[-1:])))[0], xg[-1]), nrhs
        f = w.f[:16]
        uo, _ = o.ddm_run(f, 6)
        ug, _ = g.iterate(_t(f.reshape(16, -1)), 6)
        assert relerr(_n(ug), uo.reshape(16, -1), axis=1) < tol
    finally:
        g.close()


@pytest.mark.parametrize("twisted", [True, False])
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("case", ["2d-2x2-small", "3d-2x2x2"])
def test_mma_parallel_rhs_tiles(case, mixed, twisted):
    """48 RHS on a 48-RHS handle: three 16-RHS tiles run side by side (grid
    rows with their own meeting flags), 40 RHS: a ragged third tile.  Each
    tile gives the same bits as when solved alone, and the oracle's values."""
    w = MMA_CASES[case](1)
    o, g = _pair(w, 48, mixed=mixed)
    tol = 5e-5 if mixed else 1e-10
    try:
        g.set_factor_layout(twisted)
        g.set_solve_variant("mma")
        for nrhs in (48, 40):
            gin = di.random_field((nrhs, o.etot), seed=420 + nrhs)
            xg = _n(g.local_solve(_t(gin)))
            assert relerr(xg, o.local_solve(gin), axis=1) < tol, nrhs
            for t0 in range(0, nrhs, 16):
                part = _n(g.local_solve(_t(gin[t0:t0 + 16])))
                assert np.array_equal(part, xg[t0:t0 + 16]), (nrhs, t0)
    finally:
        g.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_mma_largest_blocks(mixed):
    """Blocks of 255 and 256 unknowns (16 row tiles: 1024-thread workgroups,
    the widest the kernel takes) against the oracle, and a switch back to the
    vector kernel (the factorisation re-runs in column-major order)."""
    w = di.small_2d(M=474, N=(2, 2), n_pml=8, n_ov=4, nrhs=1)
    o, g = _pair(w, 16, mixed=mixed)
    tol = 5e-5 if mixed else 1e-10
    try:
        assert g.solve_variant() == "mma"
        gin = di.random_field((16, o.etot), seed=410)
        xo = o.local_solve(gin)
        assert relerr(_n(g.local_solve(_t(gin))), xo, axis=1) < tol
        g.set_solve_variant("chain")
        assert relerr(_n(g.local_solve(_t(gin))), xo, axis=1) < tol
        g.set_solve_variant("mma")
        assert relerr(_n(g.local_solve(_t(gin))), xo, axis=1) < tol
    finally:
        g.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_mma_stationary_and_fgmres(mixed):
    w = di.small_2d(M=192, N=(3, 3), n_pml=7, n_ov=5, nrhs=8, layered=True, seed=4)
    o, g = _pair(w, 8, mixed=mixed)
    try:
        assert g.solve_variant() == "mma"
        uref = o.global_solve(w.f).reshape(8, -1)
        f = _t(w.f.reshape(8, -1))
        for method in ("stationary", "fgmres"):
            u, info, st = g.solve(f, method=method, tol=1e-10, maxiter=400)
            assert st == 0, (method, info)
            assert relerr(_n(u), uref, axis=1) < (1e-7 if mixed else 1e-8), method
    finally:
        g.close()
