"""Edge and degenerate cases of the HIP path through the C-ABI:

* empty and oversized RHS batches are rejected (EINVAL) and leave the
  handle usable;
* a zero source: the stationary and FGMRES solves, FP64 and mixed, return
  u = 0 at once (relres is ||r|| when ||f|| = 0);
* one subdomain: the first DDM step is the global direct solve (eq. talg_1
  with N = 1), against the oracle's banded LU;
* the split substitution at its largest grid (8 x 8 subdomains: 256
  workgroups, one per CU, all resident) and on its largest blocks (255 and
  256 unknowns) against the oracle, and the one-workgroup variant as the
  default beyond the grid (9 x 9);
* the default substitution variant for block size and RHS count;
* grid rows wider than 256 nodes with a ragged last piece (the assembly
  gives every node a thread over 256-node row pieces): assembly and
  residual against the oracle.
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


def test_empty_and_oversized_batches_rejected():
    w = di.small_2d(M=64, N=(2, 2), n_pml=4, n_ov=3, nrhs=1)
    o, g = _pair(w, 2)
    try:
        empty = torch.zeros((0, g.etot), dtype=torch.complex128, device=DEV)
        with pytest.raises(ddm.DDMError) as e:
            g.local_solve(empty)
        assert e.value.code == ddm._ffi.DDM_EINVAL
        big = _t(di.random_field((3, g.etot), seed=90))
        with pytest.raises(ddm.DDMError) as e:
            g.local_solve(big)
        assert e.value.code == ddm._ffi.DDM_EINVAL
        gin = di.random_field((2, g.etot), seed=91)
        assert relerr(_n(g.local_solve(_t(gin))), o.local_solve(gin), axis=1) < 1e-10
    finally:
        g.close()


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("method", ["stationary", "fgmres"])
def test_zero_source_converges_at_once(method, mixed):
    w = di.small_2d(M=64, N=(2, 2), n_pml=4, n_ov=3, nrhs=2)
    o, g = _pair(w, 2, mixed=mixed)
    try:
        f = torch.zeros((2, g.nglob), dtype=torch.complex128, device=DEV)
        u, info, st = g.solve(f, method=method, tol=1e-8, maxiter=50)
        assert st == 0
        assert torch.count_nonzero(u).item() == 0
        assert all(x["relres"] == 0.0 for x in info)
    finally:
        g.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_single_subdomain_first_step_is_global_solve(dim):
    w = (di.small_2d(M=40, N=(1, 1), n_pml=5, nrhs=2) if dim == 2
         else di.small_3d(M=10, N=(1, 1, 1), n_pml=3, nrhs=1))
    o, g = _pair(w, w.nrhs)
    try:
        u, _ = g.iterate(_t(w.f.reshape(w.nrhs, -1)), 1)
        uref = o.global_solve(w.f).reshape(w.nrhs, -1)
        assert relerr(_n(u), uref, axis=1) < 1e-10
    finally:
        g.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_split_substitution_at_full_grid(mixed):
    w = di.small_2d(M=256, N=(8, 8), n_pml=4, n_ov=3, nrhs=3)
    o, g = _pair(w, 3, mixed=mixed)
    try:
        g.set_solve_variant("chain2")
        gin = di.random_field((3, o.etot), seed=92)
        x = _n(g.local_solve(_t(gin)))
        assert relerr(x, o.local_solve(gin), axis=1) < (5e-5 if mixed else 1e-10)
        if not mixed:
            uo, _ = o.ddm_run(w.f, 6)
            ug, _ = g.iterate(_t(w.f.reshape(w.nrhs, -1)), 6)
            assert relerr(_n(ug), uo, axis=1) < 1e-10
    finally:
        g.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_split_substitution_largest_blocks(mixed):
    """Blocks of 255 and 256 unknowns: four 64-row tiles, the largest blocks
    the split variant takes (128 partner rows per exchange); the odd complex64
    block is stored with a padded column stride.  Split and one-workgroup
    substitution against the oracle for 1 and 4 RHS; the split one is the
    default."""
    w = di.small_2d(M=474, N=(2, 2), n_pml=8, n_ov=4, nrhs=1)
    o, g = _pair(w, 4, mixed=mixed)
    try:
        assert g.solve_variant() == "chain2"
        tol = 5e-5 if mixed else 1e-10
        for nrhs in (1, 4):
            gin = di.random_field((nrhs, o.etot), seed=96 + nrhs)
            xo = o.local_solve(gin)
            for v in ("chain2", "chain"):
                g.set_solve_variant(v)
                assert relerr(_n(g.local_solve(_t(gin))), xo, axis=1) < tol, (v, nrhs)
    finally:
        g.close()


def test_beyond_full_grid_uses_one_workgroup_per_chain():
    w = di.small_2d(M=288, N=(9, 9), n_pml=4, n_ov=3, nrhs=2)
    o, g = _pair(w, 2)
    try:
        assert g.solve_variant() == "chain"
        with pytest.raises(ddm.DDMError):
            g.set_solve_variant("chain2")
        gin = di.random_field((2, o.etot), seed=93)
        assert relerr(_n(g.local_solve(_t(gin))), o.local_solve(gin), axis=1) < 1e-10
    finally:
        g.close()


def test_default_variant_choice():
    """Defaults: split chains for at most 4 RHS on blocks of >= 128 unknowns,
    one workgroup per chain for small blocks and 5-7 RHS, the matrix-core
    kernel from 8 RHS on."""
    cases = [(di.small_2d(M=256, N=(2, 2), n_pml=8, n_ov=4, nrhs=1), 2, "chain2"),
             (di.small_2d(M=256, N=(2, 2), n_pml=8, n_ov=4, nrhs=1), 6, "chain"),
             (di.small_2d(M=256, N=(2, 2), n_pml=8, n_ov=4, nrhs=1), 8, "mma"),
             (di.small_2d(M=64, N=(2, 2), n_pml=4, n_ov=3, nrhs=1), 16, "mma"),
             (di.small_2d(M=64, N=(2, 2), n_pml=4, n_ov=3, nrhs=1), 2, "chain")]
    for w, nrhs_max, want in cases:
        o, g = _pair(w, nrhs_max)
        try:
            assert g.solve_variant() == want, (w.name, nrhs_max)
            gin = di.random_field((1, o.etot), seed=94)
            assert relerr(_n(g.local_solve(_t(gin))), o.local_solve(gin), axis=1) < 1e-10
        finally:
            g.close()


@pytest.mark.parametrize("M,N", [(300, (2, 2)), (520, (4, 2))])
def test_assembly_and_residual_on_rows_wider_than_256(M, N):
    """Rows of 311 and 531 nodes: 2 and 3 row pieces, the last one ragged
    (55 and 19 nodes). Assembly (1e-14) and residual with its norms (1e-13)
    against the oracle, as on the narrower grids."""
    w = di.small_2d(M=M, N=N, n_pml=6, n_ov=4, nrhs=2, seed=7)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    G0 = int(round(o.nglob ** 0.5))
    assert G0 * G0 == o.nglob and G0 > 256 and G0 % 256 != 0
    g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w), _t(w.k2.reshape(-1)), 3)
    try:
        U = di.random_field((3, o.etot), seed=31)
        assert relerr(_n(g.assemble(_t(U))), o.assemble(U)) < 1e-14
        u = di.random_field((3, o.nglob), seed=32)
        f = di.random_field((3, o.nglob), seed=33)
        r, rn, fn = g.residual(_t(f), _t(u))
        ro = f - o.apply(u)
        assert relerr(_n(r), ro) < 1e-13
        np.testing.assert_allclose(np.sqrt(rn), np.linalg.norm(ro, axis=1), rtol=1e-13)
        np.testing.assert_allclose(np.sqrt(fn), np.linalg.norm(f, axis=1), rtol=1e-13)
    finally:
        g.close()
