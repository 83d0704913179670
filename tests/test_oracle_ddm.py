"""Pins of the oracle's Algorithm 3.1 (truncated additive overlapping DDM) and
its FGMRES driver (Sec. 4.2) to properties fixed by the paper and by the
mathematics, not by the oracle:

* one subdomain: step 1 is the global direct solve (eq. talg_1 with N = 1);
* light cone (Sec. 3.2, first paragraph; proof of Thm 2.4): with f supported in
  one core, the local solution of subdomain a is exactly zero at every step
  s <= |i - i0| + |j - j0| (+ |m - m0|), and non-zero on the front;
* discrete residual identity: for every step s and core node p of a,
  f - L_h u^(s) at p equals the sum of the transfers Psi_{b->a} of the latest
  local solutions with lags folded in (edge: uhat^s, corner: uhat^(s-1)+uhat^s;
  3D face/edge/vertex analogous).  It follows from Lemma 2.1's algebra applied
  to the discrete operators; a wrong chi, beta placement or lag breaks it;
* fixed point: run as an iterative solver the DDM converges to the global
  discrete solution for constant and layered media (2D and 3D);
* Theorem 3.4 trend: after N1+N2 steps the error in a constant medium falls
  as the PML gets stronger (exp(-k gamma0 sigma_bar / 2));
* FGMRES with K DDM steps converges to the global solution and counts
  n_Local_Solve = K n_GMRES_Iter, the identity every row of Tables 5/6 obeys.
"""
import math

import numpy as np
import pytest

import ddm_inputs as di
from oracle import Oracle


def _oracle(w):
    return Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)


def _core_view(o, a, packed, dim):
    sd = o.subdomain(a)
    lo, hi, clo, chi = sd["ext_lo"], sd["ext_hi"], sd["core_lo"], sd["core_hi"]
    n = [hi[d] - lo[d] + 1 for d in range(3)]
    box = packed[sd["off"]:sd["off"] + sd["n"]].reshape(n[2], n[1], n[0])
    return box[clo[2] - lo[2]:chi[2] - lo[2] + 1, clo[1] - lo[1]:chi[1] - lo[1] + 1,
               clo[0] - lo[0]:chi[0] - lo[0] + 1]


def _glob_core(o, a, glob, w):
    sd = o.subdomain(a)
    clo, chi = sd["core_lo"], sd["core_hi"]
    g = glob.reshape((1,) * (3 - w.dim) + w.grid_shape)
    off = [w.n_pml - 1 if d < w.dim else 0 for d in range(3)]
    return g[clo[2] + off[2]:chi[2] + off[2] + 1, clo[1] + off[1]:chi[1] + off[1] + 1,
             clo[0] + off[0]:chi[0] + off[0] + 1]


@pytest.mark.parametrize("dim", [2, 3])
def test_single_subdomain_step1_is_global_solve(dim):
    w = di.small_2d(M=24, N=(1, 1), n_pml=4) if dim == 2 else di.small_3d(M=8, N=(1, 1, 1), n_pml=3)
    o = _oracle(w)
    u, rr = o.ddm_run(w.f, 1)
    uref = o.global_solve(w.f).reshape(u.shape)
    np.testing.assert_allclose(u, uref, rtol=0, atol=1e-12 * np.abs(uref).max())
    assert rr[0, 0] < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_light_cone(dim):
    if dim == 2:
        w = di.small_2d(M=40, N=(4, 4), n_pml=3, n_ov=3)
        src_sub = (1, 2)
    else:
        w = di.small_3d(M=18, N=(3, 3, 3), n_pml=2, n_ov=2)
        src_sub = (0, 1, 2)
    o = _oracle(w)
    # delta shot inside the core of subdomain src_sub
    C = w.M[0] // w.N[0]
    node = tuple(src_sub[d] * C + C // 2 for d in range(dim))
    f = di.delta_shot(dim, w.M, w.n_pml, w.h, node)[None]
    nsub = o.nsub
    ids = [(a % w.N[0], (a // w.N[0]) % w.N[1], a // (w.N[0] * w.N[1])) for a in range(nsub)]
    dist = [sum(abs(ids[a][d] - src_sub[d]) for d in range(dim)) for a in range(nsub)]
    for s in range(1, max(dist) + 2):
        _, _, uhat, _, _ = o.ddm_run(f, s, want_relres=False, want_state=True)
        for a in range(nsub):
            sd = o.subdomain(a)
            blk = uhat[0, sd["off"]:sd["off"] + sd["n"]]
            if s <= dist[a]:
                assert np.all(blk == 0), (s, a, dist[a])
            elif s == dist[a] + 1:
                assert np.abs(blk).max() > 0, (s, a)


@pytest.mark.parametrize("case", ["2d-const", "2d-layered", "3d"])
def test_residual_identity_every_step(case):
    if case == "2d-const":
        w = di.small_2d(M=36, N=(3, 3), n_pml=3, n_ov=3, nrhs=2)
    elif case == "2d-layered":
        w = di.small_2d(M=36, N=(3, 3), n_pml=4, n_ov=4, layered=True, seed=7)
    else:
        w = di.small_3d(M=12, N=(2, 2, 2), n_pml=2, n_ov=2)
    o = _oracle(w)
    nrhs = w.nrhs
    hist = [np.zeros((nrhs, o.etot), dtype=np.complex128)] * 3
    for s in range(1, 7):
        u, _, uhat, _, _ = o.ddm_run(w.f, s, want_relres=False, want_state=True)
        hist = [uhat] + hist[:2]
        r = w.f.reshape(nrhs, -1) - o.apply(u)
        lag_sums = [hist[0], hist[0] + hist[1], hist[0] + hist[1] + hist[2]]
        t = o.transfer(lag_sums, nrhs)
        # roundoff floor: r is a difference of O(||f||) and O(|L_h| |u|) terms
        floor = 1e-13 * (np.abs(w.f).max() + 4 * w.dim / w.h ** 2 * np.abs(u).max())
        scale = np.abs(r).max()
        for rr in range(nrhs):
            for a in range(o.nsub):
                lhs = _glob_core(o, a, r[rr], w)
                rhs = _core_view(o, a, t[rr], w.dim)
                np.testing.assert_allclose(rhs, lhs, rtol=0, atol=1e-11 * scale + floor)


@pytest.mark.parametrize("case", ["2d-const", "2d-layered", "3d"])
def test_fixed_point_is_global_solution(case):
    if case == "2d-const":
        w = di.small_2d(M=48, N=(3, 3), n_pml=4, n_ov=3, nrhs=2)
        steps = 25
    elif case == "2d-layered":
        w = di.small_2d(M=48, N=(4, 4), n_pml=5, n_ov=4, layered=True, seed=5)
        steps = 120
    else:
        w = di.small_3d(M=12, N=(2, 2, 2), n_pml=3, n_ov=2)
        steps = 20
    o = _oracle(w)
    u, rr = o.ddm_run(w.f, steps)
    assert rr[-1].max() < 1e-12
    uref = o.global_solve(w.f).reshape(u.shape)
    err = np.linalg.norm(u - uref, axis=1) / np.linalg.norm(uref, axis=1)
    assert err.max() < 1e-10


def test_thm34_trend_stronger_pml_smaller_error():
    M = 48
    h = 1.0 / M
    k = 2 * math.pi / (10 * h)
    errs = []
    for n_pml in (3, 6, 12):
        k2 = di.constant_k2(2, (M, M), n_pml, k)
        f = di.gaussian_source(2, (M, M), n_pml, h, 1.0, (0.3, 0.4), 2 * h)[None]
        o = Oracle(2, (M, M), h, n_pml, 2.0, (3, 3), 3, k2)
        uref = o.global_solve(f).reshape(1, -1)
        u, _ = o.ddm_run(f, 6, want_relres=False)  # N1 + N2 steps
        errs.append(np.linalg.norm(u - uref) / np.linalg.norm(uref))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 1e-4


def test_fgmres_converges_and_counts_local_solves(golden):
    w = di.small_2d(M=48, N=(3, 3), n_pml=4, n_ov=3, layered=True, seed=8)
    o = _oracle(w)
    uref = o.global_solve(w.f).reshape(-1)
    for K in (1, 3, 6):
        x, its, rel = o.fgmres(w.f, K=K, restart=30, tol=1e-10, maxiter=200)
        assert rel <= 1e-10
        assert np.linalg.norm(x - uref) / np.linalg.norm(uref) < 1e-8
        assert its >= 1
    # the identity holds for every printed row of Tables 5 and 6
    for tab in ("table5_precond_constant", "table6_precond_layered"):
        t = golden[tab]
        for K, it, ls in zip(t["K"], t["n_gmres_iter"], t["n_local_solve"]):
            assert ls == K * it


def test_fgmres_unpreconditioned_matches_dense():
    w = di.small_2d(M=12, N=(1, 1), n_pml=3, n_ov=2)
    o = _oracle(w)
    uref = o.global_solve(w.f).reshape(-1)
    x, its, rel = o.fgmres(w.f, K=0, restart=40, tol=1e-11, maxiter=2000)
    assert rel <= 1e-11
    assert np.linalg.norm(x - uref) / np.linalg.norm(uref) < 1e-8


def test_subdomain_sizes_match_derived_layouts():
    """Per-axis subdomain sizes and the packed total for the configurations
    (interior / edge sizes differ: the global sides carry no overlap band)."""
    cases = [((80, 80), (2, 2), 10, 4, 15625), ((1024, 1024), (8, 8), 16, 8, 1896129)]
    for M, N, n_pml, n_ov, etot in cases:
        G = M[0] + 2 * n_pml - 1
        k2 = np.ones((G, G))
        o = Oracle(2, M, 1.0 / M[0], n_pml, 1.0, N, n_ov, k2)
        assert o.etot == etot
    o = Oracle(2, (80, 80), 1 / 80, 10, 1.0, (2, 2), 4, np.ones((99, 99)))
    assert [o.subdomain(a)["n"] for a in range(4)] == [62 * 62, 63 * 62, 62 * 63, 63 * 63]
