"""Pins of the oracle's discrete operator L_h (Sec. 3.1 eq. PMLweak0, Sec. 4
5/7-point scheme) to facts that do not come from the oracle itself.

* Without PML (sigma0 = 0) the 5/7-point Dirichlet Laplacian has the closed-form
  eigenpairs sin(p pi i/(G+1)) ... with eigenvalue -(4/h^2) sum sin^2(p pi/(2(G+1))):
  pins the stencil weights, the h^2 scaling, the Dirichlet ends and the k^2 term.
* J L_h (J = alpha_x alpha_y (alpha_z) at the node) is complex symmetric, as the
  discretisation of the symmetric form (A grad u, grad v) - k^2 (J u, v) of
  eq. PMLweak must be: pins the node / half-node placement of alpha.
* Constant medium, unit-mass Gaussian source: outside the source the free-space
  solution is -(i/4) exp(-k^2 s^2/2) H0^(1)(k r) (fundamental solution of
  Sec. 2.1 plus Graf's addition theorem); the PML-truncated discrete solution
  matches it on an annulus, with error ratio 4 per mesh halving (the second
  order rate printed in Table 1).  A flipped PML sign (alpha = 1 - i sigma)
  fails this by two orders of magnitude.
"""
import math

import numpy as np
import pytest

import ddm_inputs as di
from oracle import Oracle


def _dense(o, n):
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        A[:, j] = o.apply(e).reshape(-1)
    return A


@pytest.mark.parametrize("dim", [2, 3])
def test_dirichlet_eigenpairs(dim):
    M, n_pml = (10, 3) if dim == 2 else (6, 2)
    h = 1.0 / M
    k = 7.0
    shape = tuple([M + 2 * n_pml - 1] * dim)
    k2 = np.full(shape, k * k)
    o = Oracle(dim, (M,) * dim, h, n_pml, 0.0, (1,) * dim, 2, k2)
    G = M + 2 * n_pml - 1
    idx = np.arange(1, G + 1)
    rng = np.random.default_rng(5)
    for _ in range(4):
        modes = rng.integers(1, G + 1, size=dim)
        vecs = [np.sin(p * math.pi * idx / (G + 1)) for p in modes]
        u = vecs[0]
        for v in vecs[1:]:
            u = np.multiply.outer(v, u)  # C order: last axis = x
        lam = sum(4.0 / h ** 2 * math.sin(p * math.pi / (2 * (G + 1))) ** 2 for p in modes)
        Lu = o.apply(u.astype(np.complex128)).reshape(u.shape)
        np.testing.assert_allclose(Lu, (k * k - lam) * u, rtol=0, atol=1e-11 * np.abs(lam))


def _alpha_nodes(o, dim, G, a=None):
    axes = []
    for ax in range(dim):
        g = np.arange(G[ax]) - o.n_pml + 1 if a is None else None
        axes.append(g)
    return axes


@pytest.mark.parametrize("dim", [2, 3])
def test_pml_operator_complex_symmetric(dim):
    M, n_pml = (8, 4) if dim == 2 else (4, 3)
    h = 1.0 / M
    G = M + 2 * n_pml - 1
    rng = np.random.default_rng(11)
    k2 = rng.uniform(20, 60, size=(G,) * dim)
    o = Oracle(dim, (M,) * dim, h, n_pml, 2.5, (1,) * dim, 2, k2)
    n = G ** dim
    A = _dense(o, n)
    g = np.arange(G) - n_pml + 1
    alpha = [1 + 1j * np.array([o.sigma_global(ax, x) for x in g]) for ax in range(dim)]
    J = alpha[0]
    for ax in range(1, dim):
        J = np.multiply.outer(alpha[ax], J)
    JA = J.reshape(-1)[:, None] * A
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()   # L_h itself is not symmetric
    np.testing.assert_allclose(JA, JA.T, rtol=0, atol=1e-12 * np.abs(JA).max())


def test_subdomain_operator_complex_symmetric():
    w = di.small_2d(M=24, N=(2, 2), n_pml=3, n_ov=3, layered=True, seed=3)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    for a in range(o.nsub):
        sd = o.subdomain(a)
        lo, hi = sd["ext_lo"], sd["ext_hi"]
        nx, ny = hi[0] - lo[0] + 1, hi[1] - lo[1] + 1
        n = nx * ny
        A = np.empty((n, n), dtype=np.complex128)
        e = np.zeros(n, dtype=np.complex128)
        for j in range(n):
            e[:] = 0
            e[j] = 1
            A[:, j] = o.apply_local(a, e)
        ax_ = 1 + 1j * np.array([o.sigma_local(a, 0, x) for x in range(lo[0], hi[0] + 1)])
        ay_ = 1 + 1j * np.array([o.sigma_local(a, 1, y) for y in range(lo[1], hi[1] + 1)])
        J = np.multiply.outer(ay_, ax_).reshape(-1)
        JA = J[:, None] * A
        np.testing.assert_allclose(JA, JA.T, rtol=0, atol=1e-12 * np.abs(JA).max())


def test_sigma_profiles():
    """Quadratic profile sigma0 (t/n_pml)^2 outside the physical box; the
    subdomain profile is zero on the n_ov overlap cells of an interior side
    (the shifted profile of eq. PMLprofile) and reaches sigma0 at its Dirichlet
    node."""
    w = di.small_2d(M=24, N=(2, 2), n_pml=4, n_ov=3)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    s0 = w.sigma0
    assert o.sigma_global(0, 0.0) == 0.0 and o.sigma_global(0, 24.0) == 0.0
    assert o.sigma_global(0, 12.5) == 0.0
    assert o.sigma_global(0, -4.0) == pytest.approx(s0)
    assert o.sigma_global(0, 26.0) == pytest.approx(s0 * 0.25)
    # subdomain 0: core x in [-3, 11], interior side at the right
    sd = o.subdomain(0)
    assert sd["core_hi"][0] == 11 and sd["ext_hi"][0] == 11 + 3 + 4 - 1
    for m in [0.5, 1, 2, 3]:
        assert o.sigma_local(0, 0, 11 + m) == 0.0
    assert o.sigma_local(0, 0, 11 + 3 + 4) == pytest.approx(s0)
    assert o.sigma_local(0, 0, 11 + 3 + 2) == pytest.approx(s0 * 0.25)
    assert o.sigma_local(0, 0, -3.5) == pytest.approx(o.sigma_global(0, -3.5))


def test_cutoff_beta0_properties():
    """beta0 of Sec. 2.2: 1 for t <= 0, 0 for t >= 1, monotone, C^2."""
    b = Oracle.beta0
    assert b(-0.3) == 1.0 and b(0.0) == 1.0 and b(1.0) == 0.0 and b(1.7) == 0.0
    t = np.linspace(0, 1, 2001)
    v = np.array([b(x) for x in t])
    assert np.all(np.diff(v) <= 1e-15)
    eps = 1e-4
    for t0 in (0.0, 1.0):
        d1 = (b(t0 + eps) - b(t0 - eps)) / (2 * eps)
        d2 = (b(t0 + eps) - 2 * b(t0) + b(t0 - eps)) / eps ** 2
        assert abs(d1) < 1e-6 and abs(d2) < 1e-2
    assert b(0.5) == pytest.approx(0.5)


def _hankel_error(M, sign=1.0):
    from scipy.special import hankel1
    k = 2 * math.pi * 2
    s = 0.05
    c0 = (0.5, 0.5)
    h = 1.0 / M
    n_pml = M // 4
    s0 = sign * di.sigma0_for_reflection(1e-8, k, n_pml * h)
    k2 = di.constant_k2(2, (M, M), n_pml, k)
    f = di.gaussian_source(2, (M, M), n_pml, h, 1.0, c0, s)
    o = Oracle(2, (M, M), h, n_pml, s0, (1, 1), 2, k2)
    u = o.global_solve(f).reshape(f.shape)
    x = di.node_coords(M, n_pml, h)
    X, Y = np.meshgrid(x, x, indexing="xy")
    r = np.hypot(X - c0[0], Y - c0[1])
    ann = (r >= 0.25) & (r <= 0.45)
    ue = -0.25j * math.exp(-k * k * s * s / 2) * hankel1(0, k * r[ann])
    return np.linalg.norm(u[ann] - ue) / np.linalg.norm(ue)


def test_point_source_matches_hankel_second_order():
    errs = [_hankel_error(M) for M in (24, 48, 96)]
    assert errs[2] < 5e-3
    for e0, e1 in zip(errs[:-1], errs[1:]):
        assert 3.6 < e0 / e1 < 4.4, errs   # rate 2.0 +- 0.15 (Table 1)


def test_flipped_pml_sign_fails_hankel():
    assert _hankel_error(48, sign=-1.0) > 0.5


@pytest.mark.parametrize("R,layered", [(1e-6, False), (1e-8, True), (1e-3, False)])
def test_sigma0_from_reflection_damps_round_trip_by_R(R, layered):
    """PML strength for a target reflection R (the round-trip reading of the
    sigma~ the paper leaves open, Sec. 2.1): integrate the oracle's own global
    profile across the layer (scipy quadrature of sigma_global over the PML
    cells) and check that a wave of the smallest wave number of the medium,
    crossing the layer twice, is damped by exactly R."""
    from scipy.integrate import quad
    w = di.small_2d(M=32, N=(2, 2), n_pml=5, n_ov=3, layered=layered, seed=3)
    s0 = Oracle.sigma0_for_reflection(R, w.k2, w.n_pml, w.h)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, s0, w.N, w.n_ov, w.k2)
    k_ref = np.sqrt(w.k2.min())
    for lo, hi in ((w.M[0], w.M[0] + w.n_pml), (-w.n_pml, 0)):
        cells, _ = quad(lambda x: o.sigma_global(0, x), lo, hi, epsabs=0, epsrel=1e-13)
        damping = np.exp(-2.0 * k_ref * w.h * cells)
        assert damping == pytest.approx(R, rel=1e-10)
