"""Pins of the accuracy study's yardstick (Sec. 4.1, Tables 1-2): the exact
free-space solutions of the paper's 2D and 3D Gaussian sources, their
gradients, and the discrete L2/H1 error norms the study reports.

* The exact solution is a sum of two Gauss-Legendre quadratures inside the
  source and a closed form outside it: the two branches agree where they
  meet, and the quadrature branch satisfies Laplace(u) + k^2 u = f (checked
  with a fine five-point stencil, which shares nothing with the quadrature).
* The same for the 3D solution (seven-point stencil).
* The returned gradients match central differences of u.
* The oracle's discrete solution of a smaller-k copy of the experiment
  (k/2pi = 5, same points per wavelength, same source shape and PML width in
  cells per wavelength) converges to it at the second order printed in
  Table 1, in both norms.
* On the GPU (tests/test_gpu_parity.py) the DDM solution of the 560^2 mesh
  itself lands on Table 1's L2 error.
"""
import math

import numpy as np
import pytest

import bench
import ddm_inputs as di
from oracle import Oracle

K25 = 2 * math.pi * 25


def _source(x, y, k, c0):
    a = (4 * k / math.pi) ** 2
    X, Y = np.meshgrid(np.asarray(x) - c0[0], np.asarray(y) - c0[1], indexing="xy")
    return 16 * k * k / math.pi ** 3 * np.exp(-a * (X * X + Y * Y))


def test_exact_solution_branches_meet_at_the_source_edge():
    k = K25
    c0 = (0.3, 0.4)
    R = math.sqrt(40.0) / (4 * k / math.pi)
    xs = np.array([c0[0] + R * (1 - 1e-13), c0[0] + R * (1 + 1e-13)])
    u, ux, uy = bench.gaussian_free_space_2d(xs, [c0[1]], k, c0)
    assert abs(u[0, 0] - u[0, 1]) < 1e-10 * abs(u[0, 0])
    assert abs(ux[0, 0] - ux[0, 1]) < 1e-10 * abs(ux[0, 0])
    assert abs(uy[0, 0]) < 1e-12 * abs(ux[0, 0]) + 1e-300


@pytest.mark.parametrize("frac", [0.05, 0.2, 0.5, 0.9, 1.5])
def test_exact_solution_satisfies_helmholtz(frac):
    k = K25
    c0 = (0.0, 0.0)
    a = (4 * k / math.pi) ** 2
    R = math.sqrt(40.0 / a)
    p = (frac * R * math.cos(0.7), frac * R * math.sin(0.7))
    d = 1e-3 / math.sqrt(a)
    x = p[0] + d * np.arange(-1, 2)
    y = p[1] + d * np.arange(-1, 2)
    u = bench.gaussian_free_space_2d(x, y, k, c0)[0]
    lap = (u[1, 0] + u[1, 2] + u[0, 1] + u[2, 1] - 4 * u[1, 1]) / (d * d)
    f = _source([p[0]], [p[1]], k, c0)[0, 0]
    res = lap + k * k * u[1, 1] - f
    # O(d^2) stencil error and rounding of the 1/d^2 difference
    assert abs(res) < 1e-5 * (k * k * abs(u[1, 1]) + abs(f)), (frac, res, f)


def test_exact_gradient_matches_differences():
    k = K25
    c0 = (0.0, 0.0)
    d = 1e-7
    for p in ((0.004, 0.003), (0.02, -0.011), (0.2, 0.1)):
        u, ux, uy = bench.gaussian_free_space_2d([p[0]], [p[1]], k, c0)
        up = bench.gaussian_free_space_2d([p[0] - d, p[0] + d], [p[1]], k, c0)[0]
        vp = bench.gaussian_free_space_2d([p[0]], [p[1] - d, p[1] + d], k, c0)[0]
        gx = (up[0, 1] - up[0, 0]) / (2 * d)
        gy = (vp[1, 0] - vp[0, 0]) / (2 * d)
        assert abs(gx - ux[0, 0]) < 1e-6 * abs(ux[0, 0])
        assert abs(gy - uy[0, 0]) < 1e-6 * abs(uy[0, 0])


def _small_copy_errors(scale):
    # the Table 1 setting at k/2pi = 5: 112 cells per unit length at scale 1
    # (22.4 per wavelength, as 560 at k/2pi = 25), 100 physical cells, PML 6
    k = 2 * math.pi * 5
    M = 100 * scale
    L = 100 / 112
    h = L / M
    n_pml = 6 * scale
    c0 = (L / 2 + 0.09, L / 2 + 0.05)
    s0 = di.sigma0_for_reflection(1e-8, k, n_pml * h)
    k2 = di.constant_k2(2, (M, M), n_pml, k)
    f = di.paper_gaussian_source(2, (M, M), n_pml, h, L, c0, k)
    u = Oracle(2, (M, M), h, n_pml, s0, (1, 1), 2, k2).global_solve(f).reshape(f.shape)
    return bench.l2_h1_errors(u, di.node_coords(M, n_pml, h), h, L, k, c0)


def test_discrete_solution_converges_at_second_order():
    (l2a, h1a), (l2b, h1b) = _small_copy_errors(1), _small_copy_errors(2)
    assert 3.7 < l2a / l2b < 4.3, (l2a, l2b)
    assert 3.7 < h1a / h1b < 4.3, (h1a, h1b)
    assert l2b < 1e-3


def test_error_norms_on_exact_data_vanish():
    k = K25
    c0 = (0.45, 0.5)
    M, n_pml = 40, 3
    L = 0.9
    h = L / M
    x = di.node_coords(M, n_pml, h)
    u = bench.gaussian_free_space_2d(x, x, k, c0)[0]
    l2, h1 = bench.l2_h1_errors(u, x, h, L, k, c0)
    assert l2 == 0.0
    assert h1 > 0.0   # difference quotients differ from exact derivatives
    # a constant shift e on the (M + 1)^2 physical nodes: L2 error h |e| (M + 1)
    l2s, _ = bench.l2_h1_errors(u + 1e-3, x, h, L, k, c0)
    assert abs(l2s - 1e-3 * h * (M + 1)) < 1e-12


def test_paper_accuracy_recipe(golden):
    t = golden["table1_2d_convergence"]
    for scale in (1, 2):
        w = di.paper_accuracy_2d(scale)
        assert w.M[0] + 2 * w.n_pml == t["mesh"][scale - 1]
        assert w.M[0] // w.N[0] == t["local_size_without_pml"][scale - 1]
        assert abs(w.n_pml * w.h - 3.0 / 56.0) < 1e-12
        assert abs(w.omega / (2 * math.pi) - 25) < 1e-12
        # unit-mass source, all of it inside the physical box
        assert abs(w.f.real.sum() * w.h ** 2 - 1) < 1e-9


def test_paper_accuracy_3d_recipe(golden):
    t = golden["table2_3d_convergence"]
    for mesh, core in zip(t["mesh"][:2], t["local_size_without_pml"][:2]):
        w = di.paper_accuracy_3d(mesh)
        assert w.M[0] + 2 * w.n_pml == mesh and w.M[0] // w.N[0] == core
        assert abs(w.n_pml * w.h - 1.0 / 8.0) < 1e-12
        assert abs(w.f.real.sum() * w.h ** 3 - 1) < 1e-4   # unit mass, sampled at ~1 node per e-fold


K10 = 2 * math.pi * 10


def _source3(p, k):
    a = (4 * k / math.pi) ** 2
    return 64 * k ** 3 / math.pi ** 4.5 * math.exp(-a * sum(c * c for c in p))


def test_exact_3d_branches_meet_at_the_source_edge():
    k = K10
    c0 = (0.3, 0.4, 0.2)
    R = math.sqrt(40.0) / (4 * k / math.pi)
    xs = np.array([c0[0] + R * (1 - 1e-13), c0[0] + R * (1 + 1e-13)])
    u, ux, uy, uz = bench.gaussian_free_space_3d(xs, [c0[1]], [c0[2]], k, c0)
    assert abs(u[0, 0, 0] - u[0, 0, 1]) < 1e-10 * abs(u[0, 0, 0])
    assert abs(ux[0, 0, 0] - ux[0, 0, 1]) < 1e-10 * abs(ux[0, 0, 0])


@pytest.mark.parametrize("frac", [0.05, 0.3, 0.8, 1.4])
def test_exact_3d_solution_satisfies_helmholtz(frac):
    k = K10
    c0 = (0.0, 0.0, 0.0)
    a = (4 * k / math.pi) ** 2
    R = math.sqrt(40.0 / a)
    p = frac * R * np.array([0.48, 0.6, 0.64])
    d = 1e-3 / math.sqrt(a)
    x, y, z = (p[i] + d * np.arange(-1, 2) for i in range(3))
    u = bench.gaussian_free_space_3d(x, y, z, k, c0)[0]
    lap = (u[1, 1, 0] + u[1, 1, 2] + u[1, 0, 1] + u[1, 2, 1] + u[0, 1, 1] + u[2, 1, 1] - 6 * u[1, 1, 1]) / (d * d)
    f = _source3(p, k)
    res = lap + k * k * u[1, 1, 1] - f
    assert abs(res) < 1e-5 * (k * k * abs(u[1, 1, 1]) + abs(f)), (frac, res, f)


def test_exact_3d_gradient_matches_differences():
    k = K10
    c0 = (0.0, 0.0, 0.0)
    d = 1e-7
    for p in ((0.01, 0.007, -0.004), (0.05, -0.02, 0.03), (0.3, 0.1, 0.2)):
        g = bench.gaussian_free_space_3d([p[0]], [p[1]], [p[2]], k, c0)
        for ax in range(3):
            lo, hi = list(p), list(p)
            lo[ax] -= d
            hi[ax] += d
            ul = bench.gaussian_free_space_3d([lo[0]], [lo[1]], [lo[2]], k, c0)[0][0, 0, 0]
            uh = bench.gaussian_free_space_3d([hi[0]], [hi[1]], [hi[2]], k, c0)[0][0, 0, 0]
            assert abs((uh - ul) / (2 * d) - g[1 + ax][0, 0, 0]) < 1e-6 * abs(g[1 + ax][0, 0, 0])


def _probe_operator_3d(o, G):
    """The oracle's 7-point operator as a sparse matrix, read column by column
    from its apply: unit vectors on the nodes of one of 27 colour classes
    (nodes 3 apart on every axis) have disjoint stencils."""
    import scipy.sparse as sp
    idx = np.arange(G ** 3).reshape(G, G, G)
    rows, cols, vals = [], [], []
    for c in range(27):
        mask = np.zeros((G, G, G), bool)
        mask[c // 9::3, (c // 3) % 3::3, c % 3::3] = True
        y = o.apply(mask.reshape(1, -1).astype(np.complex128)).reshape(G, G, G)
        zz, yy, xx = np.nonzero(mask)
        for dz, dy, dx in ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            z2, y2, x2 = zz + dz, yy + dy, xx + dx
            ok = (z2 >= 0) & (z2 < G) & (y2 >= 0) & (y2 < G) & (x2 >= 0) & (x2 < G)
            rows.append(idx[z2[ok], y2[ok], x2[ok]])
            cols.append(idx[zz[ok], yy[ok], xx[ok]])
            vals.append(y[z2[ok], y2[ok], x2[ok]])
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(G ** 3, G ** 3))


def _small_copy_errors_3d(M, n_pml):
    # Table 2's setting shrunk: k/2pi = 2 on a box of L = 1/2 (one wavelength)
    # with a PML of n_pml cells, the paper's 3D Gaussian (Sec. 4.1.2) off
    # centre, sigma0 for a reflection of 1e-8
    import scipy.sparse.linalg as spl
    k = 2 * math.pi * 2
    L = 0.5
    h = L / M
    c0 = (L / 2 + 0.03, L / 2 - 0.02, L / 2 + 0.01)
    k2 = di.constant_k2(3, (M, M, M), n_pml, k)
    s0 = Oracle.sigma0_for_reflection(1e-8, k2, n_pml, h)
    f = di.paper_gaussian_source(3, (M, M, M), n_pml, h, L, c0, k).reshape(-1)
    o = Oracle(3, (M, M, M), h, n_pml, s0, (1, 1, 1), 2, k2)
    G = M + 2 * n_pml - 1
    u = spl.spsolve(_probe_operator_3d(o, G), f)
    # the probed matrix is the oracle's operator: its solution zeroes the
    # oracle's own residual
    assert o.relres(f.reshape(1, -1), u.reshape(1, -1))[0] < 1e-12
    return bench.l2_h1_errors(u.reshape(G, G, G), di.node_coords(M, n_pml, h), h, L, k, c0)


def test_discrete_3d_solution_converges_at_second_order():
    """The 3D twin of the 2D rate pin: the oracle's seven-point PML solution
    of the paper's 3D Gaussian source converges to the exact free-space
    solution at the second order printed in Table 2 (meshes of 12 and 18
    cells with a PML of fixed width: error ratio 1.5^2 = 2.25, order 2)."""
    (l2a, h1a), (l2b, h1b) = _small_copy_errors_3d(12, 4), _small_copy_errors_3d(18, 6)
    for a, b in ((l2a, l2b), (h1a, h1b)):
        order = math.log(a / b) / math.log(1.5)
        assert 1.8 < order < 2.3, (a, b, order)
    assert l2b < 3e-3
