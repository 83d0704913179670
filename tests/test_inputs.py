"""Seeded input generators: determinism and the serving stream's recipe."""
import numpy as np

import ddm_inputs as di


def test_gaussian_window_matches_full_evaluation():
    M, n_pml = 256, 16
    h = 1.0 / M
    for c in [(0.37, 0.61), (0.1, 0.9), (0.5, 0.5)]:
        full = di.gaussian_source(2, (M, M), n_pml, h, 1.0, c, 2 * h)
        win = di._gaussian_2d_window(M, n_pml, h, c, 2 * h)
        assert np.abs(full - win).max() <= 1e-25 * np.abs(full).max()
        assert abs(full.sum().real * h * h - 1.0) < 1e-6  # unit mass


def test_serving_stream_is_seeded_and_follows_the_recipe():
    a = di.serving_stream(n_requests=12, rate=4.0, grids=(256, 512))
    b = di.serving_stream(n_requests=12, rate=4.0, grids=(256, 512))
    assert [r.key for r in a] == [r.key for r in b]
    assert [r.t_arrival for r in a] == [r.t_arrival for r in b]
    assert all(np.array_equal(x.workload.f, y.workload.f) for x, y in zip(a, b))
    t = [r.t_arrival for r in a]
    assert all(t1 > t0 for t0, t1 in zip(t, t[1:]))
    kinds = set()
    for r in a:
        w = r.workload
        M, kind, N = r.key
        kinds.add(kind)
        assert w.M == (M, M) and w.N == N and N[0] * 128 == M
        assert 1 <= w.nrhs <= 32
        assert w.f.shape == (w.nrhs,) + w.grid_shape
        # 10 points per wavelength at the slowest velocity (8 for the second
        # constant medium of the catalog)
        k_max = np.sqrt(w.k2.max())
        ppw = 8.0 if kind == "constant-1" else 10.0
        assert abs(2 * np.pi / k_max / w.h - ppw) < 1e-9
    assert kinds <= {"constant-0", "constant-1", "layered-2", "layered-3"}
    # one problem per key: requests with the same key share the medium
    by_key = {}
    for r in a:
        by_key.setdefault(r.key, r.workload.k2)
        assert by_key[r.key] is r.workload.k2


def test_paper_weak_recipe():
    for N in (2, 3):
        w = di.paper_weak(N, "constant", core=60, n_pml=10)
        assert w.M == (60 * N, 60 * N) and w.N == (N, N)
        assert abs(w.omega / (2 * np.pi) - (25 * N + 5)) < 1e-12
        # one delta shot of mass 1 at node (15, 20): a quarter / a third of a core
        nz = np.argwhere(w.f[0] != 0)
        assert len(nz) == 1
        iy, ix = nz[0]
        assert (ix - (w.n_pml - 1), iy - (w.n_pml - 1)) == (15, 20)
        assert abs(w.f[0][iy, ix] * w.h ** 2 - 1.0) < 1e-12
    wl = di.paper_weak(2, "layered", core=60, n_pml=10)
    assert abs(wl.omega / (2 * np.pi) - 27.5) < 1e-12 and 1.5 <= wl.c_min < wl.c_max <= 4.5


def test_const_2048_layout_matches_layered():
    a = di.const_2d_2048(nrhs=2, M=256, N=4)
    b = di.layered_2d_2048(nrhs=2, M=256, N=4)
    assert (a.M, a.N, a.n_pml, a.n_ov) == (b.M, b.N, b.n_pml, b.n_ov)
    assert np.allclose(a.k2, a.omega ** 2)
