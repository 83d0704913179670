"""GPU parity: every step of the HIP path (through the C-ABI) against the CPU
oracle on the same seeded inputs, element by element.

Sizes: subdomain blocks of 75-98 nodes span two 64-row tiles of the
substitution kernel with a ragged tail; RHS counts 1, 3, 5, 9, 16 and 20 exercise
ragged RHS tiles; layouts 2x2, 3x2 and 3x3 mix interior, edge and corner
boxes of different sizes in one launch.

Tolerances (relative, max-abs or L2 per RHS as stated):
  operator, restriction, transfer, assembly : 1e-13 (same FP64 formula, only
      rounding order differs)
  FP64 local solves and DDM iterates         : 1e-10 (the stated bound for the
      FP64 path; block inverses vs banded LU differ by rounding amplified by
      the local condition number)
  mixed (complex64) local solves            : 5e-5 (c64 unit roundoff 6e-8
      times the local condition number, < 1e3 here)
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


def make_pair(w, nrhs_max=None, mixed=False):
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), _t(w.k2.reshape(-1)),
                         nrhs_max or max(w.nrhs, 1))
    return o, g


def relerr(a, b, axis=None):
    a = np.asarray(a).reshape(b.shape)
    num = np.linalg.norm(a - b, axis=axis)
    den = np.linalg.norm(b, axis=axis)
    return np.max(num / np.maximum(den, 1e-300))


CASES = {
    "2d-2x2-const": lambda: di.small_2d(M=160, N=(2, 2), n_pml=8, n_ov=4, nrhs=3),
    "2d-3x2-layered": lambda: di.small_2d(M=144, N=(3, 2), n_pml=6, n_ov=3, nrhs=1, layered=True, seed=3),
    "2d-3x3-layered": lambda: di.small_2d(M=192, N=(3, 3), n_pml=7, n_ov=5, nrhs=5, layered=True, seed=4),
    # 3D: plane blocks of 100-196 unknowns, 26 transfer directions, lags 1-3
    "3d-2x2x2": lambda: di.small_3d(M=16, N=(2, 2, 2), n_pml=3, n_ov=2, nrhs=2, seed=1),
    "3d-3x2x2": lambda: di.small_3d(M=12, N=(3, 2, 2), n_pml=3, n_ov=2, nrhs=3, seed=2),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request):
    w = CASES[request.param]()
    # 3x2: unequal subdomain counts per axis need M divisible by both
    o, g = make_pair(w, nrhs_max=9)
    yield w, o, g
    g.close()


def test_geometry_matches_oracle(pair):
    w, o, g = pair
    assert g.nglob == o.nglob and g.etot == o.etot and g.nsub == o.nsub
    for a in range(o.nsub):
        go, gg = o.subdomain(a), g.geometry(a)
        for k in ("core_lo", "core_hi", "ext_lo", "ext_hi", "off", "n"):
            assert tuple(np.atleast_1d(go[k])) == tuple(np.atleast_1d(gg[k])), (a, k)


def test_operator_and_residual(pair):
    w, o, g = pair
    u = di.random_field((3, o.nglob), seed=11)
    Lo = o.apply(u)
    Lg = _n(g.apply(_t(u)))
    assert relerr(Lg, Lo) < 1e-13
    f = di.random_field((3, o.nglob), seed=12)
    r, rn, fn = g.residual(_t(f), _t(u))
    ro = f - Lo
    assert relerr(_n(r), ro) < 1e-13
    np.testing.assert_allclose(np.sqrt(rn), np.linalg.norm(ro, axis=1), rtol=1e-13)
    np.testing.assert_allclose(np.sqrt(fn), np.linalg.norm(f, axis=1), rtol=1e-13)


def test_restrict_core_bitwise(pair):
    w, o, g = pair
    f = di.random_field((2, o.nglob), seed=13)
    assert np.array_equal(_n(g.restrict_core(_t(f))), o.restrict_core(f))


@pytest.mark.parametrize("nrhs", [1, 5])
def test_transfer(pair, nrhs):
    w, o, g = pair
    lags = [di.random_field((nrhs, o.etot), seed=20 + k) for k in range(3)]
    for use in ([0], [0, 1], [1], [0, 1, 2]):
        args = [lags[k] if k in use else None for k in range(3)]
        go = o.transfer(args, nrhs)
        gg = _n(g.transfer(*[None if a is None else _t(a) for a in args]))
        assert relerr(gg, go) < 1e-13, use


def test_assemble(pair):
    w, o, g = pair
    U = di.random_field((3, o.etot), seed=30)
    assert relerr(_n(g.assemble(_t(U))), o.assemble(U)) < 1e-14


@pytest.mark.parametrize("nrhs", [1, 3, 9])
def test_local_solve_fp64(pair, nrhs):
    w, o, g = pair
    gin = di.random_field((nrhs, o.etot), seed=40 + nrhs)
    xo = o.local_solve(gin)
    xg = _n(g.local_solve(_t(gin)))
    for a in range(o.nsub):
        sd = o.subdomain(a)
        sl = slice(sd["off"], sd["off"] + sd["n"])
        assert relerr(xg[:, sl], xo[:, sl], axis=1) < 1e-10, a


def test_iterate_fp64_matches_oracle_every_step(pair):
    w, o, g = pair
    nsteps = 2 * sum(w.N) + 2 if w.dim == 2 else sum(w.N) + 3
    uo, rro = o.ddm_run(w.f, nsteps)
    ug, rrg = g.iterate(_t(w.f.reshape(w.nrhs, -1)), nsteps)
    assert relerr(_n(ug), uo, axis=1) < 1e-10
    rrg = np.array(rrg)
    # relres agrees while it is well above roundoff
    big = rro > 1e-9
    np.testing.assert_allclose(rrg[big], rro[big], rtol=1e-8)


def test_local_solve_mixed():
    w = CASES["2d-3x3-layered"]()
    o, g = make_pair(w, nrhs_max=3, mixed=True)
    gin = di.random_field((3, o.etot), seed=50)
    xo = o.local_solve(gin)
    xg = _n(g.local_solve(_t(gin)))
    assert relerr(xg, xo, axis=1) < 5e-5
    g.close()


def test_batch_invariance_bitwise(pair):
    """Each RHS alone gives bit-for-bit the same local solves and iterates as
    inside a batch of 9."""
    w, o, g = pair
    gin = di.random_field((9, o.etot), seed=60)
    xb = _n(g.local_solve(_t(gin)))
    for q in (0, 4, 8):
        xq = _n(g.local_solve(_t(gin[q:q + 1])))
        assert np.array_equal(xq[0], xb[q])


def test_deterministic_bitwise(pair):
    w, o, g = pair
    f = _t(w.f.reshape(w.nrhs, -1))
    u1, r1 = g.iterate(f, 5)
    u2, r2 = g.iterate(f, 5)
    assert torch.equal(u1, u2) and r1 == r2


LAYOUTS = {"twisted": (True, ["chain", "chain2", "mma"]), "onedir": (False, ["perline", "chain", "mma"])}


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_local_solve_layouts_and_variants(pair, layout):
    """Both factor layouts (two-ended / one-directional elimination) and every
    substitution variant that applies: oracle parity, repeatability and
    batch invariance (bitwise)."""
    w, o, g = pair
    twisted, variants = LAYOUTS[layout]
    g.set_factor_layout(twisted)
    try:
        for variant in variants:
            g.set_solve_variant(variant)
            for nrhs in (1, 5):
                gin = di.random_field((nrhs, o.etot), seed=70 + nrhs)
                xo = o.local_solve(gin)
                xg = _n(g.local_solve(_t(gin)))
                assert relerr(xg, xo, axis=1) < 1e-10, (variant, nrhs)
                assert np.array_equal(_n(g.local_solve(_t(gin))), xg), (variant, nrhs)
                x0 = _n(g.local_solve(_t(gin[nrhs - 1:nrhs])))
                assert np.array_equal(x0[0], xg[nrhs - 1]), (variant, nrhs)
    finally:
        g.set_factor_layout(True)


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_iterate_layouts_match_oracle(pair, layout):
    w, o, g = pair
    twisted, variants = LAYOUTS[layout]
    g.set_factor_layout(twisted)
    try:
        for variant in variants:
            g.set_solve_variant(variant)
            nsteps = sum(w.N) + 3
            uo, _ = o.ddm_run(w.f, nsteps)
            ug, _ = g.iterate(_t(w.f.reshape(w.nrhs, -1)), nsteps)
            assert relerr(_n(ug), uo, axis=1) < 1e-10, variant
    finally:
        g.set_factor_layout(True)


def test_chain_mixed_matches_oracle():
    w = CASES["2d-3x3-layered"]()
    o, g = make_pair(w, nrhs_max=20, mixed=True)
    g.set_solve_variant("chain")
    # block sizes (x extents) include odd ones: complex64 inverses are stored
    # with an even column stride and read two rows per lane
    bsz = [g.geometry(a)["ext_hi"][0] - g.geometry(a)["ext_lo"][0] + 1 for a in range(9)]
    assert any(b % 2 for b in bsz) and any(b % 2 == 0 for b in bsz), bsz
    for nrhs in (3, 6, 9, 20):  # RHS tiles of 4, 8, 16 and 16 + a ragged 4
        gin = di.random_field((nrhs, o.etot), seed=51)
        assert relerr(_n(g.local_solve(_t(gin))), o.local_solve(gin), axis=1) < 5e-5
    g.close()


@pytest.mark.parametrize("case", ["2d-3x3-layered", "2d-2x2-146"])
def test_chain_16_rhs_tiles_fp64(case):
    """Complex128 batches of 16 or more RHS take 16-RHS tiles (1024-thread
    workgroups, the column groups' partial sums added in order), on blocks of
    two (75-98 nodes) and three (146 nodes) 64-row tiles: oracle parity for
    16 RHS; every RHS gives the same bits in a batch of 20 (reordered, the
    last 4 in a ragged second tile) and alone."""
    w = CASES[case]() if case in CASES else di.small_2d(M=256, N=(2, 2), n_pml=8, n_ov=4, nrhs=1)
    o, g = make_pair(w, nrhs_max=20)
    try:
        g.set_solve_variant("chain")
        assert g.solve_variant() == "chain"
        gin = di.random_field((16, o.etot), seed=54)
        x16 = _n(g.local_solve(_t(gin)))
        assert relerr(x16, o.local_solve(gin), axis=1) < 1e-10
        x20 = _n(g.local_solve(_t(np.concatenate([gin[::-1], gin[:4]]))))
        assert np.array_equal(x20[:16], x16[::-1])
        assert np.array_equal(x20[16:], x16[:4])
        assert np.array_equal(_n(g.local_solve(_t(gin[5:6])))[0], x16[5])
    finally:
        g.close()


def test_chain2_mixed_matches_oracle():
    """Split substitution (two workgroups per chain) in complex64: oracle
    parity over 1, 3 and 6 RHS (tiles of 4 and a ragged tile), and a single
    RHS bit-for-bit equal to its place in the batch."""
    w = CASES["2d-3x3-layered"]()
    o, g = make_pair(w, nrhs_max=6, mixed=True)
    g.set_solve_variant("chain2")
    assert g.solve_variant() == "chain2"
    for nrhs in (1, 3, 6):
        gin = di.random_field((nrhs, o.etot), seed=53)
        xb = _n(g.local_solve(_t(gin)))
        assert relerr(xb, o.local_solve(gin), axis=1) < 5e-5, nrhs
        assert np.array_equal(_n(g.local_solve(_t(gin[-1:])))[0], xb[-1]), nrhs
    g.close()


def test_chain2_spin_bound_drains_and_reports():
    """A spin bound of 1 makes the split substitution give up its waits (the
    per-block exchange and the middle meeting): the launch must still drain
    and report EHIP unless every partner was already there; afterwards, with
    the normal bound, results are correct again."""
    w = CASES["2d-3x3-layered"]()
    o, g = make_pair(w, nrhs_max=2)
    g.set_solve_variant("chain2")
    gin = di.random_field((2, o.etot), seed=54)
    xo = o.local_solve(gin)
    g.set_spin_limit(1)
    try:
        x = g.local_solve(_t(gin))
        assert relerr(_n(x), xo, axis=1) < 1e-10
    except ddm.DDMError as e:
        assert e.code == ddm._ffi.DDM_EHIP
    g.set_spin_limit(1 << 22)
    assert relerr(_n(g.local_solve(_t(gin))), xo, axis=1) < 1e-10
    g.close()


def test_chain_spin_bound_drains_and_reports():
    """A spin bound of 1 lets a chain give up waiting for its partner at the
    middle block: the launch must still drain (no hang) and report EHIP unless
    the partner was already there; afterwards, with the normal bound, results
    are correct again."""
    w = CASES["2d-3x3-layered"]()
    o, g = make_pair(w, nrhs_max=2)
    g.set_solve_variant("chain")
    gin = di.random_field((2, o.etot), seed=52)
    xo = o.local_solve(gin)
    g.set_spin_limit(1)
    try:
        x = g.local_solve(_t(gin))
        assert relerr(_n(x), xo, axis=1) < 1e-10
    except ddm.DDMError as e:
        assert e.code == ddm._ffi.DDM_EHIP
    g.set_spin_limit(1 << 22)
    assert relerr(_n(g.local_solve(_t(gin))), xo, axis=1) < 1e-10
    g.close()


def test_autotune_picks_an_applicable_variant(pair):
    w, o, g = pair
    g.set_factor_layout(False)
    try:
        times = g.autotune(nrhs=3, reps=2)
        assert times["perline"] is not None and times["chain"] is not None
        assert times[g.solve_variant()] == min(t for t in times.values() if t is not None)
    finally:
        g.set_factor_layout(True)


def test_mixed_stationary_residual_corrected_converges():
    """Mixed path (complex64 local solves and transfers, FP64 residual):
    with residual-corrected sources it reaches a tight FP64 tolerance, and the
    result matches the oracle's global direct solve."""
    w = CASES["2d-3x3-layered"]()
    o, g = make_pair(w, nrhs_max=w.nrhs, mixed=True)
    f = _t(w.f.reshape(w.nrhs, -1))
    u, info, st = g.solve(f, method="stationary", tol=1e-9, maxiter=400)
    assert st == 0, info
    uref = o.global_solve(w.f).reshape(w.nrhs, -1)
    assert relerr(_n(u), uref, axis=1) < 1e-7
    # FP64 path on the same problem for the step count comparison
    o2, g64 = make_pair(w, nrhs_max=w.nrhs)
    _, info64, _ = g64.solve(f, method="stationary", tol=1e-9, maxiter=400)
    assert max(i["iters"] for i in info) <= max(i["iters"] for i in info64) + 3
    g.close()
    g64.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_fgmres_matches_global_solve(mixed):
    w = CASES["2d-3x3-layered"]()
    o, g = make_pair(w, nrhs_max=w.nrhs, mixed=mixed)
    f = _t(w.f.reshape(w.nrhs, -1))
    u, info, st = g.solve(f, method="fgmres", tol=1e-10, maxiter=100, restart=30)
    assert st == 0, info
    uref = o.global_solve(w.f).reshape(w.nrhs, -1)
    assert relerr(_n(u), uref, axis=1) < 1e-8
    assert all(i["local_solves"] == i["iters"] * sum(w.N) for i in info)
    g.close()


def test_stationary_fp64_matches_global_solve():
    w = CASES["2d-2x2-const"]()
    o, g = make_pair(w, nrhs_max=w.nrhs)
    f = _t(w.f.reshape(w.nrhs, -1))
    u, info, st = g.solve(f, method="stationary", tol=1e-12, maxiter=200)
    assert st == 0
    uref = o.global_solve(w.f).reshape(w.nrhs, -1)
    assert relerr(_n(u), uref, axis=1) < 1e-10
    g.close()


def test_3d_large_planes_perline():
    """3D plane blocks of 289 unknowns (> 256): one-directional layout and the
    one-launch-per-block substitution; local solves and iterates vs oracle."""
    w = di.small_3d(M=22, N=(2, 2, 2), n_pml=3, n_ov=2, nrhs=2, seed=3)
    o, g = make_pair(w, nrhs_max=2)
    assert g.solve_variant() == "perline"
    gin = di.random_field((2, o.etot), seed=80)
    assert relerr(_n(g.local_solve(_t(gin))), o.local_solve(gin), axis=1) < 1e-10
    uo, _ = o.ddm_run(w.f, 4)
    ug, _ = g.iterate(_t(w.f.reshape(2, -1)), 4)
    assert relerr(_n(ug), uo, axis=1) < 1e-10
    g.close()


@pytest.mark.parametrize("M", [34, 36])
def test_3d_planes_above_512(M):
    """Plane blocks of 529 (M = 34: the last 32-column panel has 17 columns)
    and 576 unknowns (M = 36: whole panels): the factorisation's left-looking
    panel elimination from the workspace and the multi-workgroup Y; FP64 and
    mixed local solves vs oracle."""
    w = di.small_3d(M=M, N=(2, 2, 2), n_pml=3, n_ov=2, nrhs=2, seed=5)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    gin = di.random_field((2, o.etot), seed=81)
    xo = o.local_solve(gin)
    for mixed, tol in ((False, 1e-10), (True, 5e-5)):
        g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), _t(w.k2.reshape(-1)), 2)
        assert relerr(_n(g.local_solve(_t(gin))), xo, axis=1) < tol, mixed
        g.close()


def test_3d_uneven_planes_deferred_groups():
    """Plane blocks of 560, 595 and 630 unknowns in one handle (3x1x3
    subdomains of a 30^3 grid): 18, 19 and 20 panels, so with groups of four
    deferred panels the smaller blocks end their last group early (two and
    three panels) and every block ends on a partial panel.  Local solves vs
    the oracle's, and their residuals under the oracle's subdomain
    operators."""
    w = di.small_3d(M=30, N=(3, 1, 3), n_pml=3, n_ov=2, nrhs=2, seed=6)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    bs = set()
    for a in range(o.nsub):
        d = o.subdomain(a)
        bs.add((d["ext_hi"][0] - d["ext_lo"][0] + 1) * (d["ext_hi"][1] - d["ext_lo"][1] + 1))
    assert bs == {560, 595, 630}
    gin = di.random_field((2, o.etot), seed=83)
    xo = o.local_solve(gin)
    for mixed, tol in ((False, 1e-10), (True, 5e-5)):
        g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), _t(w.k2.reshape(-1)), 2)
        xg = _n(g.local_solve(_t(gin)))
        assert relerr(xg, xo, axis=1) < tol, mixed
        if not mixed:
            for a in range(o.nsub):
                d = o.subdomain(a)
                sl = slice(d["off"], d["off"] + d["n"])
                for q in range(2):
                    r = o.apply_local(a, xg[q, sl]) - gin[q, sl]
                    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(gin[q, sl]), (a, q)
        g.close()


@pytest.mark.parametrize("case,mixed", [("2d-3x3-layered", False), ("2d-3x3-layered", True), ("3d-2x2x2", False)])
def test_step_graph_replays_match_eager(case, mixed):
    """The stationary solve replays captured step graphs (one per ring
    phase) many times with host work and synchronisation in between; every
    solve must be bitwise identical to plain launches."""
    w = CASES[case]()
    o, g = make_pair(w, nrhs_max=w.nrhs, mixed=mixed)
    f = _t(w.f.reshape(w.nrhs, -1))
    g.set_graphs(False)
    u0, i0, _ = g.solve(f, method="stationary", tol=1e-9, maxiter=300)
    g.set_graphs(True)
    n0 = g.graph_launches()
    u1, i1, _ = g.solve(f, method="stationary", tol=1e-9, maxiter=300)
    u2, i2, _ = g.solve(f, method="stationary", tol=1e-9, maxiter=300)
    assert g.graph_launches() > n0
    assert torch.equal(u1, u0) and torch.equal(u2, u0)
    assert [i["iters"] for i in i1] == [i["iters"] for i in i0] == [i["iters"] for i in i2]
    uref = o.global_solve(w.f).reshape(w.nrhs, -1)
    assert relerr(_n(u1), uref, axis=1) < (1e-7 if mixed else 1e-8)
    g.close()


def test_paper_weak_recipe_small():
    """The weak-scaling recipe (delta shot a quarter / a third of a core into
    the first subdomain, omega/2pi = 25 N + 5, 30-cell PML scaled down):
    FP64 iterates match the oracle's and reach its global solution."""
    w = di.paper_weak(2, "constant", core=48, n_pml=8, n_ov=4)
    o, g = make_pair(w)
    uo, _ = o.ddm_run(w.f, 6)
    ug, _ = g.iterate(_t(w.f.reshape(1, -1)), 6)
    assert relerr(_n(ug), uo, axis=1) < 1e-10
    u, info, st = g.solve(_t(w.f.reshape(1, -1)), method="stationary", tol=1e-10, maxiter=200)
    assert st == 0 and info[0]["relres"] <= 1e-10
    uref = o.global_solve(w.f).reshape(1, -1)
    assert relerr(_n(u), uref, axis=1) < 1e-8
    g.close()


def test_paper_accuracy_560_lands_on_table1(golden):
    """Sec. 4.1.1: the DDM solution (N1 + N2 = 10 steps) of the 560^2 mesh,
    k/2pi = 25, 5x5 subdomains, against the exact free-space solution: its L2
    error on the physical box is Table 1's 3.13e-3 (within 2 %)."""
    import math
    import bench
    w = di.paper_accuracy_2d(1)
    g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w), _t(w.k2.reshape(-1)), 1)
    u, _ = g.iterate(_t(w.f.reshape(1, -1)), sum(w.N))
    g.close()
    x = di.node_coords(w.M[0], w.n_pml, w.h)
    l2, _ = bench.l2_h1_errors(_n(u).reshape(len(x), len(x)), x, w.h, w.L, w.omega, di.PAPER_ACCURACY_CENTRE_2D)
    ref = golden["table1_2d_convergence"]["l2_error"][0]
    assert abs(l2 - ref) < 0.02 * ref, (l2, ref)
    assert math.isfinite(l2)
