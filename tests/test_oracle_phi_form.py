"""Pins of the oracle's Phi form of the transferred source (eq. Phi, the remark
after the horizontal transfer in Sec. 2.2) and of where it holds:

* it is free of the wave number: changing k^2 leaves it unchanged, while
  the direct form -L_a(beta v) changes;
* along one axis of subdomains (the setting of the remark: every transfer
  horizontal, or every transfer vertical) the local solutions of the DDM
  satisfy L v = 0 wherever beta varies, so the Phi form equals the direct
  one on every step, including the lag sums of the residual identity;
* with subdomains along two or more axes it does not: a box's sources from
  one direction reach into the overlap bands it transfers across in another
  (the corner crossings), and run as the DDM's transfer the Phi form loses
  the fixed point (the residual stalls) while the direct form converges.
  The library therefore accepts it only for layouts split along one axis;
* on arbitrary input it differs from the direct form (the switch is real);
* for a smooth v and a cut-off of fixed physical width it converges under
  mesh refinement to the continuous Phi = -(beta'' v + 2 beta' dv/dx) of
  eq. Phi (A = J = 1 off the PML), i.e. to derivatives falling on beta.
"""
import math

import numpy as np
import pytest

import ddm_inputs as di
from oracle import Oracle


def _oracle(w, k2=None):
    return Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2 if k2 is None else k2)


def _case(name):
    if name == "2d-const":
        return di.small_2d(M=36, N=(3, 3), n_pml=3, n_ov=3, nrhs=2)
    if name == "2d-layered":
        return di.small_2d(M=36, N=(3, 3), n_pml=4, n_ov=4, layered=True, seed=7)
    if name == "2d-row":
        return di.small_2d(M=48, N=(4, 1), n_pml=4, n_ov=3, nrhs=2)
    if name == "2d-column-layered":
        return di.small_2d(M=36, N=(1, 3), n_pml=4, n_ov=4, layered=True, seed=7)
    if name == "3d-line":
        return di.small_3d(M=12, N=(1, 1, 3), n_pml=2, n_ov=2)
    return di.small_3d(M=12, N=(2, 2, 2), n_pml=2, n_ov=2)


def _ddm_with(o, w, form, steps):
    """Algorithm 3.1 assembled from the oracle's steps with the chosen form of
    the transferred source; returns the residual history."""
    f = w.f.reshape(w.nrhs, -1)
    hist = [None, None, None]
    U = np.zeros((w.nrhs, o.etot), dtype=np.complex128)
    rel = []
    for s in range(1, steps + 1):
        g = o.restrict_core(f) if s == 1 else o.transfer(hist, w.nrhs, form=form)
        us = o.local_solve(g)
        U += us
        hist = [us] + hist[:2]
        rel.append(o.relres(f, o.assemble(U)).max())
    return rel


def test_phi_form_is_k_free():
    w = _case("2d-layered")
    o1 = _oracle(w)
    o2 = _oracle(w, k2=w.k2 * 1.7 + 3.0)
    lag = [di.random_field((1, o1.etot), seed=s) for s in (11, 12)]
    p1, p2 = o1.transfer(lag, 1, form="phi"), o2.transfer(lag, 1, form="phi")
    d1, d2 = o1.transfer(lag, 1), o2.transfer(lag, 1)
    assert np.abs(p1 - p2).max() <= 1e-12 * np.abs(p1).max()
    assert np.abs(d1 - d2).max() > 1e-2 * np.abs(d1).max()


def test_phi_form_differs_on_arbitrary_input():
    w = _case("2d-const")
    o = _oracle(w)
    lag = [di.random_field((2, o.etot), seed=s) for s in (21, 22)]
    p, d = o.transfer(lag, 2, form="phi"), o.transfer(lag, 2)
    assert np.abs(p - d).max() > 1e-2 * np.abs(d).max()


@pytest.mark.parametrize("case", ["2d-row", "2d-column-layered", "3d-line"])
def test_phi_form_equals_direct_on_ddm_local_solutions(case):
    w = _case(case)
    o = _oracle(w)
    nrhs = w.nrhs
    hist = [np.zeros((nrhs, o.etot), dtype=np.complex128)] * 3
    for s in range(1, 7):
        u, _, uhat, _, _ = o.ddm_run(w.f, s, want_relres=False, want_state=True)
        hist = [uhat] + hist[:2]
        # the plain lags of the next step, and the lag sums of the residual identity
        for lag in (hist, [hist[0], hist[0] + hist[1], hist[0] + hist[1] + hist[2]]):
            d = o.transfer(lag, nrhs)
            p = o.transfer(lag, nrhs, form="phi")
            scale = max(np.abs(d).max(), 1e-300)
            # L v at a strip node is a local-solve residual: O(eps |L| |v|)
            floor = 1e-12 * (4 * w.dim / w.h ** 2) * max(np.abs(x).max() for x in lag)
            assert np.abs(p - d).max() <= 1e-11 * scale + floor, (case, s)


@pytest.mark.parametrize("case", ["2d-const", "2d-layered", "3d"])
def test_phi_form_loses_the_fixed_point_with_corner_transfers(case):
    w = _case(case)
    o = _oracle(w)
    steps = 40 if w.dim == 2 else 16
    direct = _ddm_with(o, w, "direct", steps)
    phi = _ddm_with(o, w, "phi", steps)
    assert direct[-1] < 1e-8, direct[-1]
    assert min(phi[-5:]) > 1e-2, phi[-5:]


def test_phi_form_converges_to_continuous_phi():
    # two subdomains side by side; v = exp(i 3 x) cos(2 y) on the left box,
    # overlap of fixed width 0.1 (n_ov - 1 = 4 s cells of h = 1 / (40 s))
    errs = []
    for s in (1, 2, 4):
        M, n_ov = 40 * s, 4 * s + 1
        w = di.small_2d(M=M, N=(2, 1), n_pml=4 * s, n_ov=n_ov, nrhs=1)
        o = _oracle(w)
        h = w.h
        b, a = o.subdomain(0), o.subdomain(1)
        V = np.zeros((1, o.etot), dtype=np.complex128)
        xs = np.arange(b["ext_lo"][0], b["ext_hi"][0] + 1) * h
        ys = np.arange(b["ext_lo"][1], b["ext_hi"][1] + 1) * h
        V[0, b["off"]:b["off"] + b["n"]] = (np.exp(3j * xs)[None, :] * np.cos(2 * ys)[:, None]).reshape(-1)
        g = o.transfer([V], 1, form="phi")[0, a["off"]:a["off"] + a["n"]]
        nx = a["ext_hi"][0] - a["ext_lo"][0] + 1
        g = g.reshape(-1, nx)
        W = (n_ov - 1) * h
        num, den = 0.0, 0.0
        for px in range(a["core_lo"][0], a["core_lo"][0] + n_ov):
            m = px - b["core_hi"][0]                   # offset outward from b's core
            t = (m - 1) / (n_ov - 1)
            # beta0(t) = 1 - (10 t^3 - 15 t^4 + 6 t^5); beta(x) = beta0((x - x_c - h) / W)
            d1 = -(30 * t ** 2 - 60 * t ** 3 + 30 * t ** 4) / W
            d2 = -(60 * t - 180 * t ** 2 + 120 * t ** 3) / W ** 2
            x = px * h
            rows = slice(4 * s, g.shape[0] - 4 * s)   # away from the y PML
            y = (np.arange(a["ext_lo"][1], a["ext_hi"][1] + 1) * h)[rows]
            v = np.exp(3j * x) * np.cos(2 * y)
            exact = -(d2 * v + 2 * d1 * 3j * v)
            got = g[rows, px - a["ext_lo"][0]]
            num += np.sum(np.abs(got - exact) ** 2)
            den += np.sum(np.abs(exact) ** 2)
        errs.append(math.sqrt(num / den))
    # O(h^2) inside the band, O(h) at its two ends (beta0 is C^2, not C^3)
    assert errs[2] < 0.06, errs
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs
