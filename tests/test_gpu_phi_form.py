"""GPU parity of the Phi form of the transferred source (eq. Phi, Sec. 2.2)
through the C-ABI, on layouts split along one axis (the only ones the
library accepts it for):

* geometry of the one-axis layouts against the oracle;
* ddm_transfer in the Phi form against the oracle's Phi form, element by
  element (1e-13, the same FP64 arithmetic in another order), and the
  direct form again after switching back;
* DDM iterates with the Phi form against the oracle's direct-form iterates
  (FP64: 1e-10; the forms agree to rounding on one-axis layouts), and a
  stationary solve that replays captured step graphs before and after the
  switch;
* layouts with subdomains along two axes reject the Phi form.
"""
import numpy as np
import pytest
import torch

import ddm_inputs as di
from oracle import Oracle
import paper_1807_04180_amd as ddm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = {
    "2d-4x1": lambda: di.small_2d(M=96, N=(4, 1), n_pml=5, n_ov=4, nrhs=3),
    "2d-1x3-layered": lambda: di.small_2d(M=72, N=(1, 3), n_pml=4, n_ov=4, layered=True, seed=3, nrhs=2),
    "3d-1x1x3": lambda: di.small_3d(M=12, N=(1, 1, 3), n_pml=2, n_ov=2, nrhs=2),
}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _n(t):
    return t.detach().cpu().numpy()


def relerr(a, b, axis=None):
    a = np.asarray(a).reshape(b.shape)
    return np.max(np.linalg.norm(a - b, axis=axis) / np.maximum(np.linalg.norm(b, axis=axis), 1e-300))


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request):
    w = CASES[request.param]()
    print("case", request.param, flush=True)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w), _t(w.k2.reshape(-1)), 4)
    yield w, o, g
    g.close()


def test_one_axis_geometry(pair):
    w, o, g = pair
    assert g.nglob == o.nglob and g.etot == o.etot and g.nsub == o.nsub
    for a in range(o.nsub):
        go, gg = o.subdomain(a), g.geometry(a)
        for k in ("core_lo", "core_hi", "ext_lo", "ext_hi", "off", "n"):
            assert tuple(np.atleast_1d(go[k])) == tuple(np.atleast_1d(gg[k])), (a, k)


@pytest.mark.parametrize("nrhs", [1, 3])
def test_phi_transfer_matches_oracle(pair, nrhs):
    w, o, g = pair
    lags = [di.random_field((nrhs, o.etot), seed=60 + k) for k in range(3)]
    args = [lags[0], None, None]
    g.set_transfer_form("phi")
    try:
        gp = _n(g.transfer(*[None if a is None else _t(a) for a in args]))
    finally:
        g.set_transfer_form("direct")
    assert relerr(gp, o.transfer(args, nrhs, form="phi")) < 1e-13
    gd = _n(g.transfer(*[None if a is None else _t(a) for a in args]))
    assert relerr(gd, o.transfer(args, nrhs)) < 1e-13
    assert relerr(gp, gd) > 1e-3      # arbitrary input: the forms differ


def test_phi_iterates_match_direct(pair):
    w, o, g = pair
    f = w.f.reshape(w.nrhs, -1)
    uo, ro = o.ddm_run(w.f, 6)
    g.set_transfer_form("phi")
    try:
        ug, rg = g.iterate(_t(f), 6)
    finally:
        g.set_transfer_form("direct")
    assert relerr(_n(ug), uo, axis=1) < 1e-10
    np.testing.assert_allclose(np.array(rg), ro, rtol=1e-6, atol=1e-14)


def test_phi_stationary_solve_with_graphs(pair):
    w, o, g = pair
    f = _t(w.f.reshape(w.nrhs, -1))
    g.set_graphs(True)
    ud, _, sd = g.solve(f, method="stationary", tol=1e-10, maxiter=200)
    g.set_transfer_form("phi")
    try:
        up, ip, sp = g.solve(f, method="stationary", tol=1e-10, maxiter=200)
    finally:
        g.set_transfer_form("direct")
    assert sd == 0 and sp == 0
    assert max(x["relres"] for x in ip) <= 1e-10
    uref = o.global_solve(w.f).reshape(w.nrhs, -1)
    assert relerr(_n(up), uref, axis=1) < 1e-8
    assert relerr(_n(up), _n(ud), axis=1) < 1e-9


def test_phi_form_rejected_with_corner_transfers():
    w = di.small_2d(M=64, N=(2, 2), n_pml=4, n_ov=3, nrhs=1)
    g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w), _t(w.k2.reshape(-1)), 1)
    try:
        with pytest.raises(ddm.DDMError, match="one axis"):
            g.set_transfer_form("phi")
        g.set_transfer_form("direct")
    finally:
        g.close()
