"""The autotuner (paper_1807_04180_amd.tuning) through the C-ABI on the GPU:

* every admissible (layout, substitution variant, chain RHS tile) is timed
  and the fastest is applied; the tuned handle's local solves match the
  oracle (1e-10 FP64, 5e-5 complex64);
* the plan goes to the JSON cache under its shape key, and a second handle
  of the same shape takes it from there without timing, with the same
  results bit for bit;
* each forced chain RHS tile (4, 8, 16) on 16 right-hand sides matches the
  oracle.
"""
import json

import numpy as np
import pytest
import torch

import ddm_inputs as di
from oracle import Oracle
import paper_1807_04180_amd as ddm
from paper_1807_04180_amd import tuning

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _n(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    a = np.asarray(a).reshape(b.shape)
    return np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1))


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("nrhs", [3, 16])
def test_tune_applies_fastest_and_caches(tmp_path, nrhs, mixed):
    w = di.small_2d(M=192, N=(3, 3), n_pml=7, n_ov=5, nrhs=1, layered=True, seed=4)
    print("case", w.name, "nrhs", nrhs, "mixed", mixed, flush=True)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    cache = tuning.PlanCache(str(tmp_path / "plans.json"))
    tol = 5e-5 if mixed else 1e-10
    gin = di.random_field((nrhs, o.etot), seed=500 + nrhs)
    xo = o.local_solve(gin)
    s = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), _t(w.k2.reshape(-1)), nrhs)
    try:
        plan = tuning.tune(s, nrhs, reps=2, cache=cache)
        assert not plan["cached"]
        variants = {(r["twisted"], r["variant"], r["chain_tile"]) for r in plan["table"]}
        assert (True, "chain", 16 if nrhs > 4 else 0) in variants and (False, "perline", 0) in variants
        assert (True, "mma", 0) in variants and (False, "mma", 0) in variants
        if nrhs > 4:
            assert {(True, "chain", t) for t in (4, 8, 16)} <= variants
        assert plan["ms"] == min(r["ms"] for r in plan["table"])
        assert s.solve_variant() == plan["variant"]
        x1 = _n(s.local_solve(_t(gin)))
        assert relerr(x1, xo) < tol
    finally:
        s.close()
    with open(tmp_path / "plans.json") as fh:
        assert plan["key"] in json.load(fh)
    # a second handle of the same shape: the cached plan, no timing
    s2 = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), _t(w.k2.reshape(-1)), nrhs, factor=False)
    try:
        p2 = tuning.tune(s2, nrhs, reps=2, cache=tuning.PlanCache(str(tmp_path / "plans.json")))
        assert p2["cached"] and p2["variant"] == plan["variant"] and p2["twisted"] == plan["twisted"]
        assert np.array_equal(_n(s2.local_solve(_t(gin))), x1)
    finally:
        s2.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_forced_chain_tiles(mixed):
    w = di.small_2d(M=192, N=(3, 3), n_pml=7, n_ov=5, nrhs=1, layered=True, seed=4)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    s = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), _t(w.k2.reshape(-1)), 16)
    tol = 5e-5 if mixed else 1e-10
    try:
        s.set_solve_variant("chain")
        gin = di.random_field((16, o.etot), seed=520)
        xo = o.local_solve(gin)
        for t in (4, 8, 16, 0):
            s.set_chain_tile(t)
            assert relerr(_n(s.local_solve(_t(gin))), xo) < tol, t
            assert s.time_local_solve(16, 1) > 0
        with pytest.raises(ddm.DDMError):
            s.set_chain_tile(5)
    finally:
        s.close()
