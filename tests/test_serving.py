"""Serving loop (continuous batching over slots, factor cache under an HBM
budget).  CPU: admission / LRU eviction logic with a stand-in solver.  GPU:
every request's result in a Poisson mix equals the same request solved alone,
and slots of different problems overlap on the device."""
import math

import numpy as np
import pytest
import torch

import ddm_inputs as di
import paper_1807_04180_amd as ddm
from paper_1807_04180_amd import serving


class _FakeSolver:
    """Stand-in for HelmholtzDDM: every slot converges after `need` steps."""
    live = 0

    def __init__(self, problem, k2, slots, factor=True):
        self.nrhs_max = slots
        self.steps = [-1] * slots
        self.need = int(problem.sigma0)
        _FakeSolver.live += 1

    def slot_admit(self, slot, f):
        assert self.steps[slot] < 0
        self.steps[slot] = 0

    def slots_step(self, n):
        self.steps = [s + n if s >= 0 else s for s in self.steps]

    def slots_poll(self):
        rel = [(-1.0 if s <= 0 else (1e-9 if s >= self.need else 1.0)) for s in self.steps]
        return rel, list(self.steps)

    def slot_retire(self, slot, u=None):
        self.steps[slot] = -1

    def close(self):
        _FakeSolver.live -= 1


class _FakeProblem:
    def __init__(self, need, nbytes):
        self.sigma0 = need
        self.nbytes = nbytes

    def memory_required(self, slots):
        return self.nbytes


class _Stream:
    def __init__(self, *a):
        pass

    def synchronize(self):
        pass

    def wait_stream(self, other):
        pass


def _fake_env(monkeypatch):
    monkeypatch.setattr(serving, "HelmholtzDDM", _FakeSolver)
    monkeypatch.setattr(torch.cuda, "Stream", _Stream)
    monkeypatch.setattr(torch.cuda, "stream", lambda s: __import__("contextlib").nullcontext())
    monkeypatch.setattr(torch.cuda, "current_stream", lambda *a: None)


def _req(rid, key, need, nbytes, nrhs, t):
    return serving.Request(rid, key, lambda: (_FakeProblem(need, nbytes), None), torch.zeros((nrhs, 4)),
                           tol=1e-6, t_arrival=t)


def test_admission_by_budget_and_lru_eviction(monkeypatch):
    _fake_env(monkeypatch)
    srv = serving.Server(hbm_budget_bytes=100, slots=2, device="cpu")
    reqs = [_req(0, "A", 3, 60, 3, 0.0), _req(1, "B", 2, 60, 1, 0.0), _req(2, "A", 1, 60, 1, 0.0),
            _req(3, "C", 2, 40, 2, 0.0)]
    done = srv.run(reqs, time_limit=10.0)
    assert len(done) == 4
    st = srv.stats()
    assert st["peak_hbm_bytes"] <= 100          # never above the budget
    assert srv.evictions >= 1                   # A and B cannot be resident together
    assert st["cache_hits"] + st["cache_misses"] == 4
    srv.close()
    assert _FakeSolver.live == 0


def test_request_larger_than_budget_is_refused(monkeypatch):
    _fake_env(monkeypatch)
    srv = serving.Server(hbm_budget_bytes=50, slots=2, device="cpu")
    with pytest.raises(ValueError):
        srv.run([_req(0, "A", 1, 60, 1, 0.0)], time_limit=1.0)


# ----------------------------------------------------------------------------
def _workload_request(rid, w, mixed, t, seed, nrhs):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(1000 + seed)
    centres = rng.uniform(0.15, 0.85, size=(nrhs, 2))
    f = np.stack([di.gaussian_source(2, w.M, w.n_pml, w.h, w.L, tuple(c), 2 * w.h) for c in centres])
    ft = torch.from_numpy(f.reshape(nrhs, -1)).to(dev)
    k2 = torch.from_numpy(w.k2.reshape(-1)).to(dev)
    key = (w.name, mixed)
    return serving.Request(rid, key, lambda: (ddm.Problem.from_workload(w, mixed=mixed), k2), ft, tol=1e-8,
                           t_arrival=t)


@pytest.mark.gpu
@pytest.mark.parametrize("blocks", ["small", "large"])
@pytest.mark.parametrize("mixed", [False, True])
def test_alone_vs_mix(mixed, blocks):
    # small: blocks of 84-92 unknowns (one workgroup per chain); large: blocks
    # of 148-160 unknowns, where handles of at most 4 slots use split chains
    if blocks == "small":
        wa = di.small_2d(M=128, N=(2, 2), n_pml=6, n_ov=4)
        wb = di.small_2d(M=144, N=(3, 3), n_pml=6, n_ov=4, layered=True, seed=2)
    else:
        wa = di.small_2d(M=256, N=(2, 2), n_pml=8, n_ov=4)
        wb = di.small_2d(M=288, N=(2, 2), n_pml=8, n_ov=4, layered=True, seed=2)
    rng = np.random.default_rng(7)
    t = np.cumsum(rng.exponential(0.02, size=8))
    reqs = [_workload_request(i, wa if i % 2 == 0 else wb, mixed, float(t[i]), i, 1 + i % 3) for i in range(8)]
    srv = serving.Server(hbm_budget_bytes=8 << 30, slots=4)
    done = srv.run(reqs, time_limit=120.0)
    assert len(done) == 8
    st = srv.stats()
    assert st["cache_misses"] + st["cache_hits"] == 8 and st["cache_misses"] >= 2 and st["cache_hits"] >= 2
    srv.close()
    # each request alone: a fresh handle, stationary solve to the same tolerance
    for r in reqs:
        w = wa if r.rid % 2 == 0 else wb
        s = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), torch.from_numpy(w.k2.reshape(-1)).cuda(),
                             r.nrhs)
        u, info, stt = s.solve(r.f, method="stationary", tol=r.tol, maxiter=r.max_steps)
        assert stt == 0
        assert [i["iters"] for i in info] == r.steps
        err = (torch.linalg.vector_norm(u - r.u, dim=1) / torch.linalg.vector_norm(u, dim=1)).max().item()
        assert err <= 1e-12, (r.rid, err)
        s.close()
