"""Serving loop (continuous batching over slots, factor cache under an HBM
budget).  CPU: admission / LRU eviction logic with a stand-in solver.  GPU:
every request's result in a Poisson mix equals the same request solved alone,
and slots of different problems overlap on the device."""
import math
import time

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
        self.build_delay = getattr(problem, "build_delay", 0.0)
        _FakeSolver.live += 1

    def factor(self):
        time.sleep(self.build_delay)

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
    def __init__(self, need, nbytes, build_delay=0.0):
        self.sigma0 = need
        self.nbytes = nbytes
        self.build_delay = build_delay

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


def _req(rid, key, need, nbytes, nrhs, t, build_delay=0.0):
    return serving.Request(rid, key, lambda: (_FakeProblem(need, nbytes, build_delay), None), torch.zeros((nrhs, 4)),
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


def test_cache_miss_builds_off_the_scheduling_path(monkeypatch):
    """A miss whose factorisation takes 0.5 s must not stall the other
    handles: requests on a resident problem finish while it builds."""
    _fake_env(monkeypatch)
    srv = serving.Server(hbm_budget_bytes=1000, slots=2, device="cpu")
    reqs = [_req(0, "A", 3, 60, 1, 0.0), _req(1, "B", 2, 60, 1, 0.05, build_delay=0.5),
            _req(2, "A", 3, 60, 2, 0.1), _req(3, "A", 3, 60, 1, 0.15)]
    done = srv.run(reqs, time_limit=10.0)
    assert len(done) == 4
    by = {r.rid: r for r in done}
    assert by[1].t_done >= 0.5
    assert max(by[0].t_done, by[2].t_done, by[3].t_done) < by[1].t_done
    assert srv.stats()["factor_seconds"] >= 0.5
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
@pytest.mark.parametrize("slots", [4, 16])
@pytest.mark.parametrize("blocks", ["small", "large"])
@pytest.mark.parametrize("mixed", [False, True])
def test_alone_vs_mix(mixed, blocks, slots):
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
    # 4 slots: the vector substitution kernels; 16: the matrix-core tiles
    srv = serving.Server(hbm_budget_bytes=8 << 30, slots=slots)
    done = srv.run(reqs, time_limit=120.0)
    assert len(done) == 8
    st = srv.stats()
    assert st["cache_misses"] + st["cache_hits"] == 8 and st["cache_misses"] >= 2 and st["cache_hits"] >= 2
    srv.close()
    # each request alone: a fresh handle of the same slot count (hence the same
    # kernels), stationary solve to the same tolerance
    for r in reqs:
        w = wa if r.rid % 2 == 0 else wb
        s = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), torch.from_numpy(w.k2.reshape(-1)).cuda(),
                             slots)
        u, info, stt = s.solve(r.f, method="stationary", tol=r.tol, maxiter=r.max_steps)
        assert stt == 0
        assert [i["iters"] for i in info] == r.steps
        err = (torch.linalg.vector_norm(u - r.u, dim=1) / torch.linalg.vector_norm(u, dim=1)).max().item()
        assert err <= 1e-12, (r.rid, err)
        s.close()
    # and against the oracle's global solve (one request per problem, on the
    # small grids): the served result is the discrete solution to the
    # stationary tolerance
    if blocks != "small":
        return
    from oracle import Oracle
    for w, r in ((wa, reqs[0]), (wb, reqs[1])):
        o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
        uo = o.global_solve(r.f.cpu().numpy().reshape((r.nrhs,) + tuple(w.grid_shape))).reshape(r.nrhs, -1)
        ug = r.u.cpu().numpy()
        err = np.max(np.linalg.norm(ug - uo, axis=1) / np.linalg.norm(uo, axis=1))
        assert err <= 1e-6, (r.rid, err)


@pytest.mark.gpu
@pytest.mark.parametrize("mixed", [False, True])
def test_slot_steps_cover_the_busy_range(mixed):
    """A 64-slot handle steps only the slots up to the highest busy one; a
    slot's arithmetic depends neither on that range nor on its position or
    on when it was admitted: slot 40 admitted first (steps cover 41 slots),
    slot 5 three steps later, each gives the bits of the same source alone in
    slot 0 of a fresh handle after the same number of steps."""
    w = di.small_2d(M=128, N=(2, 2), n_pml=6, n_ov=4, nrhs=2, seed=3)
    dev = torch.device("cuda:0")
    k2 = torch.from_numpy(w.k2.reshape(-1)).to(dev)
    f = torch.from_numpy(w.f.reshape(2, -1)).to(dev)
    prob = ddm.Problem.from_workload(w, mixed=mixed)
    s = ddm.HelmholtzDDM(prob, k2, 64)
    s.slot_admit(40, f[0])
    s.slots_step(3)
    s.slot_admit(5, f[1])
    s.slots_step(6)
    rel, steps = s.slots_poll()
    assert steps[40] == 9 and steps[5] == 6 and steps[0] == -1
    ua, ub = torch.zeros_like(f[0]), torch.zeros_like(f[1])
    s.slot_retire(40, ua)
    s.slot_retire(5, ub)
    s.close()
    for src, nsteps, got in ((f[0], 9, ua), (f[1], 6, ub)):
        t = ddm.HelmholtzDDM(prob, k2, 64)
        t.slot_admit(0, src)
        t.slots_step(nsteps)
        u = torch.zeros_like(src)
        t.slot_retire(0, u)
        t.close()
        assert torch.equal(u, got), nsteps
