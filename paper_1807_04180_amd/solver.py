"""Python binding of libddm: argument marshalling only.

Every array argument is a torch tensor on the HIP device (complex128 for
global / packed vectors, float64 for k^2); shapes follow include/ddm.h:
global vectors [nrhs, nglob] (C order [z][y][x] inside), packed subdomain
vectors [nrhs, etot].  All calls run on the torch stream current at
construction.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence, Tuple

import torch

from . import _ffi


class DDMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ffi.STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


@dataclasses.dataclass
class Problem:
    """The truncated PML problem and its partition (include/ddm.h ddm_problem)."""
    dim: int
    M: Sequence[int]
    h: float
    n_pml: int
    sigma0: float
    N: Sequence[int]
    n_ov: int
    mixed: bool = False
    hbm_budget_bytes: int = 0
    reflection: float = 0.0   # > 0: the library derives sigma0 (then 0) from it

    def to_c(self, k2_on_host: bool = False) -> _ffi.DdmProblem:
        p = _ffi.DdmProblem()
        p.dim = self.dim
        M = list(self.M) + [0] * (3 - len(self.M))
        N = list(self.N) + [1] * (3 - len(self.N))
        for d in range(3):
            p.M[d] = int(M[d]) if d < self.dim else 0
            p.N[d] = int(N[d]) if d < self.dim else 1
        p.h = float(self.h)
        p.n_pml = int(self.n_pml)
        p.sigma0 = float(self.sigma0)
        p.n_ov = int(self.n_ov)
        p.precision = _ffi.DDM_MIXED if self.mixed else _ffi.DDM_FP64
        p.hbm_budget_bytes = int(self.hbm_budget_bytes)
        p.reflection = float(self.reflection)
        p.k2_on_host = 1 if k2_on_host else 0
        return p

    @classmethod
    def from_workload(cls, w, mixed: bool = False, hbm_budget_bytes: int = 0) -> "Problem":
        return cls(w.dim, tuple(w.M), w.h, w.n_pml, w.sigma0, tuple(w.N), w.n_ov, mixed, hbm_budget_bytes)

    def memory_required(self, nrhs_max: int) -> int:
        b = ctypes.c_size_t(0)
        p = self.to_c()
        L = _ffi.lib()
        st = L.ddm_memory_required(ctypes.byref(p), nrhs_max, ctypes.byref(b))
        if st != 0:
            raise DDMError(st, L.ddm_last_error(None).decode())
        return b.value


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the HIP device")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check_c128(t: torch.Tensor, n: int, name: str) -> int:
    if t.dtype != torch.complex128:
        raise TypeError("%s must be complex128" % name)
    if t.numel() % n != 0:
        raise ValueError("%s has %d entries, not a multiple of %d" % (name, t.numel(), n))
    return t.numel() // n


class HelmholtzDDM:
    """Handle on one factored problem (ddm_setup + ddm_factor).  k2 (float64,
    nglob entries) may be a device tensor or host memory (a CPU tensor)."""

    def __init__(self, problem: Problem, k2: torch.Tensor, nrhs_max: int, factor: bool = True):
        self.lib = _ffi.lib()
        self.problem = problem
        if k2.dtype != torch.float64:
            raise TypeError("k2 must be float64")
        k2 = k2.contiguous()
        on_host = not k2.is_cuda
        self.device = torch.device("cuda", torch.cuda.current_device()) if on_host else k2.device
        self.stream = torch.cuda.current_stream(self.device)
        p = problem.to_c(k2_on_host=on_host)
        h = ctypes.c_void_p()
        kp = ctypes.c_void_p(k2.data_ptr()) if on_host else _ptr(k2)
        st = self.lib.ddm_setup(ctypes.byref(p), kp, int(nrhs_max), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h))
        if st != 0:
            raise DDMError(st, self.lib.ddm_last_error(None).decode())
        self._h = h
        self.nrhs_max = nrhs_max
        sz = (ctypes.c_long * 4)()
        self.lib.ddm_sizes(self._h, sz)
        self.nglob, self.etot, self.nsub, self.factor_bytes = int(sz[0]), int(sz[1]), int(sz[2]), int(sz[3])
        self.factored = False
        if factor:
            self.factor()

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self.lib.ddm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st < 0:
            raise DDMError(st, self.lib.ddm_last_error(self._h).decode())
        return st

    def factor(self):
        self._check(self.lib.ddm_factor(self._h))
        self.factored = True

    def pml_strength(self) -> float:
        v = ctypes.c_double(0.0)
        self._check(self.lib.ddm_pml_strength(self._h, ctypes.byref(v)))
        return v.value

    def device_bytes(self) -> Tuple[int, int]:
        """(bytes held now, most bytes held at once) on the device."""
        held, peak = ctypes.c_size_t(0), ctypes.c_size_t(0)
        self._check(self.lib.ddm_device_bytes(self._h, ctypes.byref(held), ctypes.byref(peak)))
        return held.value, peak.value

    # -- geometry ----------------------------------------------------------
    def geometry(self, a: int) -> dict:
        out = (ctypes.c_long * 14)()
        self._check(self.lib.ddm_geometry(self._h, a, out))
        v = list(out)
        return dict(core_lo=tuple(v[0:3]), core_hi=tuple(v[3:6]), ext_lo=tuple(v[6:9]), ext_hi=tuple(v[9:12]),
                    off=v[12], n=v[13])

    def zeros_global(self, nrhs: int) -> torch.Tensor:
        return torch.zeros((nrhs, self.nglob), dtype=torch.complex128, device=self.device)

    def zeros_packed(self, nrhs: int) -> torch.Tensor:
        return torch.zeros((nrhs, self.etot), dtype=torch.complex128, device=self.device)

    # -- single-step entry points -----------------------------------------
    def apply(self, u: torch.Tensor) -> torch.Tensor:
        nrhs = _check_c128(u, self.nglob, "u")
        out = torch.empty_like(u)
        self._check(self.lib.ddm_apply(self._h, _ptr(u), _ptr(out), nrhs))
        return out

    def residual(self, f: torch.Tensor, u: torch.Tensor, want_r: bool = True):
        nrhs = _check_c128(f, self.nglob, "f")
        r = torch.empty_like(f) if want_r else None
        rn = (ctypes.c_double * nrhs)()
        fn = (ctypes.c_double * nrhs)()
        self._check(self.lib.ddm_residual(self._h, _ptr(f), _ptr(u), _ptr(r), nrhs, rn, fn))
        return r, list(rn), list(fn)

    def residual_noalloc(self, f: torch.Tensor, u: torch.Tensor, r: Optional[torch.Tensor] = None,
                         norms: Optional[torch.Tensor] = None) -> torch.Tensor:
        """ddm_residual_noalloc: r (if given) = f - L_h u; returns the device
        tensor norms = [||r_q||^2 ..., ||f_q||^2 ...] (float64, 2 nrhs),
        written asynchronously on the handle's stream."""
        nrhs = _check_c128(f, self.nglob, "f")
        if norms is None:
            norms = torch.empty(2 * nrhs, dtype=torch.float64, device=f.device)
        if norms.dtype != torch.float64 or norms.numel() < 2 * nrhs:
            raise ValueError("norms must be float64 with at least 2 nrhs entries")
        self._check(self.lib.ddm_residual_noalloc(self._h, _ptr(f), _ptr(u), _ptr(r), nrhs, _ptr(norms)))
        return norms

    def restrict_core(self, f: torch.Tensor) -> torch.Tensor:
        nrhs = _check_c128(f, self.nglob, "f")
        g = self.zeros_packed(nrhs)
        self._check(self.lib.ddm_restrict_core(self._h, _ptr(f), _ptr(g), nrhs))
        return g

    def local_solve(self, g: torch.Tensor) -> torch.Tensor:
        nrhs = _check_c128(g, self.etot, "g")
        x = torch.empty_like(g)
        self._check(self.lib.ddm_local_solve(self._h, _ptr(g), _ptr(x), nrhs))
        return x

    def transfer(self, lag1, lag2=None, lag3=None) -> torch.Tensor:
        ref = next(t for t in (lag1, lag2, lag3) if t is not None)
        nrhs = _check_c128(ref, self.etot, "lag")
        g = self.zeros_packed(nrhs)
        self._check(self.lib.ddm_transfer(self._h, _ptr(lag1), _ptr(lag2), _ptr(lag3), _ptr(g), nrhs))
        return g

    def assemble(self, U: torch.Tensor) -> torch.Tensor:
        nrhs = _check_c128(U, self.etot, "U")
        u = self.zeros_global(nrhs)
        self._check(self.lib.ddm_assemble(self._h, _ptr(U), _ptr(u), nrhs))
        return u

    # -- tuning --------------------------------------------------------------
    def set_factor_layout(self, twisted: bool, refactor: bool = True):
        self._check(self.lib.ddm_set_factor_layout(self._h, 1 if twisted else 0))
        self.factored = False
        if refactor:
            self.factor()

    # -- tuning --------------------------------------------------------------
    def set_solve_variant(self, variant):
        v = _ffi.SOLVE_VARIANTS.index(variant) if isinstance(variant, str) else int(variant)
        self._check(self.lib.ddm_set_solve_variant(self._h, v))

    def solve_variant(self) -> str:
        return _ffi.SOLVE_VARIANTS[self.lib.ddm_get_solve_variant(self._h)]

    def autotune(self, nrhs: Optional[int] = None, reps: int = 3) -> dict:
        t = (ctypes.c_double * len(_ffi.SOLVE_VARIANTS))()
        self._check(self.lib.ddm_autotune(self._h, int(nrhs or self.nrhs_max), reps, t))
        return {name: (t[i] if t[i] >= 0 else None) for i, name in enumerate(_ffi.SOLVE_VARIANTS)}

    def set_chain_tile(self, rt: int):
        self._check(self.lib.ddm_set_chain_tile(self._h, int(rt)))

    def time_local_solve(self, nrhs: Optional[int] = None, reps: int = 3) -> float:
        ms = ctypes.c_double(0.0)
        self._check(self.lib.ddm_time_local_solve(self._h, int(nrhs or self.nrhs_max), int(reps), ctypes.byref(ms)))
        return ms.value

    def set_graphs(self, on: bool):
        self._check(self.lib.ddm_set_graphs(self._h, 1 if on else 0))

    def graph_launches(self) -> int:
        return int(self.lib.ddm_graph_launches(self._h))

    def set_spin_limit(self, limit: int):
        self._check(self.lib.ddm_set_spin_limit(self._h, int(limit)))

    def set_transfer_form(self, form: str):
        """"direct": -L_a(beta v) chi (default); "phi": the k-free commutator
        form -(L_a(beta v) - beta L_a v) chi (eq. Phi)."""
        self._check(self.lib.ddm_set_transfer_form(self._h, _ffi.TRANSFER_FORMS.index(form)))

    # -- continuous batching (slots) -------------------------------------
    def slot_admit(self, slot: int, f: torch.Tensor):
        if f.dtype != torch.complex128 or f.numel() != self.nglob:
            raise ValueError("f must be one complex128 global vector")
        self._check(self.lib.ddm_slot_admit(self._h, int(slot), _ptr(f.contiguous())))

    def slots_step(self, nsteps: int = 1):
        self._check(self.lib.ddm_slots_step(self._h, int(nsteps)))

    def slots_poll(self):
        rel = (ctypes.c_double * self.nrhs_max)()
        st = (ctypes.c_int * self.nrhs_max)()
        self._check(self.lib.ddm_slots_poll(self._h, rel, st))
        return list(rel), list(st)

    def slot_retire(self, slot: int, u: Optional[torch.Tensor] = None):
        self._check(self.lib.ddm_slot_retire(self._h, int(slot), _ptr(u)))

    # -- observability -----------------------------------------------------
    def profile_enable(self, on: bool = True):
        self._check(self.lib.ddm_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        p = _ffi.DdmProfile()
        self._check(self.lib.ddm_profile_read(self._h, ctypes.byref(p)))
        return {name: dict(launches=int(p.launches[i]), ms=float(p.ms[i]), bytes=float(p.bytes[i]))
                for i, name in enumerate(_ffi.KERNEL_CLASSES)}

    # -- drivers -------------------------------------------------------------
    def iterate(self, f: torch.Tensor, nsteps: int, want_relres: bool = True):
        nrhs = _check_c128(f, self.nglob, "f")
        u = torch.empty_like(f)
        rr = (ctypes.c_double * max(1, nsteps * nrhs))() if want_relres else None
        self._check(self.lib.ddm_iterate(self._h, _ptr(f), _ptr(u), nrhs, nsteps, rr))
        rel = None
        if want_relres:
            rel = [[rr[s * nrhs + q] for q in range(nrhs)] for s in range(nsteps)]
        return u, rel

    def solve(self, f: torch.Tensor, method: str = "stationary", tol: float = 1e-6, maxiter: int = 500,
              restart: int = 30, K: int = 0, refine_every: int = 0, u: Optional[torch.Tensor] = None,
              check_every: int = 1):
        nrhs = _check_c128(f, self.nglob, "f")
        if u is None:
            u = torch.empty_like(f)
        o = _ffi.DdmSolveOpts()
        o.method = _ffi.DDM_FGMRES if method == "fgmres" else _ffi.DDM_STATIONARY
        o.tol, o.maxiter, o.restart, o.K, o.refine_every = tol, maxiter, restart, K, refine_every
        o.check_every = check_every
        info = (_ffi.DdmRhsInfo * nrhs)()
        st = self._check(self.lib.ddm_solve(self._h, _ptr(f), _ptr(u), nrhs, ctypes.byref(o), info))
        infos = [dict(iters=i.iters, local_solves=i.local_solves, relres=i.relres, seconds=i.seconds,
                      status=_ffi.STATUS_NAMES.get(i.status, str(i.status))) for i in info]
        return u, infos, st
