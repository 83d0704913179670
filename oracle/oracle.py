"""ctypes wrapper of the C oracle (ddm_oracle.c).  Test infrastructure only.

Layouts (numpy complex128, C order):
  global vectors  [nrhs, G_z, G_y, G_x]  flattened to [nrhs, nglob]
  packed vectors  [nrhs, etot]: subdomain a occupies [off_a, off_a + |E_a|)
                  with its box stored x fastest, then y, then z.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def build_oracle(force: bool = False) -> str:
    return _build.build(force=force)


def _lib():
    global _LIB
    if _LIB is None:
        path = build_oracle(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, f64, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_long
        ip = ctypes.POINTER(ctypes.c_int)
        lib.or_create.restype = P
        lib.or_create.argtypes = [i32, ip, f64, i32, f64, ip, i32, P]
        lib.or_destroy.argtypes = [P]
        lib.or_nglob.restype = i64
        lib.or_nglob.argtypes = [P]
        lib.or_etot.restype = i64
        lib.or_etot.argtypes = [P]
        lib.or_nsub.restype = i32
        lib.or_nsub.argtypes = [P]
        lib.or_subdomain_info.argtypes = [P, i32, P]
        lib.or_apply_global.argtypes = [P, i32, P, P]
        lib.or_apply_local.argtypes = [P, i32, P, P]
        lib.or_sigma_local.restype = f64
        lib.or_sigma_local.argtypes = [P, i32, i32, f64]
        lib.or_sigma_global.restype = f64
        lib.or_sigma_global.argtypes = [P, i32, f64]
        lib.or_sigma0_for_reflection.restype = f64
        lib.or_sigma0_for_reflection.argtypes = [f64, f64, f64]
        lib.or_beta0.restype = f64
        lib.or_beta0.argtypes = [f64]
        lib.or_global_solve.restype = i32
        lib.or_global_solve.argtypes = [P, i32, P, P]
        lib.or_factor.restype = i32
        lib.or_factor.argtypes = [P]
        lib.or_local_solve.restype = i32
        lib.or_local_solve.argtypes = [P, i32, P, P]
        lib.or_restrict_core.argtypes = [P, i32, P, P]
        lib.or_transfer.argtypes = [P, i32, P, P]
        lib.or_transfer_form.argtypes = [P, i32, P, P, i32]
        lib.or_assemble.argtypes = [P, i32, P, P]
        lib.or_relres.argtypes = [P, i32, P, P, P]
        lib.or_ddm_run.restype = i32
        lib.or_ddm_run.argtypes = [P, i32, P, i32, P, P, P, P, P]
        lib.or_fgmres.restype = i32
        lib.or_fgmres.argtypes = [P, P, i32, i32, f64, i32, P, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_double)]
        _LIB = lib
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """One truncated PML problem with its DDM partition (Sec. 3.1, Alg. 3.1)."""

    def __init__(self, dim, M, h, n_pml, sigma0, N, n_ov, k2):
        lib = _lib()
        M3 = (ctypes.c_int * 3)(*(list(M) + [0] * (3 - len(M))))
        N3 = (ctypes.c_int * 3)(*(list(N) + [1] * (3 - len(N))))
        self.dim = dim
        self.M = tuple(M)[:dim]
        self.N = tuple(N)[:dim]
        self.h, self.n_pml, self.sigma0, self.n_ov = h, n_pml, sigma0, n_ov
        G = [m + 2 * n_pml - 1 for m in self.M]
        self.gshape = tuple(reversed(G))  # (Gz,) Gy, Gx
        k2 = np.ascontiguousarray(k2, dtype=np.float64).reshape(-1)
        if k2.size != int(np.prod(G)):
            raise ValueError("k2 has %d entries, grid needs %d" % (k2.size, int(np.prod(G))))
        self._k2 = k2
        self._c = lib.or_create(dim, M3, h, n_pml, sigma0, N3, n_ov, _ptr(k2))
        if not self._c:
            raise ValueError("oracle rejected the problem (divisibility, n_ov>=2, n_pml>=2, core>=n_ov+2)")
        self.nglob = lib.or_nglob(self._c)
        self.etot = lib.or_etot(self._c)
        self.nsub = lib.or_nsub(self._c)
        self._factored = False

    def __del__(self):
        if getattr(self, "_c", None):
            _lib().or_destroy(self._c)
            self._c = None

    # -- geometry ---------------------------------------------------------
    def subdomain(self, a):
        out = np.zeros(14, dtype=np.int64)
        _lib().or_subdomain_info(self._c, a, _ptr(out))
        return dict(core_lo=tuple(out[0:3]), core_hi=tuple(out[3:6]),
                    ext_lo=tuple(out[6:9]), ext_hi=tuple(out[9:12]),
                    off=int(out[12]), n=int(out[13]))

    def sigma_local(self, a, ax, x):
        return _lib().or_sigma_local(self._c, a, ax, float(x))

    def sigma_global(self, ax, x):
        return _lib().or_sigma_global(self._c, ax, float(x))

    @staticmethod
    def sigma0_for_reflection(R, k2, n_pml, h):
        """PML strength for target reflection R with k_ref = sqrt(min k^2)
        (the smallest wave number of the medium) and layer width n_pml h."""
        k_ref = float(np.sqrt(np.min(np.asarray(k2, dtype=np.float64))))
        return _lib().or_sigma0_for_reflection(float(R), k_ref, float(n_pml * h))

    @staticmethod
    def beta0(t):
        return _lib().or_beta0(float(t))

    # -- operators --------------------------------------------------------
    def apply(self, u):
        u = _c128(u)
        nrhs = u.size // self.nglob
        out = np.empty_like(u)
        _lib().or_apply_global(self._c, nrhs, _ptr(u), _ptr(out))
        return out

    def apply_local(self, a, ua):
        ua = _c128(ua)
        out = np.empty_like(ua)
        _lib().or_apply_local(self._c, a, _ptr(ua), _ptr(out))
        return out

    def global_solve(self, f):
        f = _c128(f)
        nrhs = f.size // self.nglob
        u = np.empty_like(f)
        st = _lib().or_global_solve(self._c, nrhs, _ptr(f), _ptr(u))
        if st != 0:
            raise RuntimeError("global banded LU failed, status %d" % st)
        return u

    def factor(self):
        st = _lib().or_factor(self._c)
        if st != 0:
            raise RuntimeError("local banded LU failed, status %d" % st)
        self._factored = True

    def local_solve(self, g):
        if not self._factored:
            self.factor()
        g = _c128(g)
        nrhs = g.size // self.etot
        out = np.empty_like(g)
        _lib().or_local_solve(self._c, nrhs, _ptr(g), _ptr(out))
        return out

    def restrict_core(self, f):
        f = _c128(f)
        nrhs = f.size // self.nglob
        g = np.empty((nrhs, self.etot), dtype=np.complex128)
        _lib().or_restrict_core(self._c, nrhs, _ptr(f), _ptr(g))
        return g

    def transfer(self, lagged, nrhs, form="direct"):
        """lagged[k] = packed local solutions k+1 steps back (None = zero).
        form "direct": -L_a(beta v) on chi (Sec. 2.2); "phi": the Phi form
        -(L_a(beta v) - beta L_a v) on chi (eq. Phi)."""
        keep = [None if x is None else _c128(x) for x in list(lagged) + [None] * (3 - len(lagged))]
        arr = (ctypes.c_void_p * 3)(*[_ptr(x) for x in keep])
        g = np.empty((nrhs, self.etot), dtype=np.complex128)
        _lib().or_transfer_form(self._c, nrhs, arr, _ptr(g), {"direct": 0, "phi": 1}[form])
        return g

    def assemble(self, U):
        U = _c128(U)
        nrhs = U.size // self.etot
        u = np.empty((nrhs, self.nglob), dtype=np.complex128)
        _lib().or_assemble(self._c, nrhs, _ptr(U), _ptr(u))
        return u

    def relres(self, f, u):
        f, u = _c128(f), _c128(u)
        nrhs = f.size // self.nglob
        out = np.empty(nrhs)
        _lib().or_relres(self._c, nrhs, _ptr(f), _ptr(u), _ptr(out))
        return out

    def ddm_run(self, f, nsteps, want_relres=True, want_state=False):
        """Algorithm 3.1 for nsteps steps.  Returns (u, relres[nsteps, nrhs])
        or, with want_state, (u, relres, uhat_last, U, g_last)."""
        f = _c128(f)
        nrhs = f.size // self.nglob
        u = np.empty((nrhs, self.nglob), dtype=np.complex128)
        rr = np.empty((max(nsteps, 1), nrhs)) if want_relres else None
        st = [np.empty((nrhs, self.etot), dtype=np.complex128) for _ in range(3)] if want_state else [None] * 3
        r = _lib().or_ddm_run(self._c, nrhs, _ptr(f), nsteps, _ptr(u), _ptr(rr),
                              _ptr(st[0]), _ptr(st[1]), _ptr(st[2]))
        if r != 0:
            raise RuntimeError("oracle DDM failed, status %d" % r)
        self._factored = True
        if want_state:
            return u, rr, st[0], st[1], st[2]
        return u, rr

    def fgmres(self, f, K, restart=30, tol=1e-8, maxiter=300):
        """Flexible GMRES(restart) with M_K (K DDM steps) as right
        preconditioner; K = 0 means no preconditioner.  One RHS."""
        f = _c128(f).reshape(-1)
        x = np.empty_like(f)
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        _lib().or_fgmres(self._c, _ptr(f), K, restart, tol, maxiter, _ptr(x),
                         ctypes.byref(it), ctypes.byref(rel))
        self._factored = self._factored or K > 0
        return x, it.value, rel.value
