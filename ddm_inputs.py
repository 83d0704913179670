"""Seeded synthetic inputs for the DDM Helmholtz solver and its oracle.

This module generates problem data only -- media k(x)^2, sources f and the
scalar problem parameters -- and holds none of the method's arithmetic (no
operator, cut-off, transfer or solve).  Both the CPU oracle (tests) and the HIP
library (tests, bench) are fed from here.

Grid convention (shared problem definition): per axis the physical interval
[0, L] has M cells of size h = L / M; the global unknowns are the nodes
g = -n_pml+1 ... M+n_pml-1 (x_g = g h), i.e. M + 2 n_pml - 1 of them, the
outer n_pml-1 on each side lying in the PML; arrays are C-ordered
[rhs][z][y][x].

The paper (Sec. 4) uses analytic sources (a Gaussian of unit mass and an
approximate delta shot) and constant or layered media whose velocity profile is
only shown in a figure; the layered media below are synthetic stand-ins.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 180704180


def sigma0_for_reflection(R: float, k_ref: float, delta: float) -> float:
    """PML strength for a quadratic profile sigma0 (t/delta)^2 and stretch
    alpha = 1 + i sigma: a normally incident wave crosses the layer twice and
    is damped by exp(-2 k sigma0 delta / 3); solve that for R."""
    return 3.0 * math.log(1.0 / R) / (2.0 * k_ref * delta)


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    M: Tuple[int, ...]
    L: float
    omega: float
    n_pml: int
    n_ov: int
    N: Tuple[int, ...]
    sigma0: float
    k2: np.ndarray            # global unknown grid, float64
    f: np.ndarray             # [nrhs, *grid], complex128
    c_min: float = 1.0
    c_max: float = 1.0
    notes: str = ""

    @property
    def h(self) -> float:
        return self.L / self.M[0]

    @property
    def nrhs(self) -> int:
        return self.f.shape[0]

    @property
    def grid_shape(self) -> Tuple[int, ...]:
        return tuple(m + 2 * self.n_pml - 1 for m in reversed(self.M))

    def describe(self) -> dict:
        return dict(name=self.name, dim=self.dim, M=list(self.M), N=list(self.N), n_pml=self.n_pml,
                    n_ov=self.n_ov, omega_over_2pi=self.omega / (2 * math.pi), sigma0=self.sigma0,
                    nrhs=self.nrhs, c_min=self.c_min, c_max=self.c_max)


def node_coords(M: int, n_pml: int, h: float) -> np.ndarray:
    g = np.arange(-n_pml + 1, M + n_pml, dtype=np.float64)
    return g * h


def _mesh(dim: int, M: Sequence[int], n_pml: int, h: float):
    axes = [node_coords(M[d], n_pml, h) for d in range(dim)]
    # C order [z][y][x]: reverse the axis list for meshgrid(indexing="ij")
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(grids))  # [X, Y(, Z)] each shaped like the grid


def gaussian_source(dim: int, M, n_pml: int, h: float, L: float, centre, s: float) -> np.ndarray:
    """Unit-mass Gaussian (2 pi s^2)^(-dim/2) exp(-|x - x0|^2 / (2 s^2)),
    sampled at physical nodes (0 <= x <= L) and zero in the PML."""
    X = _mesh(dim, M, n_pml, h)
    r2 = sum((X[d] - centre[d]) ** 2 for d in range(dim))
    f = (2 * math.pi * s * s) ** (-dim / 2.0) * np.exp(-r2 / (2 * s * s))
    inside = np.ones_like(f, dtype=bool)
    for d in range(dim):
        inside &= (X[d] >= -1e-12) & (X[d] <= L + 1e-12)
    return np.where(inside, f, 0.0).astype(np.complex128)


def paper_gaussian_source(dim: int, M, n_pml: int, h: float, L: float, centre, k: float) -> np.ndarray:
    """The paper's Gaussian sources of Sec. 4.1: 16 k^2/pi^3 exp(-(4k/pi)^2 r^2)
    in 2D, 64 k^3/pi^(9/2) exp(-(4k/pi)^2 r^2) in 3D (both of unit mass)."""
    X = _mesh(dim, M, n_pml, h)
    r2 = sum((X[d] - centre[d]) ** 2 for d in range(dim))
    amp = 16 * k * k / math.pi ** 3 if dim == 2 else 64 * k ** 3 / math.pi ** 4.5
    f = amp * np.exp(-((4 * k / math.pi) ** 2) * r2)
    return f.astype(np.complex128)


def delta_shot(dim: int, M, n_pml: int, h: float, node) -> np.ndarray:
    """Approximate delta source 1/h^dim at one physical node (Sec. 4.2)."""
    shape = tuple(m + 2 * n_pml - 1 for m in reversed(M))
    f = np.zeros(shape, dtype=np.complex128)
    idx = tuple(int(node[d]) + n_pml - 1 for d in reversed(range(dim)))
    f[idx] = 1.0 / h ** dim
    return f


def constant_k2(dim: int, M, n_pml: int, k: float) -> np.ndarray:
    shape = tuple(m + 2 * n_pml - 1 for m in reversed(M))
    return np.full(shape, k * k, dtype=np.float64)


def layered_velocity(dim: int, M, n_pml: int, h: float, L: float, rng: np.random.Generator,
                     n_layers: int = 8, v_lo: float = 1.5, v_hi: float = 4.5, pert: float = 0.10,
                     smooth_cells: float = 16.0) -> np.ndarray:
    """Synthetic layered medium: n_layers flat layers in the last axis (depth),
    interfaces at sorted uniform depths, layer velocities uniform in
    [v_lo, v_hi], times (1 + pert * p) with p white noise smoothed by a
    Gaussian of std smooth_cells cells and normalised to unit std, clipped to
    [v_lo, v_hi].  Constant extension into the PML (coordinates clamped)."""
    from scipy.ndimage import gaussian_filter

    depth = np.sort(rng.uniform(0.0, L, size=n_layers - 1))
    vel = rng.uniform(v_lo, v_hi, size=n_layers)
    X = _mesh(dim, M, n_pml, h)
    zc = np.clip(X[dim - 1], 0.0, L)
    layer = np.searchsorted(depth, zc)
    c = vel[layer]
    # perturbation on the physical nodes, then clamp-extended
    phys_shape = tuple(m + 1 for m in reversed(M))
    p = rng.standard_normal(phys_shape)
    p = gaussian_filter(p, sigma=smooth_cells, mode="reflect")
    p /= max(p.std(), 1e-300)
    idx = []
    for d in reversed(range(dim)):
        g = np.arange(-n_pml + 1, M[d] + n_pml)
        idx.append(np.clip(g, 0, M[d]))
    pe = p[np.ix_(*idx)]
    c = np.clip(c * (1.0 + pert * pe), v_lo, v_hi)
    return c


# ---------------------------------------------------------------------------
# The benchmark workloads (seed = BASE_SEED + a fixed per-workload offset).
# ---------------------------------------------------------------------------

def const_2d_80() -> Workload:
    """2D constant medium, omega = 2 pi 8 (10 ppw), M = 80, PML 10 cells,
    R = 1e-6, 2x2 subdomains, overlap 4, one Gaussian (s = 2h) at the centre."""
    M, n_pml, L = 80, 10, 1.0
    h = L / M
    omega = 2 * math.pi * 8
    k = omega
    s0 = sigma0_for_reflection(1e-6, k, n_pml * h)
    k2 = constant_k2(2, (M, M), n_pml, k)
    f = gaussian_source(2, (M, M), n_pml, h, L, (0.5, 0.5), 2 * h)[None]
    return Workload("2d-const-80-2x2", 2, (M, M), L, omega, n_pml, 4, (2, 2), s0, k2, f)


def const_2d_1024(nrhs: int = 4) -> Workload:
    """2D constant medium, M = 1024 (10 ppw, omega = 2 pi 102.4), PML 16,
    8x8 subdomains of 128^2, overlap 8, nrhs seeded Gaussians (s = 2h) with
    centres uniform in [0.1, 0.9]^2."""
    M, n_pml, L = 1024, 16, 1.0
    h = L / M
    omega = 2 * math.pi * 102.4
    k = omega
    s0 = sigma0_for_reflection(1e-6, k, n_pml * h)
    k2 = constant_k2(2, (M, M), n_pml, k)
    rng = np.random.default_rng(BASE_SEED + 2)
    centres = rng.uniform(0.1, 0.9, size=(nrhs, 2))
    f = np.stack([gaussian_source(2, (M, M), n_pml, h, L, tuple(c), 2 * h) for c in centres])
    return Workload("2d-const-1024-8x8", 2, (M, M), L, omega, n_pml, 8, (8, 8), s0, k2, f,
                    notes="centres=%s" % np.round(centres, 4).tolist())


def strip_2d_1024(nrhs: int = 4) -> Workload:
    """The 2D 1024^2 constant-medium problem (10 ppw, PML 16, overlap 8, the
    same seeded Gaussians) split along x only: 8 x 1 subdomains of
    128 x 1024 cells, so every transfer is horizontal (the setting in which
    the source can be written in the Phi form of eq. Phi)."""
    w = const_2d_1024(nrhs)
    return Workload("2d-const-1024-8x1", 2, w.M, w.L, w.omega, w.n_pml, w.n_ov, (8, 1), w.sigma0, w.k2, w.f,
                    notes=w.notes)


def const_2d_1024_cut(Ncut: int = 2, nrhs: int = 4) -> Workload:
    """A Ncut x Ncut block of the 2D 1024^2 workload: same mesh size h = 1/1024,
    frequency, PML, overlap and 128^2 cores (M = 128 Ncut cells), nrhs seeded
    Gaussians inside it.  Used as a bounded sample of that workload."""
    M, n_pml = 128 * Ncut, 16
    h = 1.0 / 1024
    L = M * h
    omega = 2 * math.pi * 102.4
    k = omega
    s0 = sigma0_for_reflection(1e-6, k, n_pml * h)
    k2 = constant_k2(2, (M, M), n_pml, k)
    rng = np.random.default_rng(BASE_SEED + 20 + Ncut)
    centres = rng.uniform(0.1 * L, 0.9 * L, size=(nrhs, 2))
    f = np.stack([gaussian_source(2, (M, M), n_pml, h, L, tuple(c), 2 * h) for c in centres])
    return Workload("2d-const-1024-cut-%dx%d" % (Ncut, Ncut), 2, (M, M), L, omega, n_pml, 8, (Ncut, Ncut), s0, k2, f)


def layered_2d_2048(nrhs: int = 16, M: int = 2048, N: int = 16) -> Workload:
    """2D layered medium (8 layers, 1.5-4.5, 10% smoothed perturbation),
    8 ppw at c = 1.5, PML 20, 16x16 subdomains, overlap 8, nrhs Gaussians."""
    n_pml, L = 20, 1.0
    h = L / M
    omega = 2 * math.pi * 1.5 / (8 * h)
    rng = np.random.default_rng(BASE_SEED + 3)
    c = layered_velocity(2, (M, M), n_pml, h, L, rng, smooth_cells=16.0 * M / 2048)
    k2 = (omega / c) ** 2
    s0 = sigma0_for_reflection(1e-6, omega / 4.5, n_pml * h)
    centres = rng.uniform(0.1, 0.9, size=(nrhs, 2))
    f = np.stack([gaussian_source(2, (M, M), n_pml, h, L, tuple(cc), 2 * h) for cc in centres])
    return Workload("2d-layered-%d-%dx%d" % (M, N, N), 2, (M, M), L, omega, n_pml, 8, (N, N), s0,
                    k2, f, c_min=float(c.min()), c_max=float(c.max()))


def layered_2d_2048_cut(Ncut: int = 4, nrhs: int = 16) -> Workload:
    """A bounded sample of layered_2d_2048: the Ncut x Ncut block of 128^2
    cores around the centre of the same medium (same h, omega, PML 20,
    overlap 8; the medium continued constantly into the cut's PML), nrhs
    seeded Gaussians (s = 2h) inside it."""
    full = layered_2d_2048(nrhs=1)
    M_full, n_pml = 2048, 20
    M = 128 * Ncut
    h = 1.0 / M_full
    L = M * h
    x0 = (M_full - M) // 2  # first physical node of the cut in the full grid
    c_full = full.omega / np.sqrt(full.k2.reshape(M_full + 2 * n_pml - 1, M_full + 2 * n_pml - 1))
    g = np.arange(-n_pml + 1, M + n_pml)
    idx = x0 + np.clip(g, 0, M) + n_pml - 1   # clamped cut node -> full array index
    c = c_full[np.ix_(idx, idx)]
    k2 = (full.omega / c) ** 2
    rng = np.random.default_rng(BASE_SEED + 40 + Ncut)
    centres = rng.uniform(0.1 * L, 0.9 * L, size=(nrhs, 2))
    f = np.stack([gaussian_source(2, (M, M), n_pml, h, L, tuple(cc), 2 * h) for cc in centres])
    return Workload("2d-layered-2048-cut-%dx%d" % (Ncut, Ncut), 2, (M, M), L, full.omega, n_pml, 8, (Ncut, Ncut),
                    full.sigma0, k2, f, c_min=float(c.min()), c_max=float(c.max()))


def _gaussian_2d_window(M: int, n_pml: int, h: float, centre, s: float, width: float = 12.0) -> np.ndarray:
    """The unit-mass 2D Gaussian of gaussian_source for a centre well inside
    the physical square, evaluated only within `width` standard deviations of
    the centre (outside, its value is below exp(-72) of the peak and is set to
    zero)."""
    n = M + 2 * n_pml - 1
    x = node_coords(M, n_pml, h)
    f = np.zeros((n, n), dtype=np.complex128)
    lo = [int(np.searchsorted(x, c - width * s)) for c in centre]
    hi = [int(np.searchsorted(x, c + width * s, side="right")) for c in centre]
    X, Y = np.meshgrid(x[lo[0]:hi[0]], x[lo[1]:hi[1]], indexing="xy")
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2
    f[lo[1]:hi[1], lo[0]:hi[0]] = (2 * math.pi * s * s) ** -1.0 * np.exp(-r2 / (2 * s * s))
    return f


@dataclasses.dataclass
class StreamRequest:
    """One request of the serving stream: arrival time (s), problem key
    (grid, medium, layout), the problem data (`base`: no sources) and the
    source centres; the sources are evaluated on demand (`workload`), so a
    long stream does not hold them all."""
    rid: int
    t_arrival: float
    key: Tuple
    base: Workload
    centres: np.ndarray

    @property
    def nrhs(self) -> int:
        return int(self.centres.shape[0])

    def sources(self) -> np.ndarray:
        w = self.base
        return np.stack([_gaussian_2d_window(w.M[0], w.n_pml, w.h, tuple(cc), 2 * w.h) for cc in self.centres])

    @property
    def workload(self) -> Workload:
        return dataclasses.replace(self.base, f=self.sources())


def serving_stream(n_requests: int = 48, rate: float = 4.0, grids=(256, 512, 1024), max_rhs: int = 32,
                   n_pml: int = 16, n_ov: int = 8, core: int = 128, seed: int = 0) -> List[StreamRequest]:
    """Serving stream: Poisson arrivals (exponential gaps of mean 1/rate s);
    each request draws a grid M from `grids` and a medium from a catalog of
    four per grid -- constant c = 1 at 10 and at 8 points per wavelength, and
    two seeded layered media of the 2048^2 recipe at 10 points per wavelength
    of their slowest velocity -- and 1..max_rhs Gaussian sources (std 2h,
    centres uniform in [0.1, 0.9]^2).  The layout has cores of `core` cells
    (2x2 for 256, 4x4 for 512, 8x8 for 1024).  Requests of the same (M,
    medium) share the problem: the factorisation cache key."""
    rng = np.random.default_rng(BASE_SEED + 4 + 1000 * seed)
    media = {}
    bases = {}
    out = []
    t = 0.0
    catalog = (("constant", 10.0, None), ("constant", 8.0, None), ("layered", 10.0, 0), ("layered", 10.0, 1))
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        M = int(grids[rng.integers(len(grids))])
        mi = int(rng.integers(len(catalog)))
        kind, ppw, lseed = catalog[mi]
        key = (M, "%s-%d" % (kind, mi))
        if key not in media:
            L = 1.0
            h = L / M
            if kind == "constant":
                c = np.ones(tuple(m + 2 * n_pml - 1 for m in (M, M)))
            else:
                c = layered_velocity(2, (M, M), n_pml, h, L, np.random.default_rng(BASE_SEED + 40 + M + 7 * lseed),
                                     smooth_cells=16.0 * M / 2048)
            c_min, c_max = float(c.min()), float(c.max())
            omega = 2 * math.pi * c_min / (ppw * h)
            s0 = sigma0_for_reflection(1e-6, omega / c_max, n_pml * h)
            media[key] = (L, h, omega, s0, (omega / c) ** 2, c_min, c_max)
        L, h, omega, s0, k2, c_min, c_max = media[key]
        nrhs = int(rng.integers(1, max_rhs + 1))
        centres = rng.uniform(0.1, 0.9, size=(nrhs, 2))
        N = max(M // core, 1)
        if key not in bases:
            bases[key] = Workload("serve-%d-%s" % (M, key[1]), 2, (M, M), L, omega, n_pml, n_ov, (N, N), s0, k2,
                                  np.zeros((0,) + k2.shape, dtype=np.complex128), c_min=c_min, c_max=c_max)
        out.append(StreamRequest(rid, t, key + ((N, N),), bases[key], centres))
    return out


def const_2d_2048(nrhs: int = 4, M: int = 2048, N: int = 16) -> Workload:
    """2D constant medium on the 16x16 layout of layered_2d_2048 (PML 20,
    overlap 8): omega for 10 points per wavelength, nrhs seeded Gaussians
    (s = 2h) with centres uniform in [0.1, 0.9]^2."""
    n_pml, L = 20, 1.0
    h = L / M
    omega = 2 * math.pi * M / 10.0
    s0 = sigma0_for_reflection(1e-6, omega, n_pml * h)
    k2 = constant_k2(2, (M, M), n_pml, omega)
    rng = np.random.default_rng(BASE_SEED + 6)
    centres = rng.uniform(0.1, 0.9, size=(nrhs, 2))
    f = np.stack([_gaussian_2d_window(M, n_pml, h, tuple(cc), 2 * h) for cc in centres])
    return Workload("2d-const-%d-%dx%d" % (M, N, N), 2, (M, M), L, omega, n_pml, 8, (N, N), s0, k2, f)


def paper_weak(N: int, medium: str = "constant", core: int = 300, n_pml: int = 30, n_ov: int = 8) -> Workload:
    """Weak-scaling workload shaped like the iterative-solver experiments
    (Sec. 4.2.1): N x N subdomains with core^2 cells each and n_pml PML
    cells, a delta shot (1/h^2 at one node) a quarter and a third of a core
    into the first subdomain; constant medium with omega/2pi = 25 N + 5, or
    a seeded layered medium (layered_velocity, 1.5-4.5) with
    omega/2pi = 12.5 N + 2.5.  The paper's overlap width is not stated:
    n_ov cells here."""
    M = core * N
    L = 1.0
    h = L / M
    if medium == "constant":
        omega = 2 * math.pi * (25 * N + 5)
        c = None
        k2 = constant_k2(2, (M, M), n_pml, omega)
        c_min = c_max = 1.0
    else:
        omega = 2 * math.pi * (12.5 * N + 2.5)
        c = layered_velocity(2, (M, M), n_pml, h, L, np.random.default_rng(BASE_SEED + 50 + N),
                             smooth_cells=16.0 * M / 2048)
        k2 = (omega / c) ** 2
        c_min, c_max = float(c.min()), float(c.max())
    s0 = sigma0_for_reflection(1e-6, omega / c_max, n_pml * h)
    f = delta_shot(2, (M, M), n_pml, h, (core // 4, core // 3))[None]
    return Workload("paper-weak-%s-N%d" % (medium, N), 2, (M, M), L, omega, n_pml, n_ov, (N, N), s0, k2, f,
                    c_min=c_min, c_max=c_max)


def paper_accuracy_2d(scale: int) -> Workload:
    """The 2D convergence experiment (Sec. 4.1.1, Table 1): the box
    [-1/2, 1/2]^2 meshed with 560*scale cells per side, of which the outer
    3/56 on each side is PML (30*scale cells), leaving the physical box
    [-25/56, 25/56]^2 of 500*scale cells split into 5 x 5 subdomains of
    (100*scale)^2 cells.  k/2pi = 25 (constant medium) and the paper's
    Gaussian source centred at (0.09, 0.268).  Stored on [0, 25/28]^2, i.e.
    shifted by 25/56 (the centre becomes (0.09 + 25/56, 0.268 + 25/56)).
    Overlap 8*scale cells (a fixed physical width); sigma0 for a PML
    reflection of 1e-8."""
    M = 500 * scale
    L = 25.0 / 28.0
    h = L / M
    k = 2 * math.pi * 25
    n_pml = 30 * scale
    s0 = sigma0_for_reflection(1e-8, k, n_pml * h)
    k2 = constant_k2(2, (M, M), n_pml, k)
    f = paper_gaussian_source(2, (M, M), n_pml, h, L, PAPER_ACCURACY_CENTRE_2D, k)[None]
    return Workload("paper-accuracy-2d-%d" % (560 * scale), 2, (M, M), L, k, n_pml, 8 * scale, (5, 5), s0, k2, f)


def paper_accuracy_3d(mesh: int) -> Workload:
    """The 3D convergence experiment (Sec. 4.1.2, Table 2): the box
    [-1/2, 1/2]^3 meshed with `mesh` cells per side (a multiple of 8), of
    which the outer 1/8 on each side is PML, leaving the physical box
    [-3/8, 3/8]^3 of 3 mesh / 4 cells split into 3 x 3 x 3 subdomains.
    k/2pi = 10 (constant medium), the paper's Gaussian source centred at
    (0.12, 0.133, 0.125).  Stored on [0, 3/4]^3 (shifted by 3/8); overlap
    mesh / 20 cells rounded (4 at 80, 5 at 96); sigma0 for R = 1e-8."""
    if mesh % 8:
        raise ValueError("mesh must be a multiple of 8")
    M = 3 * mesh // 4
    L = 0.75
    h = L / M
    k = 2 * math.pi * 10
    n_pml = mesh // 8
    s0 = sigma0_for_reflection(1e-8, k, n_pml * h)
    k2 = constant_k2(3, (M, M, M), n_pml, k)
    f = paper_gaussian_source(3, (M, M, M), n_pml, h, L, PAPER_ACCURACY_CENTRE_3D, k)[None]
    return Workload("paper-accuracy-3d-%d" % mesh, 3, (M, M, M), L, k, n_pml, int(round(mesh / 20)), (3, 3, 3),
                    s0, k2, f)


# source centre of the 2D convergence experiment on the stored box [0, 25/28]^2
PAPER_ACCURACY_CENTRE_2D = (0.09 + 25.0 / 56.0, 0.268 + 25.0 / 56.0)
# and of the 3D one on [0, 3/4]^3
PAPER_ACCURACY_CENTRE_3D = (0.12 + 0.375, 0.133 + 0.375, 0.125 + 0.375)


def const_3d_96(M: int = 96, N: int = 3, n_pml: int = 6, n_ov: int = 2) -> Workload:
    """3D constant medium, M = 96 (10 ppw, omega = 2 pi 9.6), PML 6, 3x3x3
    subdomains, overlap 2, Gaussian (s = 2h) at the centre."""
    L = 1.0
    h = L / M
    omega = 2 * math.pi * M / 10.0
    k = omega
    s0 = sigma0_for_reflection(1e-6, k, n_pml * h)
    k2 = constant_k2(3, (M, M, M), n_pml, k)
    f = gaussian_source(3, (M, M, M), n_pml, h, L, (0.5, 0.5, 0.5), 2 * h)[None]
    return Workload("3d-const-%d-%dx%dx%d" % (M, N, N, N), 3, (M, M, M), L, omega, n_pml, n_ov, (N, N, N),
                    s0, k2, f)


def small_2d(M: int = 32, N=(2, 2), n_pml: int = 4, n_ov: int = 3, ppw: float = 10.0, nrhs: int = 1,
             layered: bool = False, seed: int = 0) -> Workload:
    """Small 2D problem for parity tests (oracle finishes in seconds)."""
    L = 1.0
    h = L / M
    rng = np.random.default_rng(BASE_SEED + 100 + seed)
    if layered:
        c = layered_velocity(2, (M, M), n_pml, h, L, rng, n_layers=4, smooth_cells=2.0)
        omega = 2 * math.pi * float(c.min()) / (ppw * h)
        k2 = (omega / c) ** 2
        kref = omega / float(c.max())
    else:
        omega = 2 * math.pi / (ppw * h)
        k2 = constant_k2(2, (M, M), n_pml, omega)
        kref = omega
        c = np.ones(1)
    s0 = sigma0_for_reflection(1e-6, kref, n_pml * h)
    centres = rng.uniform(0.15, 0.85, size=(nrhs, 2))
    f = np.stack([gaussian_source(2, (M, M), n_pml, h, L, tuple(cc), 2 * h) for cc in centres])
    return Workload("small2d-%d-%dx%d" % (M, N[0], N[1]), 2, (M, M), L, omega, n_pml, n_ov, tuple(N), s0,
                    k2, f, c_min=float(c.min()), c_max=float(c.max()))


def small_3d(M: int = 16, N=(2, 2, 2), n_pml: int = 3, n_ov: int = 2, ppw: float = 8.0, nrhs: int = 1,
             seed: int = 0) -> Workload:
    L = 1.0
    h = L / M
    omega = 2 * math.pi / (ppw * h)
    k2 = constant_k2(3, (M, M, M), n_pml, omega)
    s0 = sigma0_for_reflection(1e-6, omega, n_pml * h)
    rng = np.random.default_rng(BASE_SEED + 200 + seed)
    centres = rng.uniform(0.2, 0.8, size=(nrhs, 3))
    f = np.stack([gaussian_source(3, (M, M, M), n_pml, h, L, tuple(cc), 2 * h) for cc in centres])
    return Workload("small3d-%d" % M, 3, (M, M, M), L, omega, n_pml, n_ov, tuple(N), s0, k2, f)


def random_field(shape, seed: int) -> np.ndarray:
    """Seeded complex normal field (for operator and solve parity tests)."""
    rng = np.random.default_rng(BASE_SEED + 1000 + seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex128)
