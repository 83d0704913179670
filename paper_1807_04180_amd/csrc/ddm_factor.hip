// Block-tridiagonal factorisation of every subdomain operator (the direct
// local solver of Algorithm 3.1; the paper used a multifrontal LU).
//
// Unknowns of a subdomain box are grouped into blocks along its last axis
// (grid lines in 2D, grid planes in 3D).  The 5/7-point operator couples block
// l only to l-1 and l+1, through C_l = cm(l) I and B_l = cp(l) I, the 1D
// coefficients of the last axis.  The factorisation is
//     S_0 = D_0,   S_l = D_l - cm(l) cp(l-1) W_{l-1},   W_l = S_l^{-1},
// and W_l is stored column-major (element (i, j) at j * ld + i, ld = bs or the
// next even number for complex64), complex128
// or complex64.  Since C_l and B_l are multiples of the identity, the Schur
// complement update is a scaled copy; the dense work is the inversion of
// every S_l, done in FP64 by blocked Gauss-Jordan elimination with partial
// pivoting:
//   * panels of kPanel columns; a panel kernel (one workgroup per chain)
//     picks the panel's pivot rows by unblocked elimination of a copy of the
//     panel (by sub-panels for blocks above 512 rows), inverts the kPanel x
//     kPanel pivot block A11 and forms
//     Y = A11^{-1} [pivot rows of S] and X = -[panel columns of S], pivot rows
//     zeroed;
//   * an update kernel applies S <- S + X Y (panel columns start from zero,
//     pivot rows become Y) over 64 x 64 tiles with FP64 MFMA
//     (v_mfma_f64_16x16x4, complex product as four real products); every
//     chain's tiles go into one launch;
//   * blocks of more than 512 rows defer the update over groups of kDefer
//     panels: each panel of a group is factored from its columns and pivot
//     rows brought up to date by narrow products, and one update of rank
//     kDefer * kPanel applies the group, so the block is read and written
//     once per group instead of once per panel;
//   * pivot rows are never swapped: row r chosen at step k is recorded
//     (ppos[r] = k, piv[k] = r) and the inverse is read back as
//     W(i, j) = N(piv[i], ppos[j]) when the block is stored.
// The elimination runs from both ends of the subdomain towards a middle
// block mid (a twisted factorisation; mid = nb - 1 is the one-directional
// case); all chains advance in lock step, one launch per panel step, then the
// middle blocks are inverted the same way.  Each chain owns two FP64 block
// buffers (the block being inverted and the next Schur complement).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "cplx.h"
#include "ddm_internal.h"
#include "ddm_mma.h"

namespace ddm {

struct FactArgs {
    int dim;
    int G0, G1;
    int glo0, glo1, glo2;
    int bs_max;
    int nsub;
};

// block-wide argmax of (value, index) over NW waves; ties go to the smaller index
template <int NW>
__device__ inline void block_argmax_n(double &v, int &idx, double *sv, int *si) {
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_down(v, o, 64);
        int oi = __shfl_down(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sv[w] = v; si[w] = idx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NW; ++i)
            if (sv[i] > sv[0] || (sv[i] == sv[0] && si[i] < si[0])) { sv[0] = sv[i]; si[0] = si[i]; }
    }
    __syncthreads();
    v = sv[0];
    idx = si[0];
    __syncthreads();
}

template <int NW>
__device__ inline double block_max_n(double v, double *sv) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sv[w] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 1; i < NW; ++i) sv[0] = fmax(sv[0], sv[i]);
    __syncthreads();
    v = sv[0];
    __syncthreads();
    return v;
}

// In-block operator D_l(i, j): in-line / in-plane part of the 5/7-point
// operator plus the diagonal of the last-axis coupling.
__device__ inline double2 block_entry(const SubDesc &s, const Coef *__restrict__ coef, const double *__restrict__ k2,
                                     const FactArgs &A, int l, int i, int j, const Coef &cl) {
    int nx = s.n[0];
    double2 v = make_double2(0, 0);
    if (A.dim == 2) {
        if (j == i) {
            Coef cx = coef[s.coff[0] + i];
            long long gi = (long long)(s.lo[0] + i - A.glo0) + (long long)A.G0 * (s.lo[1] + l - A.glo1);
            v.x = k2[gi] - cx.cp.x - cx.cm.x - cl.cp.x - cl.cm.x;
            v.y = -cx.cp.y - cx.cm.y - cl.cp.y - cl.cm.y;
        } else if (j == i + 1) {
            v = coef[s.coff[0] + i].cp;
        } else if (j == i - 1) {
            v = coef[s.coff[0] + i].cm;
        }
    } else {
        int xi = i % nx, yi = i / nx;
        if (j == i) {
            Coef cx = coef[s.coff[0] + xi], cy = coef[s.coff[1] + yi];
            long long gi = (long long)(s.lo[0] + xi - A.glo0) +
                           (long long)A.G0 * ((long long)(s.lo[1] + yi - A.glo1) + (long long)A.G1 * (s.lo[2] + l - A.glo2));
            v.x = k2[gi] - cx.cp.x - cx.cm.x - cy.cp.x - cy.cm.x - cl.cp.x - cl.cm.x;
            v.y = -cx.cp.y - cx.cm.y - cy.cp.y - cy.cm.y - cl.cp.y - cl.cm.y;
        } else if (j == i + 1 && xi + 1 < nx) {
            v = coef[s.coff[0] + xi].cp;
        } else if (j == i - 1 && xi > 0) {
            v = coef[s.coff[0] + xi].cm;
        } else if (j == i + nx) {
            v = coef[s.coff[1] + yi].cp;
        } else if (j == i - nx) {
            v = coef[s.coff[1] + yi].cm;
        }
    }
    return v;
}


constexpr int kPanel = 32;      // panel width (columns per elimination panel)
constexpr int kPThreads = 512;  // panel kernel
constexpr int kPWaves = kPThreads / 64;
constexpr int kUTile = 64;      // update tile edge
constexpr int kUThreads = 256;  // update kernel: 2 x 2 waves of 32 x 32
constexpr int kEThreads = 256;  // form / store kernels
constexpr int kEGroups = 64;    // max workgroups per chain for form / store

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Blocks of more than 512 rows defer their trailing updates: kDefer panels
// are factored against the block as it stood before the first of them (each
// panel's columns and pivot rows brought up to date by narrow products), then
// one update of rank kDefer * kPanel applies all of them.
constexpr int kDefer = 4;
constexpr int kSPRows = 4096;  // largest block of the sub-panel kernel

// deferral goes with the sub-panel kernel (blocks of 513 .. kSPRows rows)
static int defer_slots(const Plan &P) {
    return P.bs_max > 512 && P.bs_max <= kSPRows ? kDefer : 1;
}

// Per-chain factor workspace (chain c = 2 * subdomain + direction).
struct FactWs {
    double2 *M;         // [chain][2][bs_max^2] FP64 block buffers
    double *X, *Y;      // [chain][slot][re, im][kPanel][bsp] panel operands of the deferred panels
    double2 *Pw;        // [chain][kPanel][bsp] panel work (when not in LDS)
    double2 *C;         // [chain][kPanel][bsp] up-to-date columns of a deferred panel (slots > 1)
    int *ppos, *piv;    // [chain][bsp] pivot step of a row / row of a pivot step
    unsigned long long *mxb;  // [chain][buffer] max |entry|^2 of a block buffer (FP64 bits)
    long long mstride;  // bs_max^2
    int bsp;            // bs_max rounded up to kUTile
    int slots;          // panels whose update can be deferred (1 or kDefer)
};

size_t factor_ws_bytes(const Plan &P) {
    const size_t bsp = (size_t)((P.bs_max + kUTile - 1) / kUTile) * kUTile;
    const size_t nc = (size_t)2 * P.nsub;
    const size_t slots = (size_t)defer_slots(P);
    size_t b = nc * 2 * (size_t)P.bs_max * P.bs_max * sizeof(double2);
    b += nc * slots * 4 * kPanel * bsp * sizeof(double);
    b += nc * kPanel * bsp * sizeof(double2);
    if (slots > 1) b += nc * kPanel * bsp * sizeof(double2);
    b += nc * 2 * bsp * sizeof(int) + nc * 2 * sizeof(double);
    return b + 4096;
}

static FactWs carve_ws(const Plan &P, void *base) {
    FactWs w;
    w.bsp = ((P.bs_max + kUTile - 1) / kUTile) * kUTile;
    w.mstride = (long long)P.bs_max * P.bs_max;
    w.slots = defer_slots(P);
    const size_t nc = (size_t)2 * P.nsub;
    char *p = (char *)base;
    w.M = (double2 *)p;  p += nc * 2 * w.mstride * sizeof(double2);
    w.X = (double *)p;   p += nc * w.slots * 2 * kPanel * w.bsp * sizeof(double);
    w.Y = (double *)p;   p += nc * w.slots * 2 * kPanel * w.bsp * sizeof(double);
    w.Pw = (double2 *)p; p += nc * kPanel * w.bsp * sizeof(double2);
    w.C = nullptr;
    if (w.slots > 1) {
        w.C = (double2 *)p;
        p += nc * kPanel * w.bsp * sizeof(double2);
    }
    w.ppos = (int *)p;   p += nc * w.bsp * sizeof(int);
    w.piv = (int *)p;    p += nc * w.bsp * sizeof(int);
    p = (char *)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    w.mxb = (unsigned long long *)p;
    return w;
}

// Real parts of chain c's X (or Y) of deferred slot k; the imaginary parts
// follow kPanel * bsp doubles later.  Element (row i, panel column t) of X
// is at t * bsp + i, element (t, column j) of Y at t * bsp + j.
__device__ inline double *ws_x(const FactWs &w, int c, int k) {
    return w.X + ((long long)c * w.slots + k) * 2 * kPanel * w.bsp;
}
__device__ inline double *ws_y(const FactWs &w, int c, int k) {
    return w.Y + ((long long)c * w.slots + k) * 2 * kPanel * w.bsp;
}

// Where chain c stands at lock-step s (mid == false), or at its subdomain's
// middle block (mid == true; only even chains take part).
struct ChainPos {
    bool active;
    int a, dir, l, bs, nb, cur, len, last;
};

__device__ inline ChainPos chain_pos(const SubDesc *__restrict__ subs, int c, int s, bool mid) {
    ChainPos q;
    q.a = c >> 1;
    q.dir = c & 1;
    const SubDesc &sd = subs[q.a];
    q.bs = sd.bs;
    q.nb = sd.nb;
    const int len0 = sd.mid, len1 = sd.nb - 1 - sd.mid;
    if (!mid) {
        q.len = q.dir == 0 ? len0 : len1;
        q.active = s < q.len;
        q.l = q.dir == 0 ? s : sd.nb - 1 - s;
        q.cur = s & 1;
        q.last = s + 1 == q.len;
    } else {
        q.len = len0;
        q.active = q.dir == 0;
        q.l = sd.mid;
        q.cur = (len0 & 1) ^ 1;
        q.last = 1;
    }
    return q;
}

__device__ inline double2 *chain_M(const FactWs &w, int c, int buf) {
    return w.M + ((long long)c * 2 + buf) * w.mstride;
}

// fold a workgroup's max |entry|^2 into a buffer's slot (non-negative
// doubles order like their bit patterns)
__device__ inline void slot_max(unsigned long long *slot, double v) {
    __shared__ double sv[kEThreads / 64];
    v = block_max_n<kEThreads / 64>(v, sv);
    if (threadIdx.x == 0) atomicMax(slot, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double slot_read(const unsigned long long *slot) {
    return __longlong_as_double((long long)*slot);
}

// First block of every chain: M[c][0] = D_first.
__global__ __launch_bounds__(kEThreads) void k_factor_form0(const SubDesc *__restrict__ subs,
                                                            const Coef *__restrict__ coef,
                                                            const double *__restrict__ k2, FactArgs A, FactWs w,
                                                            int groups) {
    const int c = blockIdx.x / groups, grp = blockIdx.x % groups;
    const ChainPos q = chain_pos(subs, c, 0, false);
    if (!q.active) return;
    const SubDesc &s = subs[q.a];
    const Coef cl = coef[s.coff[A.dim - 1] + q.l];
    double2 *M = chain_M(w, c, 0);
    const long long n2 = (long long)q.bs * q.bs;
    double m = 0.0;
    for (long long e = (long long)grp * kEThreads + threadIdx.x; e < n2; e += (long long)groups * kEThreads) {
        const int i = (int)(e % q.bs), j = (int)(e / q.bs);
        const double2 v = block_entry(s, coef, k2, A, q.l, i, j, cl);
        M[e] = v;
        m = fmax(m, cabs2(v));
    }
    slot_max(w.mxb + 2 * c, m);
}

// Middle block of every subdomain:
// Z = D_mid - cm(mid) cp(mid-1) S_{mid-1}^{-1} - cp(mid) cm(mid+1) T_{mid+1}^{-1},
// the two inverses being the chains' final buffers.
__global__ __launch_bounds__(kEThreads) void k_factor_formmid(const SubDesc *__restrict__ subs,
                                                              const Coef *__restrict__ coef,
                                                              const double *__restrict__ k2, FactArgs A, FactWs w,
                                                              int groups) {
    const int a = blockIdx.x / groups, grp = blockIdx.x % groups;
    const SubDesc &s = subs[a];
    const int ax = A.dim - 1, l = s.mid, bs = s.bs;
    const int len0 = s.mid, len1 = s.nb - 1 - s.mid;
    const Coef cl = coef[s.coff[ax] + l];
    const double2 c1 = len0 > 0 ? cmul(cl.cm, coef[s.coff[ax] + l - 1].cp) : make_double2(0, 0);
    const double2 c2 = len1 > 0 ? cmul(cl.cp, coef[s.coff[ax] + l + 1].cm) : make_double2(0, 0);
    const double2 *I0 = len0 > 0 ? chain_M(w, 2 * a, len0 & 1) : nullptr;
    const double2 *I1 = len1 > 0 ? chain_M(w, 2 * a + 1, len1 & 1) : nullptr;
    double2 *Z = chain_M(w, 2 * a, (len0 & 1) ^ 1);
    const long long n2 = (long long)bs * bs;
    double m = 0.0;
    for (long long e = (long long)grp * kEThreads + threadIdx.x; e < n2; e += (long long)groups * kEThreads) {
        const int i = (int)(e % bs), j = (int)(e / bs);
        double2 v = block_entry(s, coef, k2, A, l, i, j, cl);
        if (I0) v = csub(v, cmul(c1, I0[e]));
        if (I1) v = csub(v, cmul(c2, I1[e]));
        Z[e] = v;
        m = fmax(m, cabs2(v));
    }
    slot_max(w.mxb + 2 * (2 * a) + ((len0 & 1) ^ 1), m);
}

// Panel kernel: pivots, A11^{-1}, X and Y of panel p (columns k0 .. k0+bw-1)
// of the block chain c is inverting; the eliminated copy of the panel lives
// in LDS (PW_LDS) or in the chain's workspace (blocks of thousands of rows).
template <bool PW_LDS>
__global__ __launch_bounds__(kPThreads) void k_factor_panel(const SubDesc *__restrict__ subs, FactWs w, int s, int p,
                                                            int mid, int *__restrict__ flags, int nsub) {
    extern __shared__ double2 lds[];
    __shared__ double sv[kPWaves];
    __shared__ int si[kPWaves];
    const int c = blockIdx.x;
    const ChainPos q = chain_pos(subs, c, s, mid != 0);
    if (!q.active) return;
    const int bs = q.bs, bsp = w.bsp, k0 = p * kPanel;
    if (k0 >= bs) return;
    const int bw = bs - k0 < kPanel ? bs - k0 : kPanel;
    const double2 *M = chain_M(w, c, q.cur);
    double *Xr = ws_x(w, c, 0), *Xi = Xr + (long long)kPanel * bsp;
    double *Yr = ws_y(w, c, 0), *Yi = Yr + (long long)kPanel * bsp;
    int *ppos = w.ppos + (long long)c * bsp, *piv = w.piv + (long long)c * bsp;
    double2 *Ainv = lds;                      // [kPanel][kPanel]
    double2 *rowr = Ainv + kPanel * kPanel;   // [kPanel]
    int *R1 = (int *)(rowr + kPanel);         // [kPanel]
    int *ppos_s = R1 + kPanel;                // [bsp]
    double2 *Pw;
    if constexpr (PW_LDS) Pw = (double2 *)(ppos_s + bsp);
    else Pw = w.Pw + (long long)c * kPanel * bsp;
    const int tid = threadIdx.x;
    const double mx = slot_read(w.mxb + 2 * c + q.cur);
    if (p == 0) {
        for (int i = tid; i < bsp; i += kPThreads) ppos_s[i] = -1;
        if (tid == 0) w.mxb[2 * c + (q.cur ^ 1)] = 0ull;  // the store of this step fills it
    } else {
        for (int i = tid; i < bsp; i += kPThreads) ppos_s[i] = ppos[i];
    }
    // working copy of the panel; X = -panel
    for (int e = tid; e < kPanel * bsp; e += kPThreads) {
        const int t = e / bsp, i = e % bsp;
        const double2 v = (t < bw && i < bs) ? M[(long long)(k0 + t) * bs + i] : make_double2(0, 0);
        Pw[e] = v;
        Xr[e] = -v.x;
        Xi[e] = -v.y;
    }
    __syncthreads();
    double tiny2 = (double)bs * DBL_EPSILON;
    tiny2 = tiny2 * tiny2 * mx;
    int status = 0;
    for (int t = 0; t < bw; ++t) {
        double best = -1.0;
        int bi = bs;
        for (int i = tid; i < bs; i += kPThreads)
            if (ppos_s[i] < 0) {
                const double v = cabs2(Pw[t * bsp + i]);
                if (v > best) { best = v; bi = i; }
            }
        block_argmax_n<kPWaves>(best, bi, sv, si);
        const int r = bi;
        if (!(best > tiny2) && status == 0) status = 1 + q.l * bs + k0 + t;
        if (tid < bw) rowr[tid] = Pw[tid * bsp + r];
        if (tid == 0) {
            ppos_s[r] = k0 + t;
            R1[t] = r;
        }
        __syncthreads();
        const double2 inv = cinv(rowr[t]);
        for (int i = tid; i < bs; i += kPThreads) {
            if (i == r) {
                for (int u = 0; u < bw; ++u) Pw[u * bsp + r] = u == t ? inv : cmul(rowr[u], inv);
            } else {
                const double2 f = cmul(Pw[t * bsp + i], inv);
                for (int u = 0; u < bw; ++u)
                    if (u != t) Pw[u * bsp + i] = csub(Pw[u * bsp + i], cmul(f, rowr[u]));
                Pw[t * bsp + i] = make_double2(-f.x, -f.y);
            }
        }
        __syncthreads();
    }
    // A11^{-1}: the pivot rows of the eliminated panel, in pivot order
    for (int e = tid; e < bw * bw; e += kPThreads) {
        const int t = e / bw, u = e % bw;
        Ainv[t * kPanel + u] = Pw[u * bsp + R1[t]];
    }
    __syncthreads();
    // pivot rows of S (all columns) into the panel work area
    for (int e = tid; e < kPanel * bsp; e += kPThreads) {
        const int u = e / bsp, j = e % bsp;
        Pw[e] = (u < bw && j < bs) ? M[(long long)j * bs + R1[u]] : make_double2(0, 0);
    }
    __syncthreads();
    // Y = A11^{-1} [pivot rows], with A11^{-1} itself in the panel columns
    for (int e = tid; e < kPanel * bsp; e += kPThreads) {
        const int t = e / bsp, j = e % bsp;
        double2 y = make_double2(0, 0);
        if (t < bw && j < bs) {
            if (j >= k0 && j < k0 + bw) {
                y = Ainv[t * kPanel + (j - k0)];
            } else {
                for (int u = 0; u < bw; ++u) cfma(y, Ainv[t * kPanel + u], Pw[u * bsp + j]);
            }
        }
        Yr[e] = y.x;
        Yi[e] = y.y;
    }
    // pivot rows take no part in X
    for (int e = tid; e < bw * kPanel; e += kPThreads) {
        const int t = e / kPanel, u = e % kPanel;
        Xr[(long long)u * bsp + R1[t]] = 0.0;
        Xi[(long long)u * bsp + R1[t]] = 0.0;
    }
    for (int i = tid; i < bsp; i += kPThreads) ppos[i] = ppos_s[i];
    if (tid < bw) piv[k0 + tid] = R1[tid];
    if (tid == 0 && status) {
        int *f = flags + (mid ? 2 * nsub + q.a : c);
        if (*f == 0) *f = status;
    }
}

// Deferred groups.  Panels p0 .. p0 + nd - 1 of a block are factored against
// the block S as it stood before panel p0; with X_n, Y_n the operands of
// panel n, the block after panels p0 .. m - 1 is
//   T_m(i, j) = base(i, j) + sum_{n = lo(i)}^{m-1} [j < 32 (n + 1) or j >= 32 m] X_n(i, :) Y_n(:, j)
// where a row that is the pivot row of step t of a deferred panel n has
// base Y_n(t, j) (kept only where the same mask holds) and lo = n + 1, and
// every other row has base S(i, j), cleared in the columns of panels p0 ..
// m - 1, and lo = p0: each panel's update zeroes its own columns and
// replaces its pivot rows by Y, so panel n's product is cleared from the
// columns of every later panel and a pivot row keeps only what came after
// its own panel.  m = p0 + nd gives the block after the whole group.

// Columns of panel p (p0 < p) of T_p, into the chain's C (column t at
// t * bsp + i): 64 rows x 4 groups of 8 columns per workgroup.
constexpr int kCThreads = 256;

__global__ __launch_bounds__(kCThreads) void k_factor_colupd(const SubDesc *__restrict__ subs, FactWs w, int s, int p,
                                                              int p0, int mid) {
    __shared__ double2 Ys[(kDefer - 1) * kPanel * kPanel];  // [n][v][t] panel p's columns of Y_n
    const int nrb = w.bsp / 64;
    const int c = blockIdx.x / nrb, rb = blockIdx.x % nrb;
    const ChainPos q = chain_pos(subs, c, s, mid != 0);
    if (!q.active) return;
    const int bs = q.bs, bsp = w.bsp, k0 = p * kPanel;
    if (k0 >= bs || rb * 64 >= bs) return;
    const int nd = p - p0;
    const int tid = threadIdx.x;
    for (int n = 0; n < nd; ++n) {
        // constant trip count: the loads issued before their LDS stores
        constexpr int kY = kPanel * kPanel / kCThreads;
        const double *yr = ws_y(w, c, n);
        double2 sy[kY];
#pragma unroll
        for (int m = 0; m < kY; ++m) {
            const int e = tid + m * kCThreads, v = e / kPanel, t = e % kPanel;
            const long long o = (long long)v * bsp + k0 + t;  // k0 + t < bsp
            sy[m] = make_double2(yr[o], yr[o + (long long)kPanel * bsp]);
        }
#pragma unroll
        for (int m = 0; m < kY; ++m) Ys[n * kPanel * kPanel + tid + m * kCThreads] = sy[m];
    }
    __syncthreads();
    const int i = rb * 64 + (tid & 63), tg = tid >> 6;
    if (i >= bs) return;
    const double2 *M = chain_M(w, c, q.cur);
    const int pp = w.ppos[(long long)c * bsp + i];
    const int pn = (pp >= p0 * kPanel && pp < k0) ? pp / kPanel : -1;  // deferred panel the row is a pivot row of
    double2 acc[8];
    if (pn >= 0) {
        const double *yr = ws_y(w, c, pn - p0);
        const long long o = (long long)(pp - pn * kPanel) * bsp + k0 + 8 * tg;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = make_double2(yr[o + k], yr[o + k + (long long)kPanel * bsp]);
    } else {
        // unconditional loads (clamped columns), zeroed past the block
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int j = k0 + 8 * tg + k;
            acc[k] = M[(long long)(j < bs ? j : bs - 1) * bs + i];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k0 + 8 * tg + k >= bs) acc[k] = make_double2(0, 0);
    }
    for (int n = pn >= 0 ? pn - p0 + 1 : 0; n < nd; ++n) {
        const double *xr = ws_x(w, c, n), *xi = xr + (long long)kPanel * bsp;
        const double2 *Yn = Ys + n * kPanel * kPanel + 8 * tg;
        for (int v0 = 0; v0 < kPanel; v0 += 8) {
            double2 x[8];  // one batch of loads in flight together
#pragma unroll
            for (int vv = 0; vv < 8; ++vv)
                x[vv] = make_double2(xr[(long long)(v0 + vv) * bsp + i], xi[(long long)(v0 + vv) * bsp + i]);
#pragma unroll
            for (int vv = 0; vv < 8; ++vv)
#pragma unroll
                for (int k = 0; k < 8; ++k) cfma(acc[k], x[vv], Yn[(v0 + vv) * kPanel + k]);
        }
    }
    double2 *C = w.C + (long long)c * kPanel * bsp;
#pragma unroll
    for (int k = 0; k < 8; ++k) C[(long long)(8 * tg + k) * bsp + i] = acc[k];
}

// Y_p = A11^{-1} [pivot rows of T_p] (kPanel x bsp, zero outside bw x bs,
// A11^{-1} itself in the panel columns) for the sub-panel kernel: one
// workgroup per chain and 64 columns (two chunks of 32).  The pivot rows of
// S are gathered (one element per row and column of the column-major block)
// into registers, the products of the deferred panels p0 .. p - 1 added to
// them (each panel's X at the pivot rows and its Y in these columns staged
// in LDS), and the rows multiplied by A11^{-1}.
constexpr int kYThreads = 256;
constexpr size_t kFormyLds = 4 * kPanel * kPanel * sizeof(double2) + kPanel * sizeof(int);

__global__ __launch_bounds__(kYThreads) void k_factor_formy(const SubDesc *__restrict__ subs, FactWs w, int s, int p,
                                                             int p0, int mid) {
    extern __shared__ double2 lds[];
    double2 *Ai = lds;                      // [t][u]
    double2 *Xs = Ai + kPanel * kPanel;     // [u][v] one deferred panel's X at the pivot rows
    double2 *Ys = Xs + kPanel * kPanel;     // [2][v][jj] its Y in the two chunks; then the rows [2][u][jj]
    int *R1 = (int *)(Ys + 2 * kPanel * kPanel);
    const int nfg = w.bsp / 64;
    const int c = blockIdx.x / nfg, j0 = (blockIdx.x % nfg) * 64;
    const ChainPos q = chain_pos(subs, c, s, mid != 0);
    if (!q.active) return;
    const int bs = q.bs, bsp = w.bsp, k0 = p * kPanel;
    if (k0 >= bs) return;
    const int bw = bs - k0 < kPanel ? bs - k0 : kPanel;
    const int nd = p - p0;
    const double2 *M = chain_M(w, c, q.cur);
    const double2 *Ainv = w.Pw + (long long)c * kPanel * bsp;
    const int *piv = w.piv + (long long)c * bsp;
    double *Yr = ws_y(w, c, nd), *Yi = Yr + (long long)kPanel * bsp;
    const int tid = threadIdx.x, jj = tid % kPanel;
    {
        constexpr int kA = kPanel * kPanel / kYThreads;
        double2 sa[kA];
#pragma unroll
        for (int m = 0; m < kA; ++m) sa[m] = Ainv[tid + m * kYThreads];
#pragma unroll
        for (int m = 0; m < kA; ++m) Ai[tid + m * kYThreads] = sa[m];
    }
    if (tid < kPanel) R1[tid] = tid < bw ? piv[k0 + tid] : 0;
    __syncthreads();
    // thread elements: rows u = tid / 32 + 8 k of the two chunks, column jj
    double2 acc[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int pc = j0 / kPanel + h;                 // the panel whose columns the chunk holds
        const bool cleared = pc >= p0 && pc < p;        // an earlier deferred panel's columns
        const int j = j0 + kPanel * h + jj;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int u = tid / kPanel + 8 * k;
            acc[h][k] = (u < bw && j < bs && !cleared) ? M[(long long)j * bs + R1[u]] : make_double2(0, 0);
        }
    }
    for (int n = 0; n < nd; ++n) {
        __syncthreads();  // the previous panel's Xs / Ys consumed
        const double *xr = ws_x(w, c, n), *yr = ws_y(w, c, n);
        // constant trip counts: every load of the staging issued before its LDS stores
        constexpr int kXs = kPanel * kPanel / kYThreads, kYs = 2 * kPanel * kPanel / kYThreads;
        double2 sx[kXs], sy[kYs];
#pragma unroll
        for (int m = 0; m < kXs; ++m) {
            const int e = tid + m * kYThreads;
            const long long o = (long long)(e % kPanel) * bsp + R1[e / kPanel];
            sx[m] = make_double2(xr[o], xr[o + (long long)kPanel * bsp]);
        }
#pragma unroll
        for (int m = 0; m < kYs; ++m) {
            const int e = tid + m * kYThreads;
            const int h = e / (kPanel * kPanel), v = (e / kPanel) % kPanel;
            const long long o = (long long)v * bsp + j0 + kPanel * h + e % kPanel;  // < kPanel * bsp
            sy[m] = make_double2(yr[o], yr[o + (long long)kPanel * bsp]);
        }
#pragma unroll
        for (int m = 0; m < kXs; ++m) Xs[tid + m * kYThreads] = sx[m];
#pragma unroll
        for (int m = 0; m < kYs; ++m) Ys[tid + m * kYThreads] = sy[m];
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // panel p0 + n's product stands in chunk pc unless p0 + n < pc < p
            const int pc = j0 / kPanel + h;
            if (pc > p0 + n && pc < p) continue;
            const double2 *yh = Ys + h * kPanel * kPanel + jj;
            for (int v = 0; v < kPanel; ++v) {
                const double2 yv = yh[v * kPanel];
#pragma unroll
                for (int k = 0; k < 4; ++k) cfma(acc[h][k], Xs[(tid / kPanel + 8 * k) * kPanel + v], yv);
            }
        }
    }
    __syncthreads();  // Ys free: the rows go there
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 4; ++k) Ys[(h * kPanel + tid / kPanel + 8 * k) * kPanel + jj] = acc[h][k];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = j0 + kPanel * h + jj;
        const double2 *rows = Ys + h * kPanel * kPanel + jj;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = tid / kPanel + 8 * k;
            double2 y = make_double2(0, 0);
            if (t < bw && j < bs) {
                if (j >= k0 && j < k0 + bw) {
                    y = Ai[t * kPanel + (j - k0)];
                } else {
                    for (int u = 0; u < bw; ++u) cfma(y, Ai[t * kPanel + u], rows[u * kPanel]);
                }
            }
            Yr[(long long)t * bsp + j] = y.x;
            Yi[(long long)t * bsp + j] = y.y;
        }
    }
}

// Pivot key of a candidate row: |value|^2 rounded to float, the low 10 bits
// replaced by 1023 - row (ties and near-ties, to 1e-4 relative, go to the
// smaller row); non-candidates have key 0.
__device__ inline unsigned pivot_key(double v2, int row) {
    return (__float_as_uint((float)v2) & ~1023u) | (unsigned)(1023 - row);
}

// Workgroup barrier that orders LDS only: this wave's LDS accesses are done,
// then every wave of the group is here.  Global accesses in flight (the
// multipliers stored at a pivot step) are not waited for, unlike
// __syncthreads(); the "memory" clobber keeps the compiler from moving
// memory accesses across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Max of a 32-bit value over the wave (DPP within rows of 16 lanes, then the
// four row results), returned to every lane.
__device__ inline unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x124, 0xF, 0xF, false));  // row_ror 4
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x128, 0xF, 0xF, false));  // row_ror 8
    const unsigned r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const unsigned r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return max(max(r0, r1), max(r2, r3));
}

// Panel kernel for blocks of at most NT rows: thread i keeps row i of the
// panel in registers through the elimination.  Per column: a wave-level max
// of the candidates' pivot keys, each wave's best row staged in LDS, one
// barrier, then every thread takes the best of the waves' candidates.
template <int NT>
__global__ __launch_bounds__(NT) void k_factor_panel_r(const SubDesc *__restrict__ subs, FactWs w, int s, int p,
                                                       int mid, int *__restrict__ flags, int nsub) {
    static_assert(NT <= 512, "pivot keys hold row indices below 1024");
    constexpr int NW = NT / 64;
    __shared__ double2 Ainv[kPanel * kPanel];
    __shared__ double2 rowc[2][NW][kPanel];
    __shared__ unsigned wkey[2][NW];
    __shared__ int R1[kPanel];
    const int c = blockIdx.x;
    const ChainPos q = chain_pos(subs, c, s, mid != 0);
    if (!q.active) return;
    const int bs = q.bs, bsp = w.bsp, k0 = p * kPanel;
    if (k0 >= bs) return;
    const int bw = bs - k0 < kPanel ? bs - k0 : kPanel;
    const double2 *M = chain_M(w, c, q.cur);
    double *Xr = ws_x(w, c, 0), *Xi = Xr + (long long)kPanel * bsp;
    double *Yr = ws_y(w, c, 0), *Yi = Yr + (long long)kPanel * bsp;
    int *ppos = w.ppos + (long long)c * bsp, *piv = w.piv + (long long)c * bsp;
    const int tid = threadIdx.x;
    const bool own = tid < bs;
    int myp = (p > 0 && own) ? ppos[tid] : -1;
    const double mx = slot_read(w.mxb + 2 * c + q.cur);
    if (p == 0 && tid == 0) w.mxb[2 * c + (q.cur ^ 1)] = 0ull;  // the store of this step fills it
    for (int e = tid; e < kPanel * kPanel; e += NT) Ainv[e] = make_double2(0, 0);
    const int wv = tid >> 6;
    // branch-free loads (clamped in-bounds addresses, then zeroed) so that all
    // of them are in flight together
    double2 pr[kPanel];
    const int rowc_ = own ? tid : bs - 1;
#pragma unroll
    for (int u = 0; u < kPanel; ++u) {
        const double2 v = M[(long long)(k0 + (u < bw ? u : bw - 1)) * bs + rowc_];
        pr[u] = (own && u < bw) ? v : make_double2(0, 0);
    }
    if (tid < bsp) {
#pragma unroll
        for (int u = 0; u < kPanel; ++u) {
            Xr[(long long)u * bsp + tid] = -pr[u].x;
            Xi[(long long)u * bsp + tid] = -pr[u].y;
        }
    }
    double tiny2 = (double)bs * DBL_EPSILON;
    tiny2 = tiny2 * tiny2 * mx;
    int status = 0;
    __syncthreads();
    // fully unrolled: the row stays in registers (static indices)
#pragma clang loop unroll(full)
    for (int t = 0; t < kPanel; ++t) {
        if (t < bw) {
            const int b = t & 1;
            const unsigned key = (own && myp < 0) ? pivot_key(cabs2(pr[t]), tid) : 0u;
            const unsigned wmax = wave_max_u32(key);
            if (key != 0u && key == wmax) {  // keys are unique: one lane per wave
#pragma unroll
                for (int u = 0; u < kPanel; ++u) rowc[b][wv][u] = pr[u];
            }
            if ((tid & 63) == 0) wkey[b][wv] = wmax;
            __syncthreads();  // rowc / wkey[b] are next written two columns later
            unsigned best = wkey[b][0];
            int wb = 0;
#pragma unroll
            for (int k = 1; k < NW; ++k)
                if (wkey[b][k] > best) { best = wkey[b][k]; wb = k; }
            int r = 1023 - (int)(best & 1023u);
            r = r < 0 ? 0 : (r >= bs ? bs - 1 : r);
            if (tid == r) {
                myp = k0 + t;
                R1[t] = r;
            }
            const double2 *rowr = rowc[b][wb];
            const double2 piv_v = rowr[t];
            if (!(cabs2(piv_v) > tiny2) && status == 0) status = 1 + q.l * bs + k0 + t;
            const double rd = 1.0 / cabs2(piv_v);
            const double2 inv = make_double2(piv_v.x * rd, -piv_v.y * rd);
            // the pivot row is read from LDS in two halves of 16, each half's
            // reads issued together (sched_barrier keeps the compiler from
            // interleaving them with the arithmetic one wait at a time)
            constexpr int kH = kPanel / 2;
            if (tid == r) {
#pragma unroll
                for (int h = 0; h < kPanel; h += kH) {
                    double2 rr[kH];
#pragma unroll
                    for (int u = 0; u < kH; ++u) rr[u] = rowr[h + u];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < kH; ++u) pr[h + u] = h + u == t ? inv : cmul(rr[u], inv);
                }
            } else {
                const double2 f = cmul(pr[t], inv);
#pragma unroll
                for (int h = 0; h < kPanel; h += kH) {
                    double2 rr[kH];
#pragma unroll
                    for (int u = 0; u < kH; ++u) rr[u] = rowr[h + u];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < kH; ++u)
                        if (h + u != t) pr[h + u] = csub(pr[h + u], cmul(f, rr[u]));
                }
                pr[t] = make_double2(-f.x, -f.y);
            }
        }
    }
    __syncthreads();  // R1 complete
    // pivot rows of this panel: rows of A11^{-1}; they take no part in X
    if (own && myp >= k0 && myp < k0 + bw) {
#pragma unroll
        for (int u = 0; u < kPanel; ++u) {
            Ainv[(myp - k0) * kPanel + u] = pr[u];
            Xr[(long long)u * bsp + tid] = 0.0;
            Xi[(long long)u * bsp + tid] = 0.0;
        }
    }
    if (own) ppos[tid] = myp;
    __syncthreads();
    if (tid < bw) piv[k0 + tid] = R1[tid];
    // Y = A11^{-1} [pivot rows of S], with A11^{-1} itself in the panel
    // columns; H thread groups split the kPanel rows of Y
    int H = 1;
    while (2 * H * bsp <= NT && 2 * H <= kPanel) H *= 2;
    const int j = tid % bsp, h = tid / bsp, th = kPanel / H;
    if (h < H) {
        double2 g[kPanel];
        const int jc = j < bs ? j : bs - 1;
#pragma unroll
        for (int u = 0; u < kPanel; ++u) {
            const int ru = R1[u < bw ? u : bw - 1];
            const double2 v = M[(long long)jc * bs + ru];
            g[u] = (u < bw && j < bs) ? v : make_double2(0, 0);
        }
        const bool inpanel = j >= k0 && j < k0 + bw;
        for (int t = h * th; t < (h + 1) * th; ++t) {
            double2 y = make_double2(0, 0);
            if (j < bs) {
                if (inpanel) {
                    y = Ainv[t * kPanel + (j - k0)];
                } else {
#pragma unroll
                    for (int u = 0; u < kPanel; ++u) cfma(y, Ainv[t * kPanel + u], g[u]);
                }
            }
            Yr[(long long)t * bsp + j] = y.x;
            Yi[(long long)t * bsp + j] = y.y;
        }
    }
    if (tid == 0 && status) {
        int *f = flags + (mid ? 2 * nsub + q.a : c);
        if (*f == 0) *f = status;
    }
}

// Panel kernel for blocks of 513 .. 4096 rows by sub-panels of SW columns:
// thread tid owns rows tid + NT k (k < NK) and keeps their values in
// the current sub-panel's columns in registers.  A sub-panel's columns are
// formed left-looking from the multipliers F of the earlier sub-panels (in
// the workspace, one batch of loads per UB of them) and the pivot rows'
// eliminated values U (LDS),
//   v(i, c) = S(i, c) - sum_{u < c0} F_u(i) U(u, c),
// then eliminated right-looking, one pivot step after another: a wave-level
// max of the candidates' pivot keys, each wave's best row staged in LDS, one
// barrier, every thread takes the best of the waves' candidates and updates
// its rows.  At the end of a sub-panel the pivot rows it chose get their U
// in the later columns, U(t, c) = S(r_t, c) - sum_{u < t} F_u(r_t) U(u, c).
// The pivots are those of partial pivoting on the panel (magnitudes compared
// to 2^-11 relative: 12 of the 23 mantissa bits of |v|^2 as a float hold
// the row; ties to the smaller row).  A11^{-1}, X and the
// workspace outputs: X = -(the panel's columns) with its pivot rows zero,
// A11^{-1} (A11 = the panel's pivot rows in pivot order, inverted by
// Gauss-Jordan with all threads) at the start of the multiplier area for
// k_factor_formy, the pivot steps of the rows and the rows of the steps.
template <int NT, int NK, int SW, int UB>
__global__ __launch_bounds__(NT) void k_factor_panel_sp(const SubDesc *__restrict__ subs, FactWs w, int s,
                                                                int p, int p0, int mid, int *__restrict__ flags,
                                                                int nsub) {
    static_assert(NK * NT <= 4096, "pivot keys hold row indices below 4096");
    constexpr int NW = NT / 64;
    static_assert(kPanel % SW == 0 && SW % 2 == 0, "sub-panels tile the panel");
    __shared__ double2 Ainv[kPanel * kPanel];  // also Lp[t][u] = F_u(r_t) while the sub-panels run
    __shared__ double2 U[kPanel * kPanel];     // [t][c] pivot row t's eliminated values
    __shared__ double2 Gbuf[kPanel * kPanel];  // second buffer of the A11 inverse
    __shared__ double2 rowc[2][NW][SW];
    __shared__ unsigned wkey[2][NW];
    __shared__ int R1[kPanel];
    const int c = blockIdx.x;
    const ChainPos q = chain_pos(subs, c, s, mid != 0);
    if (!q.active) return;
    const int bs = q.bs, bsp = w.bsp, k0 = p * kPanel;
    if (k0 >= bs) return;
    const int bw = bs - k0 < kPanel ? bs - k0 : kPanel;
    const int slot = p - p0;
    const double2 *src = slot == 0 ? chain_M(w, c, q.cur) + (long long)k0 * bs : w.C + (long long)c * kPanel * bsp;
    const long long sld = slot == 0 ? bs : bsp;
    double *Xr = ws_x(w, c, slot), *Xi = Xr + (long long)kPanel * bsp;
    double2 *F = w.Pw + (long long)c * kPanel * bsp;  // [kPanel][bsp] multipliers
    int *ppos = w.ppos + (long long)c * bsp, *piv = w.piv + (long long)c * bsp;
    double2 *Lp = Ainv;
    const int tid = threadIdx.x, wv = tid >> 6;
    const double mx = slot_read(w.mxb + 2 * c + q.cur);
    if (p == 0 && tid == 0) w.mxb[2 * c + (q.cur ^ 1)] = 0ull;  // the store of this step fills it
    // state of the thread's rows: -2 not a candidate (outside the block or an
    // earlier panel's pivot), -1 candidate, t >= 0 pivot row of step t
    int tp[NK], ic[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int i = tid + k * NT;
        ic[k] = i < bs ? i : bs - 1;  // clamped row for unconditional loads
        tp[k] = (i < bs && (p == 0 || ppos[i] < 0)) ? -1 : -2;
    }
    double tiny2 = (double)bs * DBL_EPSILON;
    tiny2 = tiny2 * tiny2 * mx;
    int status = 0;
    for (int c0 = 0; c0 < bw; c0 += SW) {
        __syncthreads();  // U of the earlier sub-panels complete
        // this sub-panel's columns of the thread's rows; X = -S there (all rows below bsp)
        // (all loads issued before the first store: a store under its branch
        // right after a load would wait for that load alone, one at a time)
        double2 v[NK][SW];
#pragma unroll
        for (int k = 0; k < NK; ++k)
#pragma unroll
            for (int cc = 0; cc < SW; ++cc) {
                const int cl = c0 + cc < bw ? c0 + cc : bw - 1;
                v[k][cc] = src[(long long)cl * sld + ic[k]];
            }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int i = tid + k * NT;
#pragma unroll
            for (int cc = 0; cc < SW; ++cc)
                if (!(i < bs && c0 + cc < bw)) v[k][cc] = make_double2(0, 0);
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int i = tid + k * NT;
            if (i < bsp) {
#pragma unroll
                for (int cc = 0; cc < SW; ++cc) {
                    Xr[(long long)(c0 + cc) * bsp + i] = -v[k][cc].x;
                    Xi[(long long)(c0 + cc) * bsp + i] = -v[k][cc].y;
                }
            }
        }
        // row by row, UB multipliers per batch (all loads of a batch in flight together)
#pragma unroll
        for (int k = 0; k < NK; ++k) {
#pragma unroll 1
            for (int u0 = 0; u0 < c0; u0 += UB) {
                double2 f[UB];
#pragma unroll
                for (int uu = 0; uu < UB; ++uu) f[uu] = F[(long long)(u0 + uu) * bsp + ic[k]];
#pragma unroll
                for (int uu = 0; uu < UB; ++uu)
#pragma unroll
                    for (int cc = 0; cc < SW; ++cc)
                        v[k][cc] = csub(v[k][cc], cmul(f[uu], U[(u0 + uu) * kPanel + c0 + cc]));
            }
        }
        // pivot steps of this sub-panel
#pragma unroll
        for (int cc = 0; cc < SW; ++cc) {
            const int t = c0 + cc;
            if (t < bw) {
                const int b = t & 1;
                unsigned key = 0u;
                int kb = 0;
#pragma unroll
                for (int k = 0; k < NK; ++k) {
                    const unsigned kk = tp[k] == -1 ? ((__float_as_uint((float)cabs2(v[k][cc])) & ~4095u) |
                                                       (unsigned)(4095 - (tid + k * NT)))
                                                    : 0u;
                    if (kk > key) { key = kk; kb = k; }
                }
                const unsigned wmax = wave_max_u32(key);
                if (key != 0u && key == wmax) {  // keys are unique: one lane per wave
#pragma unroll
                    for (int k = 0; k < NK; ++k)
                        if (k == kb)
#pragma unroll
                            for (int c2 = 0; c2 < SW; ++c2) rowc[b][wv][c2] = v[k][c2];
                }
                if ((tid & 63) == 0) wkey[b][wv] = wmax;
                lds_barrier();  // rowc / wkey[b] are next written two steps later
                unsigned best = wkey[b][0];
                int wb = 0;
#pragma unroll
                for (int k = 1; k < NW; ++k)
                    if (wkey[b][k] > best) { best = wkey[b][k]; wb = k; }
                int r = 4095 - (int)(best & 4095u);
                r = r < 0 ? 0 : (r >= bs ? bs - 1 : r);
                const double2 *prow = rowc[b][wb];
                const double2 piv_v = prow[cc];
                if (!(cabs2(piv_v) > tiny2) && status == 0) status = 1 + q.l * bs + k0 + t;
                const double2 inv = cinv(piv_v);
                if (tid == 0) R1[t] = r;
                if (tid >= cc && tid < SW) U[t * kPanel + c0 + tid] = prow[tid];  // the pivot row in this sub-panel
#pragma unroll
                for (int k = 0; k < NK; ++k) {
                    if (tp[k] != -1) continue;
                    const int i = tid + k * NT;
                    if (i == r) {
                        tp[k] = t;
                        continue;
                    }
                    const double2 fm = cmul(v[k][cc], inv);
                    F[(long long)t * bsp + i] = fm;
#pragma unroll
                    for (int c2 = cc + 1; c2 < SW; ++c2) v[k][c2] = csub(v[k][c2], cmul(fm, prow[c2]));
                }
            }
        }
        const int cn = c0 + SW;  // first column of the next sub-panel
        if (cn < bw) {
            __syncthreads();  // R1 of this sub-panel, its multipliers stored
            const int te = cn < bw ? cn : bw;
            for (int e = tid; e < SW * kPanel; e += NT) {
                const int tt = c0 + e / kPanel, u = e % kPanel;
                if (tt < te) {
                    Lp[tt * kPanel + u] = u < tt ? F[(long long)u * bsp + R1[tt]] : make_double2(0, 0);
                    if (u >= cn && u < bw) U[tt * kPanel + u] = src[(long long)u * sld + R1[tt]];
                }
            }
            __syncthreads();
            // the earlier sub-panels' pivots, in parallel over (row, column)
            for (int e = tid; e < SW * kPanel; e += NT) {
                const int tt = c0 + e / kPanel, cl = e % kPanel;
                if (tt < te && cl >= cn && cl < bw) {
                    double2 a = U[tt * kPanel + cl];
                    for (int u = 0; u < c0; ++u) a = csub(a, cmul(Lp[tt * kPanel + u], U[u * kPanel + cl]));
                    U[tt * kPanel + cl] = a;
                }
            }
            __syncthreads();
            // this sub-panel's pivots in order, one thread per later column
            if (tid >= cn && tid < bw) {
                for (int tt = c0; tt < te; ++tt) {
                    double2 a = U[tt * kPanel + tid];
                    for (int u = c0; u < tt; ++u) a = csub(a, cmul(Lp[tt * kPanel + u], U[u * kPanel + tid]));
                    U[tt * kPanel + tid] = a;
                }
            }
        }
    }
    __syncthreads();  // R1 complete; Lp no longer read
    // A11 (original pivot rows, pivot order) and its inverse by Gauss-Jordan
    // with the pivots on the diagonal: every thread, the matrix double-buffered
    // in LDS, one barrier per step
    for (int e = tid; e < kPanel * kPanel; e += NT) {
        const int t = e / kPanel, u = e % kPanel;
        Ainv[e] = (t < bw && u < bw) ? src[(long long)u * sld + R1[t]] : make_double2(0, 0);
    }
    __syncthreads();
    for (int t = 0; t < bw; ++t) {
        const double2 *Gi = (t & 1) ? Gbuf : Ainv;
        double2 *Go = (t & 1) ? Ainv : Gbuf;
        const double2 pi = cinv(Gi[t * kPanel + t]);
        for (int e = tid; e < kPanel * kPanel; e += NT) {
            const int i = e / kPanel, u = e % kPanel;
            double2 nv = make_double2(0, 0);
            if (i < bw && u < bw) {
                const double2 rt = u == t ? pi : cmul(Gi[t * kPanel + u], pi);  // new row t
                if (i == t) {
                    nv = rt;
                } else {
                    const double2 fa = Gi[i * kPanel + t];
                    nv = u == t ? make_double2(-(fa.x * pi.x - fa.y * pi.y), -(fa.x * pi.y + fa.y * pi.x))
                                : csub(Gi[i * kPanel + u], cmul(fa, rt));
                }
            }
            Go[e] = nv;
        }
        lds_barrier();
    }
    const double2 *Ares = (bw & 1) ? Gbuf : Ainv;  // the buffer the last step wrote
    // A11^{-1} to the workspace (the multipliers are done): Y is formed by
    // k_factor_formy over several workgroups per chain
    for (int e = tid; e < kPanel * kPanel; e += NT) F[e] = Ares[e];
    // pivot rows take no part in X; pivot steps of the rows
    for (int e = tid; e < bw * kPanel; e += NT) {
        const int t = e / kPanel, u = e % kPanel;
        Xr[(long long)u * bsp + R1[t]] = 0.0;
        Xi[(long long)u * bsp + R1[t]] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int i = tid + k * NT;
        if (i >= bsp) continue;
        if (tp[k] >= 0) ppos[i] = k0 + tp[k];
        else if (p == 0) ppos[i] = -1;
    }
    for (int i = tid + NK * NT; i < bsp; i += NT)
        if (p == 0) ppos[i] = -1;
    if (tid < bw) piv[k0 + tid] = R1[tid];
    if (tid == 0 && status) {
        int *fl = flags + (mid ? 2 * nsub + q.a : c);
        if (*fl == 0) *fl = status;
    }
}

// Update kernel: the block after the deferred group p0 .. p0 + nd - 1 (one
// panel when nd = 1: S <- S + X Y, panel columns starting from zero and
// pivot rows becoming Y), T_{p0+nd} of the formula above, on the block of
// every active chain.  Tile 64 x 64, four waves of 32 x 32, each as 2 x 2
// MFMA blocks of 16 x 16.
__global__ __launch_bounds__(kUThreads) void k_factor_update(const SubDesc *__restrict__ subs, FactWs w, int s,
                                                             int p0, int nd, int mid, int tpd) {
    const int ntile = tpd * tpd;
    const int c = blockIdx.x / ntile, tile = blockIdx.x % ntile;
    const ChainPos q = chain_pos(subs, c, s, mid != 0);
    if (!q.active) return;
    const int bs = q.bs, bsp = w.bsp, kd = p0 * kPanel;
    if (kd >= bs) return;
    const int npb = (bs + kPanel - 1) / kPanel;  // panels of this block
    const int ne = nd < npb - p0 ? nd : npb - p0;  // deferred panels this block has
    const int ke = (p0 + ne) * kPanel;           // end of the group's columns
    const int i0 = (tile % tpd) * kUTile, j0 = (tile / tpd) * kUTile;
    if (i0 >= bs || j0 >= bs) return;
    double2 *M = chain_M(w, c, q.cur);
    const int *ppos = w.ppos + (long long)c * bsp;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, qq = lane & 15;
    const int rw = i0 + 32 * (wv & 1), cw = j0 + 32 * (wv >> 1);
    // The product is formed transposed, S^T += Y^T X^T (A operand Y^T(j, t) at
    // lane j + 16 t, B operand X^T(t, i) at lane i + 16 t; the accumulator
    // holds D(m, n) at lane n + 16 (m % 4), register m / 4): in block (bi, bj)
    // lane qq + 16 g, register r holds S(i, j) with i = rw + 16 bi + qq and
    // j = cw + 16 bj + g + 4 r, so every load and store instruction covers 16
    // consecutive rows (256 bytes) of 4 columns.
    int lo[2];  // first deferred slot whose product reaches row rw + 16 bi + qq
    dbl4 re[2][2], im[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
        const int i = rw + 16 * bi + qq;
        const int pp = i < bs ? ppos[i] : -1;
        const int pn = (pp >= kd && pp < ke) ? pp / kPanel : -1;  // deferred panel the row is a pivot row of
        lo[bi] = pn >= 0 ? pn - p0 + 1 : 0;
        const double *yb = pn >= 0 ? ws_y(w, c, pn - p0) + (long long)(pp - pn * kPanel) * bsp : nullptr;
        const int ymask = pn >= 0 ? (pn + 1) * kPanel : kd;  // base kept in columns j < ymask or j >= ke
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = cw + 16 * bj + g + 4 * r;
                const bool keep = j < bs && i < bs && (j < ymask || j >= ke);
                double2 v = make_double2(0, 0);
                if (keep) v = pn >= 0 ? make_double2(yb[j], yb[j + (long long)kPanel * bsp]) : M[(long long)j * bs + i];
                re[bi][bj][r] = v.x;
                im[bi][bj][r] = v.y;
            }
    }
    // operands of chunk (slot n, panel columns t0 .. t0 + 3): panel n's product
    // reaches rows from slot lo on and columns outside the group's later panels
    auto kend_of = [&](int n) {
        const int kn = (p0 + n) * kPanel;
        return ((bs - kn < kPanel ? bs - kn : kPanel) + 3) & ~3;
    };
    auto load_chunk = [&](int n, int t0, double (&xr)[2], double (&xi)[2], double (&yr)[2], double (&yi)[2]) {
        const double *Xr = ws_x(w, c, n), *Xi = Xr + (long long)kPanel * bsp;
        const double *Yr = ws_y(w, c, n), *Yi = Yr + (long long)kPanel * bsp;
        const int kn = (p0 + n) * kPanel;
        const long long ko = (long long)(t0 + g) * bsp;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double ar = Xr[ko + rw + 16 * b + qq], ai = Xi[ko + rw + 16 * b + qq];
            const double br = Yr[ko + cw + 16 * b + qq], bi_ = Yi[ko + cw + 16 * b + qq];
            const bool xs = n >= lo[b];
            const int j = cw + 16 * b + qq;
            const bool ys = j < kn + kPanel || j >= ke;
            xr[b] = xs ? ar : 0.0;  // B operand: X^T(t, i) at lane i + 16 t
            xi[b] = xs ? ai : 0.0;
            yr[b] = ys ? br : 0.0;  // A operand: Y^T(j, t) at lane j + 16 t
            yi[b] = ys ? bi_ : 0.0;
        }
    };
    // chunks in order, the next chunk's operands loaded before this chunk's
    // products (loads issued unconditionally: past the last chunk the last
    // one is loaded again)
    int n = 0, t0 = 0;
    double xr[2], xi[2], yr[2], yi[2];
    load_chunk(0, 0, xr, xi, yr, yi);
    for (;;) {
        int n2 = n, t2 = t0 + 4;
        if (t2 >= kend_of(n)) {
            n2 = n + 1;
            t2 = 0;
        }
        const bool more = n2 < ne;
        double nxr[2], nxi[2], nyr[2], nyi[2];
        load_chunk(more ? n2 : n, more ? t2 : t0, nxr, nxi, nyr, nyi);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(yr[bj], xr[bi], re[bi][bj], 0, 0, 0);
                im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(yi[bj], xr[bi], im[bi][bj], 0, 0, 0);
            }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(yi[bj], -xi[bi], re[bi][bj], 0, 0, 0);
                im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(yr[bj], xi[bi], im[bi][bj], 0, 0, 0);
            }
        if (!more) break;
        n = n2;
        t0 = t2;
        xr[0] = nxr[0], xr[1] = nxr[1], xi[0] = nxi[0], xi[1] = nxi[1];
        yr[0] = nyr[0], yr[1] = nyr[1], yi[0] = nyi[0], yi[1] = nyi[1];
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
        const int i = rw + 16 * bi + qq;
        if (i >= bs) continue;
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = cw + 16 * bj + g + 4 * r;
                if (j >= bs) continue;
                M[(long long)j * bs + i] = make_double2(re[bi][bj][r], im[bi][bj][r]);
            }
    }
}

// Store the inverse of the chain's block, W_l(i, j) = N(piv[i], ppos[j]), and
// form the chain's next Schur complement in the other buffer (the inverse
// itself after the chain's last block, for the middle block).
template <typename T2>
__global__ __launch_bounds__(kEThreads) void k_factor_store(const SubDesc *__restrict__ subs,
                                                            const Coef *__restrict__ coef,
                                                            const double *__restrict__ k2, FactArgs A, FactWs w,
                                                            int s, int mid, int groups, int mma,
                                                            T2 *__restrict__ W) {
    const int c = blockIdx.x / groups, grp = blockIdx.x % groups;
    const ChainPos q = chain_pos(subs, c, s, mid != 0);
    if (!q.active) return;
    const SubDesc &sd = subs[q.a];
    const int bs = q.bs, ax = A.dim - 1;
    const double2 *N = chain_M(w, c, q.cur);
    double2 *Mn = chain_M(w, c, q.cur ^ 1);
    const int *ppos = w.ppos + (long long)c * w.bsp, *piv = w.piv + (long long)c * w.bsp;
    const int ld = sd.ld;
    // column-major with stride ld, or the matrix-core operand order (blocks
    // of bs x mpad)
    T2 *Wl = W + sd.foff + (long long)q.l * bs * (mma ? sd.mpad : ld);
    const bool next = !mid && !q.last;
    const int ln = q.dir == 0 ? q.l + 1 : q.l - 1;
    Coef cln = coef[sd.coff[ax] + (next ? ln : q.l)];
    double2 cc = make_double2(0, 0);
    if (next) cc = q.dir == 0 ? cmul(cln.cm, coef[sd.coff[ax] + q.l].cp) : cmul(cln.cp, coef[sd.coff[ax] + q.l].cm);
    const long long n2 = (long long)bs * bs;
    double m = 0.0;
    for (long long e = (long long)grp * kEThreads + threadIdx.x; e < n2; e += (long long)groups * kEThreads) {
        const int i = (int)(e % bs), j = (int)(e / bs);
        const double2 v = N[(long long)ppos[j] * bs + piv[i]];
        if (mma) {
            mma_store<T2>(Wl, bs, sd.mpad, i, j, from_d2<T2>(v));
            // padding columns of the last group: zeros
            if (j == bs - 1)
                for (int jp = bs; jp < sd.mpad; ++jp) mma_store<T2>(Wl, bs, sd.mpad, i, jp, czero<T2>());
        } else {
            Wl[(long long)j * ld + i] = from_d2<T2>(v);
            if (ld > bs && i == bs - 1) Wl[(long long)j * ld + bs] = czero<T2>();  // padding row
        }
        if (!mid) {
            const double2 mv = next ? csub(block_entry(sd, coef, k2, A, ln, i, j, cln), cmul(cc, v)) : v;
            Mn[e] = mv;
            m = fmax(m, cabs2(mv));
        }
    }
    if (!mid) {
        slot_max(w.mxb + 2 * c + (q.cur ^ 1), m);
        // the middle block of this subdomain is formed in this buffer next
        if (q.last && q.dir == 0 && grp == 0 && threadIdx.x == 0) w.mxb[2 * c + q.cur] = 0ull;
    }
}

static int groups_for(long long n2) {
    long long g = (n2 + kEThreads - 1) / kEThreads;
    return (int)(g < kEGroups ? g : kEGroups);
}

// Workgroup size, rows per thread and sub-panel width by block size (the
// registers of v[NK][SW] and of the multiplier batch within the VGPR budget
// of NT threads per CU).
static hipError_t launch_panel_sp(int bs_max, int nc, hipStream_t st, const SubDesc *subs, FactWs w, int s, int p,
                                  int p0, int mid, int *flags, int nsub) {
    if (bs_max <= 1024)
        k_factor_panel_sp<512, 2, 8, 8><<<nc, 512, 0, st>>>(subs, w, s, p, p0, mid, flags, nsub);
    else if (bs_max <= 1536)
        k_factor_panel_sp<512, 3, 8, 8><<<nc, 512, 0, st>>>(subs, w, s, p, p0, mid, flags, nsub);
    else if (bs_max <= 2048)
        k_factor_panel_sp<512, 4, 8, 8><<<nc, 512, 0, st>>>(subs, w, s, p, p0, mid, flags, nsub);
    else if (bs_max <= 2304)
        k_factor_panel_sp<768, 3, 8, 4><<<nc, 768, 0, st>>>(subs, w, s, p, p0, mid, flags, nsub);
    else if (bs_max <= 3072)
        k_factor_panel_sp<1024, 3, 4, 4><<<nc, 1024, 0, st>>>(subs, w, s, p, p0, mid, flags, nsub);
    else if (bs_max <= 4096)
        k_factor_panel_sp<1024, 4, 4, 2><<<nc, 1024, 0, st>>>(subs, w, s, p, p0, mid, flags, nsub);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_factor(ddm_handle *h, void *ws_base) {
    const Plan &P = h->plan;
    FactArgs A;
    A.dim = P.dim;
    A.G0 = P.G[0]; A.G1 = P.G[1];
    A.glo0 = P.glo[0]; A.glo1 = P.glo[1]; A.glo2 = P.glo[2];
    A.bs_max = P.bs_max;
    A.nsub = P.nsub;
    const FactWs w = carve_ws(P, ws_base);
    const int nc = 2 * P.nsub;
    const int groups = groups_for((long long)P.bs_max * P.bs_max);
    const int npan = (P.bs_max + kPanel - 1) / kPanel;
    const int tpd = w.bsp / kUTile;
    int maxlen = 0;
    for (const SubDesc &sd : P.subs) {
        maxlen = std::max(maxlen, sd.mid);
        maxlen = std::max(maxlen, sd.nb - 1 - sd.mid);
    }
    // panel kernel: registers for blocks of at most kPThreads rows, else
    // the generic kernel with its working panel in LDS when it fits
    const int panel_kind = P.bs_max <= 256 ? 0 : (P.bs_max <= 512 ? 1 : 2);
    size_t lds = (size_t)kPanel * kPanel * sizeof(double2) + kPanel * sizeof(double2) + kPanel * sizeof(int) +
                 (size_t)w.bsp * sizeof(int);
    lds = (lds + 15) & ~(size_t)15;
    const size_t lds_pw = lds + (size_t)kPanel * w.bsp * sizeof(double2);
    const bool pw_in_lds = lds_pw <= 150 * 1024;
    if (pw_in_lds) lds = lds_pw;
    hipError_t e = hipFuncSetAttribute(pw_in_lds ? (const void *)k_factor_panel<true> : (const void *)k_factor_panel<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // blocks of 513 .. 4096 rows: the sub-panel kernel and deferred groups
    const bool use_sp = panel_kind == 2 && P.bs_max <= kSPRows;
    if (use_sp) {
        e = hipFuncSetAttribute((const void *)k_factor_formy, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kFormyLds);
        if (e != hipSuccess) return e;
    }
    // panels per deferred group (the sub-panel path only)
    const int D = use_sp ? w.slots : 1;
    e = launch_fill_zero(w.mxb, (long long)2 * nc * sizeof(unsigned long long), h->stream);
    if (e != hipSuccess) return e;
    e = launch_fill_zero(h->d_flags, (long long)3 * P.nsub * sizeof(int), h->stream);
    if (e != hipSuccess) return e;
    k_factor_form0<<<nc * groups, kEThreads, 0, h->stream>>>(h->d_subs, h->d_coef, h->d_k2, A, w, groups);
    for (int s = 0; s <= maxlen; ++s) {
        const int mid = s == maxlen;  // the last round inverts the middle blocks
        if (mid)
            k_factor_formmid<<<P.nsub * groups, kEThreads, 0, h->stream>>>(h->d_subs, h->d_coef, h->d_k2, A, w,
                                                                          groups);
        const int ss = mid ? 0 : s;
        for (int p0 = 0; p0 < npan; p0 += D) {
            const int nd = npan - p0 < D ? npan - p0 : D;
            for (int p = p0; p < p0 + nd; ++p) {
                if (panel_kind == 0)
                    k_factor_panel_r<256><<<nc, 256, 0, h->stream>>>(h->d_subs, w, ss, p, mid, h->d_flags, P.nsub);
                else if (panel_kind == 1)
                    k_factor_panel_r<512><<<nc, 512, 0, h->stream>>>(h->d_subs, w, ss, p, mid, h->d_flags, P.nsub);
                else if (use_sp) {
                    if (p > p0)
                        k_factor_colupd<<<nc * (w.bsp / 64), kCThreads, 0, h->stream>>>(h->d_subs, w, ss, p, p0, mid);
                    e = launch_panel_sp(P.bs_max, nc, h->stream, h->d_subs, w, ss, p, p0, mid, h->d_flags, P.nsub);
                    if (e != hipSuccess) return e;
                    k_factor_formy<<<nc * (w.bsp / 64), kYThreads, kFormyLds, h->stream>>>(h->d_subs, w, ss, p, p0,
                                                                                            mid);
                } else if (pw_in_lds)
                    k_factor_panel<true><<<nc, kPThreads, lds, h->stream>>>(h->d_subs, w, ss, p, mid, h->d_flags,
                                                                            P.nsub);
                else
                    k_factor_panel<false><<<nc, kPThreads, lds, h->stream>>>(h->d_subs, w, ss, p, mid, h->d_flags,
                                                                             P.nsub);
            }
            k_factor_update<<<nc * tpd * tpd, kUThreads, 0, h->stream>>>(h->d_subs, w, ss, p0, nd, mid, tpd);
        }
        k_factor_store<T><<<nc * groups, kEThreads, 0, h->stream>>>(h->d_subs, h->d_coef, h->d_k2, A, w, ss, mid,
                                                                    groups, P.mma ? 1 : 0, (T *)h->d_W);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_factor<double2>(ddm_handle *, void *);
template hipError_t launch_factor<float2>(ddm_handle *, void *);

}  // namespace ddm
