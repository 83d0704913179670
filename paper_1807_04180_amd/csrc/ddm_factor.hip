// Block-tridiagonal factorisation of every subdomain operator (the direct
// local solver of Algorithm 3.1; the paper used a multifrontal LU).
//
// Unknowns of a subdomain box are grouped into blocks along its last axis
// (grid lines in 2D, grid planes in 3D).  The 5/7-point operator couples block
// l only to l-1 and l+1, through C_l = cm(l) I and B_l = cp(l) I, the 1D
// coefficients of the last axis.  The factorisation is
//     S_0 = D_0,   S_l = D_l - cm(l) cp(l-1) W_{l-1},   W_l = S_l^{-1},
// and W_l is stored column-major (element (i, j) at j * bs + i), complex128
// or complex64.  The inverse is formed by in-place Gauss-Jordan elimination
// with partial (row) pivoting inside S_l, in FP64.
//
// The elimination runs from both ends of the subdomain towards a middle
// block mid (a twisted factorisation; mid = nb - 1 is the one-directional
// case): one workgroup (1024 threads) per chain and subdomain walks its
// blocks in order, then one workgroup per subdomain inverts the middle block.
// The current block lives in an FP64 scratch matrix (L2-resident for 2D block
// sizes); row k / column k of each elimination step are staged in LDS.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "cplx.h"
#include "ddm_internal.h"

namespace ddm {

constexpr int kFThreads = 1024;
constexpr int kFWaves = kFThreads / 64;

struct FactArgs {
    int dim;
    int G0, G1;
    int glo0, glo1, glo2;
    int bs_max;
    int nsub;
};

// block-wide argmax of (value, index); ties go to the smaller index
__device__ inline void block_argmax(double &v, int &idx, double *sv, int *si) {
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_down(v, o, 64);
        int oi = __shfl_down(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sv[w] = v; si[w] = idx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kFWaves; ++i)
            if (sv[i] > sv[0] || (sv[i] == sv[0] && si[i] < si[0])) { sv[0] = sv[i]; si[0] = si[i]; }
    }
    __syncthreads();
    v = sv[0];
    idx = si[0];
    __syncthreads();
}

__device__ inline double block_max(double v, double *sv) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sv[w] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 1; i < kFWaves; ++i) sv[0] = fmax(sv[0], sv[i]);
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

// In-place Gauss-Jordan inversion of the bs x bs column-major FP64 matrix M
// with partial (row) pivoting; returns a non-zero status (1 + column) in
// every thread if a pivot falls below bs * eps * max|M|.
__device__ int gj_invert(double2 *__restrict__ M, int bs, double2 *rowk, double2 *rs, double2 *colk, int *perm,
                         double *sv, int *si) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double mx = 0.0;
    for (int j = ty; j < bs; j += kFWaves)
        for (int i = tx; i < bs; i += 64) mx = fmax(mx, cabs2(M[(long long)j * bs + i]));
    mx = block_max(mx, sv);
    double tiny2 = (double)bs * DBL_EPSILON;
    tiny2 = tiny2 * tiny2 * mx;
    int status = 0;
    for (int k = 0; k < bs; ++k) {
        double pv = -1.0;
        int pi = k;
        for (int i = k + threadIdx.x; i < bs; i += kFThreads) {
            double v = cabs2(M[(long long)k * bs + i]);
            if (v > pv) { pv = v; pi = i; }
        }
        block_argmax(pv, pi, sv, si);
        if (!(pv > tiny2) && status == 0) status = 1 + k;
        if (threadIdx.x == 0) perm[k] = pi;
        if (pi != k)
            for (int j = threadIdx.x; j < bs; j += kFThreads) {
                double2 t = M[(long long)j * bs + k];
                M[(long long)j * bs + k] = M[(long long)j * bs + pi];
                M[(long long)j * bs + pi] = t;
            }
        __syncthreads();
        for (int j = threadIdx.x; j < bs; j += kFThreads) {
            rowk[j] = M[(long long)j * bs + k];
            colk[j] = M[(long long)k * bs + j];
        }
        __syncthreads();
        double2 inv = cinv(rowk[k]);
        for (int j = threadIdx.x; j < bs; j += kFThreads) rs[j] = j == k ? inv : cmul(rowk[j], inv);
        __syncthreads();
        for (int j = ty; j < bs; j += kFWaves) {
            double2 rj = rs[j];
            for (int i = tx; i < bs; i += 64) {
                long long o = (long long)j * bs + i;
                if (i == k) {
                    M[o] = rj;
                } else if (j == k) {
                    M[o] = make_double2(-(colk[i].x * inv.x - colk[i].y * inv.y),
                                        -(colk[i].x * inv.y + colk[i].y * inv.x));
                } else {
                    double2 c = colk[i];
                    double2 m = M[o];
                    m.x -= c.x * rj.x - c.y * rj.y;
                    m.y -= c.x * rj.y + c.y * rj.x;
                    M[o] = m;
                }
            }
        }
        __syncthreads();
    }
    // undo the row interchanges: swap columns in reverse order
    for (int k = bs - 1; k >= 0; --k) {
        int p = perm[k];
        if (p != k)
            for (int i = threadIdx.x; i < bs; i += kFThreads) {
                double2 t = M[(long long)k * bs + i];
                M[(long long)k * bs + i] = M[(long long)p * bs + i];
                M[(long long)p * bs + i] = t;
            }
        __syncthreads();
    }
    return status;
}

// M = D_l - c1 * A1 - c2 * A2 (A1 / A2 may be null), in place over A1 == M
__device__ void form_block(const SubDesc &s, const Coef *__restrict__ coef, const double *__restrict__ k2,
                           const FactArgs &A, int l, double2 *__restrict__ M, double2 c1, const double2 *A1,
                           double2 c2, const double2 *A2) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int bs = s.bs;
    Coef cl = coef[s.coff[A.dim - 1] + l];
    for (int j = ty; j < bs; j += kFWaves)
        for (int i = tx; i < bs; i += 64) {
            long long o = (long long)j * bs + i;
            double2 v = block_entry(s, coef, k2, A, l, i, j, cl);
            if (A1) v = csub(v, cmul(c1, A1[o]));
            if (A2) v = csub(v, cmul(c2, A2[o]));
            M[o] = v;
        }
    __syncthreads();
}

template <typename T2>
__device__ void store_block(const SubDesc &s, int l, const double2 *__restrict__ M, T2 *__restrict__ W) {
    const int bs = s.bs;
    T2 *Wl = W + s.foff + (long long)l * bs * bs;
    for (long long o = threadIdx.x; o < (long long)bs * bs; o += kFThreads) Wl[o] = from_d2<T2>(M[o]);
    __syncthreads();
}

// Chains of the block elimination.  Block l couples to l-1 through
// C_l = cm(l) I and to l+1 through B_l = cp(l) I (1D coefficients of the last
// axis).  Chain 0 eliminates from the first block:
//     S_0 = D_0,  S_l = D_l - cm(l) cp(l-1) S_{l-1}^{-1},  l < mid;
// chain 1 from the last block:
//     T_{nb-1} = D_{nb-1},  T_l = D_l - cp(l) cm(l+1) T_{l+1}^{-1},  l > mid.
// Each chain keeps its last inverse in FP64 scratch for the middle block.
template <typename T2>
__global__ __launch_bounds__(kFThreads) void k_factor_chain(const SubDesc *__restrict__ subs,
                                                            const Coef *__restrict__ coef,
                                                            const double *__restrict__ k2, FactArgs A,
                                                            double2 *__restrict__ scratch, long long sstride,
                                                            T2 *__restrict__ W, int *__restrict__ flags) {
    extern __shared__ double2 lds[];
    double2 *rowk = lds, *rs = lds + A.bs_max, *colk = lds + 2 * A.bs_max;
    int *perm = (int *)(lds + 3 * A.bs_max);
    __shared__ double sv[kFWaves];
    __shared__ int si[kFWaves];
    const int a = blockIdx.x >> 1, chain = blockIdx.x & 1;
    const SubDesc &s = subs[a];
    const int bs = s.bs, nb = s.nb, mid = s.mid, ax = A.dim - 1;
    double2 *M = scratch + (long long)blockIdx.x * sstride;
    int status = 0;
    if (chain == 0) {
        for (int l = 0; l < mid; ++l) {
            double2 c = l > 0 ? cmul(coef[s.coff[ax] + l].cm, coef[s.coff[ax] + l - 1].cp) : make_double2(0, 0);
            form_block(s, coef, k2, A, l, M, c, l > 0 ? M : nullptr, c, nullptr);
            int st = gj_invert(M, bs, rowk, rs, colk, perm, sv, si);
            if (st && !status) status = 1 + l * bs + (st - 1);
            store_block<T2>(s, l, M, W);
        }
    } else {
        for (int l = nb - 1; l > mid; --l) {
            double2 c = l < nb - 1 ? cmul(coef[s.coff[ax] + l].cp, coef[s.coff[ax] + l + 1].cm) : make_double2(0, 0);
            form_block(s, coef, k2, A, l, M, c, l < nb - 1 ? M : nullptr, c, nullptr);
            int st = gj_invert(M, bs, rowk, rs, colk, perm, sv, si);
            if (st && !status) status = 1 + l * bs + (st - 1);
            store_block<T2>(s, l, M, W);
        }
    }
    if (threadIdx.x == 0) flags[blockIdx.x] = status;
}

// Middle block: Z = D_mid - cm(mid) cp(mid-1) S_{mid-1}^{-1} - cp(mid) cm(mid+1) T_{mid+1}^{-1}
template <typename T2>
__global__ __launch_bounds__(kFThreads) void k_factor_mid(const SubDesc *__restrict__ subs,
                                                          const Coef *__restrict__ coef,
                                                          const double *__restrict__ k2, FactArgs A,
                                                          double2 *__restrict__ scratch, long long sstride,
                                                          T2 *__restrict__ W, int *__restrict__ flags) {
    extern __shared__ double2 lds[];
    double2 *rowk = lds, *rs = lds + A.bs_max, *colk = lds + 2 * A.bs_max;
    int *perm = (int *)(lds + 3 * A.bs_max);
    __shared__ double sv[kFWaves];
    __shared__ int si[kFWaves];
    const int a = blockIdx.x;
    const SubDesc &s = subs[a];
    const int bs = s.bs, nb = s.nb, l = s.mid, ax = A.dim - 1;
    double2 *Mtop = scratch + (long long)(2 * a) * sstride;
    double2 *Mbot = scratch + (long long)(2 * a + 1) * sstride;
    double2 c1 = l > 0 ? cmul(coef[s.coff[ax] + l].cm, coef[s.coff[ax] + l - 1].cp) : make_double2(0, 0);
    double2 c2 = l < nb - 1 ? cmul(coef[s.coff[ax] + l].cp, coef[s.coff[ax] + l + 1].cm) : make_double2(0, 0);
    form_block(s, coef, k2, A, l, Mtop, c1, l > 0 ? Mtop : nullptr, c2, l < nb - 1 ? Mbot : nullptr);
    int st = gj_invert(Mtop, bs, rowk, rs, colk, perm, sv, si);
    store_block<T2>(s, l, Mtop, W);
    if (threadIdx.x == 0) flags[2 * A.nsub + a] = st ? 1 + l * bs + (st - 1) : 0;
}

template <typename T>
hipError_t launch_factor(ddm_handle *h) {
    const Plan &P = h->plan;
    FactArgs A;
    A.dim = P.dim;
    A.G0 = P.G[0]; A.G1 = P.G[1];
    A.glo0 = P.glo[0]; A.glo1 = P.glo[1]; A.glo2 = P.glo[2];
    A.bs_max = P.bs_max;
    A.nsub = P.nsub;
    size_t lds = (size_t)P.bs_max * (3 * sizeof(double2) + sizeof(int));
    long long sstride = (long long)P.bs_max * P.bs_max;
    k_factor_chain<T><<<2 * P.nsub, kFThreads, lds, h->stream>>>(h->d_subs, h->d_coef, h->d_k2, A, h->d_scratch,
                                                                 sstride, (T *)h->d_W, h->d_flags);
    k_factor_mid<T><<<P.nsub, kFThreads, lds, h->stream>>>(h->d_subs, h->d_coef, h->d_k2, A, h->d_scratch, sstride,
                                                           (T *)h->d_W, h->d_flags);
    return hipGetLastError();
}

template hipError_t launch_factor<double2>(ddm_handle *);
template hipError_t launch_factor<float2>(ddm_handle *);

}  // namespace ddm
