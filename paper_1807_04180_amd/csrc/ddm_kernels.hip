// Memory-bound kernels of the DDM step: 5/7-point PML operator and residual
// with FP64 norms (stopping test of Sec. 4.2), step-1 source restriction,
// 8/26-direction source transfer (Sec. 2.2, eq. talg_2), assembly
// u = sum_a beta_{0;a} U_a (eq. tsum), precision casts and the batched
// Krylov vector operations of the FGMRES driver.
//
// All reductions use a fixed assignment of elements to threads and a fixed
// reduction tree: results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cplx.h"
#include "ddm_internal.h"

namespace ddm {

constexpr int kBlock = 256;
static_assert(kBlock == kRowPiece, "one thread per node of a row piece");

// ---------------------------------------------------------------------------
// block-wide sum of doubles (fixed tree)
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// Operator apply / residual on the global grid.
// L u(p) = k^2 u(p) + sum_axes [cp (u(p+e) - u(p)) - cm (u(p) - u(p-e))]
// ---------------------------------------------------------------------------
struct GridArgs {
    int G0, G1, G2, dim;
    int c0, c1, c2;
    long long nglob;
};

// The node's loads are issued together (clamped in-bounds indices; a missing
// neighbour's value is replaced by 0 afterwards, as if it had not been read),
// so that they are waited for once per node and not once per axis.
__device__ inline double2 apply_global_at(const double2 *__restrict__ u, const double *__restrict__ k2,
                                          const Coef *__restrict__ gc, const GridArgs &g, long long idx, int x,
                                          int y, int z) {
    const double2 zero = make_double2(0, 0);
    const long long s1 = g.G0;
    const bool xp = x + 1 < g.G0, xm = x > 0;
    const bool yp = g.dim >= 2 && y + 1 < g.G1, ym = g.dim >= 2 && y > 0;
    const double2 uc = u[idx];
    const double kk = k2[idx];
    const double2 uxp = u[xp ? idx + 1 : idx], uxm = u[xm ? idx - 1 : idx];
    const double2 uyp = u[yp ? idx + s1 : idx], uym = u[ym ? idx - s1 : idx];
    const Coef cx = gc[g.c0 + x];
    const Coef cy = gc[g.dim >= 2 ? g.c1 + y : g.c0];
    double2 Lu = cscale(uc, kk);
    {
        const double2 up = xp ? uxp : zero, um = xm ? uxm : zero;
        Lu = cadd(Lu, csub(cmul(cx.cp, csub(up, uc)), cmul(cx.cm, csub(uc, um))));
    }
    if (g.dim >= 2) {
        const double2 up = yp ? uyp : zero, um = ym ? uym : zero;
        Lu = cadd(Lu, csub(cmul(cy.cp, csub(up, uc)), cmul(cy.cm, csub(uc, um))));
    }
    if (g.dim >= 3) {
        const long long s2 = (long long)g.G0 * g.G1;
        const bool zp = z + 1 < g.G2, zm = z > 0;
        const double2 uzp = u[zp ? idx + s2 : idx], uzm = u[zm ? idx - s2 : idx];
        const Coef cz = gc[g.c2 + z];
        const double2 up = zp ? uzp : zero, um = zm ? uzm : zero;
        Lu = cadd(Lu, csub(cmul(cz.cp, csub(up, uc)), cmul(cz.cm, csub(uc, um))));
    }
    return Lu;
}

// mode 0: out = f - L u and partial norms of out and f; mode 1: out = L u.
// One block per grid row (fixed y, z) and RHS; threads along x.  Workgroups
// go to the 8 XCDs round-robin, so block b takes row (b % 8) chunk + b / 8:
// each XCD sweeps one contiguous band of rows and the rows above and below
// a row are read from its own L2 (a plain row-per-block order spreads the
// three readers of every row over three XCDs and fetched 2.2x the bytes).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil(const double2 *__restrict__ f, const double2 *__restrict__ u,
                                                    double2 *__restrict__ out, const double *__restrict__ k2,
                                                    const Coef *__restrict__ gc, GridArgs g,
                                                    double *__restrict__ part_r, double *__restrict__ part_f) {
    __shared__ double sh[kBlock / 64];
    const int rhs = blockIdx.y;
    const int chunk = (int)gridDim.x / kXcds;
    const int rowi = ((int)blockIdx.x % kXcds) * chunk + (int)blockIdx.x / kXcds;  // y + G1 * z
    if (rowi >= g.G1 * g.G2) {  // padding block: zero partials
        if (MODE == 0 && threadIdx.x == 0) {
            part_r[(long long)rhs * gridDim.x + blockIdx.x] = 0.0;
            part_f[(long long)rhs * gridDim.x + blockIdx.x] = 0.0;
        }
        return;
    }
    const int y = rowi % g.G1, z = rowi / g.G1;
    const long long row0 = (long long)rowi * g.G0;
    const double2 *ur = u + rhs * g.nglob;
    double rn = 0.0, fn = 0.0;
    for (int x = threadIdx.x; x < g.G0; x += kBlock) {
        const long long idx = row0 + x;
        // f is loaded with the stencil's values (mode 1 reads u's own entry)
        const double2 fv = MODE == 0 ? f[rhs * g.nglob + idx] : make_double2(0, 0);
        double2 Lu = apply_global_at(ur, k2, gc, g, idx, x, y, z);
        if (MODE == 0) {
            double2 rv = csub(fv, Lu);
            if (out) out[rhs * g.nglob + idx] = rv;
            rn += cabs2(rv);
            fn += cabs2(fv);
        } else {
            out[rhs * g.nglob + idx] = Lu;
        }
    }
    if (MODE == 0) {
        double a = block_sum(rn, sh);
        if (threadIdx.x == 0) part_r[(long long)rhs * gridDim.x + blockIdx.x] = a;
        double b = block_sum(fn, sh);
        if (threadIdx.x == 0) part_f[(long long)rhs * gridDim.x + blockIdx.x] = b;
    }
}

// sum nblk partials per RHS in a fixed order: one block per RHS
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double *__restrict__ part, int nblk,
                                                         double *__restrict__ out) {
    __shared__ double sh[kBlock / 64];
    int rhs = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kBlock) s += part[(long long)rhs * nblk + i];
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[rhs] = t;
}

// squared norms of nrhs vectors (length n, stride ld)
__global__ __launch_bounds__(kBlock) void k_norm2_part(const double2 *__restrict__ x, long long n, long long ld,
                                                       double *__restrict__ part) {
    __shared__ double sh[kBlock / 64];
    int rhs = blockIdx.y;
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        s += cabs2(x[rhs * ld + i]);
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[(long long)rhs * gridDim.x + blockIdx.x] = t;
}

static GridArgs grid_args(const Plan &P) {
    GridArgs g;
    g.G0 = P.G[0]; g.G1 = P.G[1]; g.G2 = P.G[2]; g.dim = P.dim;
    g.c0 = P.gcoff[0]; g.c1 = P.gcoff[1]; g.c2 = P.gcoff[2];
    g.nglob = P.nglob;
    return g;
}

hipError_t launch_apply(ddm_handle *h, const double2 *u, double2 *out, int nrhs) {
    const Plan &P = h->plan;
    dim3 grid((unsigned)stencil_blocks(P), nrhs);
    k_stencil<1><<<grid, kBlock, 0, h->stream>>>(nullptr, u, out, h->d_k2, h->d_gcoef, grid_args(P), nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_residual(ddm_handle *h, const double2 *f, const double2 *u, double2 *r, int nrhs, double *d_rn2,
                           double *d_fn2) {
    return launch_residual_parts(h, f, u, r, nrhs, h->d_part, d_rn2, d_fn2);
}

hipError_t launch_residual_parts(ddm_handle *h, const double2 *f, const double2 *u, double2 *r, int nrhs,
                                 double *part, double *d_rn2, double *d_fn2, bool profile) {
    const Plan &P = h->plan;
    int nblk = stencil_blocks(P);
    dim3 grid(nblk, nrhs);
    double *part_r = part, *part_f = part + (long long)nrhs * nblk;
    // f and u read, r written (if requested), k^2 read
    ProfScope ps(h, DDM_K_RESIDUAL, (double)P.nglob * (nrhs * (r ? 48.0 : 32.0) + 8.0), profile);
    k_stencil<0><<<grid, kBlock, 0, h->stream>>>(f, u, r, h->d_k2, h->d_gcoef, grid_args(P), part_r, part_f);
    k_sum_partials<<<nrhs, kBlock, 0, h->stream>>>(part_r, nblk, d_rn2);
    k_sum_partials<<<nrhs, kBlock, 0, h->stream>>>(part_f, nblk, d_fn2);
    return hipGetLastError();
}

hipError_t launch_norm2(ddm_handle *h, const double2 *x, long long n, int nrhs, long long ld, double *d_out) {
    int nblk = 512;
    k_norm2_part<<<dim3(nblk, nrhs), kBlock, 0, h->stream>>>(x, n, ld, h->d_part);
    k_sum_partials<<<nrhs, kBlock, 0, h->stream>>>(h->d_part, nblk, d_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Packed subdomain vectors: helpers
// ---------------------------------------------------------------------------
struct PackArgs {
    int dim, n_ov;
    int G0, G1;
    int glo0, glo1, glo2;
    long long etot, nglob;
};

__device__ inline double side_factor(const double *__restrict__ btab, int n_ov, int m) {
    if (m <= 1) return 1.0;
    if (m >= n_ov) return 0.0;
    return btab[m];
}

__device__ inline long long glob_index(const PackArgs &A, int px, int py, int pz) {
    return (long long)(px - A.glo0) + (long long)A.G0 * ((long long)(py - A.glo1) + (long long)A.G1 * (pz - A.glo2));
}

// ---------------------------------------------------------------------------
// Step-1 sources: g_a = f on the core of a, 0 elsewhere.
// grid: (grid rows of the largest box, nsub, RHS tiles of kRestrictRQ): one
// workgroup per box row and RHS tile, the loads of the tile's RHS in flight
// together (one workgroup per row and RHS made the launch bound by the
// workgroup dispatch: 0.65 ms for the 2048^2 batch of 16 RHS)
// ---------------------------------------------------------------------------
constexpr int kRestrictRQ = 8;
template <typename TIN, typename TOUT>
__global__ __launch_bounds__(kBlock) void k_restrict(const SubDesc *__restrict__ subs, const TIN *__restrict__ f,
                                                     TOUT *__restrict__ g, PackArgs A, int nrhs) {
    const int a = blockIdx.y, r0 = blockIdx.z * kRestrictRQ;
    const int nr = nrhs - r0 < kRestrictRQ ? nrhs - r0 : kRestrictRQ;
    const SubDesc &s = subs[a];
    const int rowi = blockIdx.x;  // ly + n1 * lz
    if (rowi >= s.n[1] * s.n[2]) return;
    const int ly = rowi % s.n[1], lz = rowi / s.n[1];
    const int p1 = s.lo[1] + ly, p2 = s.lo[2] + lz;
    const bool rowcore = p1 >= s.clo[1] && p1 <= s.chi[1] && p2 >= s.clo[2] && p2 <= s.chi[2];
    TOUT *gr = g + (long long)r0 * A.etot + s.off + (long long)rowi * s.n[0];
    for (int lx = threadIdx.x; lx < s.n[0]; lx += kBlock) {
        const int p0 = s.lo[0] + lx;
        const bool core = rowcore && p0 >= s.clo[0] && p0 <= s.chi[0];
        // nodes outside the core read node 0 (always there) and store 0
        const long long gi = core ? glob_index(A, p0, p1, p2) : 0;
        TIN v[kRestrictRQ];
#pragma unroll
        for (int q = 0; q < kRestrictRQ; ++q) {
            const int qc = q < nr ? q : nr - 1;
            v[q] = f[(long long)(r0 + qc) * A.nglob + gi];
        }
#pragma unroll
        for (int q = 0; q < kRestrictRQ; ++q)
            if (q < nr) gr[(long long)q * A.etot + lx] = from_d2<TOUT>(core ? to_d2(v[q]) : make_double2(0, 0));
    }
}

// ---------------------------------------------------------------------------
// Source transfer (Sec. 2.2 transfer operators, eq. talg_2):
//   g_a(p) = - sum_b [p in chi_{b->a}] (L_a (beta_{b->a} uhat_b))(p)
// b over the 8 / 26 neighbours, lag = number of differing axes.
// Only the first n_ov core layers of a facing b can be non-zero (beta
// vanishes n_ov nodes past b's core); every other node gets 0.
//
// The Phi form (the remark on horizontal / vertical transfers in Sec. 2.2,
// eq. Phi) replaces L_a(beta v) by the commutator
//   L_a(beta v) - beta L_a v = sum_d cp_d (beta(p+e_d) - beta(p)) v(p+e_d)
//                                  + cm_d (beta(p-e_d) - beta(p)) v(p-e_d),
// the discrete product rule: first differences of beta times v, no k^2 and
// no v(p).  The two agree wherever L_a v = 0 on the support of beta.  The
// DDM's local solutions satisfy that when the subdomains are split along one
// axis (every transfer runs in one direction, the setting of the remark);
// with corner transfers a box's sources reach into its other overlap bands,
// the forms differ there and the iteration loses its fixed point, so the
// host accepts the Phi form only for one-axis layouts.  Its terms are
// O(v |grad beta| / h) with no cancellation of O(v / h^2) terms.
// ---------------------------------------------------------------------------
// The box fields of a descriptor the transfer uses, copied to registers with
// all loads issued together (read field by field where they are used, each
// load would be waited for alone inside its branch).
struct BoxR {
    int lo[3], hi[3], clo[3], chi[3], n[3];
    long long off;
};

__device__ inline BoxR box_of(const SubDesc *__restrict__ subs, int i) {
    const SubDesc &d = subs[i];
    BoxR b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = d.lo[k];
        b.hi[k] = d.hi[k];
        b.clo[k] = d.clo[k];
        b.chi[k] = d.chi[k];
        b.n[k] = d.n[k];
    }
    b.off = d.off;
    return b;
}

template <typename B>
__device__ inline bool in_box(const B &b, int q0, int q1, int q2) {
    return q0 >= b.lo[0] && q0 <= b.hi[0] && q1 >= b.lo[1] && q1 <= b.hi[1] && q2 >= b.lo[2] && q2 <= b.hi[2];
}

// beta_{b->a}(q): b's side factors facing a on every axis where they differ
template <typename B>
__device__ inline double beta_ba(const B &b, const int *dd, const double *__restrict__ btab, int n_ov, int q0,
                                 int q1, int q2) {
    int q[3] = {q0, q1, q2};
    double beta = 1.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (dd[d] < 0) beta *= side_factor(btab, n_ov, q[d] - b.chi[d]);       // b below a: b's high side
        else if (dd[d] > 0) beta *= side_factor(btab, n_ov, b.clo[d] - q[d]);  // b above a: b's low side
    }
    return beta;
}

// With rcorr (residual-corrected sources): on the core of a the source is
// built from the FP64 residual r = f - L_h u of the current iterate instead:
//     g_a(p) = r(p) - sum_{b: lag >= 2} Psi_{b->a}(uhat_b^s + ... + uhat_b^{s-lag+2})(p),
// which equals the plain transfer in exact arithmetic (discrete residual
// identity) and feeds the rounding errors of the local solves back as
// sources.  Rows outside the core keep the plain transfer.
//
// The launch first writes every node's value without neighbour terms (0, or
// r on the core in the corrected form: the restriction kernel), then one
// thread per node of the strip list (the nodes within n_ov core layers of
// a box side) adds the neighbour terms, so that no lane idles on the many
// nodes far from every interface.
// One thread per strip node and tile of up to RQ right-hand sides: the
// geometry of every neighbour term (which stencil points lie in b's box, their
// cut-off weights and packed indices) is worked out once and applied to every
// RHS of the tile.
template <typename TIN, typename TOUT, bool PHI, int RQ, bool DIM3>
__global__ __launch_bounds__(kBlock) void k_transfer(const SubDesc *__restrict__ subs, const Coef *__restrict__ coef,
                                                     const double *__restrict__ k2, const double *__restrict__ btab,
                                                     const TIN *__restrict__ l1, const TIN *__restrict__ l2,
                                                     const TIN *__restrict__ l3, TOUT *__restrict__ g, PackArgs A,
                                                     const double2 *__restrict__ rcorr, const int2 *__restrict__ strip,
                                                     long long nstrip, int nrhs) {
    const int r0 = blockIdx.y * RQ;
    const int nr = nrhs - r0 < RQ ? nrhs - r0 : RQ;
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nstrip) return;
    const int2 se = strip[t];
    const int a = se.x;
    const long long e = se.y;
    // a's box, coefficient offsets and neighbour table in registers
    constexpr int NS0 = DIM3 ? 0 : 9, NS = DIM3 ? 26 : 8;  // 2D: only the dz = 0 slots 9 .. 16
    const BoxR s = box_of(subs, a);
    int scoff[3], snbr[NS], slag[NS];
#pragma unroll
    for (int d = 0; d < 3; ++d) scoff[d] = subs[a].coff[d];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        snbr[k] = subs[a].nbr[NS0 + k];
        slag[k] = subs[a].lag[NS0 + k];
    }
    const int lx = (int)(e % s.n[0]), ly = (int)((e / s.n[0]) % s.n[1]), lz = (int)(e / ((long long)s.n[0] * s.n[1]));
    int p[3] = {s.lo[0] + lx, s.lo[1] + ly, s.lo[2] + lz};
    int l[3] = {lx, ly, lz};
    double2 acc[RQ];
    // strip membership per axis: inlo = one of the first n_ov core layers
    // (faces the lower neighbour), inhi = one of the last n_ov core layers;
    // both can hold when the core is narrower than 2 n_ov
    bool inlo[3], inhi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        inlo[d] = d < A.dim && p[d] >= s.clo[d] && p[d] <= s.clo[d] + A.n_ov - 1;
        inhi[d] = d < A.dim && p[d] <= s.chi[d] && p[d] >= s.chi[d] - A.n_ov + 1;
    }
    const bool corrected = rcorr && p[0] >= s.clo[0] && p[0] <= s.chi[0] && p[1] >= s.clo[1] &&
                           p[1] <= s.chi[1] && p[2] >= s.clo[2] && p[2] <= s.chi[2];
    const long long gi = glob_index(A, p[0], p[1], p[2]);
    // loads are issued unconditionally (clamped RHS / node indices, the value
    // masked afterwards) so that a term's loads for every RHS of the tile are
    // in flight together; under a branch each load would be waited for alone
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        const int qc = q < nr ? q : nr - 1;
        const double2 v = rcorr ? rcorr[(long long)(r0 + qc) * A.nglob + gi] : make_double2(0, 0);
        acc[q] = (corrected && q < nr) ? v : make_double2(0, 0);
    }
    const double kk = PHI ? 0.0 : k2[gi];
    Coef cf[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cf[d] = coef[scoff[d] + l[d]];
    // neighbour slots in (dz, dy, dx) order without (0, 0, 0); in 2D only the
    // dz = 0 slots 9 .. 16 exist
    int k = 0;
    for (int dz = DIM3 ? -1 : 0; dz <= (DIM3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const int slot = k++;
                const int bidx = snbr[slot];
                if (bidx < 0) continue;
                int dd[3] = {dx, dy, dz};
                // every differing axis must put p in the strip facing b
                bool ok = true;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (dd[d] < 0 && !inlo[d]) ok = false;
                    if (dd[d] > 0 && !inhi[d]) ok = false;
                }
                if (!ok) continue;
                const int lag = slag[slot];
                const TIN *src = lag == 1 ? l1 : (lag == 2 ? l2 : l3);
                const TIN *src2 = nullptr;
                if (corrected) {
                    // edge / face terms are inside r; lag >= 2 terms use the
                    // newer solutions: uhat^s (+ uhat^{s-1} for lag 3)
                    if (lag == 1) continue;
                    src = l1;
                    src2 = lag == 3 ? l2 : nullptr;
                }
                if (!src) continue;
                const BoxR b = box_of(subs, bidx);
                // stencil points: 0 = p, 2d + 1 = p + e_d, 2d + 2 = p - e_d;
                // weight of the packed value at each (direct: beta, Phi form:
                // beta - beta(p)), its packed index, -1 outside b's box or
                // a's box
                double wt[7];
                long long li[7];
                auto point = [&](int j, int q0, int q1, int q2) {
                    if (!in_box(b, q0, q1, q2)) { li[j] = -1; wt[j] = 0.0; return; }
                    wt[j] = beta_ba(b, dd, btab, A.n_ov, q0, q1, q2);
                    li[j] = b.off + (long long)(q0 - b.lo[0]) +
                            (long long)b.n[0] * ((long long)(q1 - b.lo[1]) + (long long)b.n[1] * (q2 - b.lo[2]));
                };
                point(0, p[0], p[1], p[2]);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    li[2 * d + 1] = li[2 * d + 2] = -1;
                    wt[2 * d + 1] = wt[2 * d + 2] = 0.0;
                    if (d >= A.dim) continue;
                    int qp[3] = {p[0], p[1], p[2]}, qm[3] = {p[0], p[1], p[2]};
                    qp[d] += 1;
                    qm[d] -= 1;
                    if (p[d] < s.hi[d]) point(2 * d + 1, qp[0], qp[1], qp[2]);
                    if (p[d] > s.lo[d]) point(2 * d + 2, qm[0], qm[1], qm[2]);
                }
                if constexpr (PHI) {
                    const double b0 = wt[0];
#pragma unroll
                    for (int j = 1; j < 7; ++j) wt[j] -= b0;
                }
                // clamped packed indices: a point outside b's box reads b's
                // first node and is masked by its zero weight
                long long lc[7];
                bool use[7];
#pragma unroll
                for (int j = 0; j < 7; ++j) {
                    use[j] = li[j] >= 0 && wt[j] != 0.0;
                    lc[j] = li[j] >= 0 ? li[j] : b.off;
                }
                constexpr int NP = DIM3 ? 7 : 5;  // stencil points
                // TWO: the sum of two solutions (the corrected form's lag-3 terms)
                auto term = [&](auto two) {
                constexpr bool TWO = decltype(two)::value;
                // RHS whose loads are in flight together (fewer for complex128 and
                // the 7-point stencil: registers)
                constexpr int QC0 = (sizeof(TIN) > 8 ? 2 : 4) / (DIM3 ? 2 : 1);
                constexpr int QC = RQ < QC0 ? RQ : QC0;
#pragma unroll
                for (int q0 = 0; q0 < RQ; q0 += QC) {
                TIN ld[QC][NP], ld2[QC][TWO ? NP : 1];
#pragma unroll
                for (int qq = 0; qq < QC; ++qq) {
                    const int q = q0 + qq, qc = q < nr ? q : nr - 1;
                    const long long ro = (long long)(r0 + qc) * A.etot;
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        ld[qq][j] = src[ro + lc[j]];
                        if constexpr (TWO) ld2[qq][j] = src2[ro + lc[j]];
                    }
                }
#pragma unroll
                for (int qq = 0; qq < QC; ++qq) {
                    const int q = q0 + qq;
                    double2 pv[7];
#pragma unroll
                    for (int j = 0; j < 7; ++j) pv[j] = make_double2(0, 0);
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        double2 v = to_d2(ld[qq][j]);
                        if constexpr (TWO) v = cadd(v, to_d2(ld2[qq][j]));
                        pv[j] = use[j] ? cscale(v, wt[j]) : make_double2(0, 0);
                    }
                    auto val = [&](int j) { return pv[j]; };
                    double2 Lw;
                    if constexpr (PHI) {
                        // commutator: sum_d cp (beta_+ - beta_0) v_+ + cm (beta_- - beta_0) v_-
                        Lw = make_double2(0, 0);
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            if (d >= A.dim) continue;
                            Lw = cadd(Lw, cadd(cmul(cf[d].cp, val(2 * d + 1)), cmul(cf[d].cm, val(2 * d + 2))));
                        }
                    } else {
                        const double2 w0 = val(0);
                        Lw = cscale(w0, kk);
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            if (d >= A.dim) continue;
                            const double2 wp = val(2 * d + 1), wm = val(2 * d + 2);
                            Lw = cadd(Lw, csub(cmul(cf[d].cp, csub(wp, w0)), cmul(cf[d].cm, csub(w0, wm))));
                        }
                    }
                    // plain: acc += Psi = -L(beta v); corrected: acc -= Psi
                    acc[q] = corrected ? cadd(acc[q], Lw) : csub(acc[q], Lw);
                }
                __builtin_amdgcn_sched_barrier(0);  // one chunk of loads live at a time (registers)
                }
                };
                if (src2) term(std::true_type{});
                else term(std::false_type{});
            }
#pragma unroll
    for (int q = 0; q < RQ; ++q)
        if (q < nr) g[(long long)(r0 + q) * A.etot + s.off + e] = from_d2<TOUT>(acc[q]);
}

// ---------------------------------------------------------------------------
// Assembly u(p) (+)= sum_a beta_{0;a}(p) U_a(p) (eq. tsum).  beta_{0;a} is the
// product over axes of the boxes' cut-off factors; per axis at most two boxes
// have a non-zero factor at p (the AxisOwn tables), visited in increasing
// subdomain order.  active[rhs] == 0 skips the RHS.
// ---------------------------------------------------------------------------
constexpr int kAsmRQ = 4;  // RHS per assembly thread

template <typename TIN, int RQ>
__global__ __launch_bounds__(kBlock) void k_assemble(const SubDesc *__restrict__ subs,
                                                     const AxisOwn *__restrict__ aown, int o0, int o1, int o2,
                                                     int N0, int N1, const TIN *__restrict__ U,
                                                     double2 *__restrict__ u, PackArgs A, int accumulate,
                                                     const int *__restrict__ active, int nrhs) {
    // one thread per global node (pieces of kRowPiece nodes of a grid row per
    // workgroup) and tile of up to RQ right-hand sides: the
    // node's owners (at most 2 per axis), their cut-off weights and packed
    // offsets are found once and applied to every RHS of the tile
    const int r0 = blockIdx.y * RQ;
    const int nr = nrhs - r0 < RQ ? nrhs - r0 : RQ;
    bool act[RQ];
    bool any = false;
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        act[q] = q < nr && (!active || active[r0 + q]);
        any = any || act[q];
    }
    if (!any) return;
    const int nch = (A.G0 + kRowPiece - 1) / kRowPiece;
    const int rowi = (int)blockIdx.x / nch;  // gy + G1 * gz
    const int gx = ((int)blockIdx.x % nch) * kRowPiece + (int)threadIdx.x;
    if (gx >= A.G0) return;
    const int gy = rowi % A.G1, gz = rowi / A.G1;
    const AxisOwn ey = aown[o1 + gy], ez = aown[o2 + gz];
    const AxisOwn ex = aown[o0 + gx];
    // owner k = c0 + 2 c1 + 4 c2 (weight 0 past an axis' owner count);
    // fixed bounds keep the tables in registers
    long long off[8];
    double wt[8];
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
        for (int c1 = 0; c1 < 2; ++c1) {
            const bool yz = c2 < ez.cnt && c1 < ey.cnt;
            const int ayz = yz ? N0 * (ey.i[c1] + N1 * ez.i[c2]) : 0;
            const long long lyz = yz ? (long long)ey.lc[c1] + (long long)ey.n[c1] * ez.lc[c2] : 0;
#pragma unroll
            for (int c0 = 0; c0 < 2; ++c0) {
                const int k = c0 + 2 * c1 + 4 * c2;
                const bool ok = yz && c0 < ex.cnt;
                wt[k] = ok ? ex.beta[c0] * ey.beta[c1] * ez.beta[c2] : 0.0;
                off[k] = ok ? subs[ex.i[c0] + ayz].off + (long long)ex.lc[c0] + (long long)ex.n[c0] * lyz : 0;
            }
        }
    const long long gi = (long long)rowi * A.G0 + gx;
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        if (!act[q]) continue;
        const TIN *Ur = U + (long long)(r0 + q) * A.etot;
        double2 acc = make_double2(0, 0);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (wt[k] != 0.0) acc = cadd(acc, cscale(to_d2(Ur[off[k]]), wt[k]));
        double2 *uq = u + (long long)(r0 + q) * A.nglob + gi;
        *uq = accumulate ? cadd(*uq, acc) : acc;
    }
}

static PackArgs pack_args(const Plan &P) {
    PackArgs A;
    A.dim = P.dim; A.n_ov = P.n_ov;
    A.G0 = P.G[0]; A.G1 = P.G[1];
    A.glo0 = P.glo[0]; A.glo1 = P.glo[1]; A.glo2 = P.glo[2];
    A.etot = P.etot; A.nglob = P.nglob;
    return A;
}

static int max_rows(const Plan &P) {  // grid rows (n1 * n2) of the largest box
    int m = 0;
    for (const SubDesc &s : P.subs) m = s.n[1] * s.n[2] > m ? s.n[1] * s.n[2] : m;
    return m;
}

// true when g points into the handle's source workspace
static bool in_source_ws(const ddm_handle *h, const void *g) {
    const char *b = (const char *)h->d_g;
    return b && (const char *)g >= b && (const char *)g < b + (size_t)h->nrhs_max * h->plan.etot * (h->mixed ? sizeof(float2) : sizeof(double2));
}

template <typename TIN, typename TOUT>
hipError_t launch_restrict(ddm_handle *h, const TIN *f, TOUT *g, int nrhs) {
    const Plan &P = h->plan;
    if (in_source_ws(h, g)) h->g_clean_rows = 0;  // cores written
    dim3 grid((unsigned)max_rows(P), P.nsub, (nrhs + kRestrictRQ - 1) / kRestrictRQ);
    k_restrict<TIN, TOUT><<<grid, kBlock, 0, h->stream>>>(h->d_subs, f, g, pack_args(P), nrhs);
    return hipGetLastError();
}

template <typename TIN, typename TOUT>
hipError_t launch_transfer(ddm_handle *h, const TIN *l1, const TIN *l2, const TIN *l3, TOUT *g, int nrhs,
                           const double2 *rcorr) {
    const Plan &P = h->plan;
    // packed g written; neighbour strips (n_ov + 1 layers) read
    double strip = 0.0;
    for (const SubDesc &sd : P.subs)
        for (int d = 0; d < P.dim; ++d) strip += 2.0 * (P.n_ov + 1) * (double)sd.nloc / sd.n[d];
    ProfScope ps(h, DDM_K_TRANSFER, (double)nrhs * ((double)P.etot * sizeof(TOUT) + strip * sizeof(TIN)));
    if (rcorr) {
        dim3 rg((unsigned)max_rows(P), P.nsub, (nrhs + kRestrictRQ - 1) / kRestrictRQ);
        k_restrict<double2, TOUT><<<rg, kBlock, 0, h->stream>>>(h->d_subs, rcorr, g, pack_args(P), nrhs);
        if (in_source_ws(h, g)) h->g_clean_rows = 0;
    } else if (!((void *)g == h->d_g && h->g_clean_rows >= nrhs)) {
        // the strip kernel writes only strip nodes: everything else must be
        // zero.  The handle's workspace stays so from one step to the next
        // (only restrictions write elsewhere), so it is cleared only after one
        hipError_t e = launch_fill_zero(g, (long long)nrhs * P.etot * sizeof(TOUT), h->stream);
        if (e != hipSuccess) return e;
        if ((void *)g == h->d_g) h->g_clean_rows = nrhs;
    }
    const long long ns = (long long)P.strip.size();
    if (ns > 0) {
        // RHS per thread: 4, or 8 for batches of more than 4 (the geometry of
        // a node's neighbour terms is worked out once per tile; with the
        // loads of 4 RHS in flight together, 8-RHS tiles keep the registers
        // for two waves per SIMD: 0.98 -> 0.54 ms per complex64 transfer on
        // the layered 2048^2 batch, against 0.70 ms with 16-RHS tiles)
        const bool phi = h->transfer_form == DDM_TRANSFER_PHI, d3 = P.dim == 3;
        auto launch = [&](auto rq) {
            constexpr int RQ = decltype(rq)::value;
            dim3 grid((unsigned)((ns + kBlock - 1) / kBlock), (nrhs + RQ - 1) / RQ);
            auto kern = phi ? (d3 ? k_transfer<TIN, TOUT, true, RQ, true> : k_transfer<TIN, TOUT, true, RQ, false>)
                            : (d3 ? k_transfer<TIN, TOUT, false, RQ, true> : k_transfer<TIN, TOUT, false, RQ, false>);
            kern<<<grid, kBlock, 0, h->stream>>>(h->d_subs, h->d_coef, h->d_k2, h->d_btab, l1, l2, l3, g, pack_args(P),
                                                 rcorr, h->d_strip, ns, nrhs);
        };
        if (nrhs > 4) launch(std::integral_constant<int, 8>{});
        else launch(std::integral_constant<int, 4>{});
    }
    return hipGetLastError();
}

template <typename TIN>
hipError_t launch_assemble(ddm_handle *h, const TIN *U, double2 *u, int nrhs, bool accumulate, const int *d_active) {
    const Plan &P = h->plan;
    dim3 grid((unsigned)(P.G[1] * P.G[2] * row_pieces(P)), (nrhs + kAsmRQ - 1) / kAsmRQ);
    // local solutions read once per global node, u read (if accumulating) and written
    ProfScope ps(h, DDM_K_ASSEMBLE, (double)P.nglob * nrhs * (sizeof(TIN) + (accumulate ? 32.0 : 16.0)));
    k_assemble<TIN, kAsmRQ><<<grid, kBlock, 0, h->stream>>>(h->d_subs, h->d_aown, P.aoff[0], P.aoff[1], P.aoff[2],
                                                            P.N[0], P.N[1], U, u, pack_args(P), accumulate ? 1 : 0,
                                                            d_active, nrhs);
    return hipGetLastError();
}

template hipError_t launch_restrict<double2, double2>(ddm_handle *, const double2 *, double2 *, int);
template hipError_t launch_restrict<double2, float2>(ddm_handle *, const double2 *, float2 *, int);
template hipError_t launch_transfer<double2, double2>(ddm_handle *, const double2 *, const double2 *,
                                                      const double2 *, double2 *, int, const double2 *);
template hipError_t launch_transfer<float2, float2>(ddm_handle *, const float2 *, const float2 *, const float2 *,
                                                    float2 *, int, const double2 *);
template hipError_t launch_assemble<double2>(ddm_handle *, const double2 *, double2 *, int, bool, const int *);
template hipError_t launch_assemble<float2>(ddm_handle *, const float2 *, double2 *, int, bool, const int *);

// ---------------------------------------------------------------------------
// casts and fills
// ---------------------------------------------------------------------------
__global__ void k_c128_to_c64(const double2 *__restrict__ in, float2 *__restrict__ out, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
}
__global__ void k_c64_to_c128(const float2 *__restrict__ in, double2 *__restrict__ out, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = make_double2(in[i].x, in[i].y);
}
__global__ void k_fill_zero(uint4 *__restrict__ p, long long n16, unsigned char *__restrict__ tail, int ntail) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n16; i += (long long)gridDim.x * kBlock)
        p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

static unsigned grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_convert_c128_to_c64(const double2 *in, float2 *out, long long n, hipStream_t s) {
    k_c128_to_c64<<<grid_for(n), kBlock, 0, s>>>(in, out, n);
    return hipGetLastError();
}
hipError_t launch_convert_c64_to_c128(const float2 *in, double2 *out, long long n, hipStream_t s) {
    k_c64_to_c128<<<grid_for(n), kBlock, 0, s>>>(in, out, n);
    return hipGetLastError();
}
// zero fill with a kernel (a memset node is avoided so that a captured step
// replays correctly)
hipError_t launch_fill_zero(void *p, long long bytes, hipStream_t s) {
    long long n16 = bytes / 16;
    int ntail = (int)(bytes - n16 * 16);
    k_fill_zero<<<grid_for(n16 > 0 ? n16 : 1), kBlock, 0, s>>>((uint4 *)p, n16, (unsigned char *)p + n16 * 16, ntail);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Krylov vector operations (FP64 complex; RHS r's vectors at stride ld)
// ---------------------------------------------------------------------------
// partial dot products conj(V_i) . w, grid (nblk, nvec, nrhs)
__global__ __launch_bounds__(kBlock) void k_dots_part(const double2 *__restrict__ V, long long vstride,
                                                      const double2 *__restrict__ w, long long n, long long ld,
                                                      double *__restrict__ part) {
    __shared__ double sh[kBlock / 64];
    int i = blockIdx.y, rhs = blockIdx.z, nvec = gridDim.y;
    const double2 *v = V + i * vstride + rhs * ld;
    const double2 *wr = w + rhs * ld;
    double sr = 0.0, si = 0.0;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) {
        double2 c = cconjmul(v[q], wr[q]);
        sr += c.x;
        si += c.y;
    }
    double a = block_sum(sr, sh);
    double b = block_sum(si, sh);
    if (threadIdx.x == 0) {
        long long base = ((long long)rhs * nvec + i) * gridDim.x + blockIdx.x;
        part[2 * base] = a;
        part[2 * base + 1] = b;
    }
}

__global__ __launch_bounds__(kBlock) void k_dots_sum(const double *__restrict__ part, int nblk,
                                                     double2 *__restrict__ out) {
    __shared__ double sh[kBlock / 64];
    long long item = blockIdx.x;  // rhs * nvec + i
    double sr = 0.0, si = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        sr += part[2 * (item * nblk + b)];
        si += part[2 * (item * nblk + b) + 1];
    }
    double a = block_sum(sr, sh);
    double c = block_sum(si, sh);
    if (threadIdx.x == 0) out[item] = make_double2(a, c);
}

hipError_t launch_dots(const double2 *V, int nvec, long long vstride, const double2 *w, long long n, int nrhs,
                       long long ld, double2 *d_out, double *d_part, int nblk, hipStream_t s) {
    k_dots_part<<<dim3(nblk, nvec, nrhs), kBlock, 0, s>>>(V, vstride, w, n, ld, d_part);
    k_dots_sum<<<nvec * nrhs, kBlock, 0, s>>>(d_part, nblk, d_out);
    return hipGetLastError();
}

// w_r += sign * sum_i coef[r * nvec + i] V_i,r
__global__ __launch_bounds__(kBlock) void k_axpy_multi(double2 *__restrict__ w, const double2 *__restrict__ V,
                                                       int nvec, long long vstride, const double2 *__restrict__ coef,
                                                       double sign, long long n, long long ld) {
    int rhs = blockIdx.y;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) {
        double2 acc = w[rhs * ld + q];
        for (int i = 0; i < nvec; ++i) {
            double2 c = cscale(coef[rhs * nvec + i], sign);
            acc = cadd(acc, cmul(c, V[i * vstride + rhs * ld + q]));
        }
        w[rhs * ld + q] = acc;
    }
}

hipError_t launch_axpy_multi(double2 *w, const double2 *V, int nvec, long long vstride, const double2 *coef,
                             double sign, long long n, int nrhs, long long ld, hipStream_t s) {
    k_axpy_multi<<<dim3(grid_for(n) > 2048 ? 2048 : grid_for(n), nrhs), kBlock, 0, s>>>(w, V, nvec, vstride, coef,
                                                                                      sign, n, ld);
    return hipGetLastError();
}

// y_r = x_r / sqrt(scale[r]) (0 if scale[r] == 0)
__global__ __launch_bounds__(kBlock) void k_scale(double2 *__restrict__ y, const double2 *__restrict__ x,
                                                  const double *__restrict__ scale, long long n, long long ld) {
    int rhs = blockIdx.y;
    double s = scale[rhs];
    double inv = s > 0 ? 1.0 / sqrt(s) : 0.0;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock)
        y[rhs * ld + q] = cscale(x[rhs * ld + q], inv);
}

hipError_t launch_scale(double2 *y, const double2 *x, const double *scale, long long n, int nrhs, long long ld,
                        hipStream_t s) {
    k_scale<<<dim3(grid_for(n) > 2048 ? 2048 : grid_for(n), nrhs), kBlock, 0, s>>>(y, x, scale, n, ld);
    return hipGetLastError();
}

}  // namespace ddm
