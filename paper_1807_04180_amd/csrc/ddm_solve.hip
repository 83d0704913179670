// Batched block forward / back substitution with the stored inverses
// W_l = S_l^{-1} of the block-tridiagonal factorisation: the local solves of
// every step of Algorithm 3.1, all subdomains and right-hand sides at once.
//   forward:  z_0 = W_0 g_0,  z_l = W_l (g_l - cm(l) z_{l-1})
//   backward: x_{nb-1} = z_{nb-1},  x_l = z_l - W_l (cp(l) x_{l+1})
//
// One launch per block index l covers every subdomain; work item (a, r0)
// computes rows r0 .. r0+63 of W_l v for all right-hand sides.  W_l is
// column-major, so lane = row and the 64 rows of one column are one
// contiguous 1 KB (complex128) / 512 B (complex64) load; the 4 waves of a
// workgroup split the columns and are summed through LDS.  v is staged in
// LDS in column tiles (broadcast reads).  The substitution streams every W_l
// once per sweep: it is HBM-bound.
#include <hip/hip_runtime.h>

#include "cplx.h"
#include "ddm_internal.h"
#include "ddm_sync.h"

namespace ddm {

// Loads of the stored inverses, which are read once per sweep: complex128
// ones are marked non-temporal (FP64 local solves 2-3% faster with the split
// and per-line kernels); complex64 ones stay plain (neutral with the split
// kernel, 4% slower with the per-line one).
typedef double ntv_d2 __attribute__((ext_vector_type(2)));
__device__ inline double2 ld_w(const double2 *p) {
    const ntv_d2 v = __builtin_nontemporal_load((const ntv_d2 *)p);
    return make_double2(v[0], v[1]);
}
__device__ inline float2 ld_w(const float2 *p) { return *p; }
__device__ inline float4 ld_w(const float4 *p) { return *p; }

constexpr int kSThreads = 256;
constexpr int kSWaves = kSThreads / 64;

template <typename T2, int RT, bool BACKWARD>
__global__ __launch_bounds__(kSThreads) void k_solve_line(const SubDesc *__restrict__ subs,
                                                          const SolveItem *__restrict__ items,
                                                          const Coef *__restrict__ coef, const T2 *__restrict__ W,
                                                          const T2 *__restrict__ g, T2 *__restrict__ x, int step,
                                                          int nrhs, long long etot, int dim) {
    constexpr int JT = 1024 / RT;  // columns per LDS tile
    __shared__ T2 vs[JT * RT];
    __shared__ T2 red[kSWaves * RT * 64];

    const SolveItem it = items[blockIdx.x];
    const SubDesc &s = subs[it.a];
    const int nb = s.nb, bs = s.bs;
    const int l = BACKWARD ? nb - 2 - step : step;
    if (l < 0 || l >= nb) return;
    const long long off = s.off;
    const int ld = s.ld;
    const T2 *Wl = W + s.foff + (long long)l * bs * ld;
    const Coef c = coef[s.coff[dim - 1] + l];
    const double2 cpl = BACKWARD ? c.cp : c.cm;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = it.r0 + lane;

    for (int r0 = 0; r0 < nrhs; r0 += RT) {
        const int nr = nrhs - r0 < RT ? nrhs - r0 : RT;
        T2 acc[RT];
#pragma unroll
        for (int q = 0; q < RT; ++q) acc[q] = czero<T2>();
        for (int j0 = 0; j0 < bs; j0 += JT) {
            const int jn = bs - j0 < JT ? bs - j0 : JT;
            for (int t = threadIdx.x; t < jn * RT; t += kSThreads) {
                const int jj = t / RT, q = t % RT;
                double2 v = make_double2(0, 0);
                if (q < nr) {
                    const long long base = (long long)(r0 + q) * etot + off;
                    const int j = j0 + jj;
                    if (!BACKWARD) {
                        v = to_d2(g[base + (long long)l * bs + j]);
                        if (l > 0) v = cmsub_fixed(v, cpl, to_d2(x[base + (long long)(l - 1) * bs + j]));
                    } else {
                        v = cmul_fixed(cpl, to_d2(x[base + (long long)(l + 1) * bs + j]));
                    }
                }
                vs[jj * RT + q] = from_d2<T2>(v);
            }
            __syncthreads();
            if (row < bs) {
                const T2 *col = Wl + (long long)j0 * ld + row;
                int jj = wv;
                for (; jj + 3 * kSWaves < jn; jj += 4 * kSWaves) {
                    T2 w0 = ld_w(col + (long long)jj * ld);
                    T2 w1 = ld_w(col + (long long)(jj + kSWaves) * ld);
                    T2 w2 = ld_w(col + (long long)(jj + 2 * kSWaves) * ld);
                    T2 w3 = ld_w(col + (long long)(jj + 3 * kSWaves) * ld);
#pragma unroll
                    for (int q = 0; q < RT; ++q) {
                        cfma(acc[q], w0, vs[jj * RT + q]);
                        cfma(acc[q], w1, vs[(jj + kSWaves) * RT + q]);
                        cfma(acc[q], w2, vs[(jj + 2 * kSWaves) * RT + q]);
                        cfma(acc[q], w3, vs[(jj + 3 * kSWaves) * RT + q]);
                    }
                }
                for (; jj < jn; jj += kSWaves) {
                    T2 w0 = ld_w(col + (long long)jj * ld);
#pragma unroll
                    for (int q = 0; q < RT; ++q) cfma(acc[q], w0, vs[jj * RT + q]);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < RT; ++q) red[(wv * RT + q) * 64 + lane] = acc[q];
        __syncthreads();
        if (wv == 0 && row < bs) {
            for (int q = 0; q < nr; ++q) {
                T2 sum = red[q * 64 + lane];
#pragma unroll
                for (int w = 1; w < kSWaves; ++w) {
                    T2 o = red[(w * RT + q) * 64 + lane];
                    sum.x += o.x;
                    sum.y += o.y;
                }
                const long long o = (long long)(r0 + q) * etot + off + (long long)l * bs + row;
                if (!BACKWARD) {
                    x[o] = sum;
                } else {
                    T2 z = x[o];
                    z.x -= sum.x;
                    z.y -= sum.y;
                    x[o] = z;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Chain variant: one workgroup (16 waves) owns a whole elimination chain of a
// subdomain and walks its blocks; the recurrence never leaves the compute
// unit (block vectors in LDS / registers), only W_l streams from HBM.
//   chain 0 (blocks 0 .. mid-1):  y_0 = W_0 g_0, y_l = W_l (g_l - cm(l) y_{l-1})
//   chain 1 (blocks nb-1 .. mid+1): y_l = W_l (g_l - cp(l) y_{l+1})
//   middle:  x_mid = W_mid (g_mid - cm(mid) y_{mid-1} - cp(mid) y_{mid+1})
//   back:    x_l = y_l - W_l (cp(l) x_{l+1})  (chain 0, l = mid-1 .. 0)
//            x_l = y_l - W_l (cm(l) x_{l-1})  (chain 1, l = mid+1 .. nb-1)
// (W_l here is the stored inverse of the chain's Schur block.)  The two
// chains of a subdomain meet once, at the middle block: each stores its last
// y block with relaxed agent-scope atomics and raises a flag, the other
// reads it with atomic loads once it has seen the flag (no fences).
// GEMV mapping: R = ceil(bs/64) row tiles, CG = 16 / R column groups; wave w
// takes row tile w % R and columns w / R, w / R + CG, ...  The first batch of
// the next block's W is loaded before the current block's reduction.
// ---------------------------------------------------------------------------
constexpr int kCThreads = 1024;
constexpr int kCWaves = 16;
constexpr size_t kLdsMax = 160 * 1024;  // LDS per workgroup on gfx950

// Rows per lane: complex64 lanes take two consecutive rows so that every
// load is 16 bytes (8-byte lane loads stream at about 60% of the per-CU
// rate of 16-byte ones); LT is the per-lane load type.
template <typename T2, int ROWS> struct LaneT;
template <> struct LaneT<double2, 1> { using type = double2; };
template <> struct LaneT<float2, 1> { using type = float2; };
template <> struct LaneT<float2, 2> { using type = float4; };

__device__ inline double2 lane_row(double2 v, int) { return v; }
__device__ inline float2 lane_row(float2 v, int) { return v; }
__device__ inline float2 lane_row(float4 v, int r) { return r == 0 ? make_float2(v.x, v.y) : make_float2(v.z, v.w); }

template <typename LT> __device__ inline LT lane_zero();
template <> __device__ inline double2 lane_zero<double2>() { return make_double2(0, 0); }
template <> __device__ inline float2 lane_zero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ inline float4 lane_zero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }

// columns per W batch (two batches in flight per wave)
template <typename T2, int ROWS> struct ChainBatch { static constexpr int value = 8; };
template <> struct ChainBatch<double2, 1> { static constexpr int value = 4; };
template <> struct ChainBatch<float2, 2> { static constexpr int value = 4; };
// the split variant: complex64 streams 5 columns per batch (1.8% faster than
// 4; complex128 gains nothing from 5)
template <typename T2, int ROWS> struct ChainBatch2 { static constexpr int value = ChainBatch<T2, ROWS>::value; };
template <> struct ChainBatch2<float2, 2> { static constexpr int value = 5; };

// Columns per wave staged in LDS ahead of each block step (direct
// global->LDS loads of 16 bytes per lane).
template <typename T2, int ROWS> struct kLdsCols { static constexpr int value = 0; };
template <> struct kLdsCols<double2, 1> { static constexpr int value = 4; };
template <> struct kLdsCols<float2, 2> { static constexpr int value = 4; };
// The split variant stages one column per wave: the wait for its exchange
// stores (vmcnt 0) also waits for every prefetch load the wave has in flight,
// so deeper staging lengthens the exchange (measured: 1 column is faster
// than 0, 2, 3 or 4).
template <typename T2, int ROWS> struct kLdsCols2 { static constexpr int value = 0; };
template <> struct kLdsCols2<double2, 1> { static constexpr int value = 1; };
template <> struct kLdsCols2<float2, 2> { static constexpr int value = 1; };

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima)
constexpr int kWaitVm0 = 0x0F70;

// Copy this wave's columns j = cg + CG u (u < PF) of the column-major block
// Wl (column stride ld) to LDS: lane i of the wave lands at 16-byte slot
// u * 64 + i of dst (the hardware places 16 bytes per lane consecutively
// from the wave-uniform base).  Lanes past the block copy the clamped last
// row (pair).
template <typename T2, int PF, int ROWS>
__device__ inline void lds_prefetch(const T2 *Wl, T2 *dst, int cg, int CG, int bs, int ld, int rowc, bool gemv) {
    if constexpr (PF > 0) {
        static_assert(sizeof(T2) * ROWS == 16, "direct LDS loads of 16 bytes per lane");
        if (!gemv) return;
#pragma unroll 1
        for (int u = 0; u < PF; ++u) {
            const int j = cg + CG * u;
            if (j < bs)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(Wl + (long long)j * ld + rowc),
                    (__attribute__((address_space(3))) void *)(dst + u * 64 * ROWS), 16, 0, 0);
        }
    }
}

template <typename T2, int RT, int ROWS, int NT, int NPAIR>
__global__ __launch_bounds__(NT) void k_solve_chain(const SubDesc *__restrict__ subs,
                                                           const Coef *__restrict__ coef, const T2 *__restrict__ W,
                                                           const T2 *__restrict__ g, T2 *__restrict__ x, int nrhs,
                                                           long long etot, int dim, int twisted, int *flags,
                                                           int *rflags, int *abort_flag, int spin_limit) {
    extern __shared__ unsigned char lds_raw[];
    using LT = typename LaneT<T2, ROWS>::type;
    // 512-thread workgroups (256 VGPRs) keep 8 columns per batch, also for
    // 16-RHS tiles (2048^2 layered, 16 RHS: 17.5 against 19.1 ms per local
    // solve with 4 in complex128, 9.8 against 10.8 in complex64)
    constexpr int kCBatch = NT < kCThreads ? 8 : (RT >= 16 ? 2 : ChainBatch<T2, ROWS>::value);
    const int a = twisted ? (int)(blockIdx.x >> 1) : (int)blockIdx.x;
    const int chain = twisted ? (int)(blockIdx.x & 1) : 0;
    const SubDesc &s = subs[a];
    const int nb = s.nb, bs = s.bs, mid = s.mid, ax = dim - 1;
    const long long off = s.off;
    const int ld = s.ld;
    const int R = (bs + 64 * ROWS - 1) / (64 * ROWS);
    // GEMV work units: (row tile rt, column group cg) pairs p = rt + R cg of
    // a partition into CG = NPAIR / R column groups; NPAIR = 16 whatever the
    // wave count for complex128, so that every variant adds the same partial
    // sums in the same order; wave w takes pairs w, w + NW, ...
    constexpr int NW = NT / 64;          // waves
    constexpr int NP = NPAIR / NW;      // pairs per wave
    // 16-RHS tiles on 1024-thread workgroups: the partial sums of the
    // column groups are added into one [RT][bsp] buffer in column-group
    // order (one barrier per group) instead of being kept side by side
    constexpr bool SEQ = RT >= 16 && NT == kCThreads;
    static_assert(!SEQ || NP == 1, "sequential reduction: one pair per wave");
    const int CG = NPAIR / R;
    const int npair = R * CG;
    // the wave index is uniform: keep it (and what derives from it) scalar
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rt = wv % R, cg = wv / R;  // the wave's first pair
    const bool gemv = cg < CG;
    const int row = (rt * 64 + lane) * ROWS;  // this lane's first row (first pair)
    const bool rowok = gemv && row < bs;
    const int bsp = R * 64 * ROWS;
    T2 *vs = (T2 *)lds_raw;                 // [bsp][RT]  current v
    T2 *red = vs + (size_t)bsp * RT;        // [CG][RT][bsp] partial sums ([RT][bsp] when SEQ)
    // complex128: each wave's first kLdsCols columns of the next block are
    // copied to LDS by direct global->LDS loads while the block step
    // reduces, synchronises and forms the next v (the column stream would
    // otherwise idle there); the register stream starts after them
    constexpr int PF = NT == kCThreads && !SEQ ? kLdsCols<T2, ROWS>::value : 0;
    T2 *mypf = red + (size_t)(SEQ ? 1 : CG) * RT * bsp + (size_t)wv * PF * 64 * ROWS;  // [PF][64 lanes][ROWS]
    // this chain's block sequence: forward blocks, the middle, backward blocks
    const int nf = chain == 0 ? mid : nb - 1 - mid;
    if (twisted == 0 && chain == 1) return;
    const int nsteps = 2 * nf + 1;
    const int dirf = chain == 0 ? 1 : -1;   // forward direction in l
    const int lfirst = chain == 0 ? 0 : nb - 1;

    for (int r0 = 0; r0 < nrhs; r0 += RT) {
        const int nr = nrhs - r0 < RT ? nrhs - r0 : RT;
        // flags count RHS tiles: tile k publishes k + 1 (no reset inside the
        // launch, so a fast chain cannot erase a signal)
        const int epoch = r0 / RT + 1;
        // initial v = g_{lfirst} (the middle step builds its own v)
        if (nf > 0) {
            const int l0 = lfirst;
            for (int e = threadIdx.x; e < bsp * RT; e += NT) {
                const int i = e / RT, q = e % RT;
                vs[e] = (i < bs && q < nr) ? g[(long long)(r0 + q) * etot + off + (long long)l0 * bs + i]
                                           : czero<T2>();
            }
        }
        __syncthreads();
        auto step_l = [&](int t) {  // block index of step t
            if (t < nf) return lfirst + dirf * t;
            if (t == nf) return mid;
            return mid - dirf * (t - nf);
        };
        const T2 *Wbase = W + s.foff;
        const long long bs2 = (long long)bs * ld;  // block stride
        // W streaming, double-buffered in batches of kCBatch columns; the
        // batch after a block's last is the next block's first
        const int rowc = row < bs ? row : (bs - 1) / ROWS * ROWS;  // clamped row for the LDS copies
        LT wb[kCBatch];
        {
            const T2 *Wl = Wbase + (long long)step_l(0) * bs2;
            lds_prefetch<T2, PF, ROWS>(Wl, mypf, cg, CG, bs, ld, rowc, gemv);
#pragma unroll
            for (int u = 0; u < kCBatch; ++u) {
                const int j = cg + CG * (PF + u);
                wb[u] = (rowok && j < bs) ? ld_w((const LT *)(Wl + (long long)j * ld + row)) : lane_zero<LT>();
            }
        }
        for (int t = 0; t < nsteps; ++t) {
            const int l = step_l(t);
            const int kind = t < nf ? 0 : (t == nf ? 1 : 2);  // 0 forward, 1 middle, 2 backward
            if (t == nf) {
                // entering the middle block: v = g_mid - cm(mid) y_{mid-1} - cp(mid) y_{mid+1}
                const Coef cmid = coef[s.coff[ax] + mid];
                // the last y block of each chain was stored with relaxed
                // agent-scope atomics (the other chain reads it here)
                __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are complete
                __syncthreads();
                if (twisted) {
                    if (threadIdx.x == 0)
                        __hip_atomic_store(flags + 2 * a + chain, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    wait_flag_relaxed(flags + 2 * a + (1 - chain), epoch, abort_flag, spin_limit);
                }
                for (int e = threadIdx.x; e < bsp * RT; e += NT) {
                    const int i = e / RT, q = e % RT;
                    double2 v = make_double2(0, 0);
                    if (i < bs && q < nr) {
                        const long long base = (long long)(r0 + q) * etot + off;
                        v = to_d2(g[base + (long long)mid * bs + i]);
                        if (mid > 0) v = cmsub_fixed(v, cmid.cm, to_d2(xload(x + base + (long long)(mid - 1) * bs + i)));
                        if (mid < nb - 1)
                            v = cmsub_fixed(v, cmid.cp, to_d2(xload(x + base + (long long)(mid + 1) * bs + i)));
                    }
                    vs[e] = from_d2<T2>(v);
                }
                __syncthreads();
                // every read of the partner's last y block has returned (its
                // value is in LDS): the partner may now overwrite that block
                // with its first backward result
                if (twisted && threadIdx.x == 0)
                    __hip_atomic_store(rflags + 2 * a + chain, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // ---- prefetch the block-vector entries the reduction will need
            // (forward: g of the next block; backward: this block's y) ----
            constexpr int kPre = (256 * RT + NT - 1) / NT;  // bsp * RT <= kPre * NT
            const int tn = t + 1;
            const int lnv = tn < nsteps && tn != nf ? step_l(tn) : -1;
            T2 pre[kPre];
            auto load_pre = [&]() {
#pragma unroll
                for (int u = 0; u < kPre; ++u) {
                    const int e = threadIdx.x + u * NT;
                    const int i = e / RT, q = e % RT;
                    const bool ok = e < bsp * RT && i < bs && q < nr;
                    const long long base = (long long)(ok ? r0 + q : 0) * etot + off;
                    if (kind == 2)  // the first backward block is the atomically stored one
                        pre[u] = ok ? (t == nf + 1 ? xload(x + base + (long long)l * bs + i)
                                                   : x[base + (long long)l * bs + i])
                                    : czero<T2>();
                    else if (kind == 0 && lnv >= 0) pre[u] = ok ? g[base + (long long)lnv * bs + i] : czero<T2>();
                    else pre[u] = czero<T2>();
                }
            };
            load_pre();
            // ---- GEMV: acc = W_l v, per work pair of this wave ----
            const int lnext = t + 1 < nsteps ? step_l(t + 1) : -1;
            T2 acc[ROWS][RT];
#pragma unroll
            for (int pi = 0; pi < NP; ++pi) {
                const int pp = wv + pi * NW;
                if (pp >= npair) break;  // uniform
                const int prt = pp % R, pcg = pp / R;
                const int prow = (prt * 64 + lane) * ROWS;
                const bool prowok = prow < bs;
                // after this pair's last batch the stream continues with the
                // wave's next pair of this block, else its first pair of the
                // next block
                const int pq = pp + NW;
                const bool nextpair = pi + 1 < NP && pq < npair && pq / R < bs;  // next pair has columns
                const int qrow = nextpair ? ((pq % R) * 64 + lane) * ROWS : row;
                const int qcg = nextpair ? pq / R : cg;
                const bool qrowok = nextpair ? qrow < bs : rowok;
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
#pragma unroll
                    for (int q = 0; q < RT; ++q) acc[r][q] = czero<T2>();
                const int kmax = (bs - pcg + CG - 1) / CG;  // columns of this pair
                if constexpr (PF > 0) {
                    __builtin_amdgcn_s_waitcnt(kWaitVm0);  // this wave's LDS copies have landed
#pragma unroll 1
                    for (int u = 0; u < PF; ++u) {
                        if (u < kmax) {
                            const int j = pcg + CG * u;
                            const LT w = ((const LT *)mypf)[u * 64 + lane];
#pragma unroll
                            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                                for (int q = 0; q < RT; ++q) cfma(acc[r][q], lane_row(w, r), vs[j * RT + q]);
                        }
                    }
                }
                for (int k0 = PF; k0 < kmax; k0 += kCBatch) {
                    const bool more = k0 + kCBatch < kmax;
                    const int ln = more || nextpair ? l : lnext;
                    const int kn = more ? k0 + kCBatch : PF;
                    const int ncg = more ? pcg : qcg;
                    const int nrow = more ? prow : qrow;
                    const bool nrowok = more ? prowok : qrowok;
                    LT wn[kCBatch];
                    const T2 *Wn = Wbase + (long long)(ln >= 0 ? ln : 0) * bs2;
#pragma unroll
                    for (int u = 0; u < kCBatch; ++u) {
                        const int j = ncg + CG * (kn + u);
                        wn[u] = (ln >= 0 && nrowok && j < bs) ? ld_w((const LT *)(Wn + (long long)j * ld + nrow))
                                                               : lane_zero<LT>();
                    }
#pragma unroll
                    for (int u = 0; u < kCBatch; ++u) {
                        const int j = pcg + CG * (k0 + u);
                        if (j < bs) {
#pragma unroll
                            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                                for (int q = 0; q < RT; ++q) cfma(acc[r][q], lane_row(wb[u], r), vs[j * RT + q]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kCBatch; ++u) wb[u] = wn[u];
                }
                if constexpr (!SEQ) {
#pragma unroll
                    for (int r = 0; r < ROWS; ++r)
#pragma unroll
                        for (int q = 0; q < RT; ++q) red[((size_t)pcg * RT + q) * bsp + prow + r] = acc[r][q];
                }
            }
            if constexpr (SEQ) {
                // column group c adds its rows' partial sums in round c
                const bool has = wv < npair;
                const int scg = wv / R, srow = ((wv % R) * 64 + lane) * ROWS;
                for (int c = 0; c < CG; ++c) {
                    if (has && scg == c) {
#pragma unroll
                        for (int r = 0; r < ROWS; ++r)
#pragma unroll
                            for (int q = 0; q < RT; ++q) {
                                T2 &d = red[(size_t)q * bsp + srow + r];
                                if (c == 0) {
                                    d = acc[r][q];
                                } else {
                                    T2 o = d;
                                    o.x += acc[r][q].x;
                                    o.y += acc[r][q].y;
                                    d = o;
                                }
                            }
                    }
                    __syncthreads();
                }
            }
            if (lnext >= 0)
                lds_prefetch<T2, PF, ROWS>(Wbase + (long long)lnext * bs2, mypf, cg, CG, bs, ld, rowc, gemv);
            __syncthreads();
            // the first backward step overwrites the y block the partner read
            // at the middle: wait until the partner has finished reading it
            if (twisted && t == nf + 1)
                wait_flag_relaxed(rflags + 2 * a + (1 - chain), epoch, abort_flag, spin_limit);
            // ---- reduce over column groups; update x; build the next v ----
#pragma unroll
            for (int u = 0; u < kPre; ++u) {
                const int e = threadIdx.x + u * NT;
                if (e >= bsp * RT) continue;
                const int i = e / RT, q = e % RT;
                if (i >= bs) continue;
                T2 sum = red[(size_t)q * bsp + i];
                for (int c = 1; c < (SEQ ? 1 : CG); ++c) {
                    T2 o = red[((size_t)c * RT + q) * bsp + i];
                    sum.x += o.x;
                    sum.y += o.y;
                }
                const long long base = (long long)(r0 + q) * etot + off;
                T2 res = sum;                       // forward: y_l, middle: x_mid
                if (kind == 2) {                    // backward: x_l = y_l - W_l v
                    res.x = pre[u].x - sum.x;
                    res.y = pre[u].y - sum.y;
                }
                if (q < nr && (kind != 1 || chain == 0)) {
                    if (t == nf - 1) xstore(x + base + (long long)l * bs + i, res);  // read at the middle
                    else x[base + (long long)l * bs + i] = res;
                }
                if (lnv >= 0) {
                    // next v from this block's result
                    double2 v;
                    const Coef cn = coef[s.coff[ax] + lnv];
                    if (kind == 0) {                // forward: g_ln - c * y_l
                        const double2 c = chain == 0 ? cn.cm : cn.cp;
                        v = q < nr ? cmsub_fixed(to_d2(pre[u]), c, to_d2(res)) : make_double2(0, 0);
                    } else {                        // after middle / backward: c * x_l
                        const double2 c = chain == 0 ? cn.cp : cn.cm;
                        v = q < nr ? cmul_fixed(c, to_d2(res)) : make_double2(0, 0);
                    }
                    vs[e] = from_d2<T2>(v);
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Split chain substitution: two workgroups per chain of a two-ended layout,
// for problems with too few chains to give every CU one (one workgroup per
// chain streams at the per-CU request rate, so half the chip would idle).
// Half h of a chain takes the columns [c0, c1) of every block (c1 - c0 about
// bs / 2) and the matching rows of every result.  Per block step each half
// forms the partial product of its columns for all rows, publishes the part
// that falls on the partner's rows in a double-buffered exchange area, adds
// the partner's part to its own rows and carries on with its half of the
// next vector.  Halves b and b ^ 8 of the grid land on the same XCD under the
// round-robin placement of workgroups.
// Each half uses the NPAIR = 16 partition of its own columns; the sum of the
// two halves' partials is commutative, so results do not depend on which
// half adds them, nor on the RHS tile size (RT <= 4; larger counts loop over
// tiles of 4).  Every wait is bounded (spin_limit) and stops at once after a
// sticky abort.
// ---------------------------------------------------------------------------
// elements per (unit, half) exchange slot: rows of the partner (<= 128 for
// bs <= 256) times the RHS tile (<= 4)
constexpr int kXSlot = 128 * 4;

template <typename T2, int RT, int ROWS>
__global__ __launch_bounds__(kCThreads) void k_solve_chain2(const SubDesc *__restrict__ subs,
                                                            const Coef *__restrict__ coef, const T2 *__restrict__ W,
                                                            const T2 *__restrict__ g, T2 *__restrict__ x, int nrhs,
                                                            long long etot, int dim, int nunits, int *mflags,
                                                            int *xflags, int *rflags, int *abort_flag, int spin_limit,
                                                            T2 *__restrict__ xbuf) {
    static_assert(RT <= 4, "exchange slots hold tiles of up to 4 RHS");
    extern __shared__ unsigned char lds_raw[];
    using LT = typename LaneT<T2, ROWS>::type;
    constexpr int NT = kCThreads;
    constexpr int kCBatch = ChainBatch2<T2, ROWS>::value;
    constexpr int NPAIR = kCWaves;  // one work pair per wave
    const int b = (int)blockIdx.x;
    const int half = (b >> 3) & 1;
    const int unit = (b & 7) | ((b >> 4) << 3);
    if (unit >= nunits) return;
    const int a = unit >> 1, chain = unit & 1;
    const SubDesc &s = subs[a];
    const int nb = s.nb, bs = s.bs, mid = s.mid, ax = dim - 1;
    const long long off = s.off;
    const int ld = s.ld;
    const int R = (bs + 64 * ROWS - 1) / (64 * ROWS);
    const int bh = ((bs + 3) / 4) * 2;               // even split point
    const int c0 = half ? bh : 0, c1 = half ? bs : bh;  // own columns = own result rows
    const int o0 = half ? 0 : bh, o1 = half ? bh : bs;  // the partner's rows
    const int ncol = c1 - c0;
    const int CG = NPAIR / R;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rt = wv % R, cg = wv / R;
    const bool gemv = cg < CG;  // groups past the last column still write zero partials
    const int row = (rt * 64 + lane) * ROWS;
    const bool rowok = gemv && row < bs;
    const int bsp = R * 64 * ROWS;
    T2 *vs = (T2 *)lds_raw;                  // [bsp][RT] current v (own columns used)
    T2 *red = vs + (size_t)bsp * RT;         // [CG][RT][bsp] partial sums
    constexpr int PF = kLdsCols2<T2, ROWS>::value;
    T2 *mypf = red + (size_t)CG * RT * bsp + (size_t)wv * PF * 64 * ROWS;
    const int nf = chain == 0 ? mid : nb - 1 - mid;
    const int nsteps = 2 * nf + 1;
    const int dirf = chain == 0 ? 1 : -1;
    const int lfirst = chain == 0 ? 0 : nb - 1;
    // this thread's element of the own rows and of the partner's rows
    const int eo = threadIdx.x, io = c0 + eo / RT, qo = eo % RT;
    const bool own_ok = eo < ncol * RT;
    const int ip = o0 + eo / RT;
    const bool part_ok = eo < (o1 - o0) * RT;
    int *myx = xflags + 2 * unit + half, *px = xflags + 2 * unit + (1 - half);
    int ep = 0;  // exchange epoch: block steps done in this launch

    for (int r0 = 0; r0 < nrhs; r0 += RT) {
        const int nr = nrhs - r0 < RT ? nrhs - r0 : RT;
        const int epoch = r0 / RT + 1;  // meeting epoch of this RHS tile
        if (nf > 0 && own_ok)
            vs[io * RT + qo] = qo < nr ? g[(long long)(r0 + qo) * etot + off + (long long)lfirst * bs + io] : czero<T2>();
        __syncthreads();
        auto step_l = [&](int t) {
            if (t < nf) return lfirst + dirf * t;
            if (t == nf) return mid;
            return mid - dirf * (t - nf);
        };
        const T2 *Wbase = W + s.foff + (long long)c0 * ld;  // own columns
        const long long bs2 = (long long)bs * ld;
        const int rowc = row < bs ? row : (bs - 1) / ROWS * ROWS;
        LT wb[kCBatch];
        {
            const T2 *Wl = Wbase + (long long)step_l(0) * bs2;
            lds_prefetch<T2, PF, ROWS>(Wl, mypf, cg, CG, ncol, ld, rowc, gemv);
#pragma unroll
            for (int u = 0; u < kCBatch; ++u) {
                const int j = cg + CG * (PF + u);
                wb[u] = (rowok && j < ncol) ? ld_w((const LT *)(Wl + (long long)j * ld + row)) : lane_zero<LT>();
            }
        }
        for (int t = 0; t < nsteps; ++t) {
            const int l = step_l(t);
            const int kind = t < nf ? 0 : (t == nf ? 1 : 2);
            if (t == nf) {
                // middle: v = g_mid - cm y_{mid-1} - cp y_{mid+1} on the own rows; the
                // other chain's same half wrote y_{mid+1} there
                const Coef cmid = coef[s.coff[ax] + mid];
                __builtin_amdgcn_s_waitcnt(0);  // this wave's stores of the last y block are complete
                __syncthreads();
                if (threadIdx.x == 0)
                    __hip_atomic_store(mflags + 4 * a + 2 * chain + half, epoch, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                wait_flag_relaxed(mflags + 4 * a + 2 * (1 - chain) + half, epoch, abort_flag, spin_limit);
                if (own_ok) {
                    double2 v = make_double2(0, 0);
                    if (qo < nr) {
                        const long long base = (long long)(r0 + qo) * etot + off;
                        v = to_d2(g[base + (long long)mid * bs + io]);
                        if (mid > 0) v = cmsub_fixed(v, cmid.cm, to_d2(xload(x + base + (long long)(mid - 1) * bs + io)));
                        if (mid < nb - 1)
                            v = cmsub_fixed(v, cmid.cp, to_d2(xload(x + base + (long long)(mid + 1) * bs + io)));
                    }
                    vs[io * RT + qo] = from_d2<T2>(v);
                }
                __syncthreads();
                // the reads of the other chain's last y block have returned:
                // its first backward step may overwrite that block now
                if (threadIdx.x == 0)
                    __hip_atomic_store(rflags + 4 * a + 2 * chain + half, epoch, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            const int tn = t + 1;
            const int lnv = tn < nsteps && tn != nf ? step_l(tn) : -1;
            T2 pre = czero<T2>();
            if (own_ok && qo < nr) {
                const long long base = (long long)(r0 + qo) * etot + off;
                if (kind == 2)  // the first backward block is the atomically stored one
                    pre = t == nf + 1 ? xload(x + base + (long long)l * bs + io) : x[base + (long long)l * bs + io];
                else if (kind == 0 && lnv >= 0) pre = g[base + (long long)lnv * bs + io];
            }
            // ---- GEMV over the own columns: one work pair per wave ----
            const int lnext = t + 1 < nsteps ? step_l(t + 1) : -1;
            if (gemv) {
                T2 acc[ROWS][RT];
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
#pragma unroll
                    for (int q = 0; q < RT; ++q) acc[r][q] = czero<T2>();
                const int kmax = (ncol - cg + CG - 1) / CG;
                const T2 *vc = vs + (size_t)c0 * RT;
                if constexpr (PF > 0) {
                    __builtin_amdgcn_s_waitcnt(kWaitVm0);
#pragma unroll 1
                    for (int u = 0; u < PF; ++u) {
                        if (u < kmax) {
                            const int j = cg + CG * u;
                            const LT w = ((const LT *)mypf)[u * 64 + lane];
#pragma unroll
                            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                                for (int q = 0; q < RT; ++q) cfma(acc[r][q], lane_row(w, r), vc[j * RT + q]);
                        }
                    }
                }
                for (int k0 = PF; k0 < kmax; k0 += kCBatch) {
                    const bool more = k0 + kCBatch < kmax;
                    const int ln = more ? l : lnext;
                    const int kn = more ? k0 + kCBatch : PF;
                    LT wn[kCBatch];
                    const T2 *Wn = Wbase + (long long)(ln >= 0 ? ln : 0) * bs2;
#pragma unroll
                    for (int u = 0; u < kCBatch; ++u) {
                        const int j = cg + CG * (kn + u);
                        wn[u] = (ln >= 0 && rowok && j < ncol) ? ld_w((const LT *)(Wn + (long long)j * ld + row))
                                                               : lane_zero<LT>();
                    }
#pragma unroll
                    for (int u = 0; u < kCBatch; ++u) {
                        const int j = cg + CG * (k0 + u);
                        if (j < ncol) {
#pragma unroll
                            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                                for (int q = 0; q < RT; ++q) cfma(acc[r][q], lane_row(wb[u], r), vc[j * RT + q]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kCBatch; ++u) wb[u] = wn[u];
                }
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
#pragma unroll
                    for (int q = 0; q < RT; ++q) red[((size_t)cg * RT + q) * bsp + row + r] = acc[r][q];
            }
            if (lnext >= 0) lds_prefetch<T2, PF, ROWS>(Wbase + (long long)lnext * bs2, mypf, cg, CG, ncol, ld, rowc, gemv);
            __syncthreads();
            // ---- publish the partner's rows of this half's partial product ----
            ++ep;
            T2 *slot = xbuf + ((size_t)(ep & 1) * nunits * 2 + (size_t)unit * 2) * kXSlot;
            if (part_ok) {
                const int q = eo % RT;
                T2 sum = red[(size_t)q * bsp + ip];
                for (int c = 1; c < CG; ++c) {
                    const T2 o = red[((size_t)c * RT + q) * bsp + ip];
                    sum.x += o.x;
                    sum.y += o.y;
                }
                xstore(slot + (size_t)half * kXSlot + eo, sum);
            }
            __builtin_amdgcn_s_waitcnt(0);  // this wave's exchange stores are complete
            __syncthreads();
            if (threadIdx.x == 0) __hip_atomic_store(myx, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            T2 own = czero<T2>();
            if (own_ok) {
                own = red[(size_t)qo * bsp + io];
                for (int c = 1; c < CG; ++c) {
                    const T2 o = red[((size_t)c * RT + qo) * bsp + io];
                    own.x += o.x;
                    own.y += o.y;
                }
            }
            wait_flag_relaxed(px, ep, abort_flag, spin_limit);
            // the first backward step overwrites the y block that the other
            // chain's same half read at the middle: wait for its reads
            if (t == nf + 1) wait_flag_relaxed(rflags + 4 * a + 2 * (1 - chain) + half, epoch, abort_flag, spin_limit);
            if (own_ok) {
                const T2 o = xload(slot + (size_t)(1 - half) * kXSlot + eo);
                T2 sum = own;
                sum.x += o.x;
                sum.y += o.y;
                const long long base = (long long)(r0 + qo) * etot + off;
                T2 res = sum;
                if (kind == 2) {
                    res.x = pre.x - sum.x;
                    res.y = pre.y - sum.y;
                }
                if (qo < nr && (kind != 1 || chain == 0)) {
                    if (t == nf - 1) xstore(x + base + (long long)l * bs + io, res);  // read at the middle
                    else x[base + (long long)l * bs + io] = res;
                }
                if (lnv >= 0) {
                    double2 v;
                    const Coef cn = coef[s.coff[ax] + lnv];
                    if (kind == 0) {
                        const double2 c = chain == 0 ? cn.cm : cn.cp;
                        v = qo < nr ? cmsub_fixed(to_d2(pre), c, to_d2(res)) : make_double2(0, 0);
                    } else {
                        const double2 c = chain == 0 ? cn.cp : cn.cm;
                        v = qo < nr ? cmul_fixed(c, to_d2(res)) : make_double2(0, 0);
                    }
                    vs[io * RT + qo] = from_d2<T2>(v);
                }
            }
            __syncthreads();
        }
    }
}

template <typename T2, int RT>
static hipError_t run_sweeps(ddm_handle *h, const T2 *g, T2 *x, int nrhs) {
    const Plan &P = h->plan;
    const int nitems = (int)P.items.size();
    const double es = sizeof(T2);
    for (int l = 0; l < P.nb_max; ++l) {
        // algorithmic bytes: W_l once, g_l and z_{l-1} read, z_l written
        ProfScope ps(h, DDM_K_SUBST, es * (P.w_el_by_l[l] + 3.0 * nrhs * P.v_el_by_l[l]));
        k_solve_line<T2, RT, false><<<nitems, kSThreads, 0, h->stream>>>(h->d_subs, h->d_items, h->d_coef,
                                                                           (const T2 *)h->d_W, g, x, l, nrhs, P.etot,
                                                                           P.dim);
    }
    for (int t = 0; t + 1 < P.nb_max; ++t) {
        // lines l = nb - 2 - t of every subdomain: W_l once, x_{l+1} and z_l read, x_l written
        double wb = 0.0, vb = 0.0;
        for (const SubDesc &sd : P.subs) {
            int l = sd.nb - 2 - t;
            if (l >= 0) { wb += (double)sd.bs * sd.bs; vb += sd.bs; }
        }
        ProfScope ps(h, DDM_K_SUBST, es * (wb + 3.0 * nrhs * vb));
        k_solve_line<T2, RT, true><<<nitems, kSThreads, 0, h->stream>>>(h->d_subs, h->d_items, h->d_coef,
                                                                          (const T2 *)h->d_W, g, x, t, nrhs, P.etot,
                                                                          P.dim);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t run_perline(ddm_handle *h, const T *g, T *x, int nrhs) {
    if (nrhs <= 1) return run_sweeps<T, 1>(h, g, x, nrhs);
    if (nrhs <= 2) return run_sweeps<T, 2>(h, g, x, nrhs);
    if (nrhs <= 4) return run_sweeps<T, 4>(h, g, x, nrhs);
    return run_sweeps<T, 8>(h, g, x, nrhs);
}

// dynamic LDS of the chain kernel: v, the column groups' partial sums and
// the per-wave LDS column copies
template <typename T2, int RT, int ROWS, int NT, int NPAIR = kCWaves>
static size_t chain_lds(int bs_max) {
    const int R = (bs_max + 64 * ROWS - 1) / (64 * ROWS);
    constexpr bool SEQ = RT >= 16 && NT == kCThreads;
    const int CG = SEQ ? 1 : NPAIR / R;  // partial-sum buffers
    const int PF = NT == kCThreads && !SEQ ? kLdsCols<T2, ROWS>::value : 0;
    return (size_t)R * 64 * ROWS * RT * (1 + CG) * sizeof(T2) + (size_t)(NT / 64) * PF * 64 * ROWS * sizeof(T2);
}

template <typename T2, int RT, int ROWS, int NT = kCThreads, int NPAIR = kCWaves>
static hipError_t run_chain(ddm_handle *h, const T2 *g, T2 *x, int nrhs) {
    const Plan &P = h->plan;
    const double es = sizeof(T2);
    double vb = 0.0;
    for (const SubDesc &sd : P.subs) vb += (double)sd.nloc;
    const int ntile = (nrhs + RT - 1) / RT;
    // W read once per sweep and RHS tile; block vectors: g read, y written,
    // y read back and x written
    ProfScope ps(h, DDM_K_SUBST, es * (2.0 * (double)P.fel * ntile + 4.0 * nrhs * vb));
    const int R = (P.bs_max + 64 * ROWS - 1) / (64 * ROWS);
    const size_t lds = chain_lds<T2, RT, ROWS, NT, NPAIR>(P.bs_max);
    hipError_t e = hipFuncSetAttribute((const void *)k_solve_chain<T2, RT, ROWS, NT, NPAIR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (P.twisted) {
        // meeting flags and read-done flags (4 nsub) start at zero
        e = launch_fill_zero(h->d_sync, (long long)(4 * P.nsub) * sizeof(int), h->stream);
        if (e != hipSuccess) return e;
        const SubDesc *a0 = h->d_subs;
        const Coef *a1 = h->d_coef;
        const T2 *a2 = (const T2 *)h->d_W;
        const T2 *a3 = g;
        T2 *a4 = x;
        int a5 = nrhs;
        long long a6 = P.etot;
        int a7 = P.dim, a8 = 1;
        int *a9 = h->d_sync, *a9r = h->d_sync + 2 * P.nsub, *a10 = abort_flag_ptr(h);
        int a11 = h->spin_limit;
        void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7, &a8, &a9, &a9r, &a10, &a11};
        // the two chains of a subdomain meet once: they must be co-resident
        return hipLaunchCooperativeKernel((const void *)k_solve_chain<T2, RT, ROWS, NT, NPAIR>, dim3(2 * P.nsub), dim3(NT),
                                          args, lds, h->stream);
    }
    k_solve_chain<T2, RT, ROWS, NT, NPAIR><<<P.nsub, NT, lds, h->stream>>>(h->d_subs, h->d_coef, (const T2 *)h->d_W, g, x,
                                                                 nrhs, P.etot, P.dim, 0, h->d_sync,
                                                                 h->d_sync + 2 * P.nsub, abort_flag_ptr(h),
                                                                 h->spin_limit);
    return hipGetLastError();
}

template <typename T>
static hipError_t run_chain_rt(ddm_handle *h, const T *g, T *x, int nrhs) {
    const bool coop_ok = !h->plan.twisted || 2 * h->plan.nsub <= h->plan.ncu;
    // a forced RHS tile (ddm_set_chain_tile) for batches of more than 4 RHS
    if (nrhs > 4 && h->chain_tile == 4) {
        if constexpr (sizeof(T) == sizeof(double2)) return run_chain<T, 4, 1>(h, g, x, nrhs);
        else return run_chain<T, 4, 2>(h, g, x, nrhs);
    }
    if (nrhs > 4 && h->chain_tile == 8 && coop_ok) {
        if constexpr (sizeof(T) == sizeof(double2)) {
            if (chain_lds<T, 8, 1, 512>(h->plan.bs_max) <= kLdsMax) return run_chain<T, 8, 1, 512>(h, g, x, nrhs);
        } else {
            return run_chain<T, 8, 1>(h, g, x, nrhs);
        }
    }
    if constexpr (sizeof(T) == sizeof(double2)) {
        if (nrhs <= 1) return run_chain<T, 1, 1>(h, g, x, nrhs);
        if (nrhs <= 2) return run_chain<T, 2, 1>(h, g, x, nrhs);
        if (nrhs <= 4) return run_chain<T, 4, 1>(h, g, x, nrhs);
        // more RHS: 8-RHS tiles on 512-thread workgroups (256 VGPRs per lane);
        // a twisted launch needs every workgroup resident (one per CU here).
        // Batches of 16 or more take 16-RHS tiles, which stream each inverse
        // once per 16 RHS: on 1024-thread workgroups with the 16-pair
        // partition and the column groups' partial sums added in order (the
        // same bits as every smaller tile), else on 512-thread workgroups with
        // 8 pairs (fewer waves; rounding differs from smaller batches)
        if (coop_ok && nrhs >= 16 && chain_lds<T, 16, 1, kCThreads>(h->plan.bs_max) <= kLdsMax)
            return run_chain<T, 16, 1>(h, g, x, nrhs);
        if (coop_ok && nrhs >= 16 && chain_lds<T, 16, 1, 512, 8>(h->plan.bs_max) <= kLdsMax)
            return run_chain<T, 16, 1, 512, 8>(h, g, x, nrhs);
        if (coop_ok && chain_lds<T, 8, 1, 512>(h->plan.bs_max) <= kLdsMax) return run_chain<T, 8, 1, 512>(h, g, x, nrhs);
        return run_chain<T, 4, 1>(h, g, x, nrhs);
    } else {
        if (nrhs <= 1) return run_chain<T, 1, 2>(h, g, x, nrhs);
        if (nrhs <= 2) return run_chain<T, 2, 2>(h, g, x, nrhs);
        if (nrhs <= 4) return run_chain<T, 4, 2>(h, g, x, nrhs);
        if (nrhs <= 8) return run_chain<T, 8, 1>(h, g, x, nrhs);
        // 16 RHS with 16-byte loads needs the 256-VGPR budget of 512-thread
        // workgroups (and 8 work pairs to fit the partial sums in LDS)
        if (coop_ok && chain_lds<T, 16, 2, 512, 8>(h->plan.bs_max) <= kLdsMax)
            return run_chain<T, 16, 2, 512, 8>(h, g, x, nrhs);
        return run_chain<T, 16, 1>(h, g, x, nrhs);
    }
}

// grid of the split substitution: 2 halves x 2 chains per subdomain, units
// padded to a multiple of 8 so that halves b and b ^ 8 share an XCD
static int chain2_grid(const Plan &P) { return ((2 * P.nsub + 7) / 8) * 16; }

size_t chain2_xbuf_bytes(const Plan &P) {
    return (size_t)2 * (2 * P.nsub) * 2 * kXSlot * sizeof(double2);
}

template <typename T2, int RT, int ROWS>
static size_t chain2_lds(int bs_max) {
    const int R = (bs_max + 64 * ROWS - 1) / (64 * ROWS);
    const int CG = kCWaves / R;
    return (size_t)R * 64 * ROWS * RT * (1 + CG) * sizeof(T2) +
           (size_t)kCWaves * kLdsCols2<T2, ROWS>::value * 64 * ROWS * sizeof(T2);
}

template <typename T2, int RT, int ROWS>
static hipError_t run_chain2(ddm_handle *h, const T2 *g, T2 *x, int nrhs) {
    const Plan &P = h->plan;
    const double es = sizeof(T2);
    double vb = 0.0;
    for (const SubDesc &sd : P.subs) vb += (double)sd.nloc;
    const int ntile = (nrhs + RT - 1) / RT;
    ProfScope ps(h, DDM_K_SUBST, es * (2.0 * (double)P.fel * ntile + 4.0 * nrhs * vb));
    const size_t lds = chain2_lds<T2, RT, ROWS>(P.bs_max);
    hipError_t e = hipFuncSetAttribute((const void *)k_solve_chain2<T2, RT, ROWS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // meeting flags [4 nsub], exchange flags [4 nsub] and read-done flags
    // [4 nsub] start at zero
    e = launch_fill_zero(h->d_sync2, (long long)(12 * P.nsub) * sizeof(int), h->stream);
    if (e != hipSuccess) return e;
    const SubDesc *a0 = h->d_subs;
    const Coef *a1 = h->d_coef;
    const T2 *a2 = (const T2 *)h->d_W;
    const T2 *a3 = g;
    T2 *a4 = x;
    int a5 = nrhs;
    long long a6 = P.etot;
    int a7 = P.dim, a8 = 2 * P.nsub;
    int *a9 = h->d_sync2, *a10 = h->d_sync2 + 4 * P.nsub, *a10r = h->d_sync2 + 8 * P.nsub;
    int *a11 = abort_flag_ptr(h);
    int a12 = h->spin_limit;
    T2 *a13 = (T2 *)h->d_xbuf;
    void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7, &a8, &a9, &a10, &a10r, &a11, &a12, &a13};
    // the halves and chains of a subdomain wait on each other: all co-resident
    return hipLaunchCooperativeKernel((const void *)k_solve_chain2<T2, RT, ROWS>, dim3(chain2_grid(P)),
                                      dim3(kCThreads), args, lds, h->stream);
}

template <typename T>
static hipError_t run_chain2_rt(ddm_handle *h, const T *g, T *x, int nrhs) {
    constexpr int ROWS = sizeof(T) == sizeof(double2) ? 1 : 2;
    if (nrhs <= 1) return run_chain2<T, 1, ROWS>(h, g, x, nrhs);
    if (nrhs <= 2) return run_chain2<T, 2, ROWS>(h, g, x, nrhs);
    return run_chain2<T, 4, ROWS>(h, g, x, nrhs);
}

// the split substitution fits this plan's blocks and subdomain count (it
// also needs the two-ended layout)
bool chain2_fits(const Plan &P) {
    return P.bs_max <= 256 && chain2_grid(P) <= P.ncu && chain2_lds<double2, 4, 1>(P.bs_max) <= kLdsMax &&
           chain2_lds<float2, 4, 2>(P.bs_max) <= kLdsMax;
}

bool solve_variant_ok(const Plan &P, int variant) {
    switch (variant) {
        case kSolvePerLine: return !P.twisted;
        case kSolveChain: return P.bs_max <= 256;
        case kSolveChain2: return P.twisted && chain2_fits(P);  // one workgroup per CU
        case kSolveMma: return mma_fits(P);
        default: return false;
    }
}

// g and x must not alias (the substitution reads g_l while x_l is written).
template <typename T>
hipError_t launch_local_solve(ddm_handle *h, const T *g, T *x, int nrhs) {
    // the stored inverses are in the matrix-core order exactly when that
    // variant is selected
    if (h->plan.mma) return run_mma<T>(h, g, x, nrhs);
    int v = h->solve_variant;
    if (!solve_variant_ok(h->plan, v)) v = solve_variant_ok(h->plan, kSolveChain) ? kSolveChain : kSolvePerLine;
    if (v == kSolveChain2 && h->d_xbuf) return run_chain2_rt<T>(h, g, x, nrhs);
    if (v == kSolveChain || v == kSolveChain2) return run_chain_rt<T>(h, g, x, nrhs);
    return run_perline<T>(h, g, x, nrhs);
}

template hipError_t launch_local_solve<double2>(ddm_handle *, const double2 *, double2 *, int);
template hipError_t launch_local_solve<float2>(ddm_handle *, const float2 *, float2 *, int);

}  // namespace ddm
