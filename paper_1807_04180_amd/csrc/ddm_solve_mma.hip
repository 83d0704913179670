// Matrix-core block substitution for tiles of 16 right-hand sides: the
// local solves of every step of Algorithm 3.1 (the same recurrence as the
// chain kernels of ddm_solve.hip),
//   forward:  y_l = W_l (g_l - c y_{l-1}),   backward: x_l = y_l - W_l (c' x_{l+1}),
// with every product W_l V (V: bs x 16 complex) on MFMA.
//
// Complex products in real form.  One 16x16x4 MFMA (f32 for complex64, f64
// for complex128) takes two complex columns j, j+1 of W_l as its K = 4
// (k = 2 jj + c: column j + jj, real part c = 0 / imaginary part c = 1) and 8
// right-hand sides as its N = 16 (n = 2 q + p: RHS q, output part p):
//   A[i][k] = (c == 0 ? Re : Im) W[i][j + jj],
//   B[k][n] = (p ^ c == 0 ? Re : Im) V[j + jj][q], negated for (c, p) = (1, 0),
// so D[i][2q] = Re (W V)[i][q] and D[i][2q+1] = Im (W V)[i][q]: four real
// products per complex product, nothing wasted.  Two accumulators take the
// two halves of the 16 RHS.
//
// Work split: one workgroup per elimination chain (one per subdomain, or two
// for the two-ended layout, which then meet at the middle block exactly as
// in k_solve_chain), one wave per 16-row tile of the block, each wave over all
// columns: no partial sums cross waves, one barrier per block.  The block
// vector V lives in LDS (double-buffered, [column][16 RHS] complex); the wave
// forms its rows of the next V from its accumulators.
//
// Inverse storage (written by the factorisation in this order): per block,
// row tile t (16 rows, the last one ragged with r_t rows), column group G
// (CPG columns), lane (k, i) at position k r_t + i: 16 bytes holding the A
// operand of the S = CPG / 2 consecutive MFMAs of the group.  A wave's loads
// are whole 1 KB (r_t = 16) runs; the ragged tile is stored compactly, so no
// padding rows are read; columns are padded to a whole group (zeros).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cplx.h"
#include "ddm_internal.h"
#include "ddm_mma.h"
#include "ddm_sync.h"

namespace ddm {

// NTB: the largest workgroup the instance is launched with (64 threads per
// row tile of the largest block); fewer threads leave more registers
template <typename T2, int NTB>
__global__ __launch_bounds__(NTB) void k_solve_mma(const SubDesc *__restrict__ subs, const Coef *__restrict__ coef,
                                                    const T2 *__restrict__ W, const T2 *__restrict__ g,
                                                    T2 *__restrict__ x, int nrhs, long long etot, int dim,
                                                    int twisted, int vcap, int *flags, int *rflags, int *abort_flag,
                                                    int spin_limit, int fstride) {
    using M = Mma<T2>;
    using R = typename M::R;
    using LT = typename M::LT;
    using Acc = typename M::Acc;
    extern __shared__ unsigned char lds_raw[];
    T2 *vbuf = (T2 *)lds_raw;  // 2 x [vcap][16]
    const int a = twisted ? (int)(blockIdx.x >> 1) : (int)blockIdx.x;
    const int chain = twisted ? (int)(blockIdx.x & 1) : 0;
    const SubDesc &s = subs[a];
    const int nb = s.nb, bs = s.bs, mid = s.mid, ax = dim - 1, mpad = s.mpad;
    const long long off = s.off;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NG = mpad / M::CPG;                                   // column groups
    const int NGP = (NG + kMmaRing - 1) / kMmaRing * kMmaRing;      // padded to whole ring turns
    const int ntile = (bs + 15) >> 4;
    const bool active = wv < ntile;                                 // this wave has rows
    const int rows_t = active ? (bs - 16 * wv < 16 ? bs - 16 * wv : 16) : 0;
    const int li = lane & 15, lk = lane >> 4;
    const long long bstr_b = (long long)bs * mpad * sizeof(T2);
    // Every operand load is issued unconditionally (out of range: a clamped,
    // valid address whose value is not used), so the loads in flight are a
    // fixed count and each use waits only for its own load.  Lanes past the
    // ragged tile's rows read the tile's last row (same addresses as a
    // valid lane); waves without rows read the subdomain's first bytes.
    const int lic = li < rows_t ? li : rows_t - 1;
    const char *Wt = (const char *)(W + s.foff) +
                     (active ? (long long)wv * 16 * mpad * sizeof(T2) + (long long)(lk * rows_t + lic) * 16 : 0);
    const int grp_b = rows_t * 64;
    // B operand of this lane: component p ^ c of V[j + jj][q], sign - for (c, p) = (1, 0)
    const int qq = (lane & 15) >> 1, p = lane & 1, jj = lk >> 1, c = lk & 1;
    const R sgn = (c == 1 && p == 0) ? R(-1) : R(1);
    const int boff = (jj * kMmaRhs + qq) * 2 + (p ^ c);              // in R units
    const int nf = chain == 0 ? mid : nb - 1 - mid;
    const int nsteps = 2 * nf + 1;
    const int dirf = chain == 0 ? 1 : -1;
    const int lfirst = chain == 0 ? 0 : nb - 1;
    auto step_l = [&](int t) {
        if (t < nf) return lfirst + dirf * t;
        if (t == nf) return mid;
        return mid - dirf * (t - nf);
    };
    // the block whose V step t forms (none at the last step, nor before the
    // two-ended meeting, which forms its own)
    auto lnv_of = [&](int t) { return (t + 1 < nsteps && !(twisted && t + 1 == nf)) ? step_l(t + 1) : -1; };

    // both V buffers start at zero: the padding columns [bs, mpad) stay zero
    for (int e = threadIdx.x; e < 2 * vcap * kMmaRhs; e += blockDim.x) vbuf[e] = czero<T2>();

    // RHS tiles blockIdx.y, blockIdx.y + gridDim.y, ...: the workgroups of a
    // grid row share nothing with other rows; each row has its own meeting
    // and read-done flags (fstride apart)
    flags += (size_t)blockIdx.y * fstride;
    rflags += (size_t)blockIdx.y * fstride;
    int epoch = 0;  // meeting flags count this row's tiles (never reset inside the launch)
    for (int r0 = (int)blockIdx.y * kMmaRhs; r0 < nrhs; r0 += (int)gridDim.y * kMmaRhs) {
        const int nr = nrhs - r0 < kMmaRhs ? nrhs - r0 : kMmaRhs;
        ++epoch;
        __syncthreads();  // the previous tile's readers of buffer 0 are done
        for (int e = threadIdx.x; e < bs * kMmaRhs; e += blockDim.x) {
            const int i = e >> 4, q = e & 15;
            vbuf[e] = q < nr ? g[(long long)(r0 + q) * etot + off + (long long)lfirst * bs + i] : czero<T2>();
        }
        __syncthreads();
        LT ring[kMmaRing];
        {
            const char *b0 = Wt + (long long)step_l(0) * bstr_b;
#pragma unroll
            for (int u = 0; u < kMmaRing; ++u) ring[u] = M::load_op(b0 + (long long)(u < NG ? u : NG - 1) * grp_b);
        }

        // per lane and half: the g_lnv (forward) or y_l (backward) entries
        // of step st_ that store_half moves for this lane (whole entries, the
        // same loads whatever the step: rows and RHS clamped, the values
        // dropped where unused), turned into part p of the lane's 4 rows by
        // M::pre_parts where they are used.  The y block of the first
        // backward step of the two-ended layout was stored by this lane pair
        // with atomic stores at the last forward step and has not been read
        // through this CU's cache since: a plain load returns it.
        typename M::PT pre[2][M::NPL];
        unsigned pok = 0;  // bit 4 hf + r: entry (hf, r) used (applied where it is read, so the
                           // loads are not waited for where they are issued)
#define DDM_MMA_PRE(st_)                                                                                  \
    {                                                                                                     \
        const int kd = (st_) < nf ? 0 : ((st_) == nf ? 1 : 2), lp = step_l(st_), ln = lnv_of(st_);        \
        const T2 *psrc = (kd == 2 ? x + (long long)lp * bs : g + (long long)(ln >= 0 ? ln : lp) * bs) + off; \
        const bool puse = kd == 2 || (kd == 0 && ln >= 0);                                                \
        _Pragma("unroll") for (int hf = 0; hf < 2; ++hf) {                                                \
            const int q = 8 * hf + qq, qc = q < nr ? q : nr - 1;                                          \
            M::pre_load(pre[hf], psrc + (long long)(r0 + qc) * etot, bs, 16 * wv, lane);                  \
            _Pragma("unroll") for (int r = 0; r < 4; ++r) {                                               \
                const int i = 16 * wv + M::row(lane, r);                                                  \
                const bool ok = puse && active && i < bs && q < nr;                                       \
                pok = ok ? pok | (1u << (4 * hf + r)) : pok & ~(1u << (4 * hf + r));                      \
            }                                                                                             \
        }                                                                                                 \
    }
        DDM_MMA_PRE(0)

        for (int st = 0; st < nsteps; ++st) {
            const int l = step_l(st);
            const int kind = st < nf ? 0 : (st == nf ? 1 : 2);  // forward, middle, backward
            T2 *vcur = vbuf + (size_t)(st & 1) * vcap * kMmaRhs;
            T2 *vnext = vbuf + (size_t)((st + 1) & 1) * vcap * kMmaRhs;
            if (twisted && st == nf) {
                // middle block: V = g_mid - cm y_{mid-1} - cp y_{mid+1}, the two
                // y blocks stored by the two chains with relaxed agent-scope
                // atomics; each chain publishes its own, then waits for the other
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (threadIdx.x == 0)
                    __hip_atomic_store(flags + 2 * a + chain, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                wait_flag_relaxed(flags + 2 * a + (1 - chain), epoch, abort_flag, spin_limit);
                const Coef cmid = coef[s.coff[ax] + mid];
                for (int e = threadIdx.x; e < bs * kMmaRhs; e += blockDim.x) {
                    const int i = e >> 4, q = e & 15;
                    double2 v = make_double2(0, 0);
                    if (q < nr) {
                        const long long base = (long long)(r0 + q) * etot + off;
                        v = to_d2(g[base + (long long)mid * bs + i]);
                        if (mid > 0) v = cmsub_fixed(v, cmid.cm, to_d2(xload(x + base + (long long)(mid - 1) * bs + i)));
                        if (mid < nb - 1)
                            v = cmsub_fixed(v, cmid.cp, to_d2(xload(x + base + (long long)(mid + 1) * bs + i)));
                    }
                    vcur[e] = from_d2<T2>(v);
                }
                __syncthreads();
                // every read of the partner's y block has returned: it may now
                // overwrite that block with its first backward result
                if (threadIdx.x == 0)
                    __hip_atomic_store(rflags + 2 * a + chain, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // the block index whose V this step forms (none before the
            // two-ended meeting, which forms its own)
            const int lnv = lnv_of(st);
            // ---- D = W_l V on the matrix cores ----
            Acc acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
            const R *vb = (const R *)vcur + boff;
            const char *cur_b = Wt + (long long)l * bstr_b;
            const char *nxt_b = Wt + (long long)(st + 1 < nsteps ? step_l(st + 1) : l) * bstr_b;
            // Full wait: the g / y entries of this step (loaded at the end of
            // the previous one, before the barrier) are in, and the first
            // ring turn, loaded before them, too.  It also lets the
            // compiler's counter analysis wait for one ring load per slot
            // (7 left in flight); without it the analysis carries an unknown
            // older load into the loop and waits for all eight at every turn.
            __builtin_amdgcn_s_waitcnt(0);
            for (int jb = 0; jb < NGP; jb += kMmaRing) {
                // the loads of this turn: groups jb + 8 .. of this block, or
                // the next block's first groups after this block's last turn
                const bool here = jb + kMmaRing < NGP;
                const char *rb = here ? cur_b : nxt_b;
                const int g0 = here ? jb + kMmaRing : 0;
#pragma unroll
                for (int u = 0; u < kMmaRing; ++u) {
                    const int G = jb + u;
                    const LT A = ring[u];
                    if (G < NG && active) {
#pragma unroll
                        for (int s_ = 0; s_ < M::S; ++s_) {
                            const R av = M::part(A, s_);
                            const R *bp = vb + (G * M::CPG + 2 * s_) * kMmaRhs * 2;
                            acc0 = M::mfma(av, sgn * bp[0], acc0);
                            acc1 = M::mfma(av, sgn * bp[16], acc1);
                        }
                    }
                    // refill this ring slot with the item kMmaRing ahead
                    const int gi = g0 + u < NG ? g0 + u : NG - 1;
                    ring[u] = M::load_op(rb + (long long)gi * grp_b);
                }
            }
            // the first backward step overwrites the y block the partner read
            // at the middle: wait until the partner has finished reading it
            if (twisted && st == nf + 1) wait_flag_relaxed(rflags + 2 * a + (1 - chain), epoch, abort_flag, spin_limit);
            // ---- results and the next V ----
            const Coef cn = coef[s.coff[ax] + (lnv >= 0 ? lnv : l)];
            const double2 cf = kind == 0 ? (chain == 0 ? cn.cm : cn.cp) : (chain == 0 ? cn.cp : cn.cm);
            // the block's results go out through store_half, whole entries
            // per lane (results stored by one part per lane took 21% of an
            // FP64 launch and 14% of a complex64 one); the last forward block
            // of the two-ended layout (read by the partner at the middle)
            // goes out here, one part per lane with atomic stores, and the
            // first backward step reads it back in the same lane pairs
            const bool store = kind != 1 || chain == 0;  // the middle block's x: chain 0 stores it
            const bool xchg = twisted && st == nf - 1;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                R resv[4], othv[4], pvv[4];
                M::pre_parts(pvv, pre[hf], bs, 16 * wv, lane);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * wv + M::row(lane, r), q = 8 * hf + qq;
                    const R y = hf == 0 ? acc0[r] : acc1[r];
                    const R pv = (pok >> (4 * hf + r)) & 1u ? pvv[r] : R(0);
                    const R res = kind == 2 ? pv - y : y;  // forward y_l, middle x_mid, backward x_l
                    const R oth = shfl_xor1(res);                  // the other part of the same entry
                    resv[r] = res;
                    othv[r] = oth;
                    if (!(active && i < bs)) continue;
                    const double re = p ? (double)oth : (double)res, im = p ? (double)res : (double)oth;
                    if (xchg && store && q < nr)
                        xstore_r((R *)(x + (long long)(r0 + q) * etot + off + (long long)l * bs + i) + p, res);
                    if (lnv >= 0) {
                        double v = 0.0;
                        if (q < nr) {
                            if (kind == 0) {  // g_lnv - cf y_l, rounded as cmsub_fixed
                                const double gp = (double)pv;
                                v = p ? fma(-cf.x, im, fma(-cf.y, re, gp)) : fma(-cf.x, re, fma(cf.y, im, gp));
                            } else {          // cf x_l, rounded as cmul_fixed
                                v = p ? fma(cf.x, im, cf.y * re) : fma(cf.x, re, -(cf.y * im));
                            }
                        }
                        ((R *)(vnext + i * kMmaRhs + q))[p] = (R)v;
                    }
                }
                if (store && !xchg && active)
                    M::store_half(x + (long long)(r0 + 8 * hf) * etot + off + (long long)l * bs + 16 * wv, etot,
                                  bs - 16 * wv, nr - 8 * hf, lane, resv, othv);
            }
            // the next step's g / y entries, in flight over the barrier
            if (st + 1 < nsteps) DDM_MMA_PRE(st + 1)
            __syncthreads();
        }
#undef DDM_MMA_PRE
    }
}

size_t mma_lds_bytes(const Plan &P, size_t es) { return (size_t)2 * P.mpad_max * kMmaRhs * es; }

bool mma_fits(const Plan &P) {
    return P.bs_max <= kMmaMaxBs && P.mpad_max > 0 && mma_lds_bytes(P, sizeof(double2)) <= 160 * 1024 &&
           (!P.twisted || 2 * P.nsub <= P.ncu);
}

template <typename T2>
hipError_t run_mma(ddm_handle *h, const T2 *g, T2 *x, int nrhs) {
    const Plan &P = h->plan;
    const double es = sizeof(T2);
    double vb = 0.0, wb = 0.0;
    for (const SubDesc &sd : P.subs) {
        vb += (double)sd.nloc;
        wb += (double)sd.nb * sd.bs * sd.bs;
    }
    const int ntile = (nrhs + kMmaRhs - 1) / kMmaRhs;
    // algorithmic bytes: every inverse (unpadded) once per sweep and RHS tile;
    // block vectors: g read, y written, y read back and x written
    ProfScope ps(h, DDM_K_SUBST, es * (2.0 * wb * ntile + 4.0 * nrhs * vb));
    const size_t lds = mma_lds_bytes(P, sizeof(T2));
    const int nt = 64 * ((P.bs_max + 15) / 16);
    const void *kern = nt <= 512   ? (const void *)k_solve_mma<T2, 512>
                       : nt <= 768 ? (const void *)k_solve_mma<T2, 768>
                                   : (const void *)k_solve_mma<T2, 1024>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const SubDesc *a0 = h->d_subs;
    const Coef *a1 = h->d_coef;
    const T2 *a2 = (const T2 *)h->d_W;
    const T2 *a3 = g;
    T2 *a4 = x;
    int a5 = nrhs;
    long long a6 = P.etot;
    int a7 = P.dim, a8 = P.twisted ? 1 : 0, a9 = P.mpad_max;
    int *a10 = h->d_sync, *a11 = h->d_sync + 2 * P.nsub, *a12 = abort_flag_ptr(h);
    int a13 = h->spin_limit, a14 = 4 * P.nsub;
    // RHS tiles side by side (grid rows): as many as there are tiles, flags
    // for and, in the two-ended layout, room to keep every workgroup
    // co-resident (one per CU); a row takes the tiles beyond them in turn
    int rows = std::min(ntile, h->sync_tiles);
    if (P.twisted) rows = std::max(1, std::min(rows, P.ncu / (2 * P.nsub)));
    if (P.twisted) {
        // meeting flags and read-done flags (4 nsub per row) start at zero
        e = launch_fill_zero(h->d_sync, (long long)(4 * P.nsub) * rows * sizeof(int), h->stream);
        if (e != hipSuccess) return e;
        void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7, &a8, &a9, &a10, &a11, &a12, &a13, &a14};
        // the two chains of a subdomain meet once: they must be co-resident
        return hipLaunchCooperativeKernel(kern, dim3(2 * P.nsub, rows), dim3(nt), args, lds, h->stream);
    }
    void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7, &a8, &a9, &a10, &a11, &a12, &a13, &a14};
    return hipLaunchKernel(kern, dim3(P.nsub, rows), dim3(nt), args, lds, h->stream);
}

template hipError_t run_mma<float2>(ddm_handle *, const float2 *, float2 *, int);
template hipError_t run_mma<double2>(ddm_handle *, const double2 *, double2 *, int);

}  // namespace ddm
