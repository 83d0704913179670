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

namespace ddm {

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
    const T2 *Wl = W + s.foff + (long long)l * bs * bs;
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
                        if (l > 0) v = csub(v, cmul(cpl, to_d2(x[base + (long long)(l - 1) * bs + j])));
                    } else {
                        v = cmul(cpl, to_d2(x[base + (long long)(l + 1) * bs + j]));
                    }
                }
                vs[jj * RT + q] = from_d2<T2>(v);
            }
            __syncthreads();
            if (row < bs) {
                const T2 *col = Wl + (long long)j0 * bs + row;
                int jj = wv;
                for (; jj + 3 * kSWaves < jn; jj += 4 * kSWaves) {
                    T2 w0 = col[(long long)jj * bs];
                    T2 w1 = col[(long long)(jj + kSWaves) * bs];
                    T2 w2 = col[(long long)(jj + 2 * kSWaves) * bs];
                    T2 w3 = col[(long long)(jj + 3 * kSWaves) * bs];
#pragma unroll
                    for (int q = 0; q < RT; ++q) {
                        cfma(acc[q], w0, vs[jj * RT + q]);
                        cfma(acc[q], w1, vs[(jj + kSWaves) * RT + q]);
                        cfma(acc[q], w2, vs[(jj + 2 * kSWaves) * RT + q]);
                        cfma(acc[q], w3, vs[(jj + 3 * kSWaves) * RT + q]);
                    }
                }
                for (; jj < jn; jj += kSWaves) {
                    T2 w0 = col[(long long)jj * bs];
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

// g and x must not alias (rows of z_l are written while other workgroups of
// the same subdomain still read g_l).
template <typename T>
hipError_t launch_local_solve(ddm_handle *h, const T *g, T *x, int nrhs) {
    if (nrhs <= 1) return run_sweeps<T, 1>(h, g, x, nrhs);
    if (nrhs <= 2) return run_sweeps<T, 2>(h, g, x, nrhs);
    if (nrhs <= 4) return run_sweeps<T, 4>(h, g, x, nrhs);
    return run_sweeps<T, 8>(h, g, x, nrhs);
}

template hipError_t launch_local_solve<double2>(ddm_handle *, const double2 *, double2 *, int);
template hipError_t launch_local_solve<float2>(ddm_handle *, const float2 *, float2 *, int);

}  // namespace ddm
