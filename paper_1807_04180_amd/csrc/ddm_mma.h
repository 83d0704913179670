// Matrix-core (MFMA 16x16x4) operand order of the stored block inverses,
// shared by the factorisation (which writes it) and the substitution kernel
// (which reads it), and the substitution's lane layouts: operand loads,
// result stores and the g / y entries it adds.  See ddm_solve_mma.hip for
// the layout.
#pragma once

#include <hip/hip_runtime.h>

namespace ddm {

typedef float mma_f4 __attribute__((ext_vector_type(4)));
typedef double mma_d4 __attribute__((ext_vector_type(4)));
// two complex64 values, 8-byte aligned (one 16-byte store)
typedef float mma_f4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef double mma_d2 __attribute__((ext_vector_type(2)));

// the value of the neighbouring lane (lane ^ 1), by a DPP quad permutation
// [1, 0, 3, 2] (no LDS crossbar)
__device__ inline float shfl_xor1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ inline double shfl_xor1(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The result tile of a wave, one half (8 RHS) at a time: lane
// l = 16 k + 2 qq + p holds, for accumulator register r, part p (res) of
// entry (row(l, r), RHS qq) and, swapped in from lane l ^ 1, the other part
// (oth).  store_half writes whole entries of rows [0, rows) and RHS
// [0, nr) to x + q estr + row (x at the tile's first row and the half's
// first RHS): each lane stores entries its pair holds, so a store
// instruction covers whole 128-byte runs of consecutive rows of 8 RHS
// instead of one part per lane.
template <typename T2> struct Mma;
template <> struct Mma<float2> {
    using R = float;
    using Acc = mma_f4;
    using LT = float4;                // one 16-byte operand load
    static constexpr int S = 4;       // MFMAs (column pairs) per load
    static constexpr int CPG = 8;     // columns per group
    __device__ static Acc mfma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // row (within the tile) held by accumulator register r of lane l
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
    __device__ static R part(const LT &v, int s) { return s == 0 ? v.x : (s == 1 ? v.y : (s == 2 ? v.z : v.w)); }
    // one operand load; the inverses are read once per sweep, so the load
    // is marked non-temporal (measured: complex64 launches 0.6% faster,
    // complex128 ones 4%)
    __device__ static LT load_op(const char *p) {
        const mma_f4 v = __builtin_nontemporal_load((const mma_f4 *)p);
        return make_float4(v[0], v[1], v[2], v[3]);
    }
    // a lane pair holds rows 4k .. 4k+3: lane p stores rows 4k + 2p, 4k + 2p + 1
    __device__ static void store_half(float2 *x, long long estr, int rows, int nr, int lane, const R (&res)[4],
                                      const R (&oth)[4]) {
        const int qq = (lane & 15) >> 1, p = lane & 1, i0 = 4 * (lane >> 4) + 2 * p;
        if (qq >= nr || i0 >= rows) return;
        // lane 0 of the pair holds the real parts, lane 1 the imaginary ones
        const R are = p ? oth[2] : res[0], aim = p ? res[2] : oth[0];
        const R bre = p ? oth[3] : res[1], bim = p ? res[3] : oth[1];
        float2 *dst = x + qq * estr + i0;
        if (i0 + 1 < rows) *(mma_f4a8 *)dst = mma_f4a8{are, aim, bre, bim};
        else *dst = make_float2(are, aim);
    }
    // The other direction, for the g / y entries a step adds to its
    // results: the lane loads whole entries of the rows store_half stores
    // from it (src: the tile's RHS, row 0 of the block; rows clamped into the
    // block), and pre_parts turns them into part p of the lane's rows
    // row(l, 0..3) with one lane swap per pair of values.
    using PT = mma_f4a8;
    static constexpr int NPL = 1;  // loads per lane and half
    __device__ static void pre_load(PT (&v)[NPL], const float2 *src, int bs, int row0, int lane) {
        const int i0 = row0 + 4 * (lane >> 4) + 2 * (lane & 1);
        if (bs >= 2) {
            v[0] = *(const PT *)(src + (i0 + 1 < bs ? i0 : bs - 2));
        } else {
            const float2 e = src[0];
            v[0] = PT{e.x, e.y, e.x, e.y};
        }
    }
    __device__ static void pre_parts(R (&pv)[4], const PT (&v)[NPL], int bs, int row0, int lane) {
        const int p = lane & 1, i0 = row0 + 4 * (lane >> 4) + 2 * p;
        // a clamped pair ends at the block's last row, which is then row i0
        const bool last = i0 + 1 >= bs && bs >= 2;
        const R are = last ? v[0].z : v[0].x, aim = last ? v[0].w : v[0].y;  // row i0
        const R bre = v[0].z, bim = v[0].w;                                   // row i0 + 1
        const R t0 = shfl_xor1(p ? are : aim), t1 = shfl_xor1(p ? bre : bim);
        pv[0] = p ? t0 : are;
        pv[1] = p ? t1 : bre;
        pv[2] = p ? aim : t0;
        pv[3] = p ? bim : t1;
    }
};
template <> struct Mma<double2> {
    using R = double;
    using Acc = mma_d4;
    using LT = double2;
    static constexpr int S = 2;
    static constexpr int CPG = 4;
    __device__ static Acc mfma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
    __device__ static R part(const LT &v, int s) { return s == 0 ? v.x : v.y; }
    __device__ static LT load_op(const char *p) {
        const mma_d2 v = __builtin_nontemporal_load((const mma_d2 *)p);
        return make_double2(v[0], v[1]);
    }
    // a lane pair holds rows k, k+4, k+8, k+12 (r = 0..3): lane p stores
    // registers r = p and r = 2 + p
    __device__ static void store_half(double2 *x, long long estr, int rows, int nr, int lane, const R (&res)[4],
                                      const R (&oth)[4]) {
        const int k = lane >> 4, qq = (lane & 15) >> 1, p = lane & 1;
        if (qq >= nr) return;
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            const int i = k + 4 * (2 * s2 + p);
            if (i >= rows) continue;
            const R re = p ? oth[2 * s2 + 1] : res[2 * s2];
            const R im = p ? res[2 * s2 + 1] : oth[2 * s2];
            x[qq * estr + i] = make_double2(re, im);
        }
    }
    using PT = double2;
    static constexpr int NPL = 2;
    __device__ static void pre_load(PT (&v)[NPL], const double2 *src, int bs, int row0, int lane) {
        const int k = lane >> 4, p = lane & 1;
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            const int i = row0 + k + 4 * (2 * s2 + p);
            v[s2] = src[i < bs ? i : bs - 1];
        }
    }
    __device__ static void pre_parts(R (&pv)[4], const PT (&v)[NPL], int, int, int lane) {
        const int p = lane & 1;
        const R t0 = shfl_xor1(p ? v[0].x : v[0].y), t1 = shfl_xor1(p ? v[1].x : v[1].y);
        pv[0] = p ? t0 : v[0].x;
        pv[1] = p ? v[0].y : t0;
        pv[2] = p ? t1 : v[1].x;
        pv[3] = p ? v[1].y : t1;
    }
};

constexpr int kMmaRhs = 16;    // RHS per tile
constexpr int kMmaRing = 8;    // operand loads in flight per lane

// Position of element (i, j) of a block's inverse in the matrix-core order
// (T2 offset of its real part; the imaginary part is rows_t lanes further).
template <typename T2>
__device__ inline void mma_store(T2 *Wblk, int bs, int mpad, int i, int j, T2 v) {
    using M = Mma<T2>;
    using R = typename M::R;
    const int tile = i >> 4, ii = i & 15;
    const int rows_t = bs - 16 * tile < 16 ? bs - 16 * tile : 16;
    const int G = j / M::CPG, jr = j % M::CPG, s = jr >> 1, jj = jr & 1;
    char *base = (char *)Wblk + (long long)tile * 16 * mpad * sizeof(T2) + (long long)G * rows_t * 64;
    R *re = (R *)(base + (long long)((2 * jj) * rows_t + ii) * 16) + s;
    R *im = (R *)(base + (long long)((2 * jj + 1) * rows_t + ii) * 16) + s;
    *re = v.x;
    *im = v.y;
}

}  // namespace ddm
