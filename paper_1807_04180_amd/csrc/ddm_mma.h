// Matrix-core (MFMA 16x16x4) operand order of the stored block inverses,
// shared by the factorisation (which writes it) and the substitution kernel
// (which reads it).  See ddm_solve_mma.hip for the layout.
#pragma once

#include <hip/hip_runtime.h>

namespace ddm {

typedef float mma_f4 __attribute__((ext_vector_type(4)));
typedef double mma_d4 __attribute__((ext_vector_type(4)));

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
};

constexpr int kMmaRhs = 16;    // RHS per tile
constexpr int kMmaRing = 8;    // operand loads in flight per lane

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
