// Complex arithmetic on HIP vector types (double2 = complex128, float2 =
// complex64, .x real, .y imaginary).
#pragma once

#include <hip/hip_runtime.h>

namespace ddm {

template <typename T2> struct real_of;
template <> struct real_of<double2> { using type = double; };
template <> struct real_of<float2> { using type = float; };

__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cinv(double2 a) {
    double d = a.x * a.x + a.y * a.y;
    return make_double2(a.x / d, -a.y / d);
}

// acc += a * b
__device__ inline void cfma(double2 &acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
__device__ inline void cfma(float2 &acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
}

// c * x and g - c * x with every rounding fixed by explicit fma calls, so that
// all template instantiations round identically (no contraction freedom)
__device__ inline double2 cmul_fixed(double2 c, double2 x) {
    double re = fma(c.x, x.x, -(c.y * x.y));
    double im = fma(c.x, x.y, c.y * x.x);
    return make_double2(re, im);
}
__device__ inline double2 cmsub_fixed(double2 g, double2 c, double2 x) {
    double re = fma(-c.x, x.x, fma(c.y, x.y, g.x));
    double im = fma(-c.x, x.y, fma(-c.y, x.x, g.y));
    return make_double2(re, im);
}

__device__ inline double2 to_d2(double2 a) { return a; }
__device__ inline double2 to_d2(float2 a) { return make_double2(a.x, a.y); }

template <typename T2> __device__ inline T2 from_d2(double2 a);
template <> __device__ inline double2 from_d2<double2>(double2 a) { return a; }
template <> __device__ inline float2 from_d2<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }

template <typename T2> __device__ inline T2 czero();
template <> __device__ inline double2 czero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ inline float2 czero<float2>() { return make_float2(0.f, 0.f); }

}  // namespace ddm
