// Small complex helpers for device code (interleaved re, im).
#pragma once
#include <hip/hip_runtime.h>

namespace omss {

template <typename VT> struct Scalar;
template <> struct Scalar<double2> { using type = double; };
template <> struct Scalar<float2> { using type = float; };

__host__ __device__ inline double2 mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline float2 mk(float r, float i) { return make_float2(r, i); }

template <typename VT> __host__ __device__ inline VT czero() { VT z; z.x = 0; z.y = 0; return z; }

template <typename VT> __host__ __device__ inline VT cadd(VT a, VT b) { VT r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename VT> __host__ __device__ inline VT csub(VT a, VT b) { VT r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename VT> __host__ __device__ inline VT cmul(VT a, VT b) {
    VT r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <typename VT> __host__ __device__ inline VT cmulc(VT a, VT b) {
    VT r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <typename VT> __host__ __device__ inline VT cconj(VT a) { a.y = -a.y; return a; }

// acc -= a * b
template <typename VT> __host__ __device__ inline void cfms(VT& acc, VT a, VT b) {
    acc.x -= a.x * b.x;
    acc.x += a.y * b.y;
    acc.y -= a.x * b.y;
    acc.y -= a.y * b.x;
}
// acc += a * b
template <typename VT> __host__ __device__ inline void cfma(VT& acc, VT a, VT b) {
    acc.x += a.x * b.x;
    acc.x -= a.y * b.y;
    acc.y += a.x * b.y;
    acc.y += a.y * b.x;
}

__device__ inline double2 to64(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ inline double2 to64(double2 a) { return a; }
template <typename VT> __device__ inline VT from64(double2 a);
template <> __device__ inline double2 from64<double2>(double2 a) { return a; }
template <> __device__ inline float2 from64<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }

}  // namespace omss
