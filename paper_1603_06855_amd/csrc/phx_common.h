// Common device/host helpers for the phx HIP library (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double __attribute__((ext_vector_type(4))) d4v;
typedef float __attribute__((ext_vector_type(4))) f4v;

// ---------------------------------------------------------------------------
// Complex scalar types: interleaved (re, im) pairs.
// ---------------------------------------------------------------------------
template <typename R> struct cplx_t;
template <> struct cplx_t<double> { typedef double2 type; };
template <> struct cplx_t<float> { typedef float2 type; };

template <typename R> using C_t = typename cplx_t<R>::type;

template <typename R>
__host__ __device__ __forceinline__ C_t<R> mk(R re, R im) { C_t<R> z; z.x = re; z.y = im; return z; }

template <typename C>
__host__ __device__ __forceinline__ C cadd(C a, C b) { C z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename C>
__host__ __device__ __forceinline__ C csub(C a, C b) { C z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename C>
__host__ __device__ __forceinline__ C cmul(C a, C b) { C z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z; }
// a * conj(b)
template <typename C>
__host__ __device__ __forceinline__ C cmulc(C a, C b) { C z; z.x = a.x * b.x + a.y * b.y; z.y = a.y * b.x - a.x * b.y; return z; }
template <typename C>
__host__ __device__ __forceinline__ C cconj(C a) { C z; z.x = a.x; z.y = -a.y; return z; }
template <typename C, typename R>
__host__ __device__ __forceinline__ C cscale(C a, R s) { C z; z.x = a.x * s; z.y = a.y * s; return z; }
template <typename C>
__host__ __device__ __forceinline__ double cabs2(C a) { return (double)a.x * a.x + (double)a.y * a.y; }

// ---------------------------------------------------------------------------
// MFMA 16x16x4 wrappers (one real product per call).
// ---------------------------------------------------------------------------
__device__ __forceinline__ d4v mfma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma16(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename R> struct acc_t;
template <> struct acc_t<double> { typedef d4v type; };
template <> struct acc_t<float> { typedef f4v type; };

// Status flags raised by kernels (device int, bit set with a vector atomic).
enum {
  PHX_FLAG_NOTPD = 1,      // a Cholesky pivot was not positive
  PHX_FLAG_NONFINITE = 2,  // a non-finite value reached a pivot
};

#define PHX_TILE 64
