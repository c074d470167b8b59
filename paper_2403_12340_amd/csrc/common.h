// Shared device-side definitions for the gfx950 kernels: complex storage,
// MFMA wrappers and their lane layouts, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isdf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Interleaved complex in memory (re, im).
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};
typedef cx<double> z64;   // complex128
typedef cx<float> c32;    // complex64

template <typename D, typename S>
__device__ __forceinline__ cx<D> cvt(const cx<S>& a) {
  return cx<D>{(D)a.re, (D)a.im};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // conj(a) * b
  return cx<T>{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) {
  return cx<T>{a.re, -a.im};
}

// ---------------------------------------------------------------------------
// 16x16x4 MFMA on real operands.  Lane l supplies A[i = l % 16][k = l / 16]
// and B[k = l / 16][j = l % 16].  Output register v of lane l holds
//   f64: D[4 v + l / 16][l % 16]      f32: D[4 (l / 16) + v][l % 16]
// (both measured on gfx950).  The column is l % 16 in both cases, so the two
// real columns 2c, 2c+1 of one complex output column sit in lanes l, l ^ 1.
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <>
struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Exchange with lane ^ 1 (the other half of a complex output element).
__device__ __forceinline__ float xor1(float x) { return __shfl_xor(x, 1); }
__device__ __forceinline__ double xor1(double x) { return __shfl_xor(x, 1); }

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace isdf
