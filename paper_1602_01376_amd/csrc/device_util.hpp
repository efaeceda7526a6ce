// Device helpers shared by the matrix-core kernels (LU, TRSM, grouped GEMM).
#pragma once

#include <hip/hip_runtime.h>

namespace invaskit {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
  using type = f64x4;
};
template <>
struct Vec4<float> {
  using type = f32x4;
};

// Global-memory pointers.  The kernels' problem descriptors hold generic
// pointers, and loads through a generic pointer compile to FLAT
// instructions, which count on the LDS counter as well: every wait for an
// LDS result would then also wait for all global loads in flight, defeating
// loads issued ahead.  Data pointers are therefore cast to the global
// address space once, at kernel entry.
#define INVASKIT_GLOBAL __attribute__((address_space(1)))
template <typename T>
using gptr = T INVASKIT_GLOBAL*;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// 16 x 16 x 4 MFMA.  Operand layout of both forms: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// accumulator row of element v in lane group g = lane / 16 (measured on
// gfx950): f32 4g + v, f64 g + 4v.  The column is lane % 16.
__device__ __forceinline__ constexpr int acc_row(double, int g, int v) { return g + 4 * v; }
__device__ __forceinline__ constexpr int acc_row(float, int g, int v) { return 4 * g + v; }

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Row-segment loads for an MFMA A operand from row-major memory.  The MFMA's
// reduction order over K is free as long as both operands use the same
// order; here lane group g (lane / 16) at MFMA step kk covers
//   k = sigma(kk, g) = 4 VE (kk / VE) + VE g + kk % VE,   VE = 16 / sizeof(T),
// so the four lane groups of a row read one contiguous 64-byte segment per
// 16-byte vector load.  Elements at k >= klim read as zero.
template <typename T>
__device__ __forceinline__ constexpr int sigma_k(int kk, int g) {
  constexpr int VE = 16 / sizeof(T);
  return 4 * VE * (kk / VE) + VE * g + kk % VE;
}
// Checked form: never reads at or beyond rowp[klim].
template <typename T, int KQ>
__device__ __forceinline__ void load_row_sigma(const T* __restrict__ rowp, int klim, int g,
                                               T (&a)[KQ]) {
  constexpr int VE = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VE), aligned(sizeof(T))));
#pragma unroll
  for (int i = 0; i < KQ / VE; ++i) {
    const int k0 = 4 * VE * i + VE * g;
    if (k0 + VE <= klim) {
      const vec v = *reinterpret_cast<const vec*>(rowp + k0);
#pragma unroll
      for (int e = 0; e < VE; ++e) a[VE * i + e] = v[e];
    } else {
#pragma unroll
      for (int e = 0; e < VE; ++e) a[VE * i + e] = (k0 + e < klim) ? rowp[k0 + e] : T(0);
    }
  }
}
// Branch-free form: always reads the full 4 VE * (KQ / VE) elements from
// rowp (the caller guarantees they are inside the allocation) and zeroes the
// ones at k >= klim.  No divergent paths, so loads issued ahead stay in
// flight across it.
template <typename T, int KQ>
__device__ __forceinline__ void load_row_sigma_full(const T* __restrict__ rowp, int klim, int g,
                                                    T (&a)[KQ]) {
  constexpr int VE = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VE), aligned(sizeof(T))));
#pragma unroll
  for (int i = 0; i < KQ / VE; ++i) {
    const int k0 = 4 * VE * i + VE * g;
    const vec v = *reinterpret_cast<const vec*>(rowp + k0);
#pragma unroll
    for (int e = 0; e < VE; ++e) a[VE * i + e] = (k0 + e < klim) ? v[e] : T(0);
  }
}

// load_row_sigma_full through a global pointer
template <typename T, int KQ>
__device__ __forceinline__ void load_row_sigma_full(gptr<const T> rowp, int klim, int g,
                                                    T (&a)[KQ]) {
  constexpr int VE = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VE), aligned(sizeof(T))));
#pragma unroll
  for (int i = 0; i < KQ / VE; ++i) {
    const int k0 = 4 * VE * i + VE * g;
    const vec v = *(gptr<const vec>)(rowp + k0);
#pragma unroll
    for (int e = 0; e < VE; ++e) a[VE * i + e] = (k0 + e < klim) ? v[e] : T(0);
  }
}
template <typename T, int KQ>
__device__ __forceinline__ void load_row_sigma_full(gptr<T> rowp, int klim, int g, T (&a)[KQ]) {
  load_row_sigma_full((gptr<const T>)rowp, klim, g, a);
}

// Unmasked global form: the four lane groups' 16-byte vectors of the
// segment, nothing zeroed (the caller masks where the segment passes the
// block, at the point of use, so the loads stay in flight until then).
template <typename T, int KQ>
__device__ __forceinline__ void load_row_sigma_raw(gptr<const T> rowp, int g, T (&a)[KQ]) {
  constexpr int VE = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VE), aligned(sizeof(T))));
#pragma unroll
  for (int i = 0; i < KQ / VE; ++i) {
    const vec v = *(gptr<const vec>)(rowp + 4 * VE * i + VE * g);
#pragma unroll
    for (int e = 0; e < VE; ++e) a[VE * i + e] = v[e];
  }
}
// Global form of load_row_sigma (never reads at or beyond rowp[klim]).
template <typename T, int KQ>
__device__ __forceinline__ void load_row_sigma_g(gptr<const T> rowp, int klim, int g,
                                                 T (&a)[KQ]) {
  constexpr int VE = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VE), aligned(sizeof(T))));
#pragma unroll
  for (int i = 0; i < KQ / VE; ++i) {
    const int k0 = 4 * VE * i + VE * g;
    if (k0 + VE <= klim) {
      const vec v = *(gptr<const vec>)(rowp + k0);
#pragma unroll
      for (int e = 0; e < VE; ++e) a[VE * i + e] = v[e];
    } else {
#pragma unroll
      for (int e = 0; e < VE; ++e) a[VE * i + e] = (k0 + e < klim) ? rowp[k0 + e] : T(0);
    }
  }
}
// zero the elements at k >= klim of a segment loaded in sigma order
template <typename T, int KQ>
__device__ __forceinline__ void mask_sigma(int klim, int g, T (&a)[KQ]) {
  constexpr int VE = 16 / sizeof(T);
#pragma unroll
  for (int i = 0; i < KQ / VE; ++i)
#pragma unroll
    for (int e = 0; e < VE; ++e)
      if (4 * VE * i + VE * g + e >= klim) a[VE * i + e] = T(0);
}

}  // namespace invaskit
