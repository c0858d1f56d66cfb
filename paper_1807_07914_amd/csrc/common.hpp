// common.hpp -- device-side helpers shared by the gfx950 kernels of libqsv.
//
// Amplitudes are interleaved (re, im) pairs of T = float (complex64) or
// T = double (complex128).  Qubit q is bit q of the amplitude index.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsv {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

// 16-byte vector of amplitudes: 2 x complex64 or 1 x complex128.
template <typename T>
struct VecInfo {
  static constexpr int A = 16 / (2 * sizeof(T));   // amplitudes per 16-byte vector
  static constexpr int LOG_A = (A == 2) ? 1 : 0;
};

template <typename T>
struct alignas(16) vec16 {
  cpx<T> a[VecInfo<T>::A];
};

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// a*b + c
template <typename T>
__device__ __forceinline__ cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> c) {
  return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}

// 2x2 and 4x4 complex matrices passed by value as kernel arguments.
template <typename T>
struct M2 {
  cpx<T> m[4];
};
template <typename T>
struct M4 {
  cpx<T> m[16];
};

// Insert a zero bit at position q of x.
__device__ __forceinline__ uint64_t insert0(uint64_t x, int q) {
  const uint64_t lo = x & ((1ull << q) - 1ull);
  return ((x >> q) << (q + 1)) | lo;
}

// Insert zero bits at positions a < b.
__device__ __forceinline__ uint64_t insert00(uint64_t x, int a, int b) {
  return insert0(insert0(x, a), b);
}

// Launch geometry of a one-dimensional range of nblk workgroups.  A dispatch
// keeps the global size of each grid dimension below 2^32 work-items, which
// a one-dimensional grid over the largest states HBM holds (2^35 complex64
// amplitudes, one work-item per 16-byte vector) would pass.  Ranges longer
// than kGridX workgroups therefore take a second grid dimension; kernels
// read their position in the range with block_index() and return when it is
// at or past nblk (the last row of a two-dimensional grid may overhang).
constexpr uint32_t kGridX = 1u << 16;

inline dim3 grid_for(uint64_t nblk) {
  if (nblk <= kGridX) return dim3((unsigned)(nblk ? nblk : 1), 1, 1);
  return dim3(kGridX, (unsigned)((nblk + kGridX - 1) / kGridX), 1);
}

__device__ __forceinline__ uint64_t block_index() {
  return (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
}

template <typename T>
__device__ __forceinline__ void apply2(const M2<T>& U, cpx<T>& a0, cpx<T>& a1) {
  cpx<T> y0 = cfma(U.m[1], a1, cmul(U.m[0], a0));
  cpx<T> y1 = cfma(U.m[3], a1, cmul(U.m[2], a0));
  a0 = y0;
  a1 = y1;
}

}  // namespace qsv
