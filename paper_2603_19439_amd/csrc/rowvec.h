// Row-slice helpers shared by the sparse-product kernels: 16-, 8- or 4-byte slices of a
// dense row per lane, a power-of-two group of lanes per row, and grid sizing.
#pragma once

#include <cstdint>

#include "grest_internal.h"

namespace {


constexpr int BS = 256;
constexpr int HEAVY_BS = 1024;  // threads of the workgroup that multiplies one heavy row

template <typename T, int N>
struct alignas(N * sizeof(T)) vec_t {
  T v[N];
};

template <typename T, int N>
__device__ inline void vload(const T* p, T (&o)[N]) {
  const vec_t<T, N> t = *reinterpret_cast<const vec_t<T, N>*>(p);
#pragma unroll
  for (int i = 0; i < N; ++i) o[i] = t.v[i];
}

template <typename T, int N>
__device__ inline void vstore(T* p, const T (&o)[N]) {
  vec_t<T, N> t;
#pragma unroll
  for (int i = 0; i < N; ++i) t.v[i] = o[i];
  *reinterpret_cast<vec_t<T, N>*>(p) = t;
}

inline int grid_for(int64_t threads, int cap = 8192) {
  int64_t g = (threads + BS - 1) / BS;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

inline int lanes_per_row(int w, int vec) {
  int need = (w + vec - 1) / vec;
  int l = 1;
  while (l < need && l < GREST_WAVE) l <<= 1;
  return l;
}

inline int ilog2(int v) {
  int s = 0;
  while ((1 << s) < v) ++s;
  return s;
}

template <typename T>
inline int pick_vec(int w, int64_t ld1, int64_t ld2, const void* p1, const void* p2) {
  const int v = 16 / (int)sizeof(T);
  if (w % v == 0 && ld1 % v == 0 && ld2 % v == 0 && ((uintptr_t)p1 % 16) == 0 && ((uintptr_t)p2 % 16) == 0)
    return v;
  return 1;
}

// 8-byte slices for FP32 blocks whose width or offsets are even but not multiples of four
// (a basis of odd K, e.g. 65 tracked pairs and a 194-wide basis)
template <typename T>
inline int pick_vec2(int w, int64_t ld1, int64_t ld2, const void* p1, const void* p2) {
  const int v = pick_vec<T>(w, ld1, ld2, p1, p2);
  if (v > 1 || sizeof(T) != 4) return v;
  if (w % 2 == 0 && ld1 % 2 == 0 && ld2 % 2 == 0 && ((uintptr_t)p1 % 8) == 0 && ((uintptr_t)p2 % 8) == 0) return 2;
  return 1;
}

}  // namespace
