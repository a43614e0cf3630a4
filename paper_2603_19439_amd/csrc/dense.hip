// Tall-skinny dense kernels on row-major n x w blocks (w <= 128):
//   * k_tn: C = A^T B as per-chunk partial sums (each workgroup owns a contiguous
//     row chunk, rows are staged through LDS, every lane keeps a P x P register
//     tile of the output), then a fixed-order sum of the partials, so the result
//     does not depend on scheduling;
//   * k_apply: Out = beta Out + In M with the small matrix M held in LDS (used
//     for the projection update W - Xbar C, the orthonormalisation W R^{-1} and
//     the back-projection Z F);
//   * fills and conversions.
#include "grest_internal.h"

namespace {

constexpr int TB = 256;   // 16 x 16 lanes
constexpr int RB = 16;    // rows per LDS stage
constexpr int TW = 128;   // widest column block
constexpr int TN_MAX_CHUNKS = 512;

template <typename T, typename Acc, int P>
__global__ void __launch_bounds__(TB) k_tn(int64_t n, int64_t rows_per_chunk, const T* __restrict__ A,
                                           int64_t lda, int a, const T* __restrict__ B, int64_t ldb,
                                           int b, double* __restrict__ partial) {
  __shared__ T sa[RB][TW + 1];
  __shared__ T sb[RB][TW + 1];
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;
  const int ntb = (b + TW - 1) / TW;
  const int a0 = (blockIdx.y / ntb) * TW, b0 = (blockIdx.y % ntb) * TW;
  const int aw = min(TW, a - a0), bw = min(TW, b - b0);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  Acc acc[P][P];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int q = 0; q < P; ++q) acc[p][q] = Acc(0);
  const int lr = tid / TW, lc = tid % TW;  // loader: 2 rows x 128 columns per pass
  for (int64_t rb = r0; rb < r1; rb += RB) {
#pragma unroll
    for (int it = 0; it < RB / 2; ++it) {
      const int rr = it * 2 + lr;
      const int64_t row = rb + rr;
      const bool okr = row < r1;
      sa[rr][lc] = (okr && lc < aw) ? A[row * lda + a0 + lc] : T(0);
      sb[rr][lc] = (okr && lc < bw) ? B[row * ldb + b0 + lc] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < RB; ++rr) {
      Acc av[P], bv[P];
#pragma unroll
      for (int p = 0; p < P; ++p) av[p] = (Acc)sa[rr][ti + 16 * p];
#pragma unroll
      for (int q = 0; q < P; ++q) bv[q] = (Acc)sb[rr][tj + 16 * q];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < P; ++q) acc[p][q] += av[p] * bv[q];
    }
    __syncthreads();
  }
  double* out = partial + (size_t)blockIdx.x * a * b;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int i = ti + 16 * p;
    if (i >= aw) continue;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int j = tj + 16 * q;
      if (j < bw) out[(size_t)(a0 + i) * b + b0 + j] = (double)acc[p][q];
    }
  }
}

__global__ void k_tn_finalize(int g, int64_t ab, const double* __restrict__ partial, double* __restrict__ C) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ab) return;
  double s = 0.0;
  for (int c = 0; c < g; ++c) s += partial[(size_t)c * ab + idx];
  C[idx] = s;
}

template <typename T, int PB>
__global__ void __launch_bounds__(TB) k_apply(int64_t n, const T* In, int64_t ldin, int a,
                                              const double* __restrict__ M, int b, double alpha,
                                              double beta, T* Out, int64_t ldout) {
  __shared__ T sM[TW * TW];
  __shared__ T sIn[RB][TW + 1];
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;
  for (int idx = tid; idx < a * b; idx += TB) sM[idx] = (T)(alpha * M[idx]);
  const int lr = tid / TW, lc = tid % TW;
  for (int64_t rb = (int64_t)blockIdx.x * RB; rb < n; rb += (int64_t)gridDim.x * RB) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RB / 2; ++it) {
      const int rr = it * 2 + lr;
      const int64_t row = rb + rr;
      sIn[rr][lc] = (row < n && lc < a) ? In[row * ldin + lc] : T(0);
    }
    __syncthreads();
    T acc[PB];
#pragma unroll
    for (int q = 0; q < PB; ++q) acc[q] = T(0);
    for (int i = 0; i < a; ++i) {
      const T x = sIn[ti][i];
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int j = tj + 16 * q;
        if (j < b) acc[q] += x * sM[i * b + j];
      }
    }
    const int64_t r = rb + ti;
    if (r < n) {
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int j = tj + 16 * q;
        if (j < b) {
          T v = acc[q];
          if (beta != 0.0) v += (T)beta * Out[r * ldout + j];
          Out[r * ldout + j] = v;
        }
      }
    }
  }
}

template <typename T>
__global__ void k_fill_rows(T* p, int64_t ld, int64_t row0, int64_t rows, int w) {
  const int64_t total = rows * w;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t r = idx / w;
    const int c = (int)(idx % w);
    p[(row0 + r) * ld + c] = T(0);
  }
}

template <typename Ts, typename Td>
__global__ void k_convert(const Ts* s, Td* d, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) d[i] = (Td)s[i];
}

inline int grid_cap(int64_t work, int cap = 4096) {
  int64_t g = (work + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <typename T, typename Acc>
void tn_launch(int P, dim3 grid, int64_t n, int64_t rpc, const T* A, int64_t lda, int a, const T* B,
               int64_t ldb, int b, double* partial, hipStream_t s) {
  switch (P) {
    case 2: k_tn<T, Acc, 2><<<grid, TB, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial); break;
    case 4: k_tn<T, Acc, 4><<<grid, TB, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial); break;
    case 6: k_tn<T, Acc, 6><<<grid, TB, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial); break;
    default: k_tn<T, Acc, 8><<<grid, TB, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial); break;
  }
}

}  // namespace

int tn_num_chunks(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > TN_MAX_CHUNKS) g = TN_MAX_CHUNKS;
  return (int)g;
}

template <typename T, bool ACC64>
void launch_tn(int64_t n, const T* A, int64_t lda, int a, const T* B, int64_t ldb, int b, double* partial,
               double* C, hipStream_t s) {
  if (a <= 0 || b <= 0) return;
  const int g = tn_num_chunks(n);
  int64_t rpc = (n + g - 1) / g;
  rpc = ((rpc + RB - 1) / RB) * RB;
  const int gy = ((a + TW - 1) / TW) * ((b + TW - 1) / TW);
  const int wmax = (a < TW ? a : TW) > (b < TW ? b : TW) ? (a < TW ? a : TW) : (b < TW ? b : TW);
  int P = (wmax + 15) / 16;
  P = P <= 2 ? 2 : (P <= 4 ? 4 : (P <= 6 ? 6 : 8));
  dim3 grid(g, gy);
  if (ACC64) tn_launch<T, double>(P, grid, n, rpc, A, lda, a, B, ldb, b, partial, s);
  else tn_launch<T, T>(P, grid, n, rpc, A, lda, a, B, ldb, b, partial, s);
  const int64_t ab = (int64_t)a * b;
  k_tn_finalize<<<(unsigned)((ab + 255) / 256), 256, 0, s>>>(g, ab, partial, C);
}

template <typename T>
void launch_apply(int64_t n, const T* In, int64_t ldin, int a, const double* M, int b, double alpha,
                  double beta, T* Out, int64_t ldout, hipStream_t s) {
  if (n <= 0 || b <= 0) return;
  const int g = grid_cap(n * 16, 2048);
  const int pb = (b + 15) / 16;
  if (pb <= 2) k_apply<T, 2><<<g, TB, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
  else if (pb <= 4) k_apply<T, 4><<<g, TB, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
  else if (pb <= 6) k_apply<T, 6><<<g, TB, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
  else k_apply<T, 8><<<g, TB, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
}

template <typename T>
void launch_fill_rows(T* p, int64_t ld, int64_t row0, int64_t rows, int w, hipStream_t s) {
  if (rows <= 0 || w <= 0) return;
  k_fill_rows<T><<<grid_cap(rows * w), 256, 0, s>>>(p, ld, row0, rows, w);
}

template <typename Tsrc, typename Tdst>
void launch_convert(const Tsrc* src, Tdst* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  k_convert<Tsrc, Tdst><<<grid_cap(count), 256, 0, s>>>(src, dst, count);
}

template void launch_tn<float, false>(int64_t, const float*, int64_t, int, const float*, int64_t, int,
                                      double*, double*, hipStream_t);
template void launch_tn<float, true>(int64_t, const float*, int64_t, int, const float*, int64_t, int,
                                     double*, double*, hipStream_t);
template void launch_tn<double, true>(int64_t, const double*, int64_t, int, const double*, int64_t, int,
                                      double*, double*, hipStream_t);
template void launch_apply<float>(int64_t, const float*, int64_t, int, const double*, int, double, double,
                                  float*, int64_t, hipStream_t);
template void launch_apply<double>(int64_t, const double*, int64_t, int, const double*, int, double, double,
                                   double*, int64_t, hipStream_t);
template void launch_fill_rows<float>(float*, int64_t, int64_t, int64_t, int, hipStream_t);
template void launch_fill_rows<double>(double*, int64_t, int64_t, int64_t, int, hipStream_t);
template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template void launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);
template void launch_tn<double, false>(int64_t, const double*, int64_t, int, const double*, int64_t, int,
                                       double*, double*, hipStream_t);

// ---- start block of the initial subspace iteration and a scaled update ----
namespace {
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void k_fill_random(T* p, int64_t ld, int64_t rows, int w, uint64_t seed) {
  const int64_t total = rows * w;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t r = idx / w;
    const int c = (int)(idx % w);
    // uniform in (-1, 1) from a counter hash; only a generic start block is needed
    const uint64_t h = mix64(seed ^ mix64((uint64_t)idx));
    const double u = ((double)(h >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
    p[r * ld + c] = (T)u;
  }
}

template <typename T>
__global__ void k_axpby(int64_t rows, int w, double a, const T* X, int64_t ldx, double b, T* Y, int64_t ldy) {
  const int64_t total = rows * w;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t r = idx / w;
    const int c = (int)(idx % w);
    Y[r * ldy + c] = (T)(a * (double)X[r * ldx + c] + b * (double)Y[r * ldy + c]);
  }
}
}  // namespace

template <typename T>
void launch_fill_random(T* p, int64_t ld, int64_t rows, int w, uint64_t seed, hipStream_t s) {
  if (rows <= 0 || w <= 0) return;
  k_fill_random<T><<<grid_cap(rows * w), 256, 0, s>>>(p, ld, rows, w, seed);
}

template <typename T>
void launch_axpby(int64_t rows, int w, double a, const T* X, int64_t ldx, double b, T* Y, int64_t ldy,
                  hipStream_t s) {
  if (rows <= 0 || w <= 0) return;
  k_axpby<T><<<grid_cap(rows * w), 256, 0, s>>>(rows, w, a, X, ldx, b, Y, ldy);
}

template void launch_fill_random<float>(float*, int64_t, int64_t, int, uint64_t, hipStream_t);
template void launch_fill_random<double>(double*, int64_t, int64_t, int, uint64_t, hipStream_t);
template void launch_axpby<float>(int64_t, int, double, const float*, int64_t, double, float*, int64_t, hipStream_t);
template void launch_axpby<double>(int64_t, int, double, const double*, int64_t, double, double*, int64_t,
                                   hipStream_t);
