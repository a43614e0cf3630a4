// Small element-wise kernels on row-major blocks: fills, conversions, the random
// start block of the initial subspace iteration and a scaled update.  The
// tall-skinny products live in mfma.hip.
#include "grest_internal.h"

namespace {

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

// zero the listed rows (rows[0 .. *count)) of a row-major block of width w
template <typename T>
__global__ void k_zero_listed_rows(T* p, int64_t ld, int w, const int32_t* rows, const int64_t* count) {
  const int64_t total = *count * w;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride)
    p[(int64_t)rows[idx / w] * ld + idx % w] = T(0);
}

__global__ void k_copy_i64(const int64_t* src, int64_t* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

template <typename Ts, typename Td>
__global__ void k_convert(const Ts* s, Td* d, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) d[i] = (Td)s[i];
}

// H (d x d) += C diag(theta) C^T, C d x k row-major (the low-rank term of the projected
// matrix), one entry per thread
// H += C diag(theta) C^T; with md_old (the combinatorial Laplacian, whose pairs are tracked
// as the eigenpairs nu of L) also alpha (I - C C^T - Gn) with alpha = 2 md_old and Gn the Gram
// of the appended rows of the basis (null when there are none)
__global__ void __launch_bounds__(256) k_lowrank_h(int d, int k, const double* __restrict__ Cm,
                                                   const double* __restrict__ theta, double* __restrict__ H,
                                                   const double* __restrict__ Gn, const int64_t* md_old) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int i = idx / d, j = idx % d;
  double acc = H[idx], cc = 0.0;
  for (int q = 0; q < k; ++q) {
    const double ci = Cm[(size_t)i * k + q], cj = Cm[(size_t)j * k + q];
    acc = fma(ci * theta[q], cj, acc);
    cc = fma(ci, cj, cc);
  }
  if (md_old) {
    const double alpha = 2.0 * (double)md_old[0];
    const double p = (i == j ? 1.0 : 0.0) - cc - (Gn ? Gn[idx] : 0.0);
    acc = fma(alpha, p, acc);
  }
  H[idx] = acc;
}

// C (m x q) = A (m x p) B (p x q), row-major FP64, one output per thread
__global__ void __launch_bounds__(256) k_small_gemm(int m, int p, int q, const double* __restrict__ A,
                                                    const double* __restrict__ B, double* __restrict__ C) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * q) return;
  const int i = idx / q, j = idx % q;
  double acc = 0.0;
#pragma unroll 16
  for (int k = 0; k < p; ++k) acc = fma(A[(size_t)i * p + k], B[(size_t)k * q + j], acc);
  C[idx] = acc;
}

inline int grid_cap(int64_t work, int cap = 4096) {
  int64_t g = (work + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

template <typename T>
void launch_fill_rows(T* p, int64_t ld, int64_t row0, int64_t rows, int w, hipStream_t s) {
  if (rows <= 0 || w <= 0) return;
  k_fill_rows<T><<<grid_cap(rows * w), 256, 0, s>>>(p, ld, row0, rows, w);
}

template <typename T>
void launch_zero_listed_rows(T* p, int64_t ld, int w, const int32_t* rows, const int64_t* count, int64_t bound,
                             hipStream_t s) {
  if (bound <= 0 || w <= 0) return;
  k_zero_listed_rows<T><<<grid_cap(bound * w), 256, 0, s>>>(p, ld, w, rows, count);
}

void launch_copy_i64(const int64_t* src, int64_t* dst, hipStream_t s) { k_copy_i64<<<1, 64, 0, s>>>(src, dst); }

void launch_lowrank_h(int d, int k, const double* Cm, const double* theta, double* H, hipStream_t s,
                      const double* Gn, const int64_t* md_old) {
  if (d <= 0) return;
  k_lowrank_h<<<(d * d + 255) / 256, 256, 0, s>>>(d, k, Cm, theta, H, Gn, md_old);
}

void launch_small_gemm(int m, int p, int q, const double* A, const double* B, double* C, hipStream_t s) {
  if (m <= 0 || q <= 0) return;
  k_small_gemm<<<(m * q + 255) / 256, 256, 0, s>>>(m, p, q, A, B, C);
}

template <typename Tsrc, typename Tdst>
void launch_convert(const Tsrc* src, Tdst* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  k_convert<Tsrc, Tdst><<<grid_cap(count), 256, 0, s>>>(src, dst, count);
}

template void launch_fill_rows<float>(float*, int64_t, int64_t, int64_t, int, hipStream_t);
template void launch_fill_rows<double>(double*, int64_t, int64_t, int64_t, int, hipStream_t);
template void launch_zero_listed_rows<float>(float*, int64_t, int, const int32_t*, const int64_t*, int64_t,
                                             hipStream_t);
template void launch_zero_listed_rows<double>(double*, int64_t, int, const int32_t*, const int64_t*, int64_t,
                                              hipStream_t);
template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template void launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);

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

// Out = a P + b Q + c R on an n x w block (FP64 arithmetic; R may be null).  Out may be
// P, Q or R itself: each element is read before it is written, at the same position.
template <typename T>
__global__ void k_lincomb3(int64_t rows, int w, double a, const T* P, int64_t ldp, double b, const T* Q,
                           int64_t ldq, double c, const T* R, int64_t ldr, T* Out, int64_t ldo) {
  const int64_t total = rows * w;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t r = idx / w;
    const int col = (int)(idx % w);
    double v = a * (double)P[r * ldp + col] + b * (double)Q[r * ldq + col];
    if (R) v += c * (double)R[r * ldr + col];
    Out[r * ldo + col] = (T)v;
  }
}

// residual block of tracked pairs: R[:, c] -= values[c] U[:, c] (FP64 arithmetic)
template <typename T>
__global__ void k_sub_scaled_cols(int64_t rows, int w, const double* __restrict__ values, const T* __restrict__ U,
                                  int64_t ldu, T* __restrict__ R, int64_t ldr) {
  const int64_t total = rows * w;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t r = idx / w;
    const int c = (int)(idx % w);
    R[r * ldr + c] = (T)((double)R[r * ldr + c] - values[c] * (double)U[r * ldu + c]);
  }
}
}  // namespace

template <typename T>
void launch_sub_scaled_cols(int64_t rows, int w, const double* values, const T* U, int64_t ldu, T* R, int64_t ldr,
                            hipStream_t s) {
  if (rows <= 0 || w <= 0) return;
  k_sub_scaled_cols<T><<<grid_cap(rows * w), 256, 0, s>>>(rows, w, values, U, ldu, R, ldr);
}
template void launch_sub_scaled_cols<float>(int64_t, int, const double*, const float*, int64_t, float*, int64_t,
                                            hipStream_t);
template void launch_sub_scaled_cols<double>(int64_t, int, const double*, const double*, int64_t, double*, int64_t,
                                             hipStream_t);

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

template <typename T>
void launch_lincomb3(int64_t rows, int w, double a, const T* P, int64_t ldp, double b, const T* Q, int64_t ldq,
                     double c, const T* R, int64_t ldr, T* Out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || w <= 0) return;
  k_lincomb3<T><<<grid_cap(rows * w), 256, 0, s>>>(rows, w, a, P, ldp, b, Q, ldq, c, R, ldr, Out, ldo);
}
template void launch_lincomb3<float>(int64_t, int, double, const float*, int64_t, double, const float*, int64_t,
                                     double, const float*, int64_t, float*, int64_t, hipStream_t);
template void launch_lincomb3<double>(int64_t, int, double, const double*, int64_t, double, const double*, int64_t,
                                      double, const double*, int64_t, double*, int64_t, hipStream_t);

template void launch_fill_random<float>(float*, int64_t, int64_t, int, uint64_t, hipStream_t);
template void launch_fill_random<double>(double*, int64_t, int64_t, int, uint64_t, hipStream_t);
template void launch_axpby<float>(int64_t, int, double, const float*, int64_t, double, float*, int64_t, hipStream_t);
template void launch_axpby<double>(int64_t, int, double, const double*, int64_t, double, double*, int64_t,
                                   hipStream_t);
