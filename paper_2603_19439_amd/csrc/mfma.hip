// Matrix-core (MFMA) kernels for the tall-skinny products of the update, gfx950:
//   * k_tn_mfma : C = A^T B over n rows (A: n x a, B: n x b, a, b <= 128), per-workgroup
//                 partial sums of 16 x 16 output tiles; FP64 MFMA (v_mfma_f64_16x16x4)
//                 for FP64 accumulation (Gram matrices of CholQR2, FP64 projected
//                 matrix), FP32 MFMA (v_mfma_f32_16x16x4) for FP32 accumulation, BF16
//                 MFMA (v_mfma_f32_16x16x32_bf16) for the mixed-precision Z^T (A Z);
//                 a symmetric mode computes only the upper tiles of a Gram matrix;
//   * k_apply_mfma : Out = beta Out + alpha In M (M: a x b small, in LDS); same three
//                 precisions (BF16 for the mixed back-projection Z F).
// Rows are staged through LDS in row-major order; the contraction index of the
// apply kernel is permuted inside each 16-wide block (lane group g feeds columns
// 4g..4g+3 over four MFMA steps) so that every lane reads one 16-byte vector.
// Output layouts (checked on the device): f32 and bf16 tiles give lane l, register r
// the element (4*(l/16)+r, l%16); the f64 tile gives (l/16+4r, l%16).
#include "grest_internal.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int WG = 256;
constexpr int NW = WG / GREST_WAVE;
constexpr int TW = 128;      // widest operand
constexpr int MAXT = 16;     // output tiles per wave
constexpr int CHUNKS = 512;  // row chunks (= partial sums) of a reduction

template <typename Tc>
struct Mma;

template <>
struct Mma<float> {
  using acc_t = f32x4;
  __device__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct Mma<double> {
  using acc_t = f64x4;
  __device__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

__device__ inline int bf16_row(int lane, int r) { return 4 * (lane >> 4) + r; }

// tile t of this wave -> (ti, tj); symmetric mode enumerates ti <= tj only
__device__ inline void decode_tile(int t, int TA, int TB, bool sym, int& ti, int& tj) {
  if (!sym) {
    ti = t / TB;
    tj = t % TB;
    if (ti >= TA) ti = -1;
    return;
  }
  ti = 0;
  while (ti < TA && t >= TB - ti) {
    t -= TB - ti;
    ++ti;
  }
  if (ti >= TA) { ti = -1; tj = -1; return; }
  tj = ti + t;
}

// ---------------------------------------------------------------------------------
// C = A^T B with FP32 / FP64 MFMA
// ---------------------------------------------------------------------------------
template <typename Tin, typename Tc, bool SYM>
__global__ void __launch_bounds__(WG) k_tn_mfma(int64_t n, int64_t rpc, const Tin* __restrict__ A, int64_t lda,
                                                int a, const Tin* __restrict__ B, int64_t ldb, int b,
                                                double* __restrict__ partial) {
  constexpr int RB = 16;
  __shared__ Tc sA[RB][TW + 4];
  __shared__ Tc sB[SYM ? 1 : RB][TW + 4];
  using M = Mma<Tc>;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int TA = (a + 15) >> 4, TB = (b + 15) >> 4;
  int ti[MAXT], tj[MAXT];
  typename M::acc_t acc[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    decode_tile(wid + NW * q, TA, TB, SYM, ti[q], tj[q]);
    acc[q] = typename M::acc_t{0, 0, 0, 0};
  }
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const int lr = tid >> 7, lc = tid & 127;
  for (int64_t rb = r0; rb < r1; rb += RB) {
    __syncthreads();
#pragma unroll
    for (int p = 0; p < RB / 2; ++p) {
      const int rr = 2 * p + lr;
      const int64_t row = rb + rr;
      const bool ok = row < r1;
      sA[rr][lc] = (ok && lc < a) ? (Tc)A[row * lda + lc] : Tc(0);
      if (!SYM) sB[rr][lc] = (ok && lc < b) ? (Tc)B[row * ldb + lc] : Tc(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < RB; kk += 4) {
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int q = 0; q < MAXT; ++q) {
        if (ti[q] < 0) continue;
        const Tc fa = sA[kr][ti[q] * 16 + (lane & 15)];
        const Tc fb = SYM ? sA[kr][tj[q] * 16 + (lane & 15)] : sB[kr][tj[q] * 16 + (lane & 15)];
        acc[q] = M::run(fa, fb, acc[q]);
      }
    }
  }
  double* out = partial + (size_t)blockIdx.x * a * b;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    if (ti[q] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti[q] * 16 + M::row(lane, r);
      const int j = tj[q] * 16 + (lane & 15);
      if (i < a && j < b) out[(size_t)i * b + j] = (double)acc[q][r];
    }
  }
}

// ---------------------------------------------------------------------------------
// C = A^T B with BF16 MFMA (FP32 accumulation); 32 rows per step
// ---------------------------------------------------------------------------------
template <typename Tin>
__global__ void __launch_bounds__(WG) k_tn_bf16(int64_t n, int64_t rpc, const Tin* __restrict__ A, int64_t lda,
                                                int a, const Tin* __restrict__ B, int64_t ldb, int b,
                                                double* __restrict__ partial) {
  constexpr int RB = 32;
  // column-major staging so that a lane's eight consecutive rows are one 16-byte read;
  // every value is split into hi = bf16(x) and lo = bf16(x - hi), and the product is
  // hi*hi + hi*lo + lo*hi (relative error ~ 2^-16 instead of 2^-8)
  __shared__ __attribute__((aligned(16))) __bf16 sA[TW][RB + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sB[TW][RB + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[TW][RB + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[TW][RB + 8];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int TA = (a + 15) >> 4, TB = (b + 15) >> 4;
  int ti[MAXT], tj[MAXT];
  f32x4 acc[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    decode_tile(wid + NW * q, TA, TB, false, ti[q], tj[q]);
    acc[q] = f32x4{0, 0, 0, 0};
  }
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const int lr = tid >> 7, lc = tid & 127;
  for (int64_t rb = r0; rb < r1; rb += RB) {
    __syncthreads();
#pragma unroll 4
    for (int p = 0; p < RB / 2; ++p) {
      const int rr = 2 * p + lr;
      const int64_t row = rb + rr;
      const bool ok = row < r1;
      const float xa = (ok && lc < a) ? (float)A[row * lda + lc] : 0.f;
      const float xb = (ok && lc < b) ? (float)B[row * ldb + lc] : 0.f;
      const __bf16 ha = (__bf16)xa, hb = (__bf16)xb;
      sA[lc][rr] = ha;
      sB[lc][rr] = hb;
      sAl[lc][rr] = (__bf16)(xa - (float)ha);
      sBl[lc][rr] = (__bf16)(xb - (float)hb);
    }
    __syncthreads();
    const int kr = 8 * (lane >> 4);
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
      if (ti[q] < 0) continue;
      const int ia = ti[q] * 16 + (lane & 15), ib = tj[q] * 16 + (lane & 15);
      const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&sA[ia][kr]);
      const bf16x8 fb = *reinterpret_cast<const bf16x8*>(&sB[ib][kr]);
      const bf16x8 fal = *reinterpret_cast<const bf16x8*>(&sAl[ia][kr]);
      const bf16x8 fbl = *reinterpret_cast<const bf16x8*>(&sBl[ib][kr]);
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal, fb, acc[q], 0, 0, 0);
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fbl, acc[q], 0, 0, 0);
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[q], 0, 0, 0);
    }
  }
  double* out = partial + (size_t)blockIdx.x * a * b;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    if (ti[q] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti[q] * 16 + bf16_row(lane, r);
      const int j = tj[q] * 16 + (lane & 15);
      if (i < a && j < b) out[(size_t)i * b + j] = (double)acc[q][r];
    }
  }
}

// fixed-order sum of the chunk partials; four lanes per output, combined in order;
// in symmetric mode the lower tiles are read from their mirror
__global__ void __launch_bounds__(WG) k_tn_reduce(int g, int a, int b, int sym, const double* __restrict__ partial,
                                                  double* __restrict__ C) {
  const int64_t ab = (int64_t)a * b;
  const int64_t idx = (int64_t)blockIdx.x * (WG / 4) + (threadIdx.x >> 2);
  const int part = threadIdx.x & 3;
  double s = 0.0;
  int64_t src = idx;
  if (idx < ab) {
    const int i = (int)(idx / b), j = (int)(idx % b);
    if (sym && (i >> 4) > (j >> 4)) src = (int64_t)j * b + i;
    for (int c = part; c < g; c += 4) s += partial[(size_t)c * ab + src];
  }
  // combine the four lanes in a fixed order
  const double s1 = __shfl_xor(s, 1, 4);
  const double lo = (part & 1) ? s1 + s : s + s1;
  const double s2 = __shfl_xor(lo, 2, 4);
  const double tot = (part & 2) ? s2 + lo : lo + s2;
  if (idx < ab && part == 0) C[idx] = tot;
}

// ---------------------------------------------------------------------------------
// Out = beta Out + alpha In M with FP32 / FP64 MFMA
// ---------------------------------------------------------------------------------
template <typename T, typename Tc, bool VEC>
__global__ void __launch_bounds__(WG) k_apply_mfma(int64_t n, const T* In, int64_t ldin, int a,
                                                   const double* __restrict__ Mg, int b, double alpha,
                                                   double beta, T* Out, int64_t ldout) {
  using M = Mma<Tc>;
  const int KB = (a + 15) >> 4, TB = (b + 15) >> 4;
  const int bp = TB * 16;
  __shared__ Tc sM[TW * TW];
  for (int idx = threadIdx.x; idx < KB * 16 * bp; idx += WG) {
    const int k = idx / bp, j = idx % bp;
    sM[idx] = (k < a && j < b) ? (Tc)(alpha * Mg[(size_t)k * b + j]) : Tc(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t ntile = (n + 15) >> 4;
  for (int64_t tile = (int64_t)blockIdx.x * NW + wid; tile < ntile; tile += (int64_t)gridDim.x * NW) {
    const int64_t row0 = tile * 16;
    const int64_t row = row0 + c16;
    Tc fin[8][4];
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      if (kb < KB) {
        const int k0 = kb * 16 + 4 * g;
        if (VEC && row < n && k0 + 4 <= a) {
          const T* p = In + row * ldin + k0;
#pragma unroll
          for (int m = 0; m < 4; ++m) fin[kb][m] = (Tc)p[m];
        } else {
#pragma unroll
          for (int m = 0; m < 4; ++m) fin[kb][m] = (row < n && k0 + m < a) ? (Tc)In[row * ldin + k0 + m] : Tc(0);
        }
      }
    }
    for (int jt = 0; jt < TB; ++jt) {
      typename M::acc_t acc{0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        if (kb < KB) {
#pragma unroll
          for (int m = 0; m < 4; ++m)
            acc = M::run(fin[kb][m], sM[(kb * 16 + 4 * g + m) * bp + jt * 16 + c16], acc);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = row0 + M::row(lane, r);
        const int ocol = jt * 16 + c16;
        if (orow < n && ocol < b) {
          Tc v = acc[r];
          if (beta != 0.0) v += (Tc)beta * (Tc)Out[orow * ldout + ocol];
          Out[orow * ldout + ocol] = (T)v;
        }
      }
    }
  }
}

// Out = alpha In M with BF16 MFMA (FP32 accumulation), In FP32
__global__ void __launch_bounds__(WG) k_apply_bf16(int64_t n, const float* In, int64_t ldin, int a,
                                                   const double* __restrict__ Mg, int b, double alpha,
                                                   float* Out, int64_t ldout) {
  const int KB = (a + 31) >> 5, TB = (b + 15) >> 4;
  const int kp = KB * 32;
  // transposed: sMt[j][k], so that eight consecutive k of one column are one 16-byte read;
  // hi/lo split of both operands as in k_tn_bf16
  __shared__ __attribute__((aligned(16))) __bf16 sMt[TW][TW + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sMl[TW][TW + 8];
  for (int idx = threadIdx.x; idx < TB * 16 * kp; idx += WG) {
    const int j = idx / kp, k = idx % kp;
    const float x = (k < a && j < b) ? (float)(alpha * Mg[(size_t)k * b + j]) : 0.f;
    const __bf16 h = (__bf16)x;
    sMt[j][k] = h;
    sMl[j][k] = (__bf16)(x - (float)h);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t ntile = (n + 15) >> 4;
  for (int64_t tile = (int64_t)blockIdx.x * NW + wid; tile < ntile; tile += (int64_t)gridDim.x * NW) {
    const int64_t row0 = tile * 16;
    const int64_t row = row0 + c16;
    bf16x8 fin[4], finl[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      if (kb < KB) {
        const int k0 = kb * 32 + 8 * g;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = (row < n && k0 + e < a) ? In[row * ldin + k0 + e] : 0.f;
          const __bf16 h = (__bf16)x;
          fin[kb][e] = h;
          finl[kb][e] = (__bf16)(x - (float)h);
        }
      }
    }
    for (int jt = 0; jt < TB; ++jt) {
      f32x4 acc{0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        if (kb < KB) {
          const bf16x8 fb = *reinterpret_cast<const bf16x8*>(&sMt[jt * 16 + c16][kb * 32 + 8 * g]);
          const bf16x8 fbl = *reinterpret_cast<const bf16x8*>(&sMl[jt * 16 + c16][kb * 32 + 8 * g]);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(finl[kb], fb, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fin[kb], fbl, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fin[kb], fb, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = row0 + bf16_row(lane, r);
        const int ocol = jt * 16 + c16;
        if (orow < n && ocol < b) Out[orow * ldout + ocol] = acc[r];
      }
    }
  }
}

inline int apply_grid(int64_t n) {
  int64_t tiles = (n + 15) / 16;
  int64_t g = (tiles + NW - 1) / NW;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T>
bool aligned16(const T* p, int64_t ld) {
  return ((uintptr_t)p % 16) == 0 && ((ld * (int64_t)sizeof(T)) % 16) == 0;
}

}  // namespace

int tn_num_chunks(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > CHUNKS) g = CHUNKS;
  return (int)g;
}

// kind: 0 = FP32 MFMA, 1 = FP64 MFMA, 2 = BF16 MFMA
template <typename T>
static void tn_run(int kind, int64_t n, const T* A, int64_t lda, int a, const T* B, int64_t ldb, int b,
                   double* partial, double* C, hipStream_t s) {
  if (a <= 0 || b <= 0) return;
  const int g = tn_num_chunks(n);
  const int rb = kind == 2 ? 32 : 16;
  int64_t rpc = (n + g - 1) / g;
  rpc = ((rpc + rb - 1) / rb) * rb;
  const bool sym = (A == B && lda == ldb && a == b && kind != 2);
  if (kind == 2) {
    k_tn_bf16<T><<<g, WG, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial);
  } else if (kind == 1) {
    if (sym) k_tn_mfma<T, double, true><<<g, WG, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial);
    else k_tn_mfma<T, double, false><<<g, WG, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial);
  } else {
    if (sym) k_tn_mfma<T, float, true><<<g, WG, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial);
    else k_tn_mfma<T, float, false><<<g, WG, 0, s>>>(n, rpc, A, lda, a, B, ldb, b, partial);
  }
  const int64_t ab = (int64_t)a * b;
  k_tn_reduce<<<(unsigned)((ab + WG / 4 - 1) / (WG / 4)), WG, 0, s>>>(g, a, b, sym ? 1 : 0, partial, C);
}

template <typename T, bool ACC64>
void launch_tn(int64_t n, const T* A, int64_t lda, int a, const T* B, int64_t ldb, int b, double* partial,
               double* C, hipStream_t s) {
  tn_run<T>((ACC64 || sizeof(T) == 8) ? 1 : 0, n, A, lda, a, B, ldb, b, partial, C, s);
}

void launch_tn_bf16(int64_t n, const float* A, int64_t lda, int a, const float* B, int64_t ldb, int b,
                    double* partial, double* C, hipStream_t s) {
  tn_run<float>(2, n, A, lda, a, B, ldb, b, partial, C, s);
}

template <typename T>
void launch_apply(int64_t n, const T* In, int64_t ldin, int a, const double* M, int b, double alpha,
                  double beta, T* Out, int64_t ldout, hipStream_t s) {
  if (n <= 0 || b <= 0) return;
  const int g = apply_grid(n);
  const bool vec = aligned16(In, ldin);
  if (sizeof(T) == 8) {
    if (vec) k_apply_mfma<T, double, true><<<g, WG, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
    else k_apply_mfma<T, double, false><<<g, WG, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
  } else {
    if (vec) k_apply_mfma<T, float, true><<<g, WG, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
    else k_apply_mfma<T, float, false><<<g, WG, 0, s>>>(n, In, ldin, a, M, b, alpha, beta, Out, ldout);
  }
}

void launch_apply_bf16(int64_t n, const float* In, int64_t ldin, int a, const double* M, int b, double alpha,
                       float* Out, int64_t ldout, hipStream_t s) {
  if (n <= 0 || b <= 0) return;
  k_apply_bf16<<<apply_grid(n), WG, 0, s>>>(n, In, ldin, a, M, b, alpha, Out, ldout);
}

template void launch_tn<float, false>(int64_t, const float*, int64_t, int, const float*, int64_t, int, double*,
                                      double*, hipStream_t);
template void launch_tn<float, true>(int64_t, const float*, int64_t, int, const float*, int64_t, int, double*,
                                     double*, hipStream_t);
template void launch_tn<double, true>(int64_t, const double*, int64_t, int, const double*, int64_t, int, double*,
                                      double*, hipStream_t);
template void launch_tn<double, false>(int64_t, const double*, int64_t, int, const double*, int64_t, int,
                                       double*, double*, hipStream_t);
template void launch_apply<float>(int64_t, const float*, int64_t, int, const double*, int, double, double, float*,
                                  int64_t, hipStream_t);
template void launch_apply<double>(int64_t, const double*, int64_t, int, const double*, int, double, double,
                                   double*, int64_t, hipStream_t);
