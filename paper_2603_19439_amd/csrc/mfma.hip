// Matrix-core (MFMA) kernels for the tall-skinny products of the update, gfx950.
//
//   * k_tnw    : C = A^T B over n rows (A: n x a, B: n x b, a, b <= 128) with FP32 or FP64
//                MFMA (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64).  Every wave owns
//                a disjoint set of 16-row blocks and keeps all output tiles of its slice
//                in registers; each lane loads exactly the operand elements it feeds to the
//                matrix core straight from global memory (16 rows per iteration, so that a
//                wave has 4 (PA + PB) loads in flight).  The four waves of a workgroup are
//                summed through LDS in a fixed order, and the workgroup partials are summed
//                in a fixed order by k_tn_reduce, so results do not depend on scheduling.
//                A symmetric mode (Gram matrices) computes the upper tiles only and writes
//                the lower ones as their mirrors.
//   * k_tn_bf16: the same product with split-BF16 MFMA (v_mfma_f32_16x16x32_bf16): every
//                value is split into hi = bf16(x) and lo = bf16(x - hi) and the tile gets
//                hi*hi + hi*lo + lo*hi with FP32 accumulation (relative error ~2^-16).  Rows
//                are staged through LDS column-major (a lane's eight rows are one 16-byte
//                read) and the next stage is prefetched into registers during the MFMAs.
//   * k_apply  : Out = beta Out + alpha In M (M: a x b small, in LDS) with FP32 / FP64 MFMA;
//                the contraction index is permuted inside each 16-wide block (lane group g
//                feeds columns 4g..4g+3 over four MFMA steps) so every lane reads one
//                16-byte vector; each wave works on one 16-row tile while the next
//                tile's fragments are loading.
// Output layouts (checked on the device): f32 and bf16 tiles give lane l, register r the
// element (4*(l/16)+r, l%16); the f64 tile gives (l/16+4r, l%16).
#include "grest_internal.h"

#include <algorithm>
#include <atomic>
#include <type_traits>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int WG = 256;
constexpr int NW = WG / GREST_WAVE;
constexpr int TW = 128;      // widest operand
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

// ---------------------------------------------------------------------------------
// C = A^T B, FP32 / FP64 MFMA, wave-owned rows, direct fragment loads
// slice y covers tile-rows [y*PA, y*PA + PA); all tile-columns (< PB*16 >= b)
// ---------------------------------------------------------------------------------
template <typename Tin, typename Tc, bool SYM, int PA, int PB>
__global__ void __launch_bounds__(WG) k_tnw(int64_t n, int64_t rpc, const Tin* __restrict__ A, int64_t lda, int a,
                                            const Tin* __restrict__ B, int64_t ldb, int b,
                                            double* __restrict__ partial) {
  using M = Mma<Tc>;
  using acc_t = typename M::acc_t;
  extern __shared__ double red_lds[];  // PA*PB tiles of 16x16 doubles
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int ty0 = blockIdx.y * PA;
  acc_t acc[PA][PB];
#pragma unroll
  for (int p = 0; p < PA; ++p)
#pragma unroll
    for (int q = 0; q < PB; ++q) acc[p][q] = acc_t{0, 0, 0, 0};
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  for (int64_t rb = r0 + 16 * wid; rb < r1; rb += 16 * NW) {
    Tc fa[4][PA], fb[4][PB];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t row = rb + 4 * s + g;
      const bool ok = row < r1;
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int col = q * 16 + c16;
        if (SYM) fb[s][q] = (ok && col < a) ? (Tc)A[row * lda + col] : Tc(0);
        else fb[s][q] = (ok && col < b) ? (Tc)B[row * ldb + col] : Tc(0);
      }
#pragma unroll
      for (int p = 0; p < PA; ++p) {
        if (SYM) {
          fa[s][p] = fb[s][p];  // single slice: the tile-rows are the tile-columns
        } else {
          const int col = (ty0 + p) * 16 + c16;
          fa[s][p] = (ok && col < a) ? (Tc)A[row * lda + col] : Tc(0);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int p = 0; p < PA; ++p)
#pragma unroll
        for (int q = 0; q < PB; ++q)
          if (!SYM || p <= q) acc[p][q] = M::run(fa[s][p], fb[s][q], acc[p][q]);
  }
  // fixed-order sum of the four waves through LDS, then one partial per workgroup
  for (int w = 0; w < NW; ++w) {
    if (wid == w) {
#pragma unroll
      for (int p = 0; p < PA; ++p)
#pragma unroll
        for (int q = 0; q < PB; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = ((p * PB + q) * 16 + M::row(lane, r)) * 16 + c16;
            red_lds[e] = (w == 0) ? (double)acc[p][q][r] : red_lds[e] + (double)acc[p][q][r];
          }
    }
    __syncthreads();
  }
  double* out = partial + (size_t)blockIdx.x * a * b;
  for (int e = threadIdx.x; e < PA * PB * 256; e += WG) {
    const int t = e >> 8, i = (e >> 4) & 15, j = e & 15;
    const int p = t / PB, q = t % PB;
    // symmetric mode: a lower tile is the transpose of its mirror, so the partial is full
    // and the reduction reads it row by row
    const double v = (SYM && p > q) ? red_lds[((q * PB + p) * 16 + j) * 16 + i] : red_lds[e];
    const int gi = (ty0 + p) * 16 + i, gj = q * 16 + j;
    if (gi < a && gj < b) out[(size_t)gi * b + gj] = v;
  }
}

// ---------------------------------------------------------------------------------
// C = A^T B for wide FP32 operands (more than 64 columns, up to TNL_MAXW): every output
// tile is owned by one wave for the workgroup's whole row chunk (tiles dealt out round-
// robin, upper tiles only for a Gram), rows are staged 16 at a time through LDS (the
// threads of the workgroup on consecutive columns of a row, the next stage's loads in
// flight during the MFMAs), and each lane feeds the matrix core from LDS.  So every row of
// A and B is read once per product, where the register-tiled kernel re-reads B once per
// slice of two tile-rows.  FP32 MFMA (Tc = float) or FP64 MFMA (Tc = double)
// accumulation; the workgroup's partial is written tile by tile by the owning waves (a
// Gram's lower tiles as the mirrors of the upper ones), so no two waves add into one value.
// ---------------------------------------------------------------------------------
constexpr int TNL_W = 8;         // waves of a workgroup
constexpr int TNL_MAXW = 208;    // widest operand (13 tiles); also the LDS pitch of a staged row
static_assert(TNL_MAXW % 64 == 16, "the four 16-lane groups of a fragment read hit disjoint banks");

template <typename Tc, int MT>
__global__ void __launch_bounds__(TNL_W * 64) k_tnl(int64_t n, int64_t rpc, const float* __restrict__ A, int64_t lda,
                                                    int a, const float* __restrict__ B, int64_t ldb, int b, int sym,
                                                    double* __restrict__ partial) {
  using M = Mma<Tc>;
  using acc_t = typename M::acc_t;
  __shared__ float sA[16 * TNL_MAXW];
  __shared__ float sB[16 * TNL_MAXW];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int TA = (a + 15) >> 4, TB = (b + 15) >> 4;
  // this wave's tiles: t = wid, wid + TNL_W, ... in row-major order of the (upper) tile grid
  int ti[MT], tj[MT];
  acc_t acc[MT];
  {
    int i = 0, j = 0, t = 0;  // the tile with index t
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      const int want = wid + TNL_W * q;
      while (i < TA && t < want) {
        ++t;
        if (++j == TB) {
          ++i;
          j = sym ? i : 0;
        }
      }
      const bool ok = i < TA && t == want;
      ti[q] = ok ? i : -1;
      tj[q] = ok ? j : -1;
      acc[q] = acc_t{0, 0, 0, 0};
    }
  }
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const int wcols = sym ? a : a + b;  // staged columns per row
  // loader: thread tid takes column tid of each of the 16 rows (wcols <= 2 TNL_MAXW <= 512)
  const bool lc = tid < wcols;
  const bool inA = tid < a;
  const float* src = inA ? A + tid : B + (tid - a);
  const int64_t lds = inA ? lda : ldb;
  float* dst = (inA ? sA : sB) + (inA ? tid : tid - a);
  float pre[16];
  auto fetch = [&](int64_t rb) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 16; ++r) pre[r] = (lc && rb + r < r1) ? src[(rb + r) * lds] : 0.f;
  };
  const float* sBr = sym ? sA : sB;
  if (r0 < r1) fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += 16) {
    __syncthreads();  // the previous stage's fragments have been read
    if (lc) {
#pragma unroll
      for (int r = 0; r < 16; ++r) dst[r * TNL_MAXW] = pre[r];
    }
    __syncthreads();
    if (rb + 16 < r1) fetch(rb + 16);  // in flight during the MFMAs below
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int rowoff = (4 * s + g) * TNL_MAXW + c16;
#pragma unroll
      for (int q = 0; q < MT; ++q) {
        if (ti[q] < 0) continue;
        const Tc fa = (Tc)sA[rowoff + ti[q] * 16];
        const Tc fb = (Tc)sBr[rowoff + tj[q] * 16];
        acc[q] = M::run(fa, fb, acc[q]);
      }
    }
  }
  double* out = partial + (size_t)blockIdx.x * a * b;
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    if (ti[q] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti[q] * 16 + M::row(lane, r), j = tj[q] * 16 + c16;
      if (i < a && j < b) {
        out[(size_t)i * b + j] = (double)acc[q][r];
        if (sym && ti[q] != tj[q]) out[(size_t)j * b + i] = (double)acc[q][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// C = A^T B with split-BF16 MFMA (FP32 accumulation); 32 rows per stage, prefetched
// ---------------------------------------------------------------------------------
constexpr int BT = 10;  // output tiles per wave (<= 40 tiles per workgroup)

__global__ void __launch_bounds__(WG) k_tn_bf16(int64_t n, int64_t rpc, const float* __restrict__ A, int64_t lda,
                                                int a, const float* __restrict__ B, int64_t ldb, int b,
                                                double* __restrict__ partial) {
  constexpr int RB = 32;
  constexpr int PF = RB * TW * 2 / WG;  // prefetched values per lane (A and B panels)
  __shared__ __attribute__((aligned(16))) __bf16 sA[TW][RB + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sB[TW][RB + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[TW][RB + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[TW][RB + 8];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int TA = (a + 15) >> 4, TB = (b + 15) >> 4;
  const int ntile = TA * TB;
  int ti[BT], tj[BT];
  f32x4 acc[BT];
#pragma unroll
  for (int q = 0; q < BT; ++q) {
    const int t = wid + NW * q;
    ti[q] = t < ntile ? t / TB : -1;
    tj[q] = t < ntile ? t % TB : -1;
    acc[q] = f32x4{0, 0, 0, 0};
  }
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  // loader mapping: value v of this lane is row (v*WG + tid) / TW... rows stride 2 per pass
  const int lr = tid >> 7, lc = tid & 127;
  float pa[PF / 2], pb[PF / 2];
  auto fetch = [&](int64_t rb) {
#pragma unroll
    for (int v = 0; v < PF / 2; ++v) {
      const int64_t row = rb + 2 * v + lr;
      const bool ok = row < r1;
      pa[v] = (ok && lc < a) ? A[row * lda + lc] : 0.f;
      pb[v] = (ok && lc < b) ? B[row * ldb + lc] : 0.f;
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += RB) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < PF / 2; ++v) {
      const int rr = 2 * v + lr;
      const __bf16 ha = (__bf16)pa[v], hb = (__bf16)pb[v];
      sA[lc][rr] = ha;
      sAl[lc][rr] = (__bf16)(pa[v] - (float)ha);
      sB[lc][rr] = hb;
      sBl[lc][rr] = (__bf16)(pb[v] - (float)hb);
    }
    __syncthreads();
    if (rb + RB < r1) fetch(rb + RB);  // in flight during the MFMAs below
    const int kr = 8 * (lane >> 4);
#pragma unroll
    for (int q = 0; q < BT; ++q) {
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
  for (int q = 0; q < BT; ++q) {
    if (ti[q] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti[q] * 16 + bf16_row(lane, r);
      const int j = tj[q] * 16 + (lane & 15);
      if (i < a && j < b) out[(size_t)i * b + j] = (double)acc[q][r];
    }
  }
}

// ---------------------------------------------------------------------------------
// C = A^T B with split-BF16 MFMA, FP32 rows staged transposed in LDS (the form used when
// the widths are multiples of four and the rows 16-byte aligned).  A stage is 32 rows:
// each loader thread takes four adjacent columns of eight consecutive rows (eight
// 16-byte loads), and writes each of its four columns' eight values as two 16-byte LDS
// stores into a column-major buffer (pitch 36 floats, which keeps the 16-lane phases of
// the 16-byte fragment reads on disjoint banks).  The next stage's loads are in flight
// during the MFMAs.  Wave w owns a TT x TT block of output tiles (tile rows from w / 2,
// tile columns from w % 2); each lane reads its eight k values of a fragment as two
// 16-byte vectors and splits them into hi = bf16(x) and lo = bf16(x - hi) in registers,
// and every tile gets lo*hi + hi*lo + hi*hi with FP32 accumulation.
// ---------------------------------------------------------------------------------
constexpr int TP = 36;  // LDS pitch (floats) of one staged column of 32 rows

template <int TT>
__global__ void __launch_bounds__(WG) k_tn_bf16t(int64_t n, int64_t rpc, const float* __restrict__ A, int64_t lda,
                                                 int a, const float* __restrict__ B, int64_t ldb, int b,
                                                 double* __restrict__ partial) {
  extern __shared__ double tsm_raw[];
  float* S = reinterpret_cast<float*>(tsm_raw);  // (a + b) columns x TP
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int ncg = (a + b) >> 2;  // column groups of four
  const int items = ncg * 4;     // x four row groups of eight rows
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  // loader item of this thread: column group cg, row group rg
  const bool loader = tid < items;
  const int cg = tid >> 2, rg = tid & 3;
  const int gc = 4 * cg;  // first concatenated column
  const float* src = gc < a ? A + gc : B + (gc - a);
  const int64_t ld = gc < a ? lda : ldb;
  f32x4 pre[8];
  auto fetch = [&](int64_t rb) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t row = rb + 8 * rg + e;
      pre[e] = (loader && row < r1) ? *reinterpret_cast<const f32x4*>(src + row * ld) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  const int ti0 = (wid >> 1) * TT, tj0 = (wid & 1) * TT;
  f32x4 acc[TT][TT];
#pragma unroll
  for (int p = 0; p < TT; ++p)
#pragma unroll
    for (int q = 0; q < TT; ++q) acc[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto frag = [&](int col, bool ok, bf16x8& hi, bf16x8& lo) __attribute__((always_inline)) {
    f32x4 u0{0.f, 0.f, 0.f, 0.f}, u1{0.f, 0.f, 0.f, 0.f};
    if (ok) {
      u0 = *reinterpret_cast<const f32x4*>(S + col * TP + 8 * g);
      u1 = *reinterpret_cast<const f32x4*>(S + col * TP + 8 * g + 4);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float x = e < 4 ? u0[e] : u1[e - 4];
      const __bf16 h = (__bf16)x;
      hi[e] = h;
      lo[e] = (__bf16)(x - (float)h);
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += 32) {
    __syncthreads();  // the previous stage's fragments have been read
    if (loader) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float* d = S + (gc + q) * TP + 8 * rg;
        *reinterpret_cast<f32x4*>(d) = f32x4{pre[0][q], pre[1][q], pre[2][q], pre[3][q]};
        *reinterpret_cast<f32x4*>(d + 4) = f32x4{pre[4][q], pre[5][q], pre[6][q], pre[7][q]};
      }
    }
    __syncthreads();
    if (rb + 32 < r1) fetch(rb + 32);  // in flight during the MFMAs below
    bf16x8 ahi[TT], alo[TT], bhi[TT], blo[TT];
#pragma unroll
    for (int p = 0; p < TT; ++p) {
      const int ca = (ti0 + p) * 16 + c16;
      frag(ca, ca < a, ahi[p], alo[p]);
    }
#pragma unroll
    for (int q = 0; q < TT; ++q) {
      const int cb = (tj0 + q) * 16 + c16;
      frag(a + cb, cb < b, bhi[q], blo[q]);
    }
#pragma unroll
    for (int p = 0; p < TT; ++p)
#pragma unroll
      for (int q = 0; q < TT; ++q) {
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[p], bhi[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[p], blo[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[p], bhi[q], acc[p][q], 0, 0, 0);
      }
  }
  double* out = partial + (size_t)blockIdx.x * a * b;
#pragma unroll
  for (int p = 0; p < TT; ++p)
#pragma unroll
    for (int q = 0; q < TT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = (ti0 + p) * 16 + bf16_row(lane, r);
        const int j = (tj0 + q) * 16 + c16;
        if (i < a && j < b) out[(size_t)i * b + j] = (double)acc[p][q][r];
      }
}

template <int TT>
void tn_bf16t_launch(int g, int64_t n, int64_t rpc, const float* A, int64_t lda, int a, const float* B, int64_t ldb,
                     int b, double* partial, hipStream_t s) {
  const size_t lds = (size_t)(a + b) * TP * sizeof(float);
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_tn_bf16t<TT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(2 * TW * TP * sizeof(float)));
    return true;
  }();
  (void)attr;
  k_tn_bf16t<TT><<<g, WG, lds, s>>>(n, rpc, A, lda, a, B, ldb, b, partial);
}

// ---------------------------------------------------------------------------------
// One pass over the rows for a projection round of block Gram-Schmidt with the
// Pythagorean Gram: C = X^T W and G = W^T W (upper tiles).
// X and W are separate column blocks (any widths <= 128).  G always accumulates in
// FP64; C in the working precision.
// ---------------------------------------------------------------------------------
// Every wave takes its own 16-row blocks of the workgroup's chunk and accumulates both
// the C tiles (TXC x TWC, working precision) and the upper tiles of G (packed triangle,
// FP64), so all four SIMDs share the FP64 matrix work; the fragments of the next block
// are loaded while the MFMAs of the current one run.  The four waves are summed through
// LDS in a fixed order.
__host__ __device__ constexpr int tri_idx(int p, int q, int n) { return p * n - p * (p - 1) / 2 + (q - p); }

// With a row list (rows, *nrows on the device) the pass runs over those rows only: the
// rows left out must be zero in W (the products are then the same).
template <typename T, typename Tcx, int TXC, int TWC>
__global__ void __launch_bounds__(WG, sizeof(T) == 4 ? 2 : 1) k_pip(int64_t n, int64_t rpc, const T* __restrict__ X, int64_t ldx, int kx,
                                            const T* __restrict__ W, int64_t ldw, int w, double* __restrict__ partC,
                                            double* __restrict__ partG, const int32_t* __restrict__ rows,
                                            const int64_t* __restrict__ nrows) {
  constexpr int NTG = TWC * (TWC + 1) / 2;
  using MC = Mma<Tcx>;
  using MG = Mma<double>;
  extern __shared__ double red_lds[];  // TXC*TWC + NTG tiles of 256 doubles
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  if (rows) n = min(n, *nrows);
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  typename MC::acc_t ac[TXC][TWC];
  typename MG::acc_t ag[NTG];
#pragma unroll
  for (int p = 0; p < TXC; ++p)
#pragma unroll
    for (int q = 0; q < TWC; ++q) ac[p][q] = typename MC::acc_t{0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < NTG; ++t) ag[t] = typename MG::acc_t{0, 0, 0, 0};
  T fx[4][TXC], fw[4][TWC];
  auto load = [&](int64_t rb) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t idx = rb + 4 * s + g;
      const bool ok = idx < r1;
      const int64_t row = (rows && ok) ? (int64_t)rows[idx] : idx;
#pragma unroll
      for (int p = 0; p < TXC; ++p) {
        const int c = p * 16 + c16;
        fx[s][p] = (ok && c < kx) ? X[row * ldx + c] : T(0);
      }
#pragma unroll
      for (int q = 0; q < TWC; ++q) {
        const int c = q * 16 + c16;
        fw[s][q] = (ok && c < w) ? W[row * ldw + c] : T(0);
      }
    }
  };
  int64_t rb = r0 + 16 * wid;
  if (rb < r1) load(rb);
  for (; rb < r1; rb += 16 * NW) {
    T cx[4][TXC], cw[4][TWC];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int p = 0; p < TXC; ++p) cx[s][p] = fx[s][p];
#pragma unroll
      for (int q = 0; q < TWC; ++q) cw[s][q] = fw[s][q];
    }
    if (rb + 16 * NW < r1) load(rb + 16 * NW);  // in flight during the MFMAs below
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int p = 0; p < TXC; ++p)
#pragma unroll
        for (int q = 0; q < TWC; ++q) ac[p][q] = MC::run((Tcx)cx[s][p], (Tcx)cw[s][q], ac[p][q]);
#pragma unroll
      for (int p = 0; p < TWC; ++p)
#pragma unroll
        for (int q = p; q < TWC; ++q)
          ag[tri_idx(p, q, TWC)] = MG::run((double)cw[s][p], (double)cw[s][q], ag[tri_idx(p, q, TWC)]);
    }
  }
  // fixed-order sum of the four waves
  double* lds2 = red_lds + (size_t)TXC * TWC * 256;
  for (int v = 0; v < NW; ++v) {
    if (wid == v) {
#pragma unroll
      for (int p = 0; p < TXC; ++p)
#pragma unroll
        for (int q = 0; q < TWC; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = ((p * TWC + q) * 16 + MC::row(lane, r)) * 16 + c16;
            red_lds[e] = (v == 0) ? (double)ac[p][q][r] : red_lds[e] + (double)ac[p][q][r];
          }
#pragma unroll
      for (int t = 0; t < NTG; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = (t * 16 + MG::row(lane, r)) * 16 + c16;
          lds2[e] = (v == 0) ? ag[t][r] : lds2[e] + ag[t][r];
        }
    }
    __syncthreads();
  }
  double* oc = partC + (size_t)blockIdx.x * kx * w;
  double* og = partG + (size_t)blockIdx.x * w * w;
  for (int e = threadIdx.x; e < TXC * TWC * 256; e += WG) {
    const int t = e >> 8, i = (e >> 4) & 15, j = e & 15;
    const int gi = (t / TWC) * 16 + i, gj = (t % TWC) * 16 + j;
    if (gi < kx && gj < w) oc[(size_t)gi * w + gj] = red_lds[e];
  }
  // G in full (lower tiles from their mirrors), so that the reduction reads rows
  for (int e = threadIdx.x; e < TWC * TWC * 256; e += WG) {
    const int t = e >> 8, i = (e >> 4) & 15, j = e & 15;
    const int p = t / TWC, q = t % TWC;
    const double v = p <= q ? lds2[(tri_idx(p, q, TWC) * 16 + i) * 16 + j] : lds2[(tri_idx(q, p, TWC) * 16 + j) * 16 + i];
    const int gi = p * 16 + i, gj = q * 16 + j;
    if (gi < w && gj < w) og[(size_t)gi * w + gj] = v;
  }
}

// fixed-order sum of the chunk partials: a workgroup of RWV waves owns 64 consecutive
// outputs, wave w sums the partials c = w, w + RWV, ... (all of its loads are issued
// before the first add, so the reduction costs one memory latency), and the wave sums are
// combined in a fixed order.  One launch serves up to two products (the two outputs of a
// projection round).
constexpr int RWV = 16;
constexpr int RLD = CHUNKS / RWV;  // partials per lane
static_assert(RLD * RWV == CHUNKS, "every chunk has a wave");

struct RedJob {
  const double* partial;
  double* C;
  int a, b, blocks;
  int ldc;  // leading dimension of C (b for a whole product, wider for a block of one)
};

__global__ void __launch_bounds__(RWV * 64) k_tn_reduce(int g, RedJob j0, RedJob j1) {
  __shared__ double red[RWV][64];
  const bool second = (int)blockIdx.x >= j0.blocks;
  const double* partial = second ? j1.partial : j0.partial;
  double* C = second ? j1.C : j0.C;
  const int a = second ? j1.a : j0.a, b = second ? j1.b : j0.b;
  const int64_t blk = second ? (int64_t)blockIdx.x - j0.blocks : (int64_t)blockIdx.x;
  const int64_t ab = (int64_t)a * b;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t idx = blk * 64 + lane;
  double v[RLD];
#pragma unroll
  for (int q = 0; q < RLD; ++q) {
    const int c = w + RWV * q;
    v[q] = (idx < ab && c < g) ? partial[(size_t)c * ab + idx] : 0.0;
  }
#pragma unroll
  for (int h = RLD / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int q = 0; q < h; ++q) v[q] += v[q + h];
  red[w][lane] = v[0];
  __syncthreads();
  if (w == 0 && idx < ab) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < RWV; ++q) t += red[q][lane];
    const int ldc = second ? j1.ldc : j0.ldc;
    C[(idx / b) * ldc + idx % b] = t;
  }
}

// C[j0 + c][i0 + r] = C[i0 + r][j0 + c] for the wi x wj block at (i0, j0) (leading dimension ldc)
__global__ void k_mirror_block(double* C, int ldc, int i0, int j0, int wi, int wj) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= wi * wj) return;
  const int r = idx / wj, c = idx % wj;
  C[(size_t)(j0 + c) * ldc + i0 + r] = C[(size_t)(i0 + r) * ldc + j0 + c];
}

inline RedJob red_job(const double* partial, double* C, int a, int b, int ldc = -1) {
  return RedJob{partial, C, a, b, (int)(((int64_t)a * b + 63) / 64), ldc < 0 ? b : ldc};
}

inline void launch_reduce(int g, const RedJob& j0, const RedJob& j1, hipStream_t s) {
  const int nb = j0.blocks + j1.blocks;
  if (nb > 0) k_tn_reduce<<<nb, RWV * 64, 0, s>>>(g, j0, j1);
}

// ---------------------------------------------------------------------------------
// Out = beta Out + alpha In M with FP32 / FP64 MFMA
// ---------------------------------------------------------------------------------
template <typename T, int N>
struct alignas(N * sizeof(T)) vec_t {
  T v[N];
};

// The input row is the concatenation [In1 row (a1 values) | In2 row (a2 values)].
template <typename T, typename Tc, bool VEC>
__device__ inline void load_frag(const T* In1, int64_t ld1, int a1, const T* In2, int64_t ld2, int a, int64_t row,
                                 int64_t n, int KB, int g, Tc (&fin)[8][4]) {
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    if (kb < KB) {
      const int k0 = kb * 16 + 4 * g;
      const bool in1 = k0 + 4 <= a1, in2 = k0 >= a1;
      if (VEC && row < n && k0 + 4 <= a && (in1 || in2)) {
        constexpr int NV = 16 / sizeof(T);  // elements per 16-byte load
        const T* p = in1 ? In1 + row * ld1 + k0 : In2 + row * ld2 + (k0 - a1);
#pragma unroll
        for (int h = 0; h < 4 / NV; ++h) {
          const vec_t<T, NV> v = *reinterpret_cast<const vec_t<T, NV>*>(p + h * NV);
#pragma unroll
          for (int m = 0; m < NV; ++m) fin[kb][h * NV + m] = (Tc)v.v[m];
        }
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int k = k0 + m;
          T v = T(0);
          if (row < n && k < a) v = k < a1 ? In1[row * ld1 + k] : In2[row * ld2 + (k - a1)];
          fin[kb][m] = (Tc)v;
        }
      }
    }
  }
}

// With rows, the kernel covers the listed rows rows[0 .. min(n, *nrows)) only (n is then a
// bound of the count); row idx of the tiles is matrix row rows[idx].
template <typename T, typename Tc, bool VEC>
__global__ void __launch_bounds__(WG) k_apply(int64_t n, const T* In1, int64_t ld1, int a1, const T* In2,
                                              int64_t ld2, int a2, const double* __restrict__ Mg, int b,
                                              double alpha, double beta, T* Out, int64_t ldout,
                                              const int32_t* __restrict__ rows, const int64_t* nrows) {
  using M = Mma<Tc>;
  extern __shared__ double sMraw[];
  Tc* sM = reinterpret_cast<Tc*>(sMraw);
  const int a = a1 + a2;
  const int KB = (a + 15) >> 4, TB = (b + 15) >> 4;
  const int bp = TB * 16 + 1;  // odd pitch: the four lane groups hit different banks
  for (int idx = threadIdx.x; idx < KB * 16 * bp; idx += WG) {
    const int k = idx / bp, j = idx % bp;
    sM[idx] = (k < a && j < b) ? (Tc)(alpha * Mg[(size_t)k * b + j]) : Tc(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t nl = rows ? (n < *nrows ? n : *nrows) : n;
  const int64_t ntile = (nl + 15) >> 4;
  const int64_t stride = (int64_t)gridDim.x * NW;
  // tile row idx -> matrix row, and the bound load_frag checks it against
  auto load_t = [&](int64_t t, Tc(&f)[8][4]) __attribute__((always_inline)) {
    const int64_t idx = t * 16 + c16;
    if (!rows) {
      load_frag<T, Tc, VEC>(In1, ld1, a1, In2, ld2, a, idx, n, KB, g, f);
    } else {
      const int64_t row = idx < nl ? (int64_t)rows[idx] : 0;
      load_frag<T, Tc, VEC>(In1, ld1, a1, In2, ld2, a, row, idx < nl ? row + 1 : 0, KB, g, f);
    }
  };
  // one 16-row tile at a time; the next tile's fragments are in flight during its MFMAs
  int64_t tile = (int64_t)blockIdx.x * NW + wid;
  Tc nxt[8][4];
  if (tile < ntile) load_t(tile, nxt);
  for (; tile < ntile; tile += stride) {
    Tc fin[8][4];
#pragma unroll
    for (int kb = 0; kb < 8; ++kb)
#pragma unroll
      for (int m = 0; m < 4; ++m) fin[kb][m] = nxt[kb][m];
    if (tile + stride < ntile) load_t(tile + stride, nxt);
    const int64_t row0 = tile * 16;
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
        const int64_t oidx = row0 + M::row(lane, r);
        const int ocol = jt * 16 + c16;
        if (oidx < nl && ocol < b) {
          const int64_t orow = rows ? (int64_t)rows[oidx] : oidx;
          Tc v = acc[r];
          if (beta != 0.0) v += (Tc)beta * (Tc)Out[orow * ldout + ocol];
          Out[orow * ldout + ocol] = (T)v;
        }
      }
    }
  }
}

// FP32 blocks: the tile is computed transposed, D = M^T In^T, so that lane (g, c) of the
// wave reads four consecutive input columns of row c (one 16-byte load per 16 columns)
// and ends up holding four consecutive output columns of row c (one 16-byte store).  M is
// staged in LDS as float4 groups [kb][jt][g][c] of the four coefficients a lane feeds in
// the four MFMA steps of a 16-wide k block, so each lane reads one 16-byte vector per
// (kb, jt).  KB = ceil(a / 16) is a template parameter so the fragment arrays are exact;
// two output tiles are accumulated side by side.  Every row's inputs are read before its
// outputs are written, so Out may alias In2 (in-place update of a column block).
// With flag2, the In2 part of row r is read only where flag2[r] != 0 (zero elsewhere).
// With rows, only the listed rows rows[0 .. min(n, *nrows)) are covered.
template <int KB, bool VEC, bool VOUT>
__global__ void __launch_bounds__(WG) k_apply_f32(int64_t n, const float* In1, int64_t ld1, int a1,
                                                  const float* In2, int64_t ld2, int a2,
                                                  const double* __restrict__ Mg, int b, double alpha, double beta,
                                                  float* Out, int64_t ldout, const int64_t* __restrict__ flag2,
                                                  const int32_t* __restrict__ rows, const int64_t* nrows) {
  extern __shared__ double sMraw[];
  f32x4* sM = reinterpret_cast<f32x4*>(sMraw);
  const int a = a1 + a2;
  const int TB = (b + 15) >> 4;
  for (int idx = threadIdx.x; idx < KB * TB * 64; idx += WG) {
    const int c = idx & 15, g = (idx >> 4) & 3, t = idx >> 6;
    const int kb = t / TB, jt = t % TB;
    const int j = jt * 16 + c;
    f32x4 v;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = kb * 16 + 4 * g + m;
      v[m] = (k < a && j < b) ? (float)(alpha * Mg[(size_t)k * b + j]) : 0.f;
    }
    sM[idx] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t nl = rows ? (n < *nrows ? n : *nrows) : n;
  const int64_t ntile = (nl + 15) >> 4;
  const int64_t stride = (int64_t)gridDim.x * NW;
  auto row_of = [&](int64_t idx) __attribute__((always_inline)) {
    return rows ? (idx < nl ? (int64_t)rows[idx] : (int64_t)0) : idx;
  };
  // VEC: every input row starts 16 bytes aligned and a1 is a multiple of four (or In2 is
  // empty), so a lane's four columns lie in one input block; the last group of a block may
  // pass its end, which stays inside the row (rows are whole multiples of 16 bytes), and is
  // masked to zero there
  auto load = [&](int64_t t, f32x4(&f)[KB]) __attribute__((always_inline)) {
    const int64_t idx = t * 16 + c16;
    const bool ok = idx < nl;
    const int64_t row = row_of(idx);
    const bool use2 = ok && (!flag2 || flag2[row] != 0);
    if (VEC) {
      const float* b1 = In1 + row * ld1;
      const float* b2 = In2 + row * ld2 - a1;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int k0 = kb * 16 + 4 * g;
        f[kb] = (ok && k0 < a && (k0 < a1 || use2))
                    ? *reinterpret_cast<const f32x4*>((k0 < a1 ? b1 : b2) + k0)
                    : f32x4{0.f, 0.f, 0.f, 0.f};
        const int lim = k0 < a1 ? a1 : a;  // the end of the block the group starts in
#pragma unroll
        for (int m = 1; m < 4; ++m)
          if (k0 + m >= lim) f[kb][m] = 0.f;
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int k = kb * 16 + 4 * g + m;
          float v = 0.f;
          if (ok && k < a) {
            if (k < a1) v = In1[row * ld1 + k];
            else if (use2) v = In2[row * ld2 + (k - a1)];
          }
          f[kb][m] = v;
        }
      }
    }
  };
  auto store = [&](int64_t row, bool ok, int jt, f32x4 acc) __attribute__((always_inline)) {
    const int col0 = jt * 16 + 4 * g;
    if (!ok || jt >= TB) return;
    float* o = Out + row * ldout + col0;
    if (VOUT && col0 + 4 <= b) {  // a whole 16-byte group of an aligned output row
      if (beta != 0.0) {
        const f32x4 old = *reinterpret_cast<const f32x4*>(o);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += (float)beta * old[r];
      }
      *reinterpret_cast<f32x4*>(o) = acc;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (col0 + r < b) {
          float v = acc[r];
          if (beta != 0.0) v += (float)beta * o[r];
          o[r] = v;
        }
      }
    }
  };
  int64_t tile = (int64_t)blockIdx.x * NW + wid;
  f32x4 nxt[KB];
  if (tile < ntile) load(tile, nxt);
  for (; tile < ntile; tile += stride) {
    f32x4 fin[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) fin[kb] = nxt[kb];
    if (tile + stride < ntile) load(tile + stride, nxt);  // in flight during the MFMAs below
    const int64_t ridx = tile * 16 + c16;
    const bool rok = ridx < nl;
    const int64_t row = row_of(ridx);
    for (int jt = 0; jt < TB; jt += 2) {
      const bool two = jt + 1 < TB;
      f32x4 acc0{0.f, 0.f, 0.f, 0.f}, acc1{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const f32x4 m0 = sM[(kb * TB + jt) * 64 + lane];
        const f32x4 m1 = two ? sM[(kb * TB + jt + 1) * 64 + lane] : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(m0[m], fin[kb][m], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(m1[m], fin[kb][m], acc1, 0, 0, 0);
        }
      }
      store(row, rok, jt, acc0);
      store(row, rok, jt + 1, acc1);
    }
  }
}

int device_cus() {
  static const int cus = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || v <= 0)
      v = 256;
    return v;
  }();
  return cus;
}

template <int KB, bool VEC, bool VOUT>
void apply_f32_launch(int64_t n, const float* In1, int64_t ld1, int a1, const float* In2, int64_t ld2, int a2,
                      const double* M, int b, double alpha, double beta, float* Out, int64_t ldout,
                      const int64_t* flag2, const int32_t* rows, const int64_t* nrows, hipStream_t s) {
  const int TB = (b + 15) >> 4;
  const size_t lds = (size_t)KB * TB * 64 * sizeof(f32x4);
  // resident workgroups per CU for this LDS size (queried once per size; a persistent
  // grid of that many workgroups per CU takes the tiles round-robin)
  static std::atomic<int> occ_cache[8];
  int occ = occ_cache[TB - 1].load(std::memory_order_relaxed);
  if (occ <= 0) {
    static const bool attr = [] {
      (void)hipFuncSetAttribute((const void*)k_apply_f32<KB, VEC, VOUT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(KB * 8 * 64 * sizeof(f32x4)));
      return true;
    }();
    (void)attr;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_apply_f32<KB, VEC, VOUT>, WG, lds) != hipSuccess ||
        nb < 1)
      nb = 1;
    occ = nb;
    occ_cache[TB - 1].store(occ, std::memory_order_relaxed);
  }
  const int64_t tiles = (n + 15) / 16;
  int64_t g = std::min<int64_t>((tiles + NW - 1) / NW, (int64_t)device_cus() * occ);
  if (g < 1) g = 1;
  k_apply_f32<KB, VEC, VOUT><<<(unsigned)g, WG, lds, s>>>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout,
                                                     flag2, rows, nrows);
}

template <bool VEC, bool VOUT>
void apply_f32_dispatch(int64_t n, const float* In1, int64_t ld1, int a1, const float* In2, int64_t ld2, int a2,
                        const double* M, int b, double alpha, double beta, float* Out, int64_t ldout,
                        const int64_t* flag2, const int32_t* rows, const int64_t* nrows, hipStream_t s) {
  switch ((a1 + a2 + 15) >> 4) {
    case 1: apply_f32_launch<1, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
    case 2: apply_f32_launch<2, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
    case 3: apply_f32_launch<3, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
    case 4: apply_f32_launch<4, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
    case 5: apply_f32_launch<5, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
    case 6: apply_f32_launch<6, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
    case 7: apply_f32_launch<7, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
    default: apply_f32_launch<8, VEC, VOUT>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s); break;
  }
}

inline int apply_grid(int64_t n) {
  int64_t tiles = (n + 15) / 16;
  int64_t g = (tiles + 4 * NW - 1) / (4 * NW);  // about four tiles per wave
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T>
bool aligned16(const T* p, int64_t ld) {
  return ((uintptr_t)p % 16) == 0 && ((ld * (int64_t)sizeof(T)) % 16) == 0;
}

template <typename Tin, typename Tc, bool SYM, int PA, int PB>
void tnw_launch(dim3 grid, hipStream_t s, int64_t n, int64_t rpc, const Tin* A, int64_t lda, int a, const Tin* B,
                int64_t ldb, int b, double* partial) {
  constexpr size_t lds = (size_t)PA * PB * 256 * sizeof(double);
  if (lds > 65536) {  // once per instance; function-local statics initialise thread-safely
    static const bool attr = [] {
      (void)hipFuncSetAttribute((const void*)k_tnw<Tin, Tc, SYM, PA, PB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      return true;
    }();
    (void)attr;
  }
  k_tnw<Tin, Tc, SYM, PA, PB><<<grid, WG, lds, s>>>(n, rpc, A, lda, a, B, ldb, b, partial);
}

// picks the register tile shape for a (TA x TB)-tile product; returns the slice count
template <typename Tin, typename Tc>
int tnw_dispatch(int64_t n, int g, int64_t rpc, const Tin* A, int64_t lda, int a, const Tin* B, int64_t ldb, int b,
                 bool sym, double* partial, hipStream_t s) {
  const int TA = (a + 15) >> 4, TB = (b + 15) >> 4;
  const bool f64 = sizeof(Tc) == 8;
  if (sym && TA <= 2) { tnw_launch<Tin, Tc, true, 2, 2>(dim3(g, 1), s, n, rpc, A, lda, a, B, ldb, b, partial); return 1; }
  if (sym && TA <= 4) { tnw_launch<Tin, Tc, true, 4, 4>(dim3(g, 1), s, n, rpc, A, lda, a, B, ldb, b, partial); return 1; }
  if (TA <= 1 && TB <= 8) { tnw_launch<Tin, Tc, false, 1, 8>(dim3(g, 1), s, n, rpc, A, lda, a, B, ldb, b, partial); return 1; }
  if (TA <= 2 && TB <= 2) { tnw_launch<Tin, Tc, false, 2, 2>(dim3(g, 1), s, n, rpc, A, lda, a, B, ldb, b, partial); return 1; }
  if (TA <= 2 && TB <= 4) { tnw_launch<Tin, Tc, false, 2, 4>(dim3(g, 1), s, n, rpc, A, lda, a, B, ldb, b, partial); return 1; }
  if (TA <= 4 && TB <= 4) { tnw_launch<Tin, Tc, false, 4, 4>(dim3(g, 1), s, n, rpc, A, lda, a, B, ldb, b, partial); return 1; }
  if (!f64 && TA <= 6 && TB <= 6) { tnw_launch<Tin, Tc, false, 6, 6>(dim3(g, 1), s, n, rpc, A, lda, a, B, ldb, b, partial); return 1; }
  // general case: slices of two tile-rows against up to eight tile-columns
  const int ny = (TA + 1) / 2;
  tnw_launch<Tin, Tc, false, 2, 8>(dim3(g, ny), s, n, rpc, A, lda, a, B, ldb, b, partial);
  return ny;
}

}  // namespace

int tn_num_chunks(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > CHUNKS) g = CHUNKS;
  return (int)g;
}

// kind: 0 = FP32 MFMA, 1 = FP64 MFMA, 2 = split-BF16 MFMA; C has leading dimension ldc
template <typename T>
static void tn_run(int kind, int64_t n, const T* A, int64_t lda, int a, const T* B, int64_t ldb, int b,
                   double* partial, double* C, hipStream_t s, int ldc = -1) {
  if (a <= 0 || b <= 0) return;
  if (ldc < 0) ldc = b;
  if constexpr (std::is_same<T, float>::value) {
    // wide FP32 operands: one pass over the rows with LDS staging (split BF16 has no such
    // form; its wide products take FP32 MFMA here, as they do below)
    const int TA = (a + 15) >> 4, TB = (b + 15) >> 4;
    const bool sym = A == B && lda == ldb && a == b && kind != 2;
    const bool bf16_fits = kind == 2 && a <= TW && b <= TW && TA * TB <= NW * BT;
    if ((a > 64 || b > 64) && a <= TNL_MAXW && b <= TNL_MAXW && !bf16_fits) {
      const int ntile = sym ? TA * (TA + 1) / 2 : TA * TB;
      const int per = (ntile + TNL_W - 1) / TNL_W;
      const bool f64 = kind == 1;
      if ((!f64 && per <= 24) || (f64 && per <= 12)) {
        const int g = tn_num_chunks(n);
        int64_t rpc = (n + g - 1) / g;
        rpc = ((rpc + 15) / 16) * 16;
        const float* fA = (const float*)A;
        const float* fB = (const float*)B;
        const int sy = sym ? 1 : 0;
        // the smallest register tile that holds the wave's tiles: fewer registers, more
        // resident waves to cover the loads of the next stage
        if (f64 && per <= 6) k_tnl<double, 6><<<g, TNL_W * 64, 0, s>>>(n, rpc, fA, lda, a, fB, ldb, b, sy, partial);
        else if (f64) k_tnl<double, 12><<<g, TNL_W * 64, 0, s>>>(n, rpc, fA, lda, a, fB, ldb, b, sy, partial);
        else if (per <= 6) k_tnl<float, 6><<<g, TNL_W * 64, 0, s>>>(n, rpc, fA, lda, a, fB, ldb, b, sy, partial);
        else if (per <= 12) k_tnl<float, 12><<<g, TNL_W * 64, 0, s>>>(n, rpc, fA, lda, a, fB, ldb, b, sy, partial);
        else k_tnl<float, 24><<<g, TNL_W * 64, 0, s>>>(n, rpc, fA, lda, a, fB, ldb, b, sy, partial);
        launch_reduce(g, red_job(partial, C, a, b, ldc), RedJob{nullptr, nullptr, 0, 0, 0, 0}, s);
        return;
      }
    }
  }
  if (A == B && lda == ldb && a == b && kind != 2 && ((a + 15) >> 4) > 4) {
    // a Gram wider than the symmetric kernel's 64 columns: its upper blocks of 64 columns
    // (the diagonal ones by the symmetric kernel), the lower blocks as their mirrors
    constexpr int SB = 64;
    for (int i0 = 0; i0 < a; i0 += SB)
      for (int j0 = i0; j0 < a; j0 += SB) {
        const int wi = std::min(SB, a - i0), wj = std::min(SB, a - j0);
        tn_run<T>(kind, n, A + i0, lda, wi, A + j0, lda, wj, partial, C + (size_t)i0 * ldc + j0, s, ldc);
        if (j0 > i0) k_mirror_block<<<(wi * wj + 255) / 256, 256, 0, s>>>(C, ldc, i0, j0, wi, wj);
      }
    return;
  }
  if (a > TW || b > TW) {
    // operands wider than the kernels hold: blocks of at most TW columns of each, one after
    // the other on the stream (they share the partial sums), each reduced into its block of C
    for (int a0 = 0; a0 < a; a0 += TW)
      for (int b0 = 0; b0 < b; b0 += TW)
        tn_run<T>(kind, n, A + a0, lda, std::min(TW, a - a0), B + b0, ldb, std::min(TW, b - b0), partial,
                  C + (size_t)a0 * ldc + b0, s, ldc);
    return;
  }
  const int g = tn_num_chunks(n);
  const int rb = kind == 2 ? 32 : 16;
  int64_t rpc = (n + g - 1) / g;
  rpc = ((rpc + rb - 1) / rb) * rb;
  if (kind == 2 && ((a + 15) >> 4) * ((b + 15) >> 4) > NW * BT) kind = 0;  // too many tiles: FP32 MFMA
  bool sym = (A == B && lda == ldb && a == b && kind != 2);
  if (kind == 2) {
    const int tt = std::max((((a + 15) >> 4) + 1) / 2, (((b + 15) >> 4) + 1) / 2);
    const bool staged = a % 4 == 0 && b % 4 == 0 && aligned16(A, lda) && aligned16(B, ldb);
    const float* fA = (const float*)A;
    const float* fB = (const float*)B;
    if (staged && tt <= 1) tn_bf16t_launch<1>(g, n, rpc, fA, lda, a, fB, ldb, b, partial, s);
    else if (staged && tt == 2) tn_bf16t_launch<2>(g, n, rpc, fA, lda, a, fB, ldb, b, partial, s);
    else if (staged && tt == 3) tn_bf16t_launch<3>(g, n, rpc, fA, lda, a, fB, ldb, b, partial, s);
    else if (staged && tt == 4) tn_bf16t_launch<4>(g, n, rpc, fA, lda, a, fB, ldb, b, partial, s);
    else k_tn_bf16<<<g, WG, 0, s>>>(n, rpc, fA, lda, a, fB, ldb, b, partial);
  } else if (kind == 1) {
    if (sym && ((a + 15) >> 4) > 4) sym = false;  // wide Gram: full product in slices
    tnw_dispatch<T, double>(n, g, rpc, A, lda, a, B, ldb, b, sym, partial, s);
  } else {
    if (sym && ((a + 15) >> 4) > 4) sym = false;
    tnw_dispatch<T, float>(n, g, rpc, A, lda, a, B, ldb, b, sym, partial, s);
  }
  launch_reduce(g, red_job(partial, C, a, b, ldc), RedJob{nullptr, nullptr, 0, 0, 0, 0}, s);
}

// one projection round: C = X^T W and G = W^T W (upper tiles; the reduce mirrors them)
template <typename T, typename Tcx, int TXC, int TWC>
static void pip_launch(int g, int64_t n, int64_t rpc, const T* X, int64_t ldx, int kx, const T* W, int64_t ldw,
                       int w, double* partC, double* partG, const int32_t* rows, const int64_t* nrows,
                       hipStream_t s) {
  constexpr int NTG = TWC * (TWC + 1) / 2;
  constexpr size_t lds = (size_t)(TXC * TWC + NTG) * 256 * sizeof(double);
  if (lds > 65536) {
    static const bool attr = [] {
      (void)hipFuncSetAttribute((const void*)k_pip<T, Tcx, TXC, TWC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      return true;
    }();
    (void)attr;
  }
  k_pip<T, Tcx, TXC, TWC><<<g, WG, lds, s>>>(n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows);
}

// the (kx / 16, w / 16) block shapes of the read pass
inline bool pip_shape(int tx, int tw) {
  return (tx == 2 && tw == 4) || (tx == 4 && tw == 2) || (tx == 3 && tw == 2) || (tx == 2 && tw == 1) ||
         (tx == 2 && tw == 2) || (tx == 1 && tw == 4) || (tx == 1 && tw == 2) || (tx == 1 && tw == 1);
}

template <typename T>
bool launch_pip(int64_t n, const T* X, int64_t ldx, int kx, const T* W, int64_t ldw, int w, double* partial,
                double* C, double* G, hipStream_t s, const int32_t* rows, const int64_t* nrows) {
  if (!rows) nrows = nullptr;
  const int TX = (kx + 15) >> 4, TWt = (w + 15) >> 4;
  const int g = tn_num_chunks(n);
  int64_t rpc = (n + g - 1) / g;
  rpc = ((rpc + 31) / 32) * 32;
  double* partC = partial;
  double* partG = partial + (size_t)g * kx * w;
  using Tcx = typename std::conditional<sizeof(T) == 8, double, float>::type;
  if (!pip_shape(TX, TWt)) return false;
  if (TX == 2 && TWt == 4) pip_launch<T, Tcx, 2, 4>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else if (TX == 4 && TWt == 2) pip_launch<T, Tcx, 4, 2>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else if (TX == 3 && TWt == 2) pip_launch<T, Tcx, 3, 2>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else if (TX == 2 && TWt == 1) pip_launch<T, Tcx, 2, 1>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else if (TX == 2 && TWt == 2) pip_launch<T, Tcx, 2, 2>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else if (TX == 1 && TWt == 4) pip_launch<T, Tcx, 1, 4>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else if (TX == 1 && TWt == 2) pip_launch<T, Tcx, 1, 2>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else if (TX == 1 && TWt == 1) pip_launch<T, Tcx, 1, 1>(g, n, rpc, X, ldx, kx, W, ldw, w, partC, partG, rows, nrows, s);
  else return false;
  launch_reduce(g, red_job(partC, C, kx, w), red_job(partG, G, w, w), s);
  return true;
}

template bool launch_pip<float>(int64_t, const float*, int64_t, int, const float*, int64_t, int, double*, double*,
                                double*, hipStream_t, const int32_t*, const int64_t*);
template bool launch_pip<double>(int64_t, const double*, int64_t, int, const double*, int64_t, int, double*,
                                 double*, double*, hipStream_t, const int32_t*, const int64_t*);

template <typename T, bool ACC64>
void launch_tn(int64_t n, const T* A, int64_t lda, int a, const T* B, int64_t ldb, int b, double* partial,
               double* C, hipStream_t s) {
  tn_run<T>((ACC64 || sizeof(T) == 8) ? 1 : 0, n, A, lda, a, B, ldb, b, partial, C, s);
}

void launch_tn_bf16(int64_t n, const float* A, int64_t lda, int a, const float* B, int64_t ldb, int b,
                    double* partial, double* C, hipStream_t s) {
  tn_run<float>(2, n, A, lda, a, B, ldb, b, partial, C, s);
}

template <typename T, typename Tc, bool VEC>
static void apply_launch(int64_t n, const T* In1, int64_t ld1, int a1, const T* In2, int64_t ld2, int a2,
                         const double* M, int b, double alpha, double beta, T* Out, int64_t ldout,
                         const int32_t* rows, const int64_t* nrows, hipStream_t s) {
  const int KB = (a1 + a2 + 15) >> 4, TB = (b + 15) >> 4;
  const size_t lds = (size_t)KB * 16 * (TB * 16 + 1) * sizeof(Tc);
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_apply<T, Tc, VEC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)((size_t)TW * (TW + 1) * sizeof(Tc)));
    return true;
  }();
  (void)attr;
  k_apply<T, Tc, VEC><<<apply_grid(n), WG, lds, s>>>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout,
                                                     rows, nrows);
}

template <typename T>
static void apply2_narrow(int64_t n, const T* In1, int64_t ld1, int a1, const T* In2, int64_t ld2, int a2,
                          const double* M, int b, double alpha, double beta, T* Out, int64_t ldout, hipStream_t s,
                          const int64_t* flag2, const int32_t* rows, const int64_t* nrows);

// whether columns [p, p + w) and [q, q + v) of row-major blocks with the same leading
// dimension share memory (the blocks start in the same row)
template <typename T>
static bool cols_overlap(const T* p, int w, const T* q, int v, int64_t ld, int64_t ldq) {
  if (ld != ldq || w <= 0 || v <= 0) return false;
  const int64_t d = q - p;
  return d > -(int64_t)v && d < (int64_t)w && d > -ld && d < ld;
}

template <typename T>
void launch_apply2(int64_t n, const T* In1, int64_t ld1, int a1, const T* In2, int64_t ld2, int a2,
                   const double* M, int b, double alpha, double beta, T* Out, int64_t ldout, hipStream_t s,
                   const int64_t* flag2, const int32_t* rows, const int64_t* nrows) {
  if (n <= 0 || b <= 0) return;
  if (a1 + a2 <= TW) {
    apply2_narrow<T>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, s, flag2, rows, nrows);
    return;
  }
  // A contraction wider than the kernel holds: Out = beta Out + alpha sum over blocks of at
  // most TW input columns (In1's, then In2's) of In_blk M_blk, the first launch with beta and
  // the others adding to Out.  A block whose columns Out overwrites (an in-place apply) goes
  // first, as one launch in place; every other block must not share memory with Out.
  struct Blk { const T* p; int64_t ld; int w; int row0; bool second; };
  Blk blk[8];
  int nb = 0;
  const int a = a1 + a2;
  const int c1s = (a - TW + 3) / 4 * 4;
  if (a2 > 0 && In2 == In1 + a1 && ld2 == ld1 && a <= 2 * TW && c1s < a && c1s <= TW &&
      cols_overlap(In1 + c1s, a - c1s, (const T*)Out, b, ld1, ldout) && !cols_overlap(In1, c1s, (const T*)Out, b, ld1, ldout)) {
    // In2 continues In1 in memory and Out lies in its last TW columns: two blocks, the last
    // TW columns (in place) and the rest, so that no block is a sliver that costs a whole
    // read-modify-write pass over Out
    const int c1 = (a - TW + 3) / 4 * 4;  // a multiple of four: both blocks keep 16-byte groups
    blk[nb++] = Blk{In1 + c1, ld1, a - c1, c1, false};
    blk[nb++] = Blk{In1, ld1, c1, 0, false};
  } else {
    for (int c0 = 0; c0 < a1 && nb < 8; c0 += TW) blk[nb++] = Blk{In1 + c0, ld1, std::min(TW, a1 - c0), c0, false};
    for (int c0 = 0; c0 < a2 && nb < 8; c0 += TW) blk[nb++] = Blk{In2 + c0, ld2, std::min(TW, a2 - c0), a1 + c0, true};
  }
  int first = -1;
  for (int q = 0; q < nb; ++q)
    if (cols_overlap(blk[q].p, blk[q].w, (const T*)Out, b, blk[q].ld, ldout)) first = q;
  double bt = beta;
  auto run = [&](const Blk& k) {
    apply2_narrow<T>(n, k.p, k.ld, k.w, k.p, k.ld, 0, M + (size_t)k.row0 * b, b, alpha, bt, Out, ldout, s,
                     nullptr, rows, nrows);
    bt = 1.0;
  };
  if (first >= 0) run(blk[first]);
  for (int q = 0; q < nb; ++q)
    if (q != first) run(blk[q]);
  (void)flag2;  // an optimisation only (skips reading zero rows of In2): every row is read here
}

template <typename T>
static void apply2_narrow(int64_t n, const T* In1, int64_t ld1, int a1, const T* In2, int64_t ld2, int a2,
                          const double* M, int b, double alpha, double beta, T* Out, int64_t ldout, hipStream_t s,
                          const int64_t* flag2, const int32_t* rows, const int64_t* nrows) {
  if (n <= 0 || b <= 0) return;
  if (!rows) nrows = nullptr;
  const bool vec = aligned16(In1, ld1) && (a2 == 0 || (aligned16(In2, ld2) && a1 % 4 == 0));
  if constexpr (sizeof(T) == 8) {
    if (vec) apply_launch<T, double, true>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, rows, nrows, s);
    else apply_launch<T, double, false>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, rows, nrows, s);
  } else {
    // 16-byte input groups wherever the input rows are aligned (a block's last group masked
    // past its end), 16-byte stores wherever the output rows are
    const bool vin = aligned16(In1, ld1) && (a2 == 0 || (aligned16(In2, ld2) && a1 % 4 == 0));
    const bool vout = aligned16(Out, ldout);
    if (vin && vout)
      apply_f32_dispatch<true, true>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s);
    else if (vin)
      apply_f32_dispatch<true, false>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s);
    else if (vout)
      apply_f32_dispatch<false, true>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s);
    else
      apply_f32_dispatch<false, false>(n, In1, ld1, a1, In2, ld2, a2, M, b, alpha, beta, Out, ldout, flag2, rows, nrows, s);
  }
}

template <typename T>
void launch_apply(int64_t n, const T* In, int64_t ldin, int a, const double* M, int b, double alpha,
                  double beta, T* Out, int64_t ldout, hipStream_t s) {
  launch_apply2<T>(n, In, ldin, a, In, ldin, 0, M, b, alpha, beta, Out, ldout, s);
}

template void launch_apply2<float>(int64_t, const float*, int64_t, int, const float*, int64_t, int, const double*,
                                   int, double, double, float*, int64_t, hipStream_t, const int64_t*,
                                   const int32_t*, const int64_t*);
template void launch_apply2<double>(int64_t, const double*, int64_t, int, const double*, int64_t, int,
                                    const double*, int, double, double, double*, int64_t, hipStream_t,
                                    const int64_t*, const int32_t*, const int64_t*);

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

// ---------------------------------------------------------------------------------
// The first CholQR round's apply fused with the second round's read pass, on FP32 blocks:
// W1 = [X | W] M1 for a 16-row tile as k_apply_f32 computes it (lane (g, c) holds row c,
// columns 16 jt + 4 g .. + 3), written to Out (which may be W: a row is read before it is
// written), and the tile's contributions to C = X^T W1 (FP32 MFMA) and G = W1^T W1 (FP64
// MFMA, upper tiles, mirrored on output), as k_pip accumulates them.  X and W1 reach the
// four-rows-per-step layout of those products through a per-wave LDS tile.  kx = 16 KBX,
// w = 16 NWB; W's blocks are skipped on a tile where flag2 marks no row (W is zero there).
// Each workgroup writes its partials for the fixed-order reduction.
// ---------------------------------------------------------------------------------
namespace {

template <int KBX, int NWB>
__global__ void __launch_bounds__(WG, 2) k_apply_pip(int64_t n, const float* __restrict__ X, int64_t ldx,
                                                  const float* W, int64_t ldw, const int64_t* __restrict__ flag2,
                                                  const double* __restrict__ M1, float* Out, int64_t ldout,
                                                  double* __restrict__ partC, double* __restrict__ partG) {
  constexpr int KB1 = KBX + NWB;
  constexpr int kx = 16 * KBX, w = 16 * NWB;
  constexpr int PT = kx + w + 4;  // pitch of the transposition tile (floats)
  constexpr int NTG = NWB * (NWB + 1) / 2;
  extern __shared__ double lds_raw[];
  f32x4* sM1 = reinterpret_cast<f32x4*>(lds_raw);
  float* tiles = reinterpret_cast<float*>(sM1 + KB1 * NWB * 64);
  // coefficients in the fragment order of k_apply_f32: [kb][jt][g][c] -> M1[16 kb + 4 g + m][16 jt + c]
  for (int idx = threadIdx.x; idx < KB1 * NWB * 64; idx += WG) {
    const int c = idx & 15, g = (idx >> 4) & 3, t = idx >> 6;
    const int kb = t / NWB, jt = t % NWB;
    f32x4 v;
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = (float)M1[(size_t)(kb * 16 + 4 * g + m) * w + jt * 16 + c];
    sM1[idx] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t ntile = (n + 15) >> 4;
  const int64_t stride = (int64_t)gridDim.x * NW;
  // fragments of [X | W] for row c16 of tile t; returns whether any row of the tile has W
  auto load = [&](int64_t t, f32x4(&f)[KB1]) __attribute__((always_inline)) {
    const int64_t row = t * 16 + c16;
    const bool ok = row < n;
    const bool use2 = ok && (!flag2 || flag2[row] != 0);
#pragma unroll
    for (int kb = 0; kb < KBX; ++kb)
      f[kb] = ok ? *reinterpret_cast<const f32x4*>(X + row * ldx + kb * 16 + 4 * g) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < NWB; ++kb)
      f[KBX + kb] = use2 ? *reinterpret_cast<const f32x4*>(W + row * ldw + kb * 16 + 4 * g)
                         : f32x4{0.f, 0.f, 0.f, 0.f};
    return __builtin_amdgcn_ballot_w64(use2) != 0;
  };
  typename Mma<float>::acc_t ac[KBX][NWB];
  typename Mma<double>::acc_t ag[NTG];
#pragma unroll
  for (int p = 0; p < KBX; ++p)
#pragma unroll
    for (int q = 0; q < NWB; ++q) ac[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < NTG; ++t) ag[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  float* tile = tiles + wid * 16 * PT;
  int64_t t = (int64_t)blockIdx.x * NW + wid;
  f32x4 fin[KB1];
  bool any2 = false;
  if (t < ntile) any2 = load(t, fin);
  for (; t < ntile; t += stride) {
    // X to the wave's tile (row c16)
#pragma unroll
    for (int kb = 0; kb < KBX; ++kb) *reinterpret_cast<f32x4*>(tile + c16 * PT + kb * 16 + 4 * g) = fin[kb];
    // W1 = [X | W] M1
    f32x4 w1[NWB];
#pragma unroll
    for (int jt = 0; jt < NWB; ++jt) w1[jt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
      if (kb >= KBX && !any2) break;
#pragma unroll
      for (int jt = 0; jt < NWB; ++jt) {
        const f32x4 mv = sM1[(kb * NWB + jt) * 64 + lane];
#pragma unroll
        for (int m = 0; m < 4; ++m) w1[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(mv[m], fin[kb][m], w1[jt], 0, 0, 0);
      }
    }
    const int64_t row = t * 16 + c16;
    // the next tile's fragments go into the same registers, in flight during the products
    if (t + stride < ntile) any2 = load(t + stride, fin);
    if (row < n) {
#pragma unroll
      for (int jt = 0; jt < NWB; ++jt) *reinterpret_cast<f32x4*>(Out + row * ldout + jt * 16 + 4 * g) = w1[jt];
    }
#pragma unroll
    for (int jt = 0; jt < NWB; ++jt) *reinterpret_cast<f32x4*>(tile + c16 * PT + kx + jt * 16 + 4 * g) = w1[jt];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll 1
    for (int s = 0; s < 4; ++s) {
      const float* tr = tile + (4 * s + g) * PT;
      float cx[KBX], cw[NWB];
#pragma unroll
      for (int p = 0; p < KBX; ++p) cx[p] = tr[p * 16 + c16];
#pragma unroll
      for (int q = 0; q < NWB; ++q) cw[q] = tr[kx + q * 16 + c16];
#pragma unroll
      for (int p = 0; p < KBX; ++p)
#pragma unroll
        for (int q = 0; q < NWB; ++q) ac[p][q] = Mma<float>::run(cx[p], cw[q], ac[p][q]);
#pragma unroll
      for (int p = 0; p < NWB; ++p)
#pragma unroll
        for (int q = p; q < NWB; ++q)
          ag[tri_idx(p, q, NWB)] = Mma<double>::run((double)cw[p], (double)cw[q], ag[tri_idx(p, q, NWB)]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // fixed-order sum of the four waves, then this workgroup's partials (the LDS of the
  // coefficients and tiles is reused once every wave is past its loop)
  __syncthreads();
  double* red = lds_raw;
  double* red2 = red + (size_t)KBX * NWB * 256;
  for (int v = 0; v < NW; ++v) {
    if (wid == v) {
#pragma unroll
      for (int p = 0; p < KBX; ++p)
#pragma unroll
        for (int q = 0; q < NWB; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = ((p * NWB + q) * 16 + Mma<float>::row(lane, r)) * 16 + c16;
            red[e] = (v == 0) ? (double)ac[p][q][r] : red[e] + (double)ac[p][q][r];
          }
#pragma unroll
      for (int tt = 0; tt < NTG; ++tt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = (tt * 16 + Mma<double>::row(lane, r)) * 16 + c16;
          red2[e] = (v == 0) ? ag[tt][r] : red2[e] + ag[tt][r];
        }
    }
    __syncthreads();
  }
  double* oc = partC + (size_t)blockIdx.x * kx * w;
  double* og = partG + (size_t)blockIdx.x * w * w;
  for (int e = threadIdx.x; e < KBX * NWB * 256; e += WG) {
    const int tt = e >> 8, i = (e >> 4) & 15, j = e & 15;
    oc[(size_t)((tt / NWB) * 16 + i) * w + (tt % NWB) * 16 + j] = red[e];
  }
  for (int e = threadIdx.x; e < NWB * NWB * 256; e += WG) {
    const int tt = e >> 8, i = (e >> 4) & 15, j = e & 15;
    const int p = tt / NWB, q = tt % NWB;
    const double v = p <= q ? red2[(tri_idx(p, q, NWB) * 16 + i) * 16 + j] : red2[(tri_idx(q, p, NWB) * 16 + j) * 16 + i];
    og[(size_t)(p * 16 + i) * w + q * 16 + j] = v;
  }
}

template <int KBX, int NWB>
void apply_pip_launch(int64_t n, const float* X, int64_t ldx, const float* W, int64_t ldw, const int64_t* flag2,
                      const double* M1, float* Out, int64_t ldout, double* partC, double* partG, int* grid_out,
                      hipStream_t s) {
  constexpr int KB1 = KBX + NWB;
  const size_t coef = (size_t)KB1 * NWB * 64 * 16;
  const size_t tiles = (size_t)NW * 16 * (16 * KB1 + 4) * sizeof(float);
  const size_t red = ((size_t)KBX * NWB + NWB * (NWB + 1) / 2) * 256 * sizeof(double);
  const size_t lds = std::max(coef + tiles, red);
  static std::atomic<int> occ_cache{0};
  int occ = occ_cache.load(std::memory_order_relaxed);
  if (occ <= 0) {
    (void)hipFuncSetAttribute((const void*)k_apply_pip<KBX, NWB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_apply_pip<KBX, NWB>, WG, lds) !=
            hipSuccess || nb < 1)
      nb = 1;
    occ = nb;
    occ_cache.store(occ, std::memory_order_relaxed);
  }
  const int64_t ntiles = (n + 15) / 16;
  int64_t g = std::min<int64_t>((ntiles + NW - 1) / NW, (int64_t)device_cus() * occ);
  if (g > CHUNKS) g = CHUNKS;  // one partial per workgroup
  if (g < 1) g = 1;
  *grid_out = (int)g;
  k_apply_pip<KBX, NWB><<<(unsigned)g, WG, lds, s>>>(n, X, ldx, W, ldw, flag2, M1, Out, ldout, partC, partG);
}

bool apply_pip_shape(int kxb, int wb) {
  return (kxb == 2 && wb == 4) || (kxb == 4 && wb == 2) || (kxb == 1 && wb == 2) || (kxb == 2 && wb == 1) ||
         (kxb == 1 && wb == 1) || (kxb == 2 && wb == 2) || (kxb == 1 && wb == 4) || (kxb == 4 && wb == 1);
}

}  // namespace

bool apply_pip_ok(const float* X, int64_t ldx, int kx, const float* W, int64_t ldw, int w, const float* Out,
                  int64_t ldout) {
  return kx > 0 && w > 0 && kx % 16 == 0 && w % 16 == 0 && apply_pip_shape(kx / 16, w / 16) && aligned16(X, ldx) &&
         aligned16(W, ldw) && aligned16(Out, ldout);
}

bool orth_reads_listed_rows_only(const float* X, int64_t ldx, int kx, const float* W, int64_t ldw, int w) {
  return apply_pip_ok(X, ldx, kx, W, ldw, w, W, ldw) && pip_shape((kx + 15) >> 4, (w + 15) >> 4);
}

bool launch_apply_pip(int64_t n, const float* X, int64_t ldx, int kx, const float* W, int64_t ldw, int w,
                      const int64_t* flag2, const double* M1, float* Out, int64_t ldout, double* partial, double* C,
                      double* G, hipStream_t s) {
  if (!apply_pip_ok(X, ldx, kx, W, ldw, w, Out, ldout) || n <= 0) return false;
  double* partC = partial;
  double* partG = partial + (size_t)CHUNKS * kx * w;
  int g = 0;
  const int a = kx / 16, b = w / 16;
#define GREST_AP(A, B)                                                                                  \
  if (a == A && b == B) apply_pip_launch<A, B>(n, X, ldx, W, ldw, flag2, M1, Out, ldout, partC, partG, &g, s); \
  else
  GREST_AP(2, 4) GREST_AP(4, 2) GREST_AP(1, 2) GREST_AP(2, 1) GREST_AP(1, 1) GREST_AP(2, 2) GREST_AP(1, 4)
  GREST_AP(4, 1) return false;
#undef GREST_AP
  launch_reduce(g, red_job(partC, C, kx, w), red_job(partG, G, w, w), s);
  return true;
}
