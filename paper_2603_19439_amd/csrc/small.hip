// FP64 kernels on the small matrices of the update:
//   * rank-revealing Cholesky with diagonal pivoting of a Gram matrix (the factor of
//     CholQR2); the inverse factor is returned as the matrix M that maps W to its
//     orthonormal basis W M;
//   * the dense symmetric eigensolver of the projected matrix (Alg. 1, small
//     eigenproblem) and of the sketch Gram B B^T of the randomized range finder
//     (Sec. 3.5), followed by the selection of the wanted pairs.
// The eigensolver runs as three launches:
//   1. one workgroup: Householder tridiagonalisation in LDS (each reflector written to a
//      global table, zero padded to the full row);
//   2. one wave per eigenvalue: multisection on the LDL^T inertia count, 64 probes per
//      step (one per lane), so that an eigenvalue is found in about nine steps;
//   3. one wave per selected pair: selection and inverse iteration with an LU
//      factorisation with partial pivoting of T - lambda I.  Pairs closer than 1e-7 ||T||
//      are computed one after the other by the wave of the lowest one, with
//      reorthogonalisation against the finished members;
//   4. one wave per selected pair: first-order symmetric orthogonalisation of the
//      selected tridiagonal-basis vectors, y_s <- y_s - (1/2) sum_t (y_t^T y_s) y_t, which
//      removes the eps ||T|| / gap overlap that independent inverse iterations leave
//      between neighbours, then the back-transform through the reflectors.
// Orders up to 128 are tridiagonalised with the matrix in registers; larger ones, up to
// TL_MAX = 196, with the lower triangle of the matrix packed in LDS (k_tridiag_lds).
#include <algorithm>

#include "grest_internal.h"

#include <math.h>

namespace {

constexpr int TRI_WAVES = 8;  // waves of the tridiagonalisation workgroup (two per SIMD)
constexpr int PCH_WAVES = 16;  // waves of the pivoted Cholesky workgroup
constexpr int MAXN = 256;  // order of the work layout (largest order: TL_MAX)
constexpr int NCOL = MAXN / GREST_WAVE;  // elements of a length-MAXN vector per lane
constexpr int TL_MAX = 196;              // largest order of the LDS-resident tridiagonalisation
constexpr double EPS = 2.220446049250313e-16;

// work layout of the eigensolver (doubles)
constexpr int W_HDR = 0;               // n, lo, hi, ||T||, pivmin, s1, seg2 (the index map)
constexpr int W_DG = 8;                // diagonal of T
constexpr int W_OD = W_DG + MAXN;      // off-diagonal of T
constexpr int W_E2 = W_OD + MAXN;      // squared off-diagonal
constexpr int W_HB = W_E2 + MAXN;      // reflector coefficients beta_k
constexpr int W_EV = W_HB + MAXN;      // eigenvalues of T, ascending
constexpr int W_FL = W_EV + MAXN;      // 1 for an output slot that holds a kept pair
constexpr int W_R = 2048;              // reflector k in row k (MAXN x MAXN), v_{k+1} = 1
constexpr int W_Y = W_R + MAXN * MAXN;  // tridiagonal-basis vectors of clustered pairs
constexpr int W_END = W_Y + MAXN * MAXN;

// ---- wave-level primitives (64 lanes, every lane active) ----
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over the wave, the same value in every lane: butterflies inside each row of 16
// lanes (quad swaps, half-row and row mirrors), then the four row sums.
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_max_d(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ double wave_min_d(double v) {
  v = fmin(v, dpp_d<0xB1>(v));
  v = fmin(v, dpp_d<0x4E>(v));
  v = fmin(v, dpp_d<0x141>(v));
  v = fmin(v, dpp_d<0x140>(v));
  return fmin(fmin(readlane_d(v, 0), readlane_d(v, 16)), fmin(readlane_d(v, 32), readlane_d(v, 48)));
}
// Orders LDS traffic of one wave across lanes (a write by one lane, then a read by another).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// 1/x to full precision: hardware estimate and two Newton steps.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// ------------------------------------------------------------------------------------
// Register-resident small matrices.  In the one-workgroup kernels below a matrix of order
// up to M (64 or 128) lives in registers: thread (wave w, lane l) holds rows
// i = w + 4 r (r < M / 4) at columns j = l + 64 c (c < M / 64), always addressed with
// compile-time indices.  A column j is gathered by the lane l = j mod 64 of every wave,
// which writes its registers at column block j / 64 to LDS; an element of a
// lane-distributed vector that a whole wave needs is read with readlane.
// ------------------------------------------------------------------------------------
template <int C>
__device__ __forceinline__ double pick(const double (&x)[C], int c) {
  double v = x[0];
#pragma unroll
  for (int q = 1; q < C; ++q) v = (c == q) ? x[q] : v;
  return v;
}
// element j of a vector held as x[c] at column lane + 64 c (j uniform)
template <int C>
__device__ __forceinline__ double vec_elem(const double (&x)[C], int j) {
  return readlane_d(pick<C>(x, j >> 6), j & (GREST_WAVE - 1));
}
// this wave's rows of column j (uniform) to buf[i]
template <int RW, int C, int NWV>
__device__ __forceinline__ void column_to_lds(const double (&A)[RW][C], int j, int wv, int n, double* buf) {
  const int lane = threadIdx.x & (GREST_WAVE - 1);
  if (lane == (j & (GREST_WAVE - 1))) {
    const int cj = j >> 6;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int i = wv + NWV * r;
      if (i < n) buf[i] = pick<C>(A[r], cj);
    }
  }
}
// The same for a buffer of NWV * RW entries whose entries past n are never used: every row
// is written (the rows past n hold zeros), so the writing lane issues its stores back to
// back instead of one branch per row.
template <int RW, int C, int NWV>
__device__ __forceinline__ void column_to_lds_full(const double (&A)[RW][C], int j, int wv, double* buf) {
  const int lane = threadIdx.x & (GREST_WAVE - 1);
  if (lane == (j & (GREST_WAVE - 1))) {
    const int cj = j >> 6;
#pragma unroll
    for (int r = 0; r < RW; ++r) buf[wv + NWV * r] = pick<C>(A[r], cj);
  }
}

// ------------------------------------------------------------------------------------
// pivoted Cholesky:  G(P) = R^T R  truncated at the first pivot <= (tol*scale)^2
// M[perm[a], j] = Rinv[a, j] for a <= j < rank, every other entry 0.
// ------------------------------------------------------------------------------------
// With a projection coefficient block C (kc x m) the factored matrix is the Gram of the
// projected block, G - C^T C (Pythagorean form of block Gram-Schmidt), the rank scale is
// taken from G itself (the block before projection), and the output is the stacked
// (kc + m) x m matrix [-C M; M], so that (W - X C) M = [X W] [-C M; M].
// Pivoting needs no row swaps: at step k column p = perm[k] of the current Schur
// complement (its row up to rounding) is gathered in LDS and kept there (it is
// R[k, .] R[k, k] by original index); every wave keeps the whole
// diagonal up to date, so all waves choose the same next pivot without an exchange, and
// one barrier per step suffices.  The inverse factor is formed as its transpose, whose
// rows are independent triangular solves, so that loop needs no barrier at all.
__device__ __forceinline__ bool chosen_bit(uint64_t c0, uint64_t c1, int j) {
  return j < 64 ? ((c0 >> j) & 1ull) : ((c1 >> (j - 64)) & 1ull);
}

template <int M, bool CL>
__device__ __forceinline__ void pchol_body(int m, const double* G, const double* Cg, int kc, double tol,
                                              double* Mout, int32_t* rank_out, int32_t* status,
                                              const int32_t* done, const int bx) {
  constexpr int NW = PCH_WAVES, EB = PCH_WAVES * GREST_WAVE;
  if (done && *done) return;  // the factor is already there (k_chol_np)
  constexpr int CC = M / GREST_WAVE, RW = M / NW, LP = M + 1;
  __shared__ double Rrow[M * LP];  // pivot rows by step (pitch M + 1); later X = R^{-1}
  __shared__ int perm[M], iperm[M];
  __shared__ double rdg[M], rdi[M];
  extern __shared__ double cdyn[];  // with CL: the coefficient block C (kc x m)
  double* Mblk = Mout + (size_t)kc * m;  // the m x m block of the output
  const int tid = threadIdx.x, lane = tid & (GREST_WAVE - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / GREST_WAVE);

  for (int j = tid; j < M; j += EB) iperm[j] = -1;
  if (CL) {
    for (int idx = tid; idx < kc * m; idx += EB) cdyn[idx] = Cg[idx];
    __syncthreads();
  }
  const double* Cp = CL ? cdyn : Cg;
  // S = sym(G) - C^T C in registers and its diagonal in every wave
  double S[RW][CC], d[CC];
  int bad = 0;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int i = wv + NW * r;
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int j = lane + GREST_WAVE * c;
      double g = 0.0;
      if (i < m && j < m) {
        g = 0.5 * (G[(size_t)i * m + j] + G[(size_t)j * m + i]);
        for (int l = 0; l < kc; ++l) g = fma(-Cp[(size_t)l * m + i], Cp[(size_t)l * m + j], g);
        if (!isfinite(g)) bad = 1;
      }
      S[r][c] = g;
    }
  }
  double mx = 0.0;
#pragma unroll
  for (int c = 0; c < CC; ++c) {
    const int j = lane + GREST_WAVE * c;
    double g = 0.0;
    if (j < m) {
      mx = fmax(mx, G[(size_t)j * m + j]);
      g = 0.5 * (G[(size_t)j * m + j] + G[(size_t)j * m + j]);
      for (int l = 0; l < kc; ++l) g = fma(-Cp[(size_t)l * m + j], Cp[(size_t)l * m + j], g);
    }
    d[c] = g;
  }
  if (bad) atomicOr(status, ST_NONFINITE);
  const double thr = tol * tol * fmax(1.0, wave_max_d(mx));
  __syncthreads();

  uint64_t ch0 = 0, ch1 = 0;
  int r = 0;
  for (int k = 0; k < m; ++k) {
    // pivot: the largest remaining diagonal; the key keeps the value's leading bits and
    // puts 127 - j in the last seven mantissa bits, so ties go to the lower position
    double key = -1.0;
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int j = lane + GREST_WAVE * c;
      if (j < m && !chosen_bit(ch0, ch1, j) && d[c] > 0.0)
        key = fmax(key, __longlong_as_double((__double_as_longlong(d[c]) & ~0x7FLL) | (long long)(127 - j)));
    }
    const double best = wave_max_d(key);
    if (!(best > 0.0)) break;
    const int p = 127 - (int)(__double_as_longlong(best) & 0x7F);
    const double piv = vec_elem<CC>(d, p);
    if (!(piv > thr)) break;  // also stops on NaN
    if (p < 64) ch0 |= 1ull << p; else ch1 |= 1ull << (p - 64);
    double* rowk = Rrow + k * LP;
    column_to_lds<RW, CC, NW>(S, p, wv, m, rowk);
    if (tid == 0) { perm[k] = p; iperm[p] = k; rdg[k] = piv; }  // square roots after the loop
    __syncthreads();
    double rp[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int j = lane + GREST_WAVE * c;
      rp[c] = j < m ? rowk[j] : 0.0;
    }
    const double ip = recip(piv);
    double f[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) f[q] = rowk[wv + NW * q];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int i = wv + NW * q;
      const double fq = (i < m && !chosen_bit(ch0, ch1, i)) ? f[q] * ip : 0.0;
#pragma unroll
      for (int c = 0; c < CC; ++c) S[q][c] = fma(-fq, rp[c], S[q][c]);
    }
#pragma unroll
    for (int c = 0; c < CC; ++c) d[c] = fma(-(rp[c] * ip), rp[c], d[c]);
    r = k + 1;
  }
  // X = R^{-1}, R[a][b] = Rrow[a][perm[b]] / sqrt(piv_a) (upper triangular in pivot
  // order).  Column j of X is an independent solve: for i descending, X[i][j] /= R[i][i],
  // then X[a][j] -= R[a][i] X[i][j] for a < i.
  for (int a = tid; a < M; a += EB) rdi[a] = a < r ? 1.0 / sqrt(rdg[a]) : 0.0;
  __syncthreads();
  {
    // Y = X^T in the distributed layout: row j of Y is column j of X, an independent solve
    double Y[RW][CC];
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
      for (int c = 0; c < CC; ++c) Y[q][c] = (wv + NW * q == lane + GREST_WAVE * c && wv + NW * q < r) ? 1.0 : 0.0;
    for (int i = r - 1; i >= 0; --i) {
      const int pi = perm[i], li = i & (GREST_WAVE - 1), ci = i >> 6;
      const double s = rdi[i];
      double ra[CC];
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int a = lane + GREST_WAVE * c;
        ra[c] = a < i ? Rrow[a * LP + pi] * rdi[a] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < RW; ++q) {
#pragma unroll
        for (int c = 0; c < CC; ++c) Y[q][c] = (c == ci && lane == li) ? Y[q][c] * s : Y[q][c];
        const double yi = vec_elem<CC>(Y[q], i);
#pragma unroll
        for (int c = 0; c < CC; ++c) Y[q][c] = fma(-ra[c], yi, Y[q][c]);
      }
    }
    __syncthreads();  // every read of Rrow is done; it now receives X
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int j = wv + NW * q;
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int a = lane + GREST_WAVE * c;
        if (a < r && j < m) {
          Rrow[a * LP + j] = Y[q][c];
          Mblk[(size_t)perm[a] * m + j] = Y[q][c];  // M[perm[a]][j] = X[a][j]
        }
      }
      if (j < m && iperm[j] < 0)  // rows of dropped columns are zero
        for (int t = lane; t < m; t += GREST_WAVE) Mblk[(size_t)j * m + t] = 0.0;
    }
  }
  __syncthreads();
  // -C M = -(C P) X: wave w takes rows l = l0 + 8 w + t of C (t < 8), lanes the columns;
  // X[a][j] is zero for a > j, so the sum runs over every a < r
  constexpr int LT = 8;
  for (int l0 = 0; l0 < kc; l0 += NW * LT) {
    const int lb = l0 + LT * wv;
    double acc[LT][CC];
#pragma unroll
    for (int t = 0; t < LT; ++t)
#pragma unroll
      for (int c = 0; c < CC; ++c) acc[t][c] = 0.0;
    for (int a = 0; a < r; ++a) {
      const int pa = __builtin_amdgcn_readfirstlane(perm[a]);
      double xa[CC];
#pragma unroll
      for (int c = 0; c < CC; ++c) xa[c] = Rrow[a * LP + lane + GREST_WAVE * c];
#pragma unroll
      for (int t = 0; t < LT; ++t) {
        const double cv = (lb + t < kc) ? Cp[(size_t)(lb + t) * m + pa] : 0.0;
#pragma unroll
        for (int c = 0; c < CC; ++c) acc[t][c] = fma(cv, xa[c], acc[t][c]);
      }
    }
#pragma unroll
    for (int t = 0; t < LT; ++t)
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int j = lane + GREST_WAVE * c;
        if (lb + t < kc && j < m) Mout[(size_t)(lb + t) * m + j] = -acc[t][c];
      }
  }
  if (tid == 0) *rank_out = r;
}

template <int M, bool CL>
__global__ void __launch_bounds__(PCH_WAVES * GREST_WAVE) k_pchol(int m, const double* G, const double* Cg, int kc, double tol,
                                              double* Mout, int32_t* rank_out, int32_t* status,
                                              const int32_t* done) {
  pchol_body<M, CL>(m, G, Cg, kc, tol, Mout, rank_out, status, done, (int)blockIdx.x);
}

// ------------------------------------------------------------------------------------
// Cholesky factor without pivoting, tried first in every CholQR round: the Gram matrix of
// a full-rank block (and of the second round, close to the identity on the columns the
// first round kept, which come first, and zero on the others) needs no pivoting for the
// factor itself; pivoting only decides the rank.  Same output as k_pchol with the
// identity permutation: S = G - C^T C =
// R^T R truncated at the first pivot <= thr, M = R^{-1} on the leading rank x rank block
// (zero elsewhere), preceded by the rows of -C M.  *done is set when this factor is valid:
// every pivot before the truncation is above thr and every diagonal entry left after it
// is at most thr (the truncation rule of the pivoted factor holds); otherwise it is
// cleared and the pivoted kernel runs.  S lives in LDS (upper triangle updated in place,
// one barrier per column), the inverse is formed row by row from the bottom (one barrier
// per row).  When S is within 1e-4 of the identity (Frobenius norm) M is instead the
// third-order polynomial approximation of S^(-1/2) (full rank; see the body).
// ------------------------------------------------------------------------------------
constexpr int CNP_M = 64, CNP_T = 256, CNP_P = CNP_M + 1;
constexpr size_t kCnpDynMax = (size_t)CNP_M * CNP_M * sizeof(double);  // the block C (kc <= 64)

__device__ __forceinline__ void chol_np_body(int m, const double* __restrict__ G, const double* __restrict__ Cg,
                                                  int kc, double tol, double* __restrict__ Mout,
                                                  int32_t* rank_out, int32_t* done, const int bx) {
  constexpr int NB = CNP_M / 16;  // a thread's rows (and columns) on a 16 x 16 thread grid
  // Each thread keeps its 4 x 4 entries (rows ty + 16 a, columns tx + 16 b) of S, later of
  // X = R^{-1}, in registers; what the other threads need goes through LDS one row at a
  // time: row j of the Schur complement at step j (Rr[j] = R[j][.] R[j][j]), and the
  // finished rows of X (Xr).
  __shared__ double Rr[CNP_M * CNP_P];
  __shared__ double Xr[CNP_M * CNP_P];
  __shared__ double rdi[CNP_M];
  __shared__ double red[CNP_T / GREST_WAVE], red2[CNP_T / GREST_WAVE];
  __shared__ int s_bad;
  extern __shared__ double Cs[];  // C (kc x m)
  const int tid = threadIdx.x, lane = tid & (GREST_WAVE - 1), wv = tid / GREST_WAVE;
  const int ty = tid >> 4, tx = tid & 15;
  if (tid == 0) s_bad = 0;
  for (int idx = tid; idx < kc * m; idx += CNP_T) Cs[idx] = Cg[idx];
  __syncthreads();
  // S = sym(G) - C^T C
  double v[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = ty + 16 * a, j = tx + 16 * b;
      v[a][b] = (i < m && j < m) ? 0.5 * (G[(size_t)i * m + j] + G[(size_t)j * m + i]) : 0.0;
    }
  for (int l = 0; l < kc; ++l) {
    double ci[NB], cj[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      ci[a] = Cs[l * m + (ty + 16 * a < m ? ty + 16 * a : 0)];
      cj[a] = Cs[l * m + (tx + 16 * a < m ? tx + 16 * a : 0)];
      ci[a] = ty + 16 * a < m ? ci[a] : 0.0;
      cj[a] = tx + 16 * a < m ? cj[a] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) v[a][b] = fma(-ci[a], cj[b], v[a][b]);
  }
  {
    int bad = 0;
    double mx = 0.0, e2 = 0.0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = ty + 16 * a, j = tx + 16 * b;
        if (i < m && j < m) {
          if (!isfinite(v[a][b])) bad = 1;
          if (i == j) mx = fmax(mx, G[(size_t)i * m + i]);
          const double e = v[a][b] - (i == j ? 1.0 : 0.0);
          e2 = fma(e, e, e2);
        }
      }
    mx = wave_max_d(mx);
    e2 = wave_sum_d(e2);
    if (lane == 0) { red[wv] = mx; red2[wv] = e2; }
    if (bad) s_bad = 1;
    if (ty < 2)  // rows 0 and 1, the first pair's
#pragma unroll
      for (int b = 0; b < NB; ++b) Rr[ty * CNP_P + tx + 16 * b] = v[0][b];
  }
  __syncthreads();
  double gmx = 0.0, ef2 = 0.0;
  for (int q = 0; q < CNP_T / GREST_WAVE; ++q) {
    gmx = fmax(gmx, red[q]);
    ef2 += red2[q];
  }
  const double thr = tol * tol * fmax(1.0, gmx);
  if (s_bad) {  // leave the non-finite report to the pivoted kernel
    if (tid == 0) *done = 0;
    return;
  }
  // A block that is already orthonormal to within ||S - I||_F <= 1e-4 (the second round of
  // CholQR2, whose input the first round has orthonormalised; then every eigenvalue of S
  // lies in 1 +- 1e-4 and no column is dropped) takes M = p(S), the Taylor polynomial of
  // S^(-1/2) about I to third order: p(S) = I - E/2 + 3E^2/8 - 5E^3/16 with E = S - I.  M
  // is a polynomial in S, so M^T S M = S p(S)^2 = I - (35/64) E^4 + O(E^5), within 6e-17
  // of I, and W M spans what W spans; two products of order m replace the factor and
  // the triangular inverse with their one barrier per row.
  if (m > 0 && ef2 <= 1e-8) {
    // E to Rr, E^2 to Xr, then E^3 from both
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = ty + 16 * a, j = tx + 16 * b;
        Rr[i * CNP_P + j] = (i < m && j < m) ? v[a][b] - (i == j ? 1.0 : 0.0) : 0.0;
      }
    __syncthreads();
    double e2m[NB][NB], e3m[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) { e2m[a][b] = 0.0; e3m[a][b] = 0.0; }
    for (int q = 0; q < m; ++q) {
      double ei[NB], eq[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        ei[a] = Rr[(ty + 16 * a) * CNP_P + q];
        eq[a] = Rr[q * CNP_P + tx + 16 * a];
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) e2m[a][b] = fma(ei[a], eq[b], e2m[a][b]);
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) Xr[(ty + 16 * a) * CNP_P + tx + 16 * b] = e2m[a][b];
    __syncthreads();
    for (int q = 0; q < m; ++q) {
      double ei[NB], xq[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        ei[a] = Rr[(ty + 16 * a) * CNP_P + q];
        xq[a] = Xr[q * CNP_P + tx + 16 * a];
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) e3m[a][b] = fma(ei[a], xq[b], e3m[a][b]);
    }
    double* Mblk = Mout + (size_t)kc * m;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = ty + 16 * a, j = tx + 16 * b;
        const double e = Rr[i * CNP_P + j];
        double mij = fma(-0.3125, e3m[a][b], 0.375 * e2m[a][b]);
        mij = fma(-0.5, e, mij) + (i == j ? 1.0 : 0.0);
        v[a][b] = (i < m && j < m) ? mij : 0.0;
        if (i < m && j < m) Mblk[(size_t)i * m + j] = v[a][b];
      }
    __syncthreads();  // every read of E^2 is done
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) Xr[(ty + 16 * a) * CNP_P + tx + 16 * b] = v[a][b];
    __syncthreads();
    // rows of -C M
    for (int l0 = 0; l0 < kc; l0 += CNP_M) {
      double acc[NB][NB];
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = 0.0;
      for (int q = 0; q < m; ++q) {
        double cl[NB], xq[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          const int l = l0 + ty + 16 * a;
          cl[a] = Cs[(l < kc ? l : 0) * m + q];
          cl[a] = l < kc ? cl[a] : 0.0;
          xq[a] = Xr[q * CNP_P + tx + 16 * a];
        }
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[a][b] = fma(cl[a], xq[b], acc[a][b]);
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int l = l0 + ty + 16 * a, j = tx + 16 * b;
          if (l < kc && j < m) Mout[(size_t)l * m + j] = -acc[a][b];
        }
    }
    if (tid == 0) {
      *rank_out = m;
      *done = 1;
    }
    return;
  }
  // right-looking factor: step j subtracts S[i][j] S[j][k] / S[j][j] (i, k > j), with
  // S[i][j] = S[j][i] read from row j.  Two steps per barrier: rows j and j + 1 of the
  // Schur complement before step j are in LDS, and every thread forms row j + 1 after
  // step j itself (the same fma as the update), so the pair applies both rank-1 updates
  // in the order and rounding of two single steps.  Row j + 1's final values (its factor
  // row) stay in the registers of its owners and go to LDS after the loop: no later step
  // changes them, and writing them during the pair would race with its readers.
  int r = m;
  for (int j = 0; j < m; j += 2) {
    const double* r0 = Rr + j * CNP_P;
    const double d0 = r0[j];
    if (!(d0 > thr)) { r = j; break; }
    const double inv0 = recip(d0);
    const bool has1 = j + 1 < m;
    const double* r1 = Rr + (has1 ? j + 1 : j) * CNP_P;
    const double c10 = has1 ? r0[j + 1] * inv0 : 0.0;
    const double d1 = has1 ? fma(-c10, r0[j + 1], r1[j + 1]) : 0.0;
    const bool two = has1 && d1 > thr;
    const double inv1 = two ? recip(d1) : 0.0;
    double f0[NB], g0[NB], f1[NB], g1[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = ty + 16 * a, k = tx + 16 * a;
      const double a0i = r0[i], a0k = r0[k], a1i = r1[i], a1k = r1[k];
      f0[a] = (i > j && i < m) ? a0i * inv0 : 0.0;
      g0[a] = (k > j && k < m) ? a0k : 0.0;
      f1[a] = (two && i > j + 1 && i < m) ? fma(-c10, a0i, a1i) * inv1 : 0.0;
      g1[a] = (two && k > j + 1 && k < m) ? fma(-c10, a0k, a1k) : 0.0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) v[a][b] = fma(-f0[a], g0[b], v[a][b]);
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) v[a][b] = fma(-f1[a], g1[b], v[a][b]);
    // rows j + 2 and j + 3 for the next pair (not read by this one)
#pragma unroll
    for (int a = 0; a < NB; ++a)
      if (ty + 16 * a == j + 2 || ty + 16 * a == j + 3)
#pragma unroll
        for (int b = 0; b < NB; ++b) Rr[(ty + 16 * a) * CNP_P + tx + 16 * b] = v[a][b];
    __syncthreads();
    if (!two) {  // row j + 1 fails the rank rule (or there is none)
      if (has1) r = j + 1;
      break;
    }
  }
  // the second rows of the pairs: their factor rows from the registers
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int q = ty + 16 * a;
    if ((q & 1) && q < r)
#pragma unroll
      for (int b = 0; b < NB; ++b) Rr[q * CNP_P + tx + 16 * b] = v[a][b];
  }
  __syncthreads();
  // valid only if every diagonal entry left is at most thr
  for (int j = tid; j < r; j += CNP_T) rdi[j] = 1.0 / sqrt(Rr[j * CNP_P + j]);
  bool ok = true;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = ty + 16 * a;
      if (i == tx + 16 * b && i >= r && i < m && v[a][b] > thr) ok = false;
    }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  if (!ok) s_bad = 1;
  __syncthreads();
  if (s_bad) {
    if (tid == 0) *done = 0;
    return;
  }
  // X = R^{-1} by rows from the bottom.  X starts as I; at step k row k has all its terms,
  // X[k][c] = B[k][c] / R[k][k], and every row i < k subtracts R[i][k] X[k][c]; the
  // division of each row by its R[i][i] comes at the end.
  // Two steps per barrier, as in the factor: rows k and k - 1 of X before step k are in
  // LDS, every thread forms row k - 1 after step k itself, and the final values of the
  // pairs' second rows go to LDS after the loop.
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) v[a][b] = (ty + 16 * a == tx + 16 * b) ? 1.0 : 0.0;
#pragma unroll
  for (int a = 0; a < NB; ++a)
    if (ty + 16 * a < r && ty + 16 * a >= r - 2)
#pragma unroll
      for (int b = 0; b < NB; ++b) Xr[(ty + 16 * a) * CNP_P + tx + 16 * b] = v[a][b];
  __syncthreads();
  for (int k = r - 1; k > 0; k -= 2) {
    const bool has1 = k > 1;  // step k - 1 (rows below k - 1) exists
    const double rk = rdi[k];
    const double rk1 = rdi[k - 1];
    const double fkk1 = Rr[(k - 1) * CNP_P + k] * rdi[k - 1] * rk;  // row k - 1's multiplier in step k
    double f0[NB], x0[NB], f1[NB], x1[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = ty + 16 * a, c = tx + 16 * a;
      const int i0 = i < k ? i : 0, i1 = i < k - 1 ? i : 0;
      f0[a] = Rr[i0 * CNP_P + k] * rdi[i0];
      f1[a] = Rr[i1 * CNP_P + k - 1] * rdi[i1];
      const double xkc = Xr[k * CNP_P + c], xk1c = Xr[(k - 1) * CNP_P + c];
      f0[a] = i < k ? f0[a] * rk : 0.0;
      x0[a] = (c >= k && c < r) ? xkc : 0.0;
      f1[a] = (has1 && i < k - 1) ? f1[a] * rk1 : 0.0;
      x1[a] = (has1 && c >= k - 1 && c < r) ? fma(-fkk1, x0[a], xk1c) : 0.0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) v[a][b] = fma(-f0[a], x0[b], v[a][b]);
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) v[a][b] = fma(-f1[a], x1[b], v[a][b]);
    // rows k - 2 and k - 3 for the next pair (not read by this one)
#pragma unroll
    for (int a = 0; a < NB; ++a)
      if (ty + 16 * a == k - 2 || ty + 16 * a == k - 3)
#pragma unroll
        for (int b = 0; b < NB; ++b) Xr[(ty + 16 * a) * CNP_P + tx + 16 * b] = v[a][b];
    __syncthreads();
  }
  // the pairs' second rows k - 1 (rows r - 2, r - 4, ...): final from the registers
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int q = ty + 16 * a;
    if (q <= r - 2 && ((r - q) & 1) == 0)
#pragma unroll
      for (int b = 0; b < NB; ++b) Xr[q * CNP_P + tx + 16 * b] = v[a][b];
  }
  __syncthreads();
  // output: rows of -C M, then M (zero outside the leading r x r upper triangle)
  double* Mblk = Mout + (size_t)kc * m;
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int i = ty + 16 * a;
    const double ri = i < r ? rdi[i] : 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = tx + 16 * b;
      if (i < m && j < m) Mblk[(size_t)i * m + j] = (i <= j && j < r) ? v[a][b] * ri : 0.0;
    }
  }
  for (int l0 = 0; l0 < kc; l0 += CNP_M) {
    double acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = 0.0;
#pragma unroll 4
    for (int q = 0; q < r; ++q) {
      const double rq = rdi[q];
      double cl[NB], xq[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int l = l0 + ty + 16 * a, j = tx + 16 * a;
        cl[a] = Cs[(l < kc ? l : 0) * m + q];
        xq[a] = Xr[q * CNP_P + j];
        cl[a] = l < kc ? cl[a] : 0.0;
        xq[a] = (j >= q && j < r) ? xq[a] * rq : 0.0;
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = fma(cl[a], xq[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int l = l0 + ty + 16 * a, j = tx + 16 * b;
        if (l < kc && j < m) Mout[(size_t)l * m + j] = -acc[a][b];
      }
  }
  if (tid == 0) {
    *rank_out = r;
    *done = 1;
  }
}

__global__ void __launch_bounds__(CNP_T) k_chol_np(int m, const double* __restrict__ G, const double* __restrict__ Cg,
                                                  int kc, double tol, double* __restrict__ Mout,
                                                  int32_t* rank_out, int32_t* done) {
  chol_np_body(m, G, Cg, kc, tol, Mout, rank_out, done, (int)blockIdx.x);
}

// ------------------------------------------------------------------------------------
// 1. tridiagonalisation T = Q^T A Q, Q = P_0 ... P_{n-3}, P_k = I - beta_k v_k v_k^T
// The tridiagonal T (diagonal sdg, off-diagonal sod, reflector coefficients shb, all of
// order n) to the work table with the Gershgorin interval, the norm and the pivot floor of
// the inertia counts, and the index map of the reduced matrix; run by one wave.
__device__ void tridiag_finish(int n, int s1, int seg2, const double* sdg, const double* sod, const double* shb,
                               double* work) {
  const int lane = threadIdx.x & (GREST_WAVE - 1);
  double lo = INFINITY, hi = -INFINITY, tn = 0.0, emax = 0.0;
  for (int i = lane; i < n; i += GREST_WAVE) {
    const double r = (i > 0 ? fabs(sod[i - 1]) : 0.0) + (i + 1 < n ? fabs(sod[i]) : 0.0);
    lo = fmin(lo, sdg[i] - r);
    hi = fmax(hi, sdg[i] + r);
    tn = fmax(tn, fabs(sdg[i]) + r);
    const double e2 = (i + 1 < n) ? sod[i] * sod[i] : 0.0;
    emax = fmax(emax, e2);
    work[W_DG + i] = sdg[i];
    work[W_OD + i] = (i + 1 < n) ? sod[i] : 0.0;
    work[W_E2 + i] = e2;
    work[W_HB + i] = shb[i];
  }
  lo = wave_min_d(lo);
  hi = wave_max_d(hi);
  tn = wave_max_d(tn);
  emax = wave_max_d(emax);
  if (lane == 0) {
    if (n == 0) { lo = 0.0; hi = 0.0; }
    const double pad = 4.0 * EPS * fmax(tn, 1e-300) + 1e-300;
    work[W_HDR + 0] = (double)n;
    work[W_HDR + 1] = lo - pad;
    work[W_HDR + 2] = hi + pad;
    work[W_HDR + 3] = tn;
    work[W_HDR + 4] = 1e-290 * fmax(1.0, emax);
    work[W_HDR + 5] = (double)s1;
    work[W_HDR + 6] = (double)seg2;
  }
}

// ------------------------------------------------------------------------------------
// A lives in registers (see above).  Iteration k:
//   every wave holds column k in registers and forms the reflector itself (identical
//   arithmetic in every wave, so nothing needs to be published); v is zero outside rows
//   k+1 .. n-1, so the full-width updates below
//   leave the rest of A unchanged;
//   p = beta A v: each wave sums over its rows (symmetry turns row sums into column
//   sums), the per-wave partial vectors meet in LDS and are summed in a fixed order;
//   w = p - (beta p^T v / 2) v;  A <- A - v w^T - w v^T in registers;
//   column k+1 of A before the reflection is published with the partial sums, and every
//   wave forms the reflected column k+1 from it and v, w itself.
// One barrier per iteration (the LDS buffers alternate with k).
// The matrix reduced is H restricted to the index set [0, s1) + [seg2, seg2 + r2) with
// s1 = base + rank_p[0] and r2 = rank2_p[0] (the kept columns of a basis made of two
// packed blocks); index i of the reduced matrix is H index i for i < s1, else
// seg2 + i - s1.  The back-transform writes F through the same map.
template <int M>
__device__ __forceinline__ void tridiag_body(int d_full, int base, const int32_t* rank_p,
                                                                    int seg2, const int32_t* rank2_p,
                                                                    const double* H, double* work,
                                                                    int32_t* status, const int bx) {
  constexpr int NW = TRI_WAVES;
  constexpr int C = M / GREST_WAVE, RW = M / NW;
  __shared__ double pwv[2][NW][M];
  __shared__ double colb[2][M];
  __shared__ double vwb[NW][2][M];  // each wave's own copy of v and w
  __shared__ double sdg[M], sod[M], shb[M];
  const int tid = threadIdx.x, lane = tid & (GREST_WAVE - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / GREST_WAVE);
  int s1 = base + (rank_p ? rank_p[0] : 0);
  s1 = s1 < 0 ? 0 : (s1 > d_full ? d_full : s1);
  int r2 = rank2_p ? rank2_p[0] : 0;
  if (!rank2_p) seg2 = s1;
  if (seg2 < s1) seg2 = s1;
  r2 = r2 < 0 ? 0 : (r2 > d_full - seg2 ? d_full - seg2 : r2);
  int n = s1 + r2;
  if (n > M) n = M;
  auto mp = [&](int i) { return i < s1 ? i : seg2 + (i - s1); };
  double* R = work + W_R;

  double A[RW][C];
  int bad = 0;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int i = wv + NW * r;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = lane + GREST_WAVE * c;
      double h = 0.0;
      if (i < n && j < n) {
        const int mi = mp(i), mj = mp(j);
        h = 0.5 * (H[(size_t)mi * d_full + mj] + H[(size_t)mj * d_full + mi]);
        if (!isfinite(h)) { bad = 1; h = 0.0; }
      }
      A[r][c] = h;
    }
  }
  if (bad) atomicOr(status, ST_NONFINITE_H);
  // column k of the current matrix is kept in registers by every wave (colk); column 0 is
  // gathered through LDS once
  if (n >= 1) column_to_lds_full<RW, C, NW>(A, 0, wv, colb[1]);
  __syncthreads();
  double colk[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int j = lane + GREST_WAVE * c;
    colk[c] = j < n ? colb[1][j] : 0.0;
  }

  for (int k = 0; k + 2 < n; ++k) {
    const int pb = k & 1;
    // reflector annihilating column k below k+1
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = lane + GREST_WAVE * c;
      const double xc = (j > k + 1 && j < n) ? colk[c] : 0.0;
      s2 = fma(xc, xc, s2);
    }
    const double x0 = vec_elem<C>(colk, k + 1);
    const double sigma = wave_sum_d(s2);
    double beta = 0.0, v0 = 1.0, ek = x0;
    if (sigma > 0.0) {
      const double mu = sqrt(x0 * x0 + sigma);
      v0 = (x0 <= 0.0) ? (x0 - mu) : (-sigma * recip(x0 + mu));
      beta = 2.0 * v0 * v0 * recip(sigma + v0 * v0);
      ek = mu;
    }
    const double inv = recip(v0);
    double v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = lane + GREST_WAVE * c;
      v[c] = (j == k + 1) ? 1.0 : ((j > k + 1 && j < n) ? colk[c] * inv : 0.0);
    }
    if (wv == 0) {
      const double dk = vec_elem<C>(colk, k);
#pragma unroll
      for (int c = 0; c < C; ++c) R[(size_t)k * MAXN + lane + GREST_WAVE * c] = v[c];
#pragma unroll
      for (int c = C; c < NCOL; ++c) R[(size_t)k * MAXN + lane + GREST_WAVE * c] = 0.0;
      if (lane == 0) { sdg[k] = dk; sod[k] = ek; shb[k] = beta; }
    }
    double vr[RW];
    if (beta != 0.0) {
#pragma unroll
      for (int c = 0; c < C; ++c) vwb[wv][0][lane + GREST_WAVE * c] = v[c];
      wave_lds_fence();
#pragma unroll
      for (int r = 0; r < RW; ++r) vr[r] = vwb[wv][0][wv + NW * r];
      double pp[C];
#pragma unroll
      for (int c = 0; c < C; ++c) pp[c] = 0.0;
      // rows and columns outside the active block have v = 0: no branches needed
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) pp[c] = fma(A[r][c], vr[r], pp[c]);
#pragma unroll
      for (int c = 0; c < C; ++c) pwv[pb][wv][lane + GREST_WAVE * c] = pp[c];
    }
    // column k+1 before this reflection, for the next reflector
    column_to_lds_full<RW, C, NW>(A, k + 1, wv, colb[pb]);
    __syncthreads();  // the only barrier of the step (buffers alternate with k)
    if (beta != 0.0) {
      double w[C];  // first p = beta A v, then w = p - K v
      double pv = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int j = lane + GREST_WAVE * c;
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) sum += pwv[pb][q][j];
        w[c] = (j > k && j < n) ? beta * sum : 0.0;
        pv = fma(w[c], v[c], pv);
      }
      const double Kc = 0.5 * beta * wave_sum_d(pv);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        w[c] = fma(-Kc, v[c], w[c]);
        vwb[wv][1][lane + GREST_WAVE * c] = w[c];
      }
      wave_lds_fence();
      double wr[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) wr[r] = vwb[wv][1][wv + NW * r];
      // v and w vanish outside rows/cols k+1 .. n-1, so the update leaves the rest as is
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) A[r][c] = fma(-vr[r], w[c], fma(-wr[r], v[c], A[r][c]));
      // the next column after the reflection: a[:, k+1] - v w[k+1] - w (v[k+1] = 1)
      const double wk1 = vec_elem<C>(w, k + 1);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int j = lane + GREST_WAVE * c;
        colk[c] = j < n ? colb[pb][j] - fma(v[c], wk1, w[c]) : 0.0;
      }
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int j = lane + GREST_WAVE * c;
        colk[c] = j < n ? colb[pb][j] : 0.0;
      }
    }
  }
  // the last two diagonal entries and the last off-diagonal one: column n-2 is colk, then
  // column n-1 is gathered
  __syncthreads();  // every read of colb in the loop is done
  if (n >= 2) {
    const double d2 = vec_elem<C>(colk, n - 2), e2 = vec_elem<C>(colk, n - 1);
    if (tid == 0) { sdg[n - 2] = d2; sod[n - 2] = e2; shb[n - 2] = 0.0; }
    column_to_lds_full<RW, C, NW>(A, n - 1, wv, colb[0]);
    __syncthreads();
    if (tid == 0) { sdg[n - 1] = colb[0][n - 1]; sod[n - 1] = 0.0; shb[n - 1] = 0.0; }
  } else if (n == 1) {
    const double d0 = vec_elem<C>(colk, 0);
    if (tid == 0) { sdg[0] = d0; sod[0] = 0.0; shb[0] = 0.0; }
  }
  __syncthreads();
  if (wv == 0) tridiag_finish(n, s1, seg2, sdg, sod, shb, work);
}

template <int M>
__global__ void __launch_bounds__(TRI_WAVES * GREST_WAVE) k_tridiag(int d_full, int base, const int32_t* rank_p,
                                                                    int seg2, const int32_t* rank2_p,
                                                                    const double* H, double* work,
                                                                    int32_t* status) {
  tridiag_body<M>(d_full, base, rank_p, seg2, rank2_p, H, work, status, (int)blockIdx.x);
}

// Householder tridiagonalisation of orders above 128 (up to TL_MAX), with the same
// reflector convention and outputs as k_tridiag: the lower triangle of the matrix lives in
// LDS, packed by rows (row i holds columns 0..i at offset i (i + 1) / 2), and one
// workgroup of 1024 threads works on it.  Each step forms the reflector of the column
// below the diagonal (a block sum of squares), p = beta A v with four threads per row of
// the trailing block (reading the packed triangle by rows left of the diagonal and by
// columns right of it), the correction K = beta / 2 (beta p)^T v (a block sum), w = beta p
// - K v, and the rank-two update A -= v w^T + w v^T of the trailing triangle, again four
// threads per row.  The block sums add the per-wave sums in a fixed order.
constexpr int TL_THREADS = 1024;
constexpr int TL_WAVES = TL_THREADS / GREST_WAVE;
constexpr size_t TL_LDS = ((size_t)TL_MAX * (TL_MAX + 1) / 2 + 2 * TL_MAX + TL_WAVES) * sizeof(double);

__device__ __forceinline__ int tri_at(int i, int j) { return (i * (i + 1)) / 2 + j; }  // i >= j

// sum of v over the workgroup, the same in every thread (red: TL_WAVES doubles)
__device__ __forceinline__ double tl_block_sum(double v, double* red) {
  v = wave_sum_d(v);
  __syncthreads();  // earlier readers of red are done
  if ((threadIdx.x & (GREST_WAVE - 1)) == 0) red[threadIdx.x / GREST_WAVE] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < TL_WAVES; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ void tridiag_lds_body(int d_full, int base, const int32_t* rank_p, int seg2,
                                                            const int32_t* rank2_p, const double* H, double* work,
                                                            int32_t* status, const int bx) {
  extern __shared__ double tl_smem[];
  double* L = tl_smem;                           // packed lower triangle
  double* vb = L + TL_MAX * (TL_MAX + 1) / 2;    // v
  double* wb = vb + TL_MAX;                      // w
  double* red = wb + TL_MAX;                     // per-wave sums
  __shared__ double sdg[TL_MAX], sod[TL_MAX], shb[TL_MAX];
  const int tid = threadIdx.x, lane = tid & (GREST_WAVE - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / GREST_WAVE);
  int s1 = base + (rank_p ? rank_p[0] : 0);
  s1 = s1 < 0 ? 0 : (s1 > d_full ? d_full : s1);
  int r2 = rank2_p ? rank2_p[0] : 0;
  if (!rank2_p) seg2 = s1;
  if (seg2 < s1) seg2 = s1;
  r2 = r2 < 0 ? 0 : (r2 > d_full - seg2 ? d_full - seg2 : r2);
  int n = s1 + r2;
  if (n > TL_MAX) n = TL_MAX;
  auto mp = [&](int i) { return i < s1 ? i : seg2 + (i - s1); };
  double* R = work + W_R;
  int bad = 0;
  for (int i = wv; i < n; i += TL_WAVES) {
    const int mi = mp(i);
    for (int j = lane; j <= i; j += GREST_WAVE) {
      const int mj = mp(j);
      double h = 0.5 * (H[(size_t)mi * d_full + mj] + H[(size_t)mj * d_full + mi]);
      if (!isfinite(h)) { bad = 1; h = 0.0; }
      L[tri_at(i, j)] = h;
    }
  }
  if (bad) atomicOr(status, ST_NONFINITE_H);
  __syncthreads();
  const int q = tid & 3;   // quarter of a row
  const int row = tid >> 2;  // the row of this thread's quad
  for (int k = 0; k + 2 < n; ++k) {
    const int j2 = k + 2 + tid;
    double part = 0.0;
    if (j2 < n) {
      const double x = L[tri_at(j2, k)];
      part = x * x;
    }
    const double sigma = tl_block_sum(part, red);
    const double x0 = L[tri_at(k + 1, k)];
    double beta = 0.0, v0 = 1.0, ek = x0;
    if (sigma > 0.0) {
      const double mu = sqrt(x0 * x0 + sigma);
      v0 = (x0 <= 0.0) ? (x0 - mu) : (-sigma * recip(x0 + mu));
      beta = 2.0 * v0 * v0 * recip(sigma + v0 * v0);
      ek = mu;
    }
    const double inv = recip(v0);
    if (tid < MAXN) {
      const int j = tid;
      const double vj = (j == k + 1) ? 1.0 : ((j > k + 1 && j < n) ? L[tri_at(j, k)] * inv : 0.0);
      if (j < TL_MAX) vb[j] = vj;
      R[(size_t)k * MAXN + j] = vj;
    }
    if (tid == 0) { sdg[k] = L[tri_at(k, k)]; sod[k] = ek; shb[k] = beta; }
    __syncthreads();  // v visible
    if (beta != 0.0) {
      const int i = row;
      const bool act = i > k && i < n;
      double pp = 0.0;
      if (act) {
        for (int j = k + 1 + q; j < n; j += 4) {
          const double a = j <= i ? L[tri_at(i, j)] : L[tri_at(j, i)];
          pp = fma(a, vb[j], pp);
        }
      }
      pp += __shfl_xor(pp, 1);
      pp += __shfl_xor(pp, 2);
      const double bp = beta * pp;
      const double pv = tl_block_sum((q == 0 && act) ? bp * vb[i] : 0.0, red);
      const double Kc = 0.5 * beta * pv;
      if (q == 0 && i < TL_MAX) wb[i] = act ? fma(-Kc, vb[i], bp) : 0.0;
      __syncthreads();  // w visible
      if (act) {
        const double vi = vb[i], wi = wb[i];
        for (int j = k + 1 + q; j <= i; j += 4) {
          const int e = tri_at(i, j);
          L[e] = fma(-vi, wb[j], fma(-wi, vb[j], L[e]));
        }
      }
    }
    __syncthreads();  // the step's update is done before the next column is read
  }
  if (tid == 0) {
    if (n >= 2) {
      sdg[n - 2] = L[tri_at(n - 2, n - 2)];
      sod[n - 2] = L[tri_at(n - 1, n - 2)];
      shb[n - 2] = 0.0;
      sdg[n - 1] = L[tri_at(n - 1, n - 1)];
      sod[n - 1] = 0.0;
      shb[n - 1] = 0.0;
    } else if (n == 1) {
      sdg[0] = L[0];
      sod[0] = 0.0;
      shb[0] = 0.0;
    }
  }
  __syncthreads();
  if (wv == 0) tridiag_finish(n, s1, seg2, sdg, sod, shb, work);
}

__global__ void __launch_bounds__(TL_THREADS) k_tridiag_lds(int d_full, int base, const int32_t* rank_p, int seg2,
                                                            const int32_t* rank2_p, const double* H, double* work,
                                                            int32_t* status) {
  tridiag_lds_body(d_full, base, rank_p, seg2, rank2_p, H, work, status, (int)blockIdx.x);
}

// ------------------------------------------------------------------------------------
// 2. eigenvalues: one wave per index t, 64-way multisection on the inertia count
// ------------------------------------------------------------------------------------
// Number of eigenvalues of the tridiagonal (dg, e2 = off-diagonal squared) below x, from
// the pivots of the LDL^T factorisation of T - x I; tiny pivots become -pivmin.
__device__ __forceinline__ int sturm_count(const double* dg, const double* e2, int n, double x, double pivmin) {
  double q = dg[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    q = fma(-e2[i - 1], recip(q), dg[i] - x);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

__device__ __forceinline__ double probe_at(double lo, double w, int s) { return lo + w * ((double)s * (1.0 / 65.0)); }

__device__ __forceinline__ void bisect_body(double* work, const int bx) {
  __shared__ double sdg[MAXN], se2[MAXN];
  const int t = bx, lane = threadIdx.x;
  const int n = (int)work[W_HDR];
  if (t >= n) return;
  for (int i = lane; i < n; i += GREST_WAVE) { sdg[i] = work[W_DG + i]; se2[i] = work[W_E2 + i]; }
  __syncthreads();
  double lo = work[W_HDR + 1], hi = work[W_HDR + 2];
  const double tnorm = work[W_HDR + 3], pivmin = work[W_HDR + 4];
  const double atol = fmax(EPS * tnorm, pivmin);
  for (int it = 0; it < 24; ++it) {
    const double w = hi - lo;
    if (!(w > fmax(atol, 2.0 * EPS * fmax(fabs(lo), fabs(hi))))) break;
    // probe s = lane + 1; the first probe whose count exceeds t closes the bracket
    const int c = sturm_count(sdg, se2, n, probe_at(lo, w, lane + 1), pivmin);
    const unsigned long long above = __ballot(c > t);
    const int a = above ? __builtin_ctzll(above) : GREST_WAVE;  // probes 1..a have count <= t
    const double nlo = a == 0 ? lo : probe_at(lo, w, a);
    const double nhi = a == GREST_WAVE ? hi : probe_at(lo, w, a + 1);
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) work[W_EV + t] = 0.5 * (lo + hi);
}

__global__ void __launch_bounds__(GREST_WAVE) k_bisect(double* work) {
  bisect_body(work, (int)blockIdx.x);
}

// ------------------------------------------------------------------------------------
// 3. selection, inverse iteration and back-transform: one wave per output slot
// ------------------------------------------------------------------------------------
// true if (ta, ia) comes before (tb, ib) in output order; WHICH 0: largest magnitude, then
// larger algebraic, then lower index; 1: smallest algebraic, then lower index; 2: largest
// algebraic, then lower index.  Written without branches (it runs in the inner loop of
// the ranking).
template <int WHICH>
__device__ __forceinline__ bool sel_before(double ta, int ia, double tb, int ib) {
  const bool tie = (ta == tb) & (ia < ib);
  if (WHICH == 1) return (ta < tb) | tie;
  if (WHICH == 2) return (ta > tb) | tie;
  const double aa = fabs(ta), ab = fabs(tb);
  return (aa > ab) | ((aa == ab) & ((ta > tb) | tie));
}

// rank of every entry of sev[0, n) in output order, each lane ranking its own entries
// against all n values, which are broadcast from the lanes' registers one at a time
template <int WHICH>
__device__ __forceinline__ void rank_values(const double* sev, int n, int (&rk)[NCOL]) {
  const int lane = threadIdx.x & (GREST_WAVE - 1);
  double tv[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) {
    const int i = lane + GREST_WAVE * c;
    tv[c] = i < n ? sev[i] : 0.0;
    rk[c] = 0;
  }
#pragma unroll
  for (int cj = 0; cj < NCOL; ++cj) {
    const int lmax = n - GREST_WAVE * cj < GREST_WAVE ? n - GREST_WAVE * cj : GREST_WAVE;
    for (int l = 0; l < lmax; ++l) {
      const int j = GREST_WAVE * cj + l;
      const double tj = readlane_d(tv[cj], l);
#pragma unroll
      for (int c = 0; c < NCOL; ++c)
        if (GREST_WAVE * c < n) {
          const int i = lane + GREST_WAVE * c;
          rk[c] += (int)((i < n) & (j != i) & sel_before<WHICH>(tj, j, tv[c], i));
        }
    }
  }
}

__device__ __forceinline__ double hash_unit(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)(h & 0xFFFFFF) / 16777216.0) - 0.5;
}

__device__ __forceinline__ void eigvec_body(int d_full, int which, int kk, double drop_tol,
                                                       double* work, double* theta_out, double* F,
                                                       int32_t* kept_out, int32_t* status, const int bx) {
  __shared__ double sev[MAXN], sdg[MAXN], sod[MAXN];
  __shared__ double u0i[MAXN], u1[MAXN], u2[MAXN], lm[MAXN], yv[MAXN];
  __shared__ unsigned char pv[MAXN];
  __shared__ int ssel[MAXN], sslot[MAXN], mslot[MAXN];
  const int slot = bx, lane = threadIdx.x;
  const int n = (int)work[W_HDR];
  const double tnorm = work[W_HDR + 3];
  double* Yb = work + W_Y;
  for (int i = lane; i < MAXN; i += GREST_WAVE) ssel[i] = 0;
  for (int i = lane; i < n; i += GREST_WAVE) {
    sev[i] = work[W_EV + i];
    sdg[i] = work[W_DG + i];
    sod[i] = work[W_OD + i];
  }
  __syncthreads();
  // rank of every eigenvalue in output order
  {
    int rk[NCOL];
    if (which == 0) rank_values<0>(sev, n, rk);
    else if (which == 1) rank_values<1>(sev, n, rk);
    else rank_values<2>(sev, n, rk);
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
      const int i = lane + GREST_WAVE * c;
      if (i < n) {
        sslot[i] = rk[c] < kk ? rk[c] : -1;
        if (rk[c] < kk) ssel[rk[c]] = i;
      }
    }
  }
  double tmax = -INFINITY;
  for (int i = lane; i < n; i += GREST_WAVE) tmax = fmax(tmax, sev[i]);
  tmax = wave_max_d(tmax);
  __syncthreads();
  const int nsel = kk < n ? kk : n;
  const double keep_thr = drop_tol > 0.0 ? drop_tol * drop_tol * fmax(1.0, tmax) : -INFINITY;
  // a selected index is kept unless its value falls below the drop threshold
  auto kept_idx = [&](int i) { return sslot[i] >= 0 && !(sev[i] <= keep_thr); };
  if (slot == 0 && lane == 0 && kept_out) {
    int c = 0;
    for (int s = 0; s < nsel; ++s) c += kept_idx(ssel[s]);
    *kept_out = c;
  }
  auto zero_column = [&](int s) {
    for (int r = lane; r < d_full; r += GREST_WAVE) F[(size_t)r * kk + s] = 0.0;
    if (lane == 0) { theta_out[s] = 0.0; work[W_FL + s] = 0.0; }
  };
  if (slot >= nsel) { zero_column(slot); return; }
  const int idx = ssel[slot];
  if (!kept_idx(idx)) { zero_column(slot); return; }
  if (lane == 0) work[W_FL + slot] = 1.0;
  // cluster: consecutive kept selected indices (ascending eigenvalue order) whose gaps are
  // at most ortol; the lowest member computes the whole cluster
  const double ortol = 1e-7 * tnorm;
  int prev = -1;
  for (int j = idx - 1; j >= 0; --j)
    if (kept_idx(j)) { prev = j; break; }
  if (prev >= 0 && sev[idx] - sev[prev] <= ortol) return;

  const double tiny = fmax(EPS * tnorm, 1e-290);
  const double y_eps = 10.0 * EPS * fmax(tnorm, 1e-300);
  double shift_prev = -INFINITY;
  int nmem = 0;
  int cur = idx;
  while (cur >= 0) {
    const int cslot = sslot[cur];
    double lam = sev[cur];
    if (nmem > 0) lam = fmax(lam, shift_prev + y_eps);
    shift_prev = lam;
    // LU with partial pivoting of T - lam I (U has three diagonals; 1/U_ii is stored),
    // pivots below tiny are raised to tiny
    // The sequential loops below (lane 0) are written without branches but the rare
    // rescaling, so that consecutive steps can be unrolled and their LDS reads issued early.
    if (lane == 0) {
      double a = sdg[0] - lam, bsup = n > 1 ? sod[0] : 0.0;
#pragma unroll 4
      for (int i = 0; i + 1 < n; ++i) {
        const double c = sod[i];
        const double an = sdg[i + 1] - lam;
        const double bn = i + 2 < n ? sod[i + 1] : 0.0;
        const bool sw = !(fabs(a) >= fabs(c));  // row interchange
        const double pa = fabs(a) < tiny ? (a < 0.0 ? -tiny : tiny) : a;
        const double ip = recip(sw ? c : pa);
        const double l = (sw ? a : c) * ip;
        u0i[i] = ip;
        u1[i] = sw ? an : bsup;
        u2[i] = sw ? bn : 0.0;
        lm[i] = l;
        pv[i] = sw ? 1 : 0;
        const double a_next = sw ? fma(-l, an, bsup) : fma(-l, bsup, an);
        bsup = sw ? -l * bn : bn;
        a = a_next;
      }
      const double pa = fabs(a) < tiny ? (a < 0.0 ? -tiny : tiny) : a;
      u0i[n - 1] = recip(pa);
      u1[n - 1] = 0.0;  // read (times zero) by the back-substitution
      u2[n - 1] = 0.0;
    }
    for (int i = lane; i < n; i += GREST_WAVE) yv[i] = hash_unit(i, cslot + 1);
    __syncthreads();
    for (int it = 0; it < 2; ++it) {
      if (lane == 0) {
        double x = yv[0];
#pragma unroll 4
        for (int i = 0; i + 1 < n; ++i) {  // L^{-1} with the row interchanges
          const double xn = yv[i + 1];
          const bool sw = pv[i] != 0;
          const double xa = sw ? xn : x, xb = sw ? x : xn;
          yv[i] = xa;
          x = fma(-lm[i], xa, xb);
        }
        yv[n - 1] = x;
        double x1 = 0.0, x2 = 0.0;  // U^{-1}; rescaled when it grows (tiny pivots)
        for (int i = n - 1; i >= 0; --i) {
          double v = fma(-u2[i], x2, fma(-u1[i], x1, yv[i])) * u0i[i];
          if (fabs(v) > 1e150) {  // scale the whole system: solved part and the rest
            for (int q = 0; q < n; ++q) yv[q] *= 1e-150;
            x1 *= 1e-150;
            x2 *= 1e-150;
            v = fma(-u2[i], x2, fma(-u1[i], x1, yv[i])) * u0i[i];
          }
          yv[i] = v;
          x2 = x1;
          x1 = v;
        }
      }
      __syncthreads();
      double y[NCOL];
#pragma unroll
      for (int c = 0; c < NCOL; ++c) y[c] = lane + GREST_WAVE * c < n ? yv[lane + GREST_WAVE * c] : 0.0;
      // classical Gram-Schmidt, twice, against the finished members of the cluster
      for (int pass = 0; pass < (nmem > 0 ? 2 : 0); ++pass) {
        for (int q = 0; q < nmem; ++q) {
          const double* yq = Yb + (size_t)mslot[q] * MAXN;
          double dp = 0.0;
#pragma unroll
          for (int c = 0; c < NCOL; ++c) dp = fma(y[c], yq[lane + GREST_WAVE * c], dp);
          const double d = wave_sum_d(dp);
#pragma unroll
          for (int c = 0; c < NCOL; ++c) y[c] = fma(-d, yq[lane + GREST_WAVE * c], y[c]);
        }
      }
      double n2p = 0.0;
#pragma unroll
      for (int c = 0; c < NCOL; ++c) n2p = fma(y[c], y[c], n2p);
      const double nrm2 = wave_sum_d(n2p);
      double s = (nrm2 > 0.0 && isfinite(nrm2)) ? 1.0 / sqrt(nrm2) : 0.0;
      if (s == 0.0) {  // breakdown: fall back to the unit vector of the index
        if (lane == 0) atomicOr(status, ST_NOT_CONVERGED);
#pragma unroll
        for (int c = 0; c < NCOL; ++c) y[c] = (lane + GREST_WAVE * c == cur) ? 1.0 : 0.0;
        s = 1.0;
      }
#pragma unroll
      for (int c = 0; c < NCOL; ++c) {
        y[c] *= s;
        if (lane + GREST_WAVE * c < n) yv[lane + GREST_WAVE * c] = y[c];
      }
      __syncthreads();
    }
    double y[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) y[c] = lane + GREST_WAVE * c < n ? yv[lane + GREST_WAVE * c] : 0.0;
    // next member of the cluster, if any
    int nxt = -1;
    for (int j = cur + 1; j < n; ++j)
      if (kept_idx(j)) { nxt = j; break; }
    if (nxt >= 0 && !(sev[nxt] - sev[cur] <= ortol)) nxt = -1;
    // the tridiagonal-basis vector, for the later members and for the last launch
    double* yq = Yb + (size_t)cslot * MAXN;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) yq[lane + GREST_WAVE * c] = y[c];
    if (lane == 0) { mslot[nmem] = cslot; theta_out[cslot] = sev[cur]; }
    __threadfence_block();
    ++nmem;
    cur = nxt;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(GREST_WAVE) k_eigvec(int d_full, int which, int kk, double drop_tol,
                                                       double* work, double* theta_out, double* F,
                                                       int32_t* kept_out, int32_t* status) {
  eigvec_body(d_full, which, kk, drop_tol, work, theta_out, F, kept_out, status, (int)blockIdx.x);
}

// The loops of the back-transform walk rows of the work table (the other slots' vectors,
// then the reflectors) whose loads do not depend on the running vector: each keeps the
// next PF rows in flight in a ring of registers, refilled as soon as a row is consumed, so
// that a step waits for its dot product and not for a round trip to memory (PF steps of a
// few hundred cycles cover it; the workgroup is one wave, so registers are plentiful).
// Entries past n are zero in every row and are left out.
constexpr int BT_PF = 16;

__device__ __forceinline__ void backtr_body(int d_full, int kk, const double* work, double* F, const int bx) {
  __shared__ double ysh[MAXN];
  __shared__ unsigned char sfl[MAXN];
  const int slot = bx, lane = threadIdx.x;
  if (work[W_FL + slot] == 0.0) return;
  const int n = (int)work[W_HDR];
  const int s1 = (int)work[W_HDR + 5], seg2 = (int)work[W_HDR + 6];
  const int nc = (n + GREST_WAVE - 1) / GREST_WAVE;  // elements of a length-n vector per lane
  const double* R = work + W_R;
  const double* hb = work + W_HB;
  const double* Yb = work + W_Y;
  for (int t = lane; t < kk; t += GREST_WAVE) sfl[t] = work[W_FL + t] != 0.0;
  wave_lds_fence();
  auto get_y = [&](int t, double(&o)[NCOL]) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < NCOL; ++c) o[c] = (t < kk && c < nc) ? Yb[(size_t)t * MAXN + lane + GREST_WAVE * c] : 0.0;
  };
  auto get_r = [&](int k, double(&o)[NCOL], double& b) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < NCOL; ++c) o[c] = (k >= 0 && c < nc) ? R[(size_t)k * MAXN + lane + GREST_WAVE * c] : 0.0;
    b = k >= 0 ? hb[k] : 0.0;
  };
  constexpr int PF = BT_PF;
  double ys[NCOL], cc[NCOL];
  get_y(slot, ys);
#pragma unroll
  for (int c = 0; c < NCOL; ++c) cc[c] = 0.0;
  double ring[PF][NCOL];
#pragma unroll
  for (int p = 0; p < PF; ++p) get_y(p, ring[p]);
  for (int t0 = 0; t0 < kk; t0 += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int t = t0 + p;
      double yt[NCOL];
#pragma unroll
      for (int c = 0; c < NCOL; ++c) yt[c] = ring[p][c];
      get_y(t + PF, ring[p]);
      if (t < kk && t != slot && sfl[t]) {
        double ep = 0.0;
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
          if (c < nc) ep = fma(yt[c], ys[c], ep);
        const double e = wave_sum_d(ep);
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
          if (c < nc) cc[c] = fma(e, yt[c], cc[c]);
      }
    }
  }
  double y[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) y[c] = fma(-0.5, cc[c], ys[c]);
  // back-transform y <- P_0 ... P_{n-3} y
  double bring[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) get_r(n - 3 - p, ring[p], bring[p]);
  for (int k0 = n - 3; k0 >= 0; k0 -= PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int k = k0 - p;
      double rk[NCOL];
#pragma unroll
      for (int c = 0; c < NCOL; ++c) rk[c] = ring[p][c];
      const double beta = bring[p];
      get_r(k - PF, ring[p], bring[p]);
      if (k >= 0) {
        double dp = 0.0;
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
          if (c < nc) dp = fma(rk[c], y[c], dp);
        const double d = beta * wave_sum_d(dp);
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
          if (c < nc) y[c] = fma(-d, rk[c], y[c]);
      }
    }
  }
  // F row of reduced index i is mp(i); the rows outside the map are zero
#pragma unroll
  for (int c = 0; c < NCOL; ++c) ysh[lane + GREST_WAVE * c] = y[c];
  wave_lds_fence();
  for (int r = lane; r < d_full; r += GREST_WAVE) {
    const int i = r < s1 ? r : ((r >= seg2 && r - seg2 < n - s1) ? s1 + (r - seg2) : -1);
    F[(size_t)r * kk + slot] = i >= 0 ? ysh[i] : 0.0;
  }
}

__global__ void __launch_bounds__(GREST_WAVE) k_backtr(int d_full, int kk, const double* work, double* F) {
  backtr_body(d_full, kk, work, F, (int)blockIdx.x);
}

__global__ void k_symmetrize(int d, double* H) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  int i = idx / d, j = idx % d;
  if (i < j) {
    double v = 0.5 * (H[i * d + j] + H[j * d + i]);
    H[i * d + j] = v;
    H[j * d + i] = v;
  }
}

}  // namespace

int64_t eig_work_elems(int d) { return d <= TL_MAX ? (int64_t)W_END : 0; }

int64_t pchol_work_elems(int, int) { return 0; }

// the coefficient block goes to LDS when it fits beside the static arrays
template <int M>
void pchol_launch(int m, const double* G, const double* C, int kc, double tol, double* Mout, int32_t* rank,
                  int32_t* status, hipStream_t s, const int32_t* done = nullptr) {
  constexpr size_t kStatic = (size_t)M * (M + 1) * 8 + (size_t)M * 24;
  constexpr size_t kDynMax = 160 * 1024 - kStatic - 1024;
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_pchol<M, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kDynMax);
    return true;
  }();
  (void)attr;
  const size_t dyn = (size_t)kc * m * sizeof(double);
  if (kc > 0 && dyn <= kDynMax)
    k_pchol<M, true><<<1, PCH_WAVES * GREST_WAVE, dyn, s>>>(m, G, C, kc, tol, Mout, rank, status, done);
  else
    k_pchol<M, false><<<1, PCH_WAVES * GREST_WAVE, 0, s>>>(m, G, C, kc, tol, Mout, rank, status, done);
}

void launch_pchol(int m, const double* G, const double* C, int kc, double tol, double* Mout, int32_t* rank,
                  int32_t* status, double*, hipStream_t s) {
  if (!C) kc = 0;
  if (m <= 64) pchol_launch<64>(m, G, C, kc, tol, Mout, rank, status, s);
  else pchol_launch<128>(m, G, C, kc, tol, Mout, rank, status, s);
}

// The factor of a CholQR round: without pivoting first (k_chol_np); where that does not
// satisfy the truncation rule (a rank-deficient block), the pivoted kernel runs.
void launch_pchol2(int m, const double* G, const double* C, int kc, double tol, double* Mout, int32_t* rank,
                   int32_t* status, double* work, hipStream_t s) {
  if (!C) kc = 0;
  int32_t* done = reinterpret_cast<int32_t*>(work);
  const size_t dyn = (size_t)kc * CNP_M * sizeof(double);
  if (m > CNP_M || dyn > kCnpDynMax) {
    launch_pchol(m, G, C, kc, tol, Mout, rank, status, work, s);
    return;
  }
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_chol_np, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCnpDynMax);
    return true;
  }();
  (void)attr;
  k_chol_np<<<1, CNP_T, dyn, s>>>(m, G, C, kc, tol, Mout, rank, done);
  if (m <= 64) pchol_launch<64>(m, G, C, kc, tol, Mout, rank, status, s, done);
  else pchol_launch<128>(m, G, C, kc, tol, Mout, rank, status, s, done);
}

bool launch_small_eig(int d_full, int base, const int32_t* rank, const double* H, int which, int kk,
                      double drop_tol, double* theta, double* F, int32_t* kept, double* work,
                      int32_t* status, hipStream_t s, int seg2, const int32_t* rank2) {
  if (d_full < 1 || d_full > TL_MAX || kk < 1 || kk > d_full) return false;
  if (rank2 && (seg2 < base || seg2 > d_full)) return false;
  if (d_full <= 64) {
    k_tridiag<64><<<1, TRI_WAVES * GREST_WAVE, 0, s>>>(d_full, base, rank, seg2, rank2, H, work, status);
  } else if (d_full <= 128) {
    k_tridiag<128><<<1, TRI_WAVES * GREST_WAVE, 0, s>>>(d_full, base, rank, seg2, rank2, H, work, status);
  } else {
    static const bool attr = [] {
      (void)hipFuncSetAttribute((const void*)k_tridiag_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TL_LDS);
      return true;
    }();
    (void)attr;
    k_tridiag_lds<<<1, TL_THREADS, TL_LDS, s>>>(d_full, base, rank, seg2, rank2, H, work, status);
  }
  k_bisect<<<d_full, GREST_WAVE, 0, s>>>(work);
  k_eigvec<<<kk, GREST_WAVE, 0, s>>>(d_full, which, kk, drop_tol, work, theta, F, kept, status);
  k_backtr<<<kk, GREST_WAVE, 0, s>>>(d_full, kk, work, F);
  return true;
}

void launch_symmetrize(int d, double* H, hipStream_t s) {
  int nthr = d * d;
  k_symmetrize<<<(nthr + 255) / 256, 256, 0, s>>>(d, H);
}

// ------------------------------------------------------------------------------------
// Batched launches: the same factor and eigensolve kernels for many graphs at once, one
// workgroup per graph (or per graph and pair), each reading its graph's arguments from a
// descriptor array in device memory.  Every workgroup runs the code of the single-graph
// kernel on its own graph's data, so a graph's results do not depend on the others.
// ------------------------------------------------------------------------------------
namespace {

// instance of the factor kernels a job needs: k_chol_np first (np), then k_pchol<M, CL>
struct CholPlan {
  bool np;
  int M;
  bool cl;
  size_t dyn_np, dyn_p;
};

template <int M>
constexpr size_t pchol_dyn_max() {
  return 160 * 1024 - ((size_t)M * (M + 1) * 8 + (size_t)M * 24) - 1024;
}

CholPlan chol_plan(const CholJob& j) {
  CholPlan p{};
  const int kc = j.C ? j.kc : 0;
  p.dyn_np = (size_t)kc * CNP_M * sizeof(double);
  p.np = j.m <= CNP_M && p.dyn_np <= kCnpDynMax;
  p.M = j.m <= 64 ? 64 : 128;
  p.dyn_p = (size_t)kc * j.m * sizeof(double);
  p.cl = kc > 0 && p.dyn_p <= (p.M == 64 ? pchol_dyn_max<64>() : pchol_dyn_max<128>());
  if (!p.cl) p.dyn_p = 0;
  return p;
}

int chol_key(const CholJob& j) {
  const CholPlan p = chol_plan(j);
  return (p.np ? 0 : 4) + (p.M == 64 ? 0 : 2) + (p.cl ? 1 : 0);
}

int eig_key(const EigJob& j) { return j.d_full <= 64 ? 0 : (j.d_full <= 128 ? 1 : 2); }

__global__ void __launch_bounds__(CNP_T) k_chol_np_batch(const CholJob* J) {
  const CholJob& j = J[blockIdx.x];
  chol_np_body(j.m, j.G, j.C, j.C ? j.kc : 0, j.tol, j.Mout, j.rank, reinterpret_cast<int32_t*>(j.work), 0);
}

template <int M, bool CL>
__global__ void __launch_bounds__(PCH_WAVES * GREST_WAVE) k_pchol_batch(const CholJob* J, int after_np) {
  const CholJob& j = J[blockIdx.x];
  pchol_body<M, CL>(j.m, j.G, j.C, j.C ? j.kc : 0, j.tol, j.Mout, j.rank, j.status,
                    after_np ? reinterpret_cast<const int32_t*>(j.work) : nullptr, 0);
}

template <int M>
__global__ void __launch_bounds__(TRI_WAVES * GREST_WAVE) k_tridiag_batch(const EigJob* J) {
  const EigJob& j = J[blockIdx.x];
  tridiag_body<M>(j.d_full, j.base, j.rank, j.seg2, j.rank2, j.H, j.work, j.status, 0);
}

__global__ void __launch_bounds__(TL_THREADS) k_tridiag_lds_batch(const EigJob* J) {
  const EigJob& j = J[blockIdx.x];
  tridiag_lds_body(j.d_full, j.base, j.rank, j.seg2, j.rank2, j.H, j.work, j.status, 0);
}

// the job whose block range [b0, b0 + count) holds block b (jobs in ascending b0)
__device__ __forceinline__ int job_of(const EigJob* J, int nj, int b, bool vec) {
  int g = 0;
  for (int i = 1; i < nj; ++i)
    if ((vec ? J[i].b0_vec : J[i].b0_bisect) <= b) g = i;
  return g;
}

__global__ void __launch_bounds__(GREST_WAVE) k_bisect_batch(const EigJob* J, int nj) {
  const int b = blockIdx.x;
  const EigJob& j = J[job_of(J, nj, b, false)];
  bisect_body(j.work, b - j.b0_bisect);
}

__global__ void __launch_bounds__(GREST_WAVE) k_eigvec_batch(const EigJob* J, int nj) {
  const int b = blockIdx.x;
  const EigJob& j = J[job_of(J, nj, b, true)];
  eigvec_body(j.d_full, j.which, j.kk, j.drop_tol, j.work, j.theta, j.F, j.kept, j.status, b - j.b0_vec);
}

__global__ void __launch_bounds__(GREST_WAVE) k_backtr_batch(const EigJob* J, int nj) {
  const int b = blockIdx.x;
  const EigJob& j = J[job_of(J, nj, b, true)];
  backtr_body(j.d_full, j.kk, j.work, j.F, b - j.b0_vec);
}

template <typename K>
void set_dyn_max(K kernel, size_t bytes) {
  (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

bool small_eig_job_ok(const EigJob& j) {
  if (j.d_full < 1 || j.d_full > TL_MAX || j.kk < 1 || j.kk > j.d_full) return false;
  if (j.rank2 && (j.seg2 < j.base || j.seg2 > j.d_full)) return false;
  return true;
}

void chol_batch_prepare(CholJob* jobs, int nj) {
  std::stable_sort(jobs, jobs + nj, [](const CholJob& a, const CholJob& b) { return chol_key(a) < chol_key(b); });
}

void batch_kernels_init() {
  static const bool attr = [] {
    set_dyn_max(k_chol_np_batch, kCnpDynMax);
    set_dyn_max(k_pchol_batch<64, true>, pchol_dyn_max<64>());
    set_dyn_max(k_pchol_batch<128, true>, pchol_dyn_max<128>());
    set_dyn_max(k_tridiag_lds_batch, TL_LDS);
    return true;
  }();
  (void)attr;
}

int chol_job_key(const CholJob& j) { return chol_key(j); }

int eig_job_key(const EigJob& j) { return eig_key(j); }

void chol_batch_launch(const CholJob* jobs, const CholJob* dev, int nj, hipStream_t s) {
  batch_kernels_init();
  // k_chol_np over the leading jobs that take it (sorted first), then k_pchol per instance
  int np = 0;
  size_t dyn = 0;
  while (np < nj && chol_plan(jobs[np]).np) dyn = std::max(dyn, chol_plan(jobs[np++]).dyn_np);
  if (np > 0) k_chol_np_batch<<<np, CNP_T, dyn, s>>>(dev);
  for (int a = 0; a < nj;) {
    const int key = chol_key(jobs[a]);
    int b = a;
    size_t d = 0;
    while (b < nj && chol_key(jobs[b]) == key) d = std::max(d, chol_plan(jobs[b++]).dyn_p);
    const CholPlan p = chol_plan(jobs[a]);
    const int after_np = p.np ? 1 : 0;
    const unsigned g = (unsigned)(b - a);
    if (p.M == 64 && p.cl) k_pchol_batch<64, true><<<g, PCH_WAVES * GREST_WAVE, d, s>>>(dev + a, after_np);
    else if (p.M == 64) k_pchol_batch<64, false><<<g, PCH_WAVES * GREST_WAVE, 0, s>>>(dev + a, after_np);
    else if (p.cl) k_pchol_batch<128, true><<<g, PCH_WAVES * GREST_WAVE, d, s>>>(dev + a, after_np);
    else k_pchol_batch<128, false><<<g, PCH_WAVES * GREST_WAVE, 0, s>>>(dev + a, after_np);
    a = b;
  }
}

void small_eig_batch_prepare(EigJob* jobs, int nj) {
  std::stable_sort(jobs, jobs + nj, [](const EigJob& a, const EigJob& b) { return eig_key(a) < eig_key(b); });
  int bb = 0, bv = 0;
  for (int i = 0; i < nj; ++i) {
    jobs[i].b0_bisect = bb;
    jobs[i].b0_vec = bv;
    bb += jobs[i].d_full;
    bv += jobs[i].kk;
  }
}

void small_eig_batch_launch(const EigJob* jobs, const EigJob* dev, int nj, hipStream_t s) {
  batch_kernels_init();
  for (int a = 0; a < nj;) {
    const int key = eig_key(jobs[a]);
    int b = a;
    while (b < nj && eig_key(jobs[b]) == key) ++b;
    const unsigned g = (unsigned)(b - a);
    if (key == 0) k_tridiag_batch<64><<<g, TRI_WAVES * GREST_WAVE, 0, s>>>(dev + a);
    else if (key == 1) k_tridiag_batch<128><<<g, TRI_WAVES * GREST_WAVE, 0, s>>>(dev + a);
    else k_tridiag_lds_batch<<<g, TL_THREADS, TL_LDS, s>>>(dev + a);
    a = b;
  }
  const EigJob& last = jobs[nj - 1];
  k_bisect_batch<<<last.b0_bisect + last.d_full, GREST_WAVE, 0, s>>>(dev, nj);
  k_eigvec_batch<<<last.b0_vec + last.kk, GREST_WAVE, 0, s>>>(dev, nj);
  k_backtr_batch<<<last.b0_vec + last.kk, GREST_WAVE, 0, s>>>(dev, nj);
}
