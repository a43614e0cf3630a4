// One-workgroup FP64 kernels on the small matrices of the update:
//   * rank-revealing Cholesky with diagonal pivoting of a Gram matrix (the
//     factor of CholQR2); the inverse factor is returned as the matrix M that
//     maps W to its orthonormal basis W M;
//   * the dense symmetric eigensolver of the projected matrix (Alg. 1, small
//     eigenproblem) and of the sketch Gram B B^T of the randomized range finder
//     (Sec. 3.5), followed by the selection of the wanted pairs.
// The eigensolver is Householder tridiagonalisation, explicit accumulation of the
// orthogonal factor, and implicit symmetric QR steps with the Wilkinson shift; the
// bulge chase runs on one lane and every lane applies the sweep's plane rotations
// to its own row of the eigenvector matrix.  Matrices up to SMALL_LDS_D live in LDS,
// larger ones in a global workspace.
#include "grest_internal.h"

#include <math.h>

namespace {

constexpr int EB = 256;           // threads per workgroup
constexpr int SMALL_LDS_D = 128;  // largest order kept in LDS (128 x 129 doubles = 132 KB)
constexpr int MAXD = 256;         // largest supported order

__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = GREST_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, GREST_WAVE);
  const int lane = threadIdx.x & (GREST_WAVE - 1), wid = threadIdx.x / GREST_WAVE;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < EB / GREST_WAVE; ++w) t += red[w];
  return t;
}

// ------------------------------------------------------------------------------------
// pivoted Cholesky:  G(P) = R^T R  truncated at the first pivot <= (tol*scale)^2
// M[perm[i], j] = Rinv[i, j] for i <= j < rank, every other entry 0.
// ------------------------------------------------------------------------------------
template <bool IN_LDS>
__global__ void __launch_bounds__(EB) k_pchol(int m, const double* G, const double* c1,
                                              const double* c2, int kc, double tol, double* M,
                                              int32_t* rank_out, int32_t* status, double* work) {
  __shared__ double sS[IN_LDS ? (SMALL_LDS_D + 1) * (SMALL_LDS_D + 1) : 1];
  __shared__ int perm[MAXD];
  __shared__ double red[EB / GREST_WAVE];
  __shared__ double sh_val[2];
  __shared__ int sh_idx;
  double* S = IN_LDS ? sS : work;
  const int lds = m + 1;
  const int tid = threadIdx.x;

  // load and find the scale: max_j (G_jj + |C1[:,j]|^2 + |C2[:,j]|^2)
  double mx = 0.0;
  int bad = 0;
  for (int idx = tid; idx < m * m; idx += EB) {
    int i = idx / m, j = idx % m;
    double g = 0.5 * (G[(size_t)i * m + j] + G[(size_t)j * m + i]);
    if (!isfinite(g)) bad = 1;
    S[i * lds + j] = g;
  }
  for (int j = tid; j < m; j += EB) {
    double v = G[(size_t)j * m + j];
    if (c1) for (int i = 0; i < kc; ++i) v += c1[(size_t)i * m + j] * c1[(size_t)i * m + j];
    if (c2) for (int i = 0; i < kc; ++i) v += c2[(size_t)i * m + j] * c2[(size_t)i * m + j];
    mx = fmax(mx, v);
    perm[j] = j;
  }
  for (int o = GREST_WAVE / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, GREST_WAVE));
  if ((tid & (GREST_WAVE - 1)) == 0) red[tid / GREST_WAVE] = mx;
  if (bad) atomicOr(status, ST_NONFINITE);
  __syncthreads();
  double scale2 = 1.0;
  for (int w = 0; w < EB / GREST_WAVE; ++w) scale2 = fmax(scale2, red[w]);
  const double thr = tol * tol * scale2;
  __syncthreads();

  int r = 0;
  for (int k = 0; k < m; ++k) {
    // pivot: largest remaining diagonal (ties to the lower position)
    if (tid < GREST_WAVE) {
      double best = -1.0;
      int bi = -1;
      for (int j = k + tid; j < m; j += GREST_WAVE) {
        double v = S[j * lds + j];
        if (v > best) { best = v; bi = j; }
      }
      for (int o = GREST_WAVE / 2; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, GREST_WAVE);
        int oi = __shfl_xor(bi, o, GREST_WAVE);
        if (ob > best || (ob == best && oi >= 0 && (bi < 0 || oi < bi))) { best = ob; bi = oi; }
      }
      if (tid == 0) { sh_val[0] = best; sh_idx = bi; }
    }
    __syncthreads();
    const double piv = sh_val[0];
    const int p = sh_idx;
    if (!(piv > thr) || p < 0) break;  // also stops on NaN
    if (p != k) {  // symmetric swap of rows/cols k and p
      for (int j = tid; j < m; j += EB) {
        double t = S[k * lds + j]; S[k * lds + j] = S[p * lds + j]; S[p * lds + j] = t;
      }
      __syncthreads();
      for (int i = tid; i < m; i += EB) {
        double t = S[i * lds + k]; S[i * lds + k] = S[i * lds + p]; S[i * lds + p] = t;
      }
      if (tid == 0) { int t = perm[k]; perm[k] = perm[p]; perm[p] = t; }
      __syncthreads();
    }
    const double rkk = sqrt(piv);
    for (int j = k + 1 + tid; j < m; j += EB) S[k * lds + j] /= rkk;
    __syncthreads();
    if (tid == 0) S[k * lds + k] = rkk;
    const int t = m - k - 1;
    for (int idx = tid; idx < t * t; idx += EB) {
      int i = k + 1 + idx / t, j = k + 1 + idx % t;
      S[i * lds + j] -= S[k * lds + i] * S[k * lds + j];
    }
    __syncthreads();
    r = k + 1;
  }
  // inverse of the leading r x r upper-triangular block, column j by thread j;
  // Rinv[i][j] is kept in row j+1 of S (below the factor) at column i
  for (int j = tid; j < r; j += EB) {
    for (int i = j; i >= 0; --i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int l = i + 1; l <= j; ++l) acc -= S[i * lds + l] * S[(j + 1) * lds + l];
      S[(j + 1) * lds + i] = acc / S[i * lds + i];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < m * m; idx += EB) {
    int a = idx / m, j = idx % m;  // output M[a][j]
    M[idx] = 0.0;
    (void)a;
  }
  __syncthreads();
  for (int idx = tid; idx < m * m; idx += EB) {
    int i = idx / m, j = idx % m;
    if (i < r && j < r && i <= j) M[(size_t)perm[i] * m + j] = S[(j + 1) * lds + i];
  }
  if (tid == 0) *rank_out = r;
}

// ------------------------------------------------------------------------------------
// symmetric eigensolver + selection
// ------------------------------------------------------------------------------------
__device__ inline bool sel_less(int which, double ta, int ia, double tb, int ib) {
  // true if (ta, ia) comes before (tb, ib) in output order
  if (which == 0) {  // largest magnitude, then larger algebraic, then lower index
    double aa = fabs(ta), ab = fabs(tb);
    if (aa != ab) return aa > ab;
    if (ta != tb) return ta > tb;
    return ia < ib;
  }
  if (which == 1) {  // smallest algebraic
    if (ta != tb) return ta < tb;
    return ia < ib;
  }
  if (ta != tb) return ta > tb;  // largest algebraic
  return ia < ib;
}

template <bool IN_LDS>
__global__ void __launch_bounds__(EB) k_small_eig(int d_full, int base, const int32_t* rank_p,
                                                  const double* H, int which, int kk, double drop_tol,
                                                  double* theta_out, double* F, int32_t* kept_out,
                                                  double* work, int32_t* status) {
  __shared__ double sA[IN_LDS ? SMALL_LDS_D * (SMALL_LDS_D + 1) : 1];
  __shared__ double dg[MAXD], od[MAXD], vv[MAXD], pw[MAXD], hb[MAXD];
  __shared__ double rc[MAXD], rs[MAXD];
  __shared__ double red[EB / GREST_WAVE];
  __shared__ int sh[4];
  const int tid = threadIdx.x;
  int n = base + (rank_p ? rank_p[0] : 0);
  if (n > d_full) n = d_full;
  if (n < 0) n = 0;
  double* A = IN_LDS ? sA : work;
  const int lda = n + 1;

  int bad = 0;
  for (int idx = tid; idx < n * n; idx += EB) {
    int i = idx / n, j = idx % n;
    double h = 0.5 * (H[(size_t)i * d_full + j] + H[(size_t)j * d_full + i]);
    if (!isfinite(h)) { bad = 1; h = 0.0; }
    A[i * lda + j] = h;
  }
  if (bad) atomicOr(status, ST_NONFINITE);
  __syncthreads();

  // ---- Householder tridiagonalisation (A = Q T Q^T) ----
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += EB) {
      double x = A[(k + 1 + i) * lda + k];
      part += x * x;
    }
    const double sigma = block_sum(part, red);
    const double x0 = A[(k + 1) * lda + k];
    double beta = 0.0, v0 = 1.0, ek = x0;
    if (sigma > 0.0) {
      const double mu = sqrt(x0 * x0 + sigma);
      v0 = (x0 <= 0.0) ? (x0 - mu) : (-sigma / (x0 + mu));
      beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
      ek = mu;
    }
    for (int i = tid; i < m; i += EB) vv[i] = (i == 0) ? 1.0 : A[(k + 1 + i) * lda + k] / v0;
    if (tid == 0) { dg[k] = A[k * lda + k]; od[k] = ek; hb[k] = beta; }
    __syncthreads();
    if (beta != 0.0) {
      // p = beta * A22 v
      for (int i = tid; i < m; i += EB) {
        const double* row = A + (k + 1 + i) * lda + (k + 1);
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += row[j] * vv[j];
        pw[i] = beta * acc;
      }
      __syncthreads();
      double pv = 0.0;
      for (int i = tid; i < m; i += EB) pv += pw[i] * vv[i];
      const double K = 0.5 * beta * block_sum(pv, red);
      for (int i = tid; i < m; i += EB) pw[i] -= K * vv[i];  // w
      __syncthreads();
      for (int idx = tid; idx < m * m; idx += EB) {
        int i = idx / m, j = idx % m;
        A[(k + 1 + i) * lda + (k + 1 + j)] -= vv[i] * pw[j] + pw[i] * vv[j];
      }
    }
    // keep v (below its implicit leading 1) in column k
    for (int i = 1 + tid; i < m; i += EB) A[(k + 1 + i) * lda + k] = vv[i];
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      dg[n - 2] = A[(n - 2) * lda + (n - 2)];
      od[n - 2] = A[(n - 1) * lda + (n - 2)];
      hb[n - 2] = 0.0;
    }
    if (n >= 1) dg[n - 1] = A[(n - 1) * lda + (n - 1)];
  }
  __syncthreads();

  // ---- explicit Q = P_0 P_1 ... P_{n-3}, accumulated backwards in place ----
  if (n >= 1 && tid == 0) A[(n - 1) * lda + (n - 1)] = 1.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    for (int i = tid; i < m; i += EB) vv[i] = (i == 0) ? 1.0 : A[(k + 1 + i) * lda + k];
    __syncthreads();
    // row k+1 and column k+1 of the block become the identity's
    for (int j = tid; j < m; j += EB) {
      A[(k + 1) * lda + (k + 1 + j)] = (j == 0) ? 1.0 : 0.0;
      if (j > 0) A[(k + 1 + j) * lda + (k + 1)] = 0.0;
    }
    __syncthreads();
    const double beta = hb[k];
    if (beta != 0.0) {
      for (int j = tid; j < m; j += EB) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += vv[i] * A[(k + 1 + i) * lda + (k + 1 + j)];
        pw[j] = beta * acc;
      }
      __syncthreads();
      for (int idx = tid; idx < m * m; idx += EB) {
        int i = idx / m, j = idx % m;
        A[(k + 1 + i) * lda + (k + 1 + j)] -= vv[i] * pw[j];
      }
      __syncthreads();
    }
  }
  if (n >= 2) {
    for (int j = tid; j < n; j += EB) {
      A[0 * lda + j] = (j == 0) ? 1.0 : 0.0;
      if (j > 0) A[j * lda + 0] = 0.0;
    }
    if (n == 2 && tid == 0) { A[1 * lda + 1] = 1.0; }
  } else if (n == 1 && tid == 0) {
    A[0] = 1.0;
  }
  __syncthreads();

  // ---- implicit symmetric QR with the Wilkinson shift ----
  const double eps = 2.220446049250313e-16;
  int sweeps = 0;
  const int max_sweeps = 30 * (n > 1 ? n : 1);
  while (true) {
    if (tid == 0) {
      int hi = sh[1];
      if (sweeps == 0) hi = n - 1;
      while (hi > 0 && fabs(od[hi - 1]) <= eps * (fabs(dg[hi - 1]) + fabs(dg[hi])) + 1e-300) {
        od[hi - 1] = 0.0;
        --hi;
      }
      if (hi <= 0 || sweeps >= max_sweeps) {
        if (hi > 0) atomicOr(status, ST_NOT_CONVERGED);
        sh[0] = -1;
      } else {
        int lo = hi - 1;
        while (lo > 0 && fabs(od[lo - 1]) > eps * (fabs(dg[lo - 1]) + fabs(dg[lo])) + 1e-300) --lo;
        const double b = od[hi - 1];
        const double delta = 0.5 * (dg[hi - 1] - dg[hi]);
        const double h = hypot(delta, b);
        const double den = delta + (delta >= 0.0 ? h : -h);
        const double mu = (den != 0.0) ? dg[hi] - b * b / den : dg[hi];
        double p = dg[lo] - mu, q = od[lo];
        for (int k = lo; k < hi; ++k) {
          double r = hypot(p, q);
          double c = 1.0, s = 0.0;
          if (r > 0.0) { c = p / r; s = -q / r; }
          if (k > lo) od[k - 1] = r;
          const double a = dg[k], bb = od[k], e2 = dg[k + 1];
          const double cc = c * c, ss = s * s, cs = c * s;
          dg[k] = cc * a - 2.0 * cs * bb + ss * e2;
          dg[k + 1] = ss * a + 2.0 * cs * bb + cc * e2;
          od[k] = cs * (a - e2) + (cc - ss) * bb;
          if (k + 1 < hi) {
            q = -s * od[k + 1];
            od[k + 1] = c * od[k + 1];
            p = od[k];
          }
          rc[k] = c;
          rs[k] = s;
        }
        sh[0] = lo;
        sh[1] = hi;
      }
    }
    __syncthreads();
    const int lo = sh[0];
    if (lo < 0) break;
    const int hi = sh[1];
    ++sweeps;
    for (int i = tid; i < n; i += EB) {
      double* row = A + i * lda;
      double cur = row[lo];
      for (int k = lo; k < hi; ++k) {
        const double c = rc[k], s = rs[k];
        const double nxt = row[k + 1];
        row[k] = c * cur - s * nxt;
        cur = s * cur + c * nxt;
      }
      row[hi] = cur;
    }
    __syncthreads();
  }

  // ---- selection ----
  if (tid == 0) sh[2] = 0;
  __syncthreads();
  double tmax = 0.0;
  for (int i = 0; i < n; ++i) tmax = fmax(tmax, dg[i]);
  const double keep_thr = drop_tol > 0.0 ? drop_tol * drop_tol * fmax(1.0, tmax) : -INFINITY;
  for (int i = tid; i < n; i += EB) {
    const double ti = dg[i];
    int rank = 0;
    for (int j = 0; j < n; ++j)
      if (j != i && sel_less(which, dg[j], j, ti, i)) ++rank;
    if (rank < kk) {
      const bool keep = !(drop_tol > 0.0) || ti > keep_thr;
      theta_out[rank] = keep ? ti : 0.0;
      if (keep) atomicAdd(&sh[2], 1);
      for (int r = 0; r < d_full; ++r)
        F[(size_t)r * kk + rank] = (keep && r < n) ? A[r * lda + i] : 0.0;
    }
  }
  // slots beyond n (fewer pairs than requested) are zero
  for (int slot = n + tid; slot < kk; slot += EB) {
    theta_out[slot] = 0.0;
    for (int r = 0; r < d_full; ++r) F[(size_t)r * kk + slot] = 0.0;
  }
  __syncthreads();
  if (tid == 0 && kept_out) *kept_out = sh[2];
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

int64_t eig_work_elems(int d) { return (int64_t)(d + 1) * (d + 1); }

void launch_pchol(int m, const double* G, const double* colsq1, const double* colsq2, int kc,
                  double tol, double* M, int32_t* rank, int32_t* status, hipStream_t s) {
  // the global-memory variant keeps its factor in the trailing part of M's buffer
  if (m <= SMALL_LDS_D) {
    k_pchol<true><<<1, EB, 0, s>>>(m, G, colsq1, colsq2, kc, tol, M, rank, status, nullptr);
  } else {
    k_pchol<false><<<1, EB, 0, s>>>(m, G, colsq1, colsq2, kc, tol, M, rank, status,
                                    M + (size_t)m * m);
  }
}

void launch_small_eig(int d_full, int base, const int32_t* rank, const double* H, int which, int kk,
                      double drop_tol, double* theta, double* F, int32_t* kept, double* work,
                      int32_t* status, hipStream_t s) {
  if (d_full <= SMALL_LDS_D) {
    k_small_eig<true><<<1, EB, 0, s>>>(d_full, base, rank, H, which, kk, drop_tol, theta, F, kept,
                                       work, status);
  } else {
    k_small_eig<false><<<1, EB, 0, s>>>(d_full, base, rank, H, which, kk, drop_tol, theta, F, kept,
                                        work, status);
  }
}

void launch_symmetrize(int d, double* H, hipStream_t s) {
  int nthr = d * d;
  k_symmetrize<<<(nthr + 255) / 256, 256, 0, s>>>(d, H);
}
