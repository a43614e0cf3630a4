// One-workgroup FP64 kernels on the small matrices of the update:
//   * rank-revealing Cholesky with diagonal pivoting of a Gram matrix (the
//     factor of CholQR2); the inverse factor is returned as the matrix M that
//     maps W to its orthonormal basis W M;
//   * the dense symmetric eigensolver of the projected matrix (Alg. 1, small
//     eigenproblem) and of the sketch Gram B B^T of the randomized range finder
//     (Sec. 3.5), followed by the selection of the wanted pairs.
// The eigensolver is Householder tridiagonalisation (reflectors kept in place), all
// eigenvalues of the tridiagonal by bisection on the LDL^T inertia (one lane per
// eigenvalue), eigenvectors of the selected ones only by inverse iteration with an
// LU factorisation with partial pivoting (clusters closer than 1e-3 ||T|| get distinct
// shifts and reorthogonalisation on one lane), and the back-transform through the
// reflectors with eight lanes per vector.  Matrices up to SMALL_LDS_D live in LDS,
// larger ones in a global workspace.
#include "grest_internal.h"

#include <math.h>

// Optional phase clocks for profiling builds (-DGREST_PHASE_CLOCKS): thread 0 records the
// 100 MHz wall clock at phase boundaries of the small kernels.
#ifdef GREST_PHASE_CLOCKS
__device__ long long g_phase_clk[64];
#define PHASE_MARK(slot)                                  \
  do {                                                    \
    __syncthreads();                                      \
    if (threadIdx.x == 0) g_phase_clk[slot] = wall_clock64(); \
  } while (0)
extern "C" int grest_debug_phase_clocks(long long* out, int n) {
  return (int)hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_clk), sizeof(long long) * (n < 64 ? n : 64));
}
#else
#define PHASE_MARK(slot) \
  do {                   \
  } while (0)
#endif

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
// With a projection coefficient block C (kc x m) the factored matrix is the Gram of the
// projected block, G - C^T C (Pythagorean form of block Gram-Schmidt), the rank scale is
// taken from G itself (the block before projection), and the output is the stacked
// (kc + m) x m matrix [-C M; M], so that (W - X C) M = [X W] [-C M; M].
template <bool IN_LDS>
__global__ void __launch_bounds__(EB) k_pchol(int m, const double* G, const double* C, int kc, double tol,
                                              double* Mout, int32_t* rank_out, int32_t* status, double* work) {
  extern __shared__ double dyn[];
  __shared__ int perm[MAXD];
  __shared__ double red[EB / GREST_WAVE];
  __shared__ double sh_val[2];
  __shared__ int sh_idx;
  const int lds = m + 1;
  double* S = IN_LDS ? dyn : work;
  double* Cs = IN_LDS ? dyn + (size_t)lds * lds : work + (size_t)lds * lds;
  double* M = Mout + (size_t)kc * m;  // the m x m block
  const int tid = threadIdx.x;

  for (int idx = tid; idx < kc * m; idx += EB) Cs[idx] = C[idx];
  __syncthreads();
  // load, subtract C^T C, and find the scale max_j G_jj
  double mx = 0.0;
  int bad = 0;
  for (int idx = tid; idx < m * m; idx += EB) {
    int i = idx / m, j = idx % m;
    double g = 0.5 * (G[(size_t)i * m + j] + G[(size_t)j * m + i]);
    for (int l = 0; l < kc; ++l) g -= Cs[l * m + i] * Cs[l * m + j];
    if (!isfinite(g)) bad = 1;
    S[i * lds + j] = g;
  }
  for (int j = tid; j < m; j += EB) {
    mx = fmax(mx, G[(size_t)j * m + j]);
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

  PHASE_MARK(10);
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
  PHASE_MARK(11);
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
  for (int idx = tid; idx < m * m; idx += EB) M[idx] = 0.0;
  __syncthreads();
  for (int idx = tid; idx < m * m; idx += EB) {
    int i = idx / m, j = idx % m;
    if (i < r && j < r && i <= j) M[(size_t)perm[i] * m + j] = S[(j + 1) * lds + i];
  }
  // -C M: row l, column j < r sums over the pivoted rows i <= j
  for (int idx = tid; idx < kc * m; idx += EB) {
    const int l = idx / m, j = idx % m;
    double acc = 0.0;
    if (j < r)
      for (int i = 0; i <= j; ++i) acc += Cs[l * m + perm[i]] * S[(j + 1) * lds + i];
    Mout[idx] = -acc;
  }
  if (tid == 0) *rank_out = r;
  PHASE_MARK(12);
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

// LDL^T inertia of T - x I: the number of eigenvalues of the tridiagonal (dg, e2 = e^2)
// below x (Sturm count); tiny pivots are replaced by -pivmin.
__device__ inline int sturm_count(const double* dg, const double* e2, int n, double x, double pivmin) {
  double q = dg[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (dg[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

__device__ inline double hash_unit(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)(h & 0xFFFFFF) / 16777216.0) - 0.5;
}

template <bool IN_LDS>
__global__ void __launch_bounds__(EB) k_small_eig(int d_full, int base, const int32_t* rank_p,
                                                  const double* H, int which, int kk, double drop_tol,
                                                  double* theta_out, double* F, int32_t* kept_out,
                                                  double* work, int32_t* status) {
  __shared__ double sA[IN_LDS ? SMALL_LDS_D * (SMALL_LDS_D + 1) : 1];
  __shared__ double dg[MAXD], od[MAXD], e2[MAXD], vv[MAXD], pw[MAXD], hb[MAXD], ev[MAXD];
  __shared__ double red[EB / GREST_WAVE];
  __shared__ int sel[MAXD], slot_of[MAXD], srt[MAXD];
  __shared__ double sh_d[4];
  __shared__ int sh_i[2];
  const int tid = threadIdx.x;
  int n = base + (rank_p ? rank_p[0] : 0);
  if (n > d_full) n = d_full;
  if (n < 0) n = 0;
  double* A = IN_LDS ? sA : work;
  double* scratch = IN_LDS ? work : work + (size_t)(d_full + 1) * (d_full + 1);
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

  PHASE_MARK(0);
  // ---- Householder tridiagonalisation; reflector k stored below the subdiagonal ----
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
      for (int i = tid; i < m; i += EB) pw[i] -= K * vv[i];
      __syncthreads();
      for (int idx = tid; idx < m * m; idx += EB) {
        int i = idx / m, j = idx % m;
        A[(k + 1 + i) * lda + (k + 1 + j)] -= vv[i] * pw[j] + pw[i] * vv[j];
      }
    }
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
    // Gershgorin interval, norm, pivot floor
    double lo = 0.0, hi = 0.0, tn = 0.0, emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(od[i - 1]) : 0.0) + (i + 1 < n ? fabs(od[i]) : 0.0);
      lo = (i == 0) ? dg[i] - r : fmin(lo, dg[i] - r);
      hi = (i == 0) ? dg[i] + r : fmax(hi, dg[i] + r);
      tn = fmax(tn, fabs(dg[i]) + r);
      if (i + 1 < n) { e2[i] = od[i] * od[i]; emax = fmax(emax, e2[i]); }
    }
    const double pad = 4.0 * 2.220446049250313e-16 * fmax(tn, 1e-300) + 1e-300;
    sh_d[0] = lo - pad;
    sh_d[1] = hi + pad;
    sh_d[2] = tn;
    sh_d[3] = 1e-290 * fmax(1.0, emax);
  }
  __syncthreads();

  PHASE_MARK(1);
  // ---- eigenvalues: one lane per index, bisection on the inertia count ----
  const double eps = 2.220446049250313e-16;
  const double pivmin = sh_d[3];
  const double tnorm = sh_d[2];
  for (int t = tid; t < n; t += EB) {
    double lo = sh_d[0], hi = sh_d[1];
    for (int it = 0; it < 80; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
      if (sturm_count(dg, e2, n, mid, pivmin) > t) hi = mid; else lo = mid;
    }
    ev[t] = 0.5 * (lo + hi);
  }
  for (int i = tid; i < MAXD; i += EB) { slot_of[i] = -1; }
  __syncthreads();

  PHASE_MARK(2);
  // ---- selection of kk pairs (ev is ascending) ----
  double tmax = 0.0;
  for (int i = 0; i < n; ++i) tmax = fmax(tmax, ev[i]);
  const double keep_thr = drop_tol > 0.0 ? drop_tol * drop_tol * fmax(1.0, tmax) : -INFINITY;
  for (int i = tid; i < n; i += EB) {
    int rank = 0;
    for (int j = 0; j < n; ++j)
      if (j != i && sel_less(which, ev[j], j, ev[i], i)) ++rank;
    if (rank < kk) { sel[rank] = i; slot_of[i] = rank; }
  }
  __syncthreads();
  const int nsel = kk < n ? kk : n;
  if (tid == 0) {  // selected indices in ascending order
    int c = 0;
    for (int i = 0; i < n; ++i)
      if (slot_of[i] >= 0) srt[c++] = i;
  }
  __syncthreads();

  PHASE_MARK(3);
  // ---- eigenvectors of T by inverse iteration; a cluster (gaps below 1e-3 ||T||) is
  //      handled by one lane with distinct shifts and reorthogonalisation ----
  const double ortol = 1e-3 * tnorm;
  // The reflectors move to global memory so that the LDS matrix becomes the scratch of
  // the inverse iterations (six vectors of length n per cluster leader).
  double* refl = work;
  if (IN_LDS) {
    for (int idx = tid; idx < n * lda; idx += EB) refl[idx] = A[idx];
  }
  __syncthreads();
  const int per = 6 * (n > 0 ? n : 1);
  const int cap = IN_LDS ? (SMALL_LDS_D * (SMALL_LDS_D + 1)) / per : EB;
  int lrank = 0;  // rank of this lane's leader among the leaders
  bool leader = false;
  const int q = tid;
  if (q < nsel) {
    leader = !(q > 0 && ev[srt[q]] - ev[srt[q - 1]] <= ortol);
    for (int qq = 1; qq < q; ++qq) lrank += !(ev[srt[qq]] - ev[srt[qq - 1]] <= ortol);
    if (q > 0) lrank += 1;  // q == 0 is always a leader
  }
  const int nlead_max = nsel;  // upper bound on leaders, for the round count
  for (int round = 0; round * cap < nlead_max; ++round) {
   if (leader && lrank / cap == round) {
    const int slot_l = lrank % cap;
    double* u0 = IN_LDS ? sA + (size_t)slot_l * per : scratch + (size_t)q * 6 * MAXD;
    const int st = IN_LDS ? n : MAXD;
    double* u1 = u0 + st;
    double* u2 = u1 + st;
    double* lm = u2 + st;
    double* x = lm + st;
    double* piv = x + st;
    double shift_prev = -INFINITY;
    for (int p = q; p < nsel && (p == q || ev[srt[p]] - ev[srt[p - 1]] <= ortol); ++p) {
      const int idx = srt[p];
      const int slot = slot_of[idx];
      double lam = ev[idx];
      if (p > q) lam = fmax(lam, shift_prev + 10.0 * eps * fmax(tnorm, 1e-300));
      shift_prev = lam;
      // LU with partial pivoting of T - lam I (three upper diagonals)
      double a = dg[0] - lam, bsup = n > 1 ? od[0] : 0.0;
      for (int i = 0; i + 1 < n; ++i) {
        const double c = od[i];                    // (i+1, i)
        const double an = dg[i + 1] - lam;         // (i+1, i+1)
        const double bn = i + 2 < n ? od[i + 1] : 0.0;  // (i+1, i+2)
        if (fabs(a) >= fabs(c)) {
          const double piv_a = (a == 0.0) ? pivmin : a;
          const double l = c / piv_a;
          u0[i] = piv_a; u1[i] = bsup; u2[i] = 0.0; lm[i] = l; piv[i] = 0.0;
          a = an - l * bsup;
          bsup = bn;
        } else {
          const double l = a / c;
          u0[i] = c; u1[i] = an; u2[i] = bn; lm[i] = l; piv[i] = 1.0;
          a = bsup - l * an;
          bsup = -l * bn;
        }
      }
      u0[n - 1] = (a == 0.0) ? pivmin : a;
      for (int i = 0; i < n; ++i) x[i] = hash_unit(i, slot + 1);
      for (int it = 0; it < 2; ++it) {
        for (int i = 0; i + 1 < n; ++i) {  // L^{-1} with the row interchanges
          if (piv[i] != 0.0) { const double t = x[i]; x[i] = x[i + 1]; x[i + 1] = t; }
          x[i + 1] -= lm[i] * x[i];
        }
        for (int i = n - 1; i >= 0; --i) {  // U^{-1}
          double v = x[i];
          if (i + 1 < n) v -= u1[i] * x[i + 1];
          if (i + 2 < n) v -= u2[i] * x[i + 2];
          x[i] = v / u0[i];
        }
        for (int pp = q; pp < p; ++pp) {  // against the finished members of the cluster
          const int sl = slot_of[srt[pp]];
          double dot = 0.0;
          for (int i = 0; i < n; ++i) dot += x[i] * F[(size_t)i * kk + sl];
          for (int i = 0; i < n; ++i) x[i] -= dot * F[(size_t)i * kk + sl];
        }
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) nrm += x[i] * x[i];
        nrm = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        for (int i = 0; i < n; ++i) x[i] *= nrm;
      }
      for (int i = 0; i < n; ++i) F[(size_t)i * kk + slot] = x[i];
    }
   }
   __syncthreads();
  }

  PHASE_MARK(4);
  // ---- back-transform x <- P_0 ... P_{n-3} x; eight lanes per vector, rows interleaved ----
  constexpr int G = 8, RMAX = MAXD / G;
  const int grp = tid / G, gl = tid % G;
  for (int s0 = 0; s0 < nsel; s0 += EB / G) {
    const int slot = s0 + grp;
    const bool act = slot < nsel;
    double xr[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      const int r = gl + G * c;
      xr[c] = (act && r < n) ? F[(size_t)r * kk + slot] : 0.0;
    }
    for (int k = n - 3; k >= 0; --k) {
      const double beta = hb[k];
      if (beta == 0.0) continue;
      double dot = 0.0;
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        const int r = gl + G * c;
        if (r >= k + 1 && r < n) dot += (r == k + 1 ? 1.0 : refl[r * lda + k]) * xr[c];
      }
#pragma unroll
      for (int o = 1; o < G; o <<= 1) dot += __shfl_xor(dot, o, G);
      dot *= beta;
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        const int r = gl + G * c;
        if (r >= k + 1 && r < n) xr[c] -= dot * (r == k + 1 ? 1.0 : refl[r * lda + k]);
      }
    }
    if (act) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        const int r = gl + G * c;
        if (r < d_full) F[(size_t)r * kk + slot] = (r < n) ? xr[c] : 0.0;
      }
    }
  }
  __syncthreads();

  PHASE_MARK(5);
  // ---- values, dropped columns, kept count ----
  if (tid == 0) sh_i[0] = 0;
  __syncthreads();
  for (int slot = tid; slot < kk; slot += EB) {
    if (slot < nsel) {
      const double ti = ev[sel[slot]];
      const bool keep = !(drop_tol > 0.0) || ti > keep_thr;
      theta_out[slot] = keep ? ti : 0.0;
      if (keep) atomicAdd(&sh_i[0], 1);
      else for (int r = 0; r < d_full; ++r) F[(size_t)r * kk + slot] = 0.0;
    } else {
      theta_out[slot] = 0.0;
      for (int r = 0; r < d_full; ++r) F[(size_t)r * kk + slot] = 0.0;
    }
  }
  __syncthreads();
  if (tid == 0 && kept_out) *kept_out = sh_i[0];
  PHASE_MARK(6);
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

int64_t eig_work_elems(int d) { return (int64_t)(d + 1) * (d + 1) + (int64_t)6 * MAXD * MAXD; }

int64_t pchol_work_elems(int m, int kc) { return (int64_t)(m + 1) * (m + 1) + (int64_t)kc * m; }

void launch_pchol(int m, const double* G, const double* C, int kc, double tol, double* Mout, int32_t* rank,
                  int32_t* status, double* work, hipStream_t s) {
  const size_t lds = (size_t)pchol_work_elems(m, C ? kc : 0) * sizeof(double);
  if (!C) kc = 0;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_pchol<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    attr = true;
  }
  if (lds <= 150 * 1024) k_pchol<true><<<1, EB, lds, s>>>(m, G, C, kc, tol, Mout, rank, status, nullptr);
  else k_pchol<false><<<1, EB, 0, s>>>(m, G, C, kc, tol, Mout, rank, status, work);
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
