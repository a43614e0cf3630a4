// Products with the update of the tracked operator:
//   * k_delta: the Prop. 3 block Delta_1 Xbar, the sketch Delta_2 Omega of the randomized
//     range finder, the transpose product Delta_2^T M, and the dense Delta_2 of G-REST3;
//   * k_nlap_dx: Delta_Tn Xbar for the normalised Laplacian, where the update rescales
//     whole rows: computed as S'A'S' Xbar - [S A S X; 0] row by row.
#include <algorithm>

#include "rowvec.h"

namespace {
// ---------------------------------------------------------------------------------
// products with the update of the tracked operator
// ---------------------------------------------------------------------------------
struct DeltaArgs {
  int64_t n_old, n_new;
  const int64_t* dptr;
  const int32_t* dcol;
  const int8_t* dsg;
  const int64_t* maxdeg;  // maximum degree of the updated graph (alpha' = 2 maxdeg)
  const int32_t* rows;    // modes 0 and 1: only these rows (a superset of the rows written), or null
  const int64_t* rcount;  // their count (device)
};

// weight of the Delta_2 entry (r, c) with c an appended node, and the diagonal of the
// new block, for the three operators (adj: Delta_2 of A; lap: alpha' I - L' restricted
// to the new columns; nlap: T_n' restricted to the new columns).
template <typename T, int OP>
__device__ inline T d2_weight(int8_t s, const T* snew, int64_t r, int64_t c) {
  if (OP == OPK_NLAP) return snew[r] * snew[c];
  (void)r; (void)c;
  return T(s);
}

template <typename T, int OP>
__device__ inline T d2_diag(const DeltaArgs& a, int64_t node) {
  if (OP == OPK_ADJ) return T(0);
  if (OP == OPK_NLAP) return T(1);
  const int64_t deg = a.dptr[node + 1] - a.dptr[node];  // every edge of an appended node is in Delta
  return T(2 * (double)a.maxdeg[0] - (double)deg);
}

// mode 0: out[r] = (Delta_T)[r, 0:n_old] X  for every r < n_old + n_new (zero rows included);
//         with acc set, also acc[r] += out[r] on the old rows that have entries and
//         acc[r] = out[r] on the appended rows (the product of the updated operator with the
//         padded block, from the old operator's product kept in acc)
// mode 1: out[r] = (Delta_T)[r, n_old:] Omega, written only on the appended rows and the
//         rows with an entry in an appended column (every other row is zero and is left
//         as it is: the caller keeps those rows zero)
// mode 2: out[j] = (Delta_T)[n_old + j, :] M  (= (Delta_T,2^T M)[j] by symmetry)
// With a row list (modes 0 and 1) just the listed rows are visited: for mode 0 the rows of
// Delta with an entry, the caller having zeroed out (and acc_io's appended rows)
// beforehand; for mode 1 the appended rows and the rows with an entry in an appended column.
template <typename T, int VEC, int OP, int MODE>
__global__ void __launch_bounds__(BS) k_delta(DeltaArgs a, const T* __restrict__ snew,
                                              const T* __restrict__ in, int64_t ldin, int w,
                                              T* __restrict__ out, int64_t ldout, T* __restrict__ acc_io,
                                              int64_t ldacc, int lpr_shift, int64_t skip_deg) {
  const int lpr = 1 << lpr_shift;
  const int64_t gid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int gl = (int)(gid & (lpr - 1));
  const int64_t ngroups = ((int64_t)gridDim.x * BS) >> lpr_shift;
  const int64_t n2 = a.n_old + a.n_new;
  const bool listed = MODE <= 1 && a.rows;
  const int64_t nrows = listed ? *a.rcount : (MODE == 2) ? a.n_new : n2;
  for (int64_t q = gid >> lpr_shift; q < nrows; q += ngroups) {
    const int64_t r = listed ? (int64_t)a.rows[q] : (MODE == 2) ? a.n_old + q : q;
    const int64_t orow = (MODE == 2) ? q : r;
    int64_t beg = a.dptr[r];
    const int64_t end = a.dptr[r + 1];
    if (MODE != 1 && end - beg > skip_deg) continue;  // a heavy row: k_delta_heavy
    if (MODE == 1) {  // the row is sorted by column: start at its first appended column
      int64_t lo = beg, hi = end;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)a.dcol[mid] < a.n_old) lo = mid + 1;
        else hi = mid;
      }
      beg = lo;
    }
    for (int c0 = gl * VEC; c0 < w; c0 += lpr * VEC) {
      T acc[VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) acc[i] = T(0);
      int32_t ssum = 0;
      bool any_new = false;  // mode 1: an entry in an appended column
      for (int64_t e = beg; e < end; ++e) {
        const int64_t c = a.dcol[e];
        const int8_t sg = a.dsg[e];
        ssum += sg;
        T wgt;
        int64_t src;
        if (MODE == 0) {
          if (c >= a.n_old) continue;
          wgt = T(sg);
          src = c;
        } else if (MODE == 1) {
          if (c < a.n_old) continue;
          any_new = true;
          wgt = d2_weight<T, OP>(sg, snew, r, c);
          src = c - a.n_old;
        } else {
          wgt = d2_weight<T, OP>(sg, snew, r, c);
          src = c;
        }
        T z[VEC];
        vload<T, VEC>(in + src * ldin + c0, z);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] += wgt * z[i];
      }
      if (MODE == 0 && OP == OPK_LAP && r < a.n_old && ssum != 0) {
        // -(D' - D) Xbar on the old rows (the alpha' - alpha shift lies in span(Xbar))
        T z[VEC];
        vload<T, VEC>(in + r * ldin + c0, z);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] -= T(ssum) * z[i];
      }
      if (MODE != 0 && r >= a.n_old) {
        const T dgl = d2_diag<T, OP>(a, r);
        if (dgl != T(0)) {
          T z[VEC];
          vload<T, VEC>(in + (MODE == 1 ? r - a.n_old : r) * ldin + c0, z);
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc[i] += dgl * z[i];
        }
      }
      // mode 1 leaves the old rows without an entry in an appended column alone: they are
      // zero, and the caller keeps them zero
      if (MODE != 1 || r >= a.n_old || any_new) vstore<T, VEC>(out + orow * ldout + c0, acc);
      if (MODE == 0 && acc_io) {
        T* pa = acc_io + r * ldacc + c0;
        if (r >= a.n_old) {
          vstore<T, VEC>(pa, acc);
        } else if (end > beg) {
          T old[VEC];
          vload<T, VEC>(pa, old);
#pragma unroll
          for (int i = 0; i < VEC; ++i) old[i] += acc[i];
          vstore<T, VEC>(pa, old);
        }
      }
    }
  }
}

// Modes 0 and 2 on the heavy rows of Delta (more than HEAVY_DEG entries: a hub that gains
// or loses many edges in one update, or an appended node with many edges), one workgroup of
// HEAVY_BS threads per row: its lane groups take contiguous, equal shares of the row's
// entries and keep their partial sums (and partial sign sums) in LDS, the workgroup adds
// them in a fixed order and applies the mode's epilogue (mode 0: the Laplacian's degree term
// and the kept product; mode 2: the diagonal of the appended block, rows of appended nodes
// only).  The row-split kernel would leave a row of thousands of entries to one lane group.
template <typename T, int VEC, int OP, int MODE>
__global__ void __launch_bounds__(HEAVY_BS) k_delta_heavy(DeltaArgs a, const T* __restrict__ snew,
                                                          const int32_t* __restrict__ hrows,
                                                          const int64_t* __restrict__ hcount,
                                                          const T* __restrict__ in, int64_t ldin, int w,
                                                          T* __restrict__ out, int64_t ldout, T* __restrict__ acc_io,
                                                          int64_t ldacc, int lpr_shift) {
  extern __shared__ char delta_smem[];
  T* part = reinterpret_cast<T*>(delta_smem);  // [groups][w]
  __shared__ int32_t gsum[HEAVY_BS];           // sign sum of each group's share
  if ((int64_t)blockIdx.x >= *hcount) return;
  const int64_t r = hrows[blockIdx.x];
  if (MODE == 2 && r < a.n_old) return;  // mode 2 covers the appended rows only
  const int lpr = 1 << lpr_shift;
  const int groups = HEAVY_BS >> lpr_shift;
  const int grp = threadIdx.x >> lpr_shift, gl = threadIdx.x & (lpr - 1);
  const int64_t beg = a.dptr[r], end = a.dptr[r + 1];
  const int64_t share = (end - beg + groups - 1) / groups;
  const int64_t e0 = min(end, beg + grp * share), e1 = min(end, e0 + share);
  if (MODE == 0 && gl == 0) {
    int32_t ss = 0;
    for (int64_t e = e0; e < e1; ++e) ss += a.dsg[e];
    gsum[grp] = ss;
  }
  for (int c0 = gl * VEC; c0 < w; c0 += lpr * VEC) {
    T acc[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) acc[i] = T(0);
    for (int64_t e = e0; e < e1; ++e) {
      const int64_t c = a.dcol[e];
      if (MODE == 0 && c >= a.n_old) continue;
      const T wgt = MODE == 0 ? T(a.dsg[e]) : d2_weight<T, OP>(a.dsg[e], snew, r, c);
      T z[VEC];
      vload<T, VEC>(in + c * ldin + c0, z);
#pragma unroll
      for (int i = 0; i < VEC; ++i) acc[i] += wgt * z[i];
    }
#pragma unroll
    for (int i = 0; i < VEC; ++i) part[(size_t)grp * w + c0 + i] = acc[i];
  }
  __syncthreads();
  int32_t ssum = 0;
  if (MODE == 0)
    for (int g = 0; g < groups; ++g) ssum += gsum[g];
  const T dgl = MODE == 2 ? d2_diag<T, OP>(a, r) : T(0);
  for (int c = threadIdx.x; c < w; c += HEAVY_BS) {
    T sum = T(0);
    for (int g = 0; g < groups; ++g) sum += part[(size_t)g * w + c];
    if (MODE == 0) {
      if (OP == OPK_LAP && r < a.n_old && ssum != 0) sum -= T(ssum) * in[r * ldin + c];
      out[r * ldout + c] = sum;
      if (acc_io) {
        if (r >= a.n_old) acc_io[r * ldacc + c] = sum;
        else acc_io[r * ldacc + c] += sum;
      }
    } else {
      if (dgl != T(0)) sum += dgl * in[r * ldin + c];
      out[(r - a.n_old) * ldout + c] = sum;
    }
  }
}

// mode 3: out[:, j] = (Delta_T)[:, n_old + j] densely (out zero-filled beforehand)
template <typename T, int OP>
__global__ void __launch_bounds__(BS) k_delta_dense2(DeltaArgs a, const T* __restrict__ snew,
                                                     T* __restrict__ out, int64_t ldout) {
  const int64_t gid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * BS;
  for (int64_t j = gid; j < a.n_new; j += nth) {
    const int64_t r = a.n_old + j;
    for (int64_t e = a.dptr[r]; e < a.dptr[r + 1]; ++e) {
      const int64_t c = a.dcol[e];
      out[c * ldout + j] = d2_weight<T, OP>(a.dsg[e], snew, c, r);
    }
    const T dgl = d2_diag<T, OP>(a, r);
    if (dgl != T(0)) out[r * ldout + j] = dgl;
  }
}

// One row of Delta_Tn Xbar for the normalised Laplacian, columns c0 .. c0 + VEC, over the
// entries [e0, e1) of the new row and [f0, f1) of the old one: the sums of s'_c x_c over
// the new row's old columns and of s_c x_c over the old row (four gathers in flight).
template <typename T, int VEC>
__device__ inline void nlap_dx_range(int64_t n_old, int64_t e0, int64_t e1, const int32_t* __restrict__ coln,
                                     const T* __restrict__ sn, int64_t f0, int64_t f1,
                                     const int32_t* __restrict__ colo, const T* __restrict__ so,
                                     const T* __restrict__ X, int64_t ldx, int c0, T (&a1)[VEC], T (&a0)[VEC]) {
  int64_t e = e0;
  for (; e + 4 <= e1; e += 4) {
    int32_t c[4];
    T z[4][VEC];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = coln[e + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c[u] < n_old) vload<T, VEC>(X + (int64_t)c[u] * ldx + c0, z[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c[u] >= n_old) continue;
      const T scu = sn[c[u]];
#pragma unroll
      for (int i = 0; i < VEC; ++i) a1[i] += scu * z[u][i];
    }
  }
  for (; e < e1; ++e) {
    const int32_t c = coln[e];
    if (c >= n_old) continue;
    T z[VEC];
    vload<T, VEC>(X + (int64_t)c * ldx + c0, z);
    const T scu = sn[c];
#pragma unroll
    for (int i = 0; i < VEC; ++i) a1[i] += scu * z[i];
  }
  int64_t f = f0;
  for (; f + 4 <= f1; f += 4) {
    int32_t c[4];
    T z[4][VEC];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = colo[f + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) vload<T, VEC>(X + (int64_t)c[u] * ldx + c0, z[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T scu = so[c[u]];
#pragma unroll
      for (int i = 0; i < VEC; ++i) a0[i] += scu * z[u][i];
    }
  }
  for (; f < f1; ++f) {
    const int32_t c = colo[f];
    T z[VEC];
    vload<T, VEC>(X + (int64_t)c * ldx + c0, z);
    const T scu = so[c];
#pragma unroll
    for (int i = 0; i < VEC; ++i) a0[i] += scu * z[i];
  }
}

// Rows whose new row has more than skip_deg entries are left to k_nlap_dx_heavy.
template <typename T, int VEC>
__global__ void __launch_bounds__(BS) k_nlap_dx(int64_t n_old, int64_t n2, const int64_t* __restrict__ rpo,
                                                const int32_t* __restrict__ colo, const T* __restrict__ so,
                                                const int64_t* __restrict__ rpn,
                                                const int32_t* __restrict__ coln, const T* __restrict__ sn,
                                                const T* __restrict__ X, int64_t ldx, int w,
                                                T* __restrict__ V, int64_t ldv, int lpr_shift, int64_t skip_deg) {
  const int lpr = 1 << lpr_shift;
  const int64_t gid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int gl = (int)(gid & (lpr - 1));
  const int64_t ngroups = ((int64_t)gridDim.x * BS) >> lpr_shift;
  for (int64_t r = gid >> lpr_shift; r < n2; r += ngroups) {
    const int64_t e0 = rpn[r], e1 = rpn[r + 1];
    if (e1 - e0 > skip_deg) continue;
    const int64_t f0 = r < n_old ? rpo[r] : 0, f1 = r < n_old ? rpo[r + 1] : 0;
    for (int c0 = gl * VEC; c0 < w; c0 += lpr * VEC) {
      T a1[VEC], a0[VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) { a1[i] = T(0); a0[i] = T(0); }
      nlap_dx_range<T, VEC>(n_old, e0, e1, coln, sn, f0, f1, colo, so, X, ldx, c0, a1, a0);
      const T s1 = sn[r];
      const T s0 = r < n_old ? so[r] : T(0);
      T o[VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) o[i] = s1 * a1[i] - s0 * a0[i];
      vstore<T, VEC>(V + r * ldv + c0, o);
    }
  }
}

// The heavy rows (of the new graph) of Delta_Tn Xbar: a workgroup per row, its lane groups
// taking equal shares of the new row's and of the old row's entries, partial sums added in
// LDS in a fixed order (as k_spmm_heavy).
template <typename T, int VEC>
__global__ void __launch_bounds__(HEAVY_BS) k_nlap_dx_heavy(const int32_t* __restrict__ hrows,
                                                            const int64_t* __restrict__ hcount, int64_t n_old,
                                                            const int64_t* __restrict__ rpo,
                                                            const int32_t* __restrict__ colo,
                                                            const T* __restrict__ so, const int64_t* __restrict__ rpn,
                                                            const int32_t* __restrict__ coln,
                                                            const T* __restrict__ sn, const T* __restrict__ X,
                                                            int64_t ldx, int w, T* __restrict__ V, int64_t ldv,
                                                            int lpr_shift) {
  extern __shared__ char nlap_smem[];
  T* p1 = reinterpret_cast<T*>(nlap_smem);  // [groups][w], then the old row's [groups][w]
  if ((int64_t)blockIdx.x >= *hcount) return;
  const int64_t r = hrows[blockIdx.x];
  const int lpr = 1 << lpr_shift;
  const int groups = HEAVY_BS >> lpr_shift;
  T* p0 = p1 + (size_t)groups * w;
  const int grp = threadIdx.x >> lpr_shift, gl = threadIdx.x & (lpr - 1);
  const int64_t b1 = rpn[r], l1 = rpn[r + 1] - b1;
  const int64_t b0 = r < n_old ? rpo[r] : 0, l0 = r < n_old ? rpo[r + 1] - b0 : 0;
  const int64_t sh1 = (l1 + groups - 1) / groups, sh0 = (l0 + groups - 1) / groups;
  const int64_t e0 = b1 + min(l1, grp * sh1), e1 = b1 + min(l1, (grp + 1) * sh1);
  const int64_t f0 = b0 + min(l0, grp * sh0), f1 = b0 + min(l0, (grp + 1) * sh0);
  for (int c0 = gl * VEC; c0 < w; c0 += lpr * VEC) {
    T a1[VEC], a0[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) { a1[i] = T(0); a0[i] = T(0); }
    nlap_dx_range<T, VEC>(n_old, e0, e1, coln, sn, f0, f1, colo, so, X, ldx, c0, a1, a0);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      p1[(size_t)grp * w + c0 + i] = a1[i];
      p0[(size_t)grp * w + c0 + i] = a0[i];
    }
  }
  __syncthreads();
  const T s1 = sn[r];
  const T s0 = r < n_old ? so[r] : T(0);
  for (int c = threadIdx.x; c < w; c += HEAVY_BS) {
    T t1 = T(0), t0 = T(0);
    for (int g = 0; g < groups; ++g) {
      t1 += p1[(size_t)g * w + c];
      t0 += p0[(size_t)g * w + c];
    }
    V[r * ldv + c] = s1 * t1 - s0 * t0;
  }
}

}  // namespace

template <typename T, int OP, int MODE>
static void delta_dispatch(int vec, const DeltaArgs& a, const T* snew, const T* in, int64_t ldin, int w,
                           T* out, int64_t ldout, T* acc_io, int64_t ldacc, hipStream_t s, int64_t bound,
                           const HeavyRows* heavy) {
  const int64_t rows = (MODE <= 1 && a.rows) ? bound : (MODE == 2) ? a.n_new : a.n_old + a.n_new;
  if (rows <= 0 || w <= 0) return;
  const int lpr = lanes_per_row(w, vec);
  const int g = grid_for(rows * lpr);
  const bool hv = MODE != 1 && heavy && heavy->bound > 0;
  const int64_t skip = hv ? HEAVY_DEG : INT64_MAX;
  constexpr int V = 16 / sizeof(T);
  if (vec == V)
    k_delta<T, V, OP, MODE><<<g, BS, 0, s>>>(a, snew, in, ldin, w, out, ldout, acc_io, ldacc, ilog2(lpr), skip);
  else
    k_delta<T, 1, OP, MODE><<<g, BS, 0, s>>>(a, snew, in, ldin, w, out, ldout, acc_io, ldacc, ilog2(lpr), skip);
  if constexpr (MODE != 1) {
    if (!hv) return;
    const size_t lds = (size_t)(HEAVY_BS / lpr) * w * sizeof(T);
    const unsigned hg = (unsigned)std::min<int64_t>(heavy->bound, a.n_old + a.n_new);
    if (vec == V)
      k_delta_heavy<T, V, OP, MODE><<<hg, HEAVY_BS, lds, s>>>(a, snew, heavy->rows, heavy->count, in, ldin, w, out,
                                                              ldout, acc_io, ldacc, ilog2(lpr));
    else
      k_delta_heavy<T, 1, OP, MODE><<<hg, HEAVY_BS, lds, s>>>(a, snew, heavy->rows, heavy->count, in, ldin, w, out,
                                                              ldout, acc_io, ldacc, ilog2(lpr));
  }
}

template <typename T, int OP>
static void delta_mode(int mode, int vec, const DeltaArgs& a, const T* snew, const T* in, int64_t ldin,
                       int w, T* out, int64_t ldout, T* acc_io, int64_t ldacc, hipStream_t s, int64_t bound,
                       const HeavyRows* heavy) {
  if (mode == 0) delta_dispatch<T, OP, 0>(vec, a, snew, in, ldin, w, out, ldout, acc_io, ldacc, s, bound, heavy);
  else if (mode == 1) delta_dispatch<T, OP, 1>(vec, a, snew, in, ldin, w, out, ldout, nullptr, 0, s, bound, nullptr);
  else if (mode == 2) delta_dispatch<T, OP, 2>(vec, a, snew, in, ldin, w, out, ldout, nullptr, 0, s, 0, heavy);
  else if (a.n_new > 0) k_delta_dense2<T, OP><<<grid_for(a.n_new), BS, 0, s>>>(a, snew, out, ldout);
}

template <typename T>
void launch_delta_mul(int mode, int op, int64_t n_old, int64_t n_new, const int64_t* dptr,
                      const int32_t* dcol, const int8_t* dsg, const int64_t* maxdeg, const T* snew,
                      const T* in, int64_t ldin, int w, T* out, int64_t ldout, hipStream_t s, T* acc_io,
                      int64_t ldacc, const int32_t* rows, const int64_t* rcount, int64_t bound,
                      const HeavyRows* heavy) {
  if (mode > 1 || bound <= 0) rows = nullptr;
  DeltaArgs a{n_old, n_new, dptr, dcol, dsg, maxdeg, rows, rows ? rcount : nullptr};
  int vec = (mode == 3) ? 1 : pick_vec<T>(w, ldin, ldout, in, out);
  if (acc_io && vec > 1 && (ldacc % vec != 0 || ((uintptr_t)acc_io % 16) != 0)) vec = 1;
  if (op == OPK_ADJ)
    delta_mode<T, OPK_ADJ>(mode, vec, a, snew, in, ldin, w, out, ldout, acc_io, ldacc, s, bound, heavy);
  else if (op == OPK_LAP)
    delta_mode<T, OPK_LAP>(mode, vec, a, snew, in, ldin, w, out, ldout, acc_io, ldacc, s, bound, heavy);
  else delta_mode<T, OPK_NLAP>(mode, vec, a, snew, in, ldin, w, out, ldout, acc_io, ldacc, s, bound, heavy);
}

template <typename T>
void launch_nlap_delta_x(int64_t n_old, int64_t n_new, const int64_t* rp_old, const int32_t* col_old,
                         const T* s_old, const int64_t* rp_new, const int32_t* col_new, const T* s_new,
                         const T* X, int64_t ldx, int k, T* V, int64_t ldv, hipStream_t s, const HeavyRows* heavy) {
  const int64_t n2 = n_old + n_new;
  if (n2 <= 0 || k <= 0) return;
  const int vec = pick_vec<T>(k, ldx, ldv, X, V);
  const int lpr = lanes_per_row(k, vec);
  const int g = grid_for(n2 * lpr);
  const bool hv = heavy && heavy->bound > 0;
  const int64_t skip = hv ? HEAVY_DEG : INT64_MAX;
  if (vec == 16 / (int)sizeof(T))
    k_nlap_dx<T, 16 / sizeof(T)><<<g, BS, 0, s>>>(n_old, n2, rp_old, col_old, s_old, rp_new, col_new,
                                                  s_new, X, ldx, k, V, ldv, ilog2(lpr), skip);
  else
    k_nlap_dx<T, 1><<<g, BS, 0, s>>>(n_old, n2, rp_old, col_old, s_old, rp_new, col_new, s_new, X, ldx,
                                     k, V, ldv, ilog2(lpr), skip);
  if (!hv) return;
  const int groups = HEAVY_BS / lpr;
  const size_t lds = 2 * (size_t)groups * k * sizeof(T);
  const unsigned hg = (unsigned)std::min<int64_t>(heavy->bound, n2);
  if (vec == 16 / (int)sizeof(T))
    k_nlap_dx_heavy<T, 16 / sizeof(T)><<<hg, HEAVY_BS, lds, s>>>(heavy->rows, heavy->count, n_old, rp_old, col_old,
                                                                 s_old, rp_new, col_new, s_new, X, ldx, k, V, ldv,
                                                                 ilog2(lpr));
  else
    k_nlap_dx_heavy<T, 1><<<hg, HEAVY_BS, lds, s>>>(heavy->rows, heavy->count, n_old, rp_old, col_old, s_old,
                                                    rp_new, col_new, s_new, X, ldx, k, V, ldv, ilog2(lpr));
}

#define INST(T)                                                                                       \
  template void launch_delta_mul<T>(int, int, int64_t, int64_t, const int64_t*, const int32_t*,        \
                                    const int8_t*, const int64_t*, const T*, const T*, int64_t, int,  \
                                    T*, int64_t, hipStream_t, T*, int64_t, const int32_t*,            \
                                    const int64_t*, int64_t, const HeavyRows*);                       \
  template void launch_nlap_delta_x<T>(int64_t, int64_t, const int64_t*, const int32_t*, const T*,     \
                                       const int64_t*, const int32_t*, const T*, const T*, int64_t,   \
                                       int, T*, int64_t, hipStream_t, const HeavyRows*);
INST(float)
INST(double)
#undef INST
