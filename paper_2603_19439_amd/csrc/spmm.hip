// The product of the updated operator with the basis, (op Z): row-split CSR with a group of
// lanes per row, each lane owning a 16-, 8- or 4-byte slice of the dense row; the Laplacians
// use the difference form sum_c (z_r - z_c) so that small eigenvalues keep their relative
// accuracy in FP32.  Rows with more than HEAVY_DEG entries go to a workgroup each.
#include <algorithm>

#include "rowvec.h"

namespace {
// ---------------------------------------------------------------------------------
// (op Z) for the stored graph
// ---------------------------------------------------------------------------------
// A row's entries [e0, e1) against columns c0 .. c0 + VEC of Z: the sum of the gathered
// rows, or of (z_r - z_c) for the Laplacians (with zr = s_r z_r and s_c z_c for L_n).
template <typename T, int VEC, int OP>
__device__ inline void spmm_range(int64_t e0, int64_t e1, const int32_t* __restrict__ col, const T* __restrict__ sc,
                                  const T* __restrict__ Z, int64_t ldz, int c0, const T (&zr)[VEC], T (&acc)[VEC]) {
  int64_t e = e0;
  for (; e + 4 <= e1; e += 4) {
    int32_t c[4];
    T z[4][VEC];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = col[e + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) vload<T, VEC>(Z + (int64_t)c[u] * ldz + c0, z[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T scu = (OP == OPK_NLAP) ? sc[c[u]] : T(1);
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        if (OP == OPK_ADJ) acc[i] += z[u][i];
        else if (OP == OPK_LAP) acc[i] += zr[i] - z[u][i];
        else acc[i] += zr[i] - scu * z[u][i];
      }
    }
  }
  for (; e < e1; ++e) {
    const int32_t c = col[e];
    T z[VEC];
    vload<T, VEC>(Z + (int64_t)c * ldz + c0, z);
    const T scu = (OP == OPK_NLAP) ? sc[c] : T(1);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      if (OP == OPK_ADJ) acc[i] += z[i];
      else if (OP == OPK_LAP) acc[i] += zr[i] - z[i];
      else acc[i] += zr[i] - scu * z[i];
    }
  }
}

// Rows with more than skip_deg entries are left to k_spmm_heavy.
template <typename T, int VEC, int OP>
__global__ void __launch_bounds__(BS) k_spmm(int64_t n, const int64_t* __restrict__ rp,
                                             const int32_t* __restrict__ col, const T* __restrict__ sc,
                                             const T* __restrict__ Z, int64_t ldz, int w,
                                             T* __restrict__ Y, int64_t ldy, int lpr_shift, int64_t skip_deg) {
  const int lpr = 1 << lpr_shift;
  const int64_t gid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int gl = (int)(gid & (lpr - 1));
  const int64_t ngroups = ((int64_t)gridDim.x * BS) >> lpr_shift;
  for (int64_t r = gid >> lpr_shift; r < n; r += ngroups) {
    const int64_t beg = rp[r], end = rp[r + 1];
    if (end - beg > skip_deg) continue;
    const T sr = (OP == OPK_NLAP) ? sc[r] : T(1);
    for (int c0 = gl * VEC; c0 < w; c0 += lpr * VEC) {
      T acc[VEC], zr[VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) { acc[i] = T(0); zr[i] = T(0); }
      if (OP != OPK_ADJ) vload<T, VEC>(Z + r * ldz + c0, zr);
      if (OP == OPK_NLAP) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) zr[i] *= sr;
      }
      spmm_range<T, VEC, OP>(beg, end, col, sc, Z, ldz, c0, zr, acc);
      if (OP == OPK_NLAP) {
        if (end == beg) {  // isolated node: (L_n)_rr = 1
          vload<T, VEC>(Z + r * ldz + c0, acc);
        } else {
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc[i] *= sr;
        }
      }
      vstore<T, VEC>(Y + r * ldy + c0, acc);
    }
  }
}

// Heavy rows (more than HEAVY_DEG entries; the hubs of power-law graphs): one workgroup of
// HEAVY_BS threads per row.  Its lane groups take contiguous, equal shares of the row's
// entries (the row is split by entries, not by rows), keep their partial sums in LDS, and
// the workgroup adds the partials in a fixed order, so the result does not depend on
// scheduling.  A row-split kernel would leave a whole hub of thousands of entries to one
// lane group.
template <typename T, int VEC, int OP>
__global__ void __launch_bounds__(HEAVY_BS) k_spmm_heavy(const int32_t* __restrict__ hrows,
                                                         const int64_t* __restrict__ hcount,
                                                         const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col, const T* __restrict__ sc,
                                                         const T* __restrict__ Z, int64_t ldz, int w,
                                                         T* __restrict__ Y, int64_t ldy, int lpr_shift) {
  extern __shared__ char spmm_smem[];
  T* part = reinterpret_cast<T*>(spmm_smem);  // [groups][w]
  if ((int64_t)blockIdx.x >= *hcount) return;
  const int64_t r = hrows[blockIdx.x];
  const int lpr = 1 << lpr_shift;
  const int groups = HEAVY_BS >> lpr_shift;
  const int grp = threadIdx.x >> lpr_shift, gl = threadIdx.x & (lpr - 1);
  const int64_t beg = rp[r], end = rp[r + 1];
  const int64_t share = (end - beg + groups - 1) / groups;
  const int64_t e0 = min(end, beg + grp * share), e1 = min(end, e0 + share);
  const T sr = (OP == OPK_NLAP) ? sc[r] : T(1);
  for (int c0 = gl * VEC; c0 < w; c0 += lpr * VEC) {
    T acc[VEC], zr[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) { acc[i] = T(0); zr[i] = T(0); }
    if (OP != OPK_ADJ) vload<T, VEC>(Z + r * ldz + c0, zr);
    if (OP == OPK_NLAP) {
#pragma unroll
      for (int i = 0; i < VEC; ++i) zr[i] *= sr;
    }
    spmm_range<T, VEC, OP>(e0, e1, col, sc, Z, ldz, c0, zr, acc);
#pragma unroll
    for (int i = 0; i < VEC; ++i) part[(size_t)grp * w + c0 + i] = acc[i];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < w; c += HEAVY_BS) {
    T sum = T(0);
    for (int g = 0; g < groups; ++g) sum += part[(size_t)g * w + c];
    if (OP == OPK_NLAP) sum *= sr;  // a heavy row is never isolated
    Y[r * ldy + c] = sum;
  }
}

template <typename T, int OP>
void spmm_dispatch(int vec, int64_t n, const int64_t* rp, const int32_t* col, const T* sc, const T* Z,
                   int64_t ldz, int w, T* Y, int64_t ldy, const HeavyRows* heavy, hipStream_t s) {
  const int lpr = lanes_per_row(w, vec);
  const int g = grid_for(n * lpr);
  const bool hv = heavy && heavy->bound > 0;
  const int64_t skip = hv ? HEAVY_DEG : INT64_MAX;
  if (vec == 16 / (int)sizeof(T))
    k_spmm<T, 16 / sizeof(T), OP><<<g, BS, 0, s>>>(n, rp, col, sc, Z, ldz, w, Y, ldy, ilog2(lpr), skip);
  else if (vec == 2)
    k_spmm<T, 2, OP><<<g, BS, 0, s>>>(n, rp, col, sc, Z, ldz, w, Y, ldy, ilog2(lpr), skip);
  else
    k_spmm<T, 1, OP><<<g, BS, 0, s>>>(n, rp, col, sc, Z, ldz, w, Y, ldy, ilog2(lpr), skip);
  if (!hv) return;
  const int groups = HEAVY_BS / lpr;
  const size_t lds = (size_t)groups * w * sizeof(T);
  const unsigned hg = (unsigned)std::min<int64_t>(heavy->bound, n);
  if (vec == 16 / (int)sizeof(T))
    k_spmm_heavy<T, 16 / sizeof(T), OP><<<hg, HEAVY_BS, lds, s>>>(heavy->rows, heavy->count, rp, col, sc, Z, ldz,
                                                                  w, Y, ldy, ilog2(lpr));
  else if (vec == 2)
    k_spmm_heavy<T, 2, OP><<<hg, HEAVY_BS, lds, s>>>(heavy->rows, heavy->count, rp, col, sc, Z, ldz, w, Y, ldy,
                                                     ilog2(lpr));
  else
    k_spmm_heavy<T, 1, OP><<<hg, HEAVY_BS, lds, s>>>(heavy->rows, heavy->count, rp, col, sc, Z, ldz, w, Y, ldy,
                                                     ilog2(lpr));
}

__global__ void k_heavy_flag(int64_t n, const int64_t* __restrict__ rp, int64_t* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * BS;
  for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n; r += stride)
    flag[r] = (rp[r + 1] - rp[r] > HEAVY_DEG) ? 1 : 0;
}

__global__ void k_heavy_compact(int64_t n, const int64_t* __restrict__ flag, const int64_t* __restrict__ pos,
                                int32_t* __restrict__ rows, int64_t* __restrict__ count) {
  const int64_t stride = (int64_t)gridDim.x * BS;
  for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n; r += stride)
    if (flag[r]) rows[pos[r]] = (int32_t)r;
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = pos[n];
}

}  // namespace

template <typename T>
void launch_spmm(int op, int64_t n, const int64_t* rp, const int32_t* col, const T* sc, const T* Z,
                 int64_t ldz, int64_t nz_rows, int w, T* Y, int64_t ldy, hipStream_t s, const HeavyRows* heavy) {
  (void)nz_rows;
  if (n <= 0 || w <= 0) return;
  const int vec = pick_vec2<T>(w, ldz, ldy, Z, Y);
  if (op == OPK_ADJ) spmm_dispatch<T, OPK_ADJ>(vec, n, rp, col, sc, Z, ldz, w, Y, ldy, heavy, s);
  else if (op == OPK_LAP) spmm_dispatch<T, OPK_LAP>(vec, n, rp, col, sc, Z, ldz, w, Y, ldy, heavy, s);
  else spmm_dispatch<T, OPK_NLAP>(vec, n, rp, col, sc, Z, ldz, w, Y, ldy, heavy, s);
}

void launch_heavy_rows(int64_t n, const int64_t* rp, int64_t* flag, int64_t* pos, int64_t* scan_tmp, int32_t* rows,
                       int64_t* count, hipStream_t s) {
  if (n <= 0) {
    launch_fill_i64(count, 0, 1, s);
    return;
  }
  k_heavy_flag<<<grid_for(n), BS, 0, s>>>(n, rp, flag);
  launch_scan_excl(flag, pos, n, scan_tmp, s);
  k_heavy_compact<<<grid_for(n), BS, 0, s>>>(n, flag, pos, rows, count);
}

#define INST(T)                                                                                       \
  template void launch_spmm<T>(int, int64_t, const int64_t*, const int32_t*, const T*, const T*,       \
                               int64_t, int64_t, int, T*, int64_t, hipStream_t, const HeavyRows*);
INST(float)
INST(double)
#undef INST
