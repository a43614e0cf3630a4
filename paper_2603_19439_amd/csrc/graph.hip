// Update of the stored graph: assembly of the symmetric update Delta and the merge
// A^(t+1) = pad(A^(t)) + Delta of the transition model (paper Sec. 2, eq. adj_update).
//
// The graph is a CSR with both triangles, int64 row offsets and int32 column ids
// sorted inside each row.  Delta arrives as a list of undirected changes (i < j, sign).
// Steps (all on the device):
//   1. the two directed entries of every change become keys (row, column) packed in
//      64 bits; the entries per row are counted                      (atomics)
//   2. exclusive scan of the counts -> row offsets of Delta          (3-kernel scan)
//   3. the keys are placed in their rows (each row's slots counted down from its count,
//      atomics) and every row is sorted by column: a thread per short row (insertion
//      sort), a workgroup per long row (bitonic sort in LDS), so every row of Delta is
//      contiguous and sorted whatever its length
//   4. a group of lanes per row, linear in the row: duplicates, insert/delete checks
//      against the old row (binary search), per-row prefix counts of insertions and
//      the new row length
//   5. exclusive scan of the new lengths -> new row offsets
//   6. blocks of rows: rows without changes are copied as one coalesced range per block;
//      rows with changes are merged by ranks (old entries not deleted + inserted
//      entries) by a group of lanes, fully parallel inside the row.
// Every write is bounds-checked against the row and the column capacity, so an
// invalid change list (reported through the status word before anything reads the
// new graph) can never write out of bounds.
#include <algorithm>

#include "grest_internal.h"

namespace {

constexpr int BS = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_CHUNK = BS * SCAN_IPT;

__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t count) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ void k_zero16(uint4* p, int64_t count) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_zero1(uint8_t* p, int64_t count) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
}

inline int grid_for(int64_t work, int per_block = BS, int cap = 4096) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// ---- block-wide exclusive scan of one int64 per thread (BS threads) ----
__device__ int64_t block_excl_scan(int64_t v, int64_t* lds, int64_t* total) {
  const int lane = threadIdx.x & (GREST_WAVE - 1);
  const int wid = threadIdx.x / GREST_WAVE;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < GREST_WAVE; o <<= 1) {
    int64_t y = __shfl_up(x, o, GREST_WAVE);
    if (lane >= o) x += y;
  }
  if (lane == GREST_WAVE - 1) lds[wid] = x;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int w = 0; w < BS / GREST_WAVE; ++w) {
    int64_t s = lds[w];
    if (w < wid) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return x - v + off;
}

__global__ void __launch_bounds__(BS) k_scan_reduce(const int64_t* in, int64_t n, int64_t* bsum) {
  __shared__ int64_t lds[BS / GREST_WAVE];
  int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
  int64_t acc = 0;
  for (int q = 0; q < SCAN_IPT; ++q) {
    int64_t i = base + (int64_t)q * BS + threadIdx.x;
    if (i < n) acc += in[i];
  }
  int64_t tot;
  block_excl_scan(acc, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of nb block sums in chunks of BS * 16 with a running
// carry (one chunk up to 8.4M scanned entries), writes out[n] = total
__global__ void __launch_bounds__(BS) k_scan_blocks(int64_t* bsum, int64_t nb, int64_t* out_total) {
  __shared__ int64_t lds[BS / GREST_WAVE];
  constexpr int IPT = 16;
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += (int64_t)BS * IPT) {
    int64_t vals[IPT];
    int64_t acc = 0;
    for (int q = 0; q < IPT; ++q) {
      const int64_t i = c0 + (int64_t)threadIdx.x * IPT + q;
      vals[q] = i < nb ? bsum[i] : 0;
      acc += vals[q];
    }
    int64_t tot;
    int64_t off = carry + block_excl_scan(acc, lds, &tot);
    for (int q = 0; q < IPT; ++q) {
      const int64_t i = c0 + (int64_t)threadIdx.x * IPT + q;
      if (i < nb) bsum[i] = off;
      off += vals[q];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) *out_total = carry;
}

__global__ void __launch_bounds__(BS) k_scan_final(const int64_t* in, int64_t n, const int64_t* boff,
                                                   int64_t* out) {
  __shared__ int64_t lds[BS / GREST_WAVE];
  __shared__ int64_t tile[SCAN_CHUNK];
  int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
  for (int q = 0; q < SCAN_IPT; ++q) {
    int64_t i = base + (int64_t)q * BS + threadIdx.x;
    tile[q * BS + threadIdx.x] = i < n ? in[i] : 0;
  }
  __syncthreads();
  int64_t acc = 0;
  for (int q = 0; q < SCAN_IPT; ++q) acc += tile[threadIdx.x * SCAN_IPT + q];
  int64_t tot;
  int64_t off = block_excl_scan(acc, lds, &tot) + boff[blockIdx.x];
  for (int q = 0; q < SCAN_IPT; ++q) {
    int64_t v = tile[threadIdx.x * SCAN_IPT + q];
    tile[threadIdx.x * SCAN_IPT + q] = off;
    off += v;
  }
  __syncthreads();
  for (int q = 0; q < SCAN_IPT; ++q) {
    int64_t i = base + (int64_t)q * BS + threadIdx.x;
    if (i < n) out[i] = tile[q * BS + threadIdx.x];
  }
}

// ---- Delta assembly ----
__device__ inline bool change_ok(int32_t i, int32_t j, int8_t s, int64_t n_old, int64_t n2) {
  if (i < 0 || j <= i || (int64_t)j >= n2) return false;
  if (s != 1 && s != -1) return false;
  if ((int64_t)j >= n_old && s != 1) return false;  // an edge of an appended node is an insertion
  return true;
}

// keys of the directed entries: (row << shift) | column; an invalid change gets all-ones
// keys, which sort after every valid one and are never read
__global__ void k_delta_keys(const int32_t* ei, const int32_t* ej, const int8_t* sg, int64_t nc, int64_t n_old,
                             int64_t n2, int shift, uint64_t* keys, int8_t* vals, int64_t* cnt, int32_t* status) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += stride) {
    const int32_t i = ei[c], j = ej[c];
    const int8_t s = sg[c];
    if (!change_ok(i, j, s, n_old, n2)) {
      atomicOr(status, ST_BAD_FORMAT);
      keys[2 * c] = ~0ull;
      keys[2 * c + 1] = ~0ull;
      vals[2 * c] = 0;
      vals[2 * c + 1] = 0;
      continue;
    }
    keys[2 * c] = ((uint64_t)i << shift) | (uint64_t)j;
    keys[2 * c + 1] = ((uint64_t)j << shift) | (uint64_t)i;
    vals[2 * c] = s;
    vals[2 * c + 1] = s;
    atomicAdd((unsigned long long*)&cnt[i], 1ull);
    atomicAdd((unsigned long long*)&cnt[j], 1ull);
  }
}

// column ids of the sorted valid entries (the first dptr[n2] keys)
__global__ void k_delta_extract(const uint64_t* keys, int64_t items, const int64_t* total, int shift,
                                int32_t* dcol) {
  const int64_t lim = min(items, *total);
  const uint64_t mask = (1ull << shift) - 1ull;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < lim; p += stride)
    dcol[p] = (int32_t)(keys[p] & mask);
}

__device__ inline int64_t lower_bound_i32(const int32_t* a, int64_t len, int32_t key) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// a group of LPR lanes per row (grid-stride) over the sorted row: duplicates, validation,
// dins[p] = insertions before p in the row, new length
template <int LPR>
__global__ void __launch_bounds__(BS) k_delta_rows(int64_t n_old, int64_t n2, const int64_t* dptr,
                                                   const int32_t* dcol, const int8_t* dsg, int32_t* dins,
                                                   const int64_t* rp_old, const int32_t* col_old,
                                                   int64_t* newlen, int32_t* status) {
  const int sl = threadIdx.x & (LPR - 1);  // lane within the row group
  const int64_t grp = ((int64_t)blockIdx.x * BS + threadIdx.x) / LPR;
  const int64_t ngrp = (int64_t)gridDim.x * (BS / LPR);
  for (int64_t r = grp; r < n2; r += ngrp) {
    const int64_t beg = dptr[r];
    const int64_t len = dptr[r + 1] - beg;
    const bool old_row = rp_old != nullptr && r < n_old;  // no old graph: membership unchecked
    const int64_t ob = old_row ? rp_old[r] : 0;
    const int64_t olen = old_row ? rp_old[r + 1] - ob : 0;
    if (len == 0) {
      if (sl == 0) newlen[r] = olen;
      continue;
    }
    int64_t sum_s = 0;
    int32_t bad = 0;
    int32_t carry = 0;  // insertions in the earlier chunks of the row
    for (int64_t e0 = 0; e0 < len; e0 += LPR) {
      const int64_t e = e0 + sl;
      const bool ve = e < len;
      const int32_t ce = ve ? dcol[beg + e] : 0;
      const int8_t se = ve ? dsg[beg + e] : 0;
      if (ve && e > 0 && dcol[beg + e - 1] == ce) bad |= ST_DUPLICATE;
      const int32_t ins = (ve && se > 0) ? 1 : 0;
      int32_t incl = ins;  // inclusive prefix sum over the group
#pragma unroll
      for (int o = 1; o < LPR; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, LPR);
        if (sl >= o) incl += y;
      }
      if (ve) {
        dins[beg + e] = carry + incl - ins;
        sum_s += se;
        if (old_row && (int64_t)ce < n_old) {
          const int64_t p = lower_bound_i32(col_old + ob, olen, ce);
          const bool found = p < olen && col_old[ob + p] == ce;
          if (found && se > 0) bad |= ST_INSERT_EXISTING;
          if (!found && se < 0) bad |= ST_DELETE_MISSING;
        }
      }
      carry += __shfl(incl, LPR - 1, LPR);
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
      sum_s += __shfl_xor(sum_s, o, LPR);
      bad |= __shfl_xor(bad, o, LPR);
    }
    if (sl == 0) {
      int64_t nl = olen + sum_s;
      newlen[r] = nl < 0 ? 0 : nl;
      if (bad) atomicOr(status, bad);
    }
  }
}

// The merge works on blocks of BS consecutive rows.  Rows without changes are shifted
// copies: the block's old column ids are one contiguous range, which the workgroup copies
// element by element (coalesced), finding each element's row by a binary search over the
// block's row starts in LDS.  Rows with changes are collected in LDS and merged by ranks
// by groups of LPR lanes (fully parallel inside the row, so hub rows do not serialise).
template <int LPR>
__global__ void __launch_bounds__(BS) k_csr_merge(int64_t n_old, int64_t n2, const int64_t* rp_old,
                                                  const int32_t* col_old, const int64_t* dptr,
                                                  const int32_t* dcol, const int8_t* dsg,
                                                  const int32_t* dins, const int64_t* rp_new,
                                                  int32_t* col_new, int64_t cap_m) {
  __shared__ int64_t s_ob[BS + 1];  // old row starts of the block (rows >= n_old: empty)
  __shared__ int64_t s_shift[BS];   // new start - old start
  __shared__ int s_list[BS];        // rows with changes (block offsets)
  __shared__ int s_cnt;
  const int t = threadIdx.x;
  const int sl = t & (LPR - 1), grp = t / LPR;
  const int64_t old_end = rp_old[n_old];
  for (int64_t r0 = (int64_t)blockIdx.x * BS; r0 < n2; r0 += (int64_t)gridDim.x * BS) {
    if (t == 0) s_cnt = 0;
    const int64_t r = r0 + t;
    s_ob[t] = r < n_old ? rp_old[r] : old_end;
    if (t == BS - 1) s_ob[BS] = r + 1 < n_old ? rp_old[r + 1] : old_end;
    __syncthreads();
    if (r < n2) {
      s_shift[t] = rp_new[r] - s_ob[t];
      if (dptr[r + 1] > dptr[r]) s_list[atomicAdd(&s_cnt, 1)] = t;
    } else {
      s_shift[t] = -1;
    }
    __syncthreads();
    // shifted copies of the rows without changes
    const int64_t e0 = s_ob[0], e1 = s_ob[BS];
    for (int64_t e = e0 + t; e < e1; e += BS) {
      int lo = 0, hi = BS;  // last row whose start is <= e
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_ob[mid] <= e) lo = mid; else hi = mid;
      }
      const int64_t rr = r0 + lo;
      if (rr < n2 && dptr[rr + 1] == dptr[rr]) {
        const int64_t dst = e + s_shift[lo];
        if (dst >= 0 && dst < cap_m) col_new[dst] = col_old[e];
      }
    }
    // rows with changes: merge by ranks
    const int cnt = s_cnt;
    for (int li = grp; li < cnt; li += BS / LPR) {
      const int64_t rr = r0 + s_list[li];
      const int64_t ob = s_ob[s_list[li]];
      const int64_t olen = (rr < n_old ? s_ob[s_list[li] + 1] : ob) - ob;
      const int64_t db = dptr[rr];
      const int64_t dlen = dptr[rr + 1] - db;
      const int64_t nb = rp_new[rr];
      const int64_t nlen = rp_new[rr + 1] - nb;
      if (nb < 0 || nlen <= 0 || nb + nlen > cap_m) continue;
      const int64_t tot_ins = (int64_t)dins[db + dlen - 1] + (dsg[db + dlen - 1] > 0 ? 1 : 0);
      for (int64_t a = sl; a < olen; a += LPR) {
        const int32_t c = col_old[ob + a];
        const int64_t p = lower_bound_i32(dcol + db, dlen, c);
        const bool hit = p < dlen && dcol[db + p] == c;
        if (hit && dsg[db + p] < 0) continue;  // deleted
        const int64_t insb = p < dlen ? (int64_t)dins[db + p] : tot_ins;
        const int64_t pos = a - (p - insb) + insb;
        if (pos >= 0 && pos < nlen) col_new[nb + pos] = c;
      }
      for (int64_t b = sl; b < dlen; b += LPR) {
        if (dsg[db + b] < 0) continue;
        const int32_t c = dcol[db + b];
        const int64_t q = rr < n_old ? lower_bound_i32(col_old + ob, olen, c) : 0;
        const int64_t insb = dins[db + b];
        const int64_t pos = q - (b - insb) + insb;
        if (pos >= 0 && pos < nlen) col_new[nb + pos] = c;
      }
    }
    __syncthreads();  // the block's LDS is reused by the next block
  }
}

// the rows where Delta_2 Omega can be nonzero: the appended rows (for the Laplacians the
// diagonal of the new block reaches every one of them) and the old rows of Delta with an
// entry in an appended column (its columns are sorted, so the last entry decides)
__global__ void __launch_bounds__(BS) k_sketch_flags(int64_t n_old, int64_t n2, const int64_t* dptr,
                                                     const int32_t* dcol, int64_t* flag) {
  for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n2; r += (int64_t)gridDim.x * BS) {
    const int64_t e = dptr[r + 1];
    flag[r] = (r >= n_old || (e > dptr[r] && (int64_t)dcol[e - 1] >= n_old)) ? 1 : 0;
  }
}

// the rows of Delta with any entry: the rows where Delta_1 X can be nonzero (an entry in
// an old column, or for the unnormalised Laplacian a degree change on an old row)
__global__ void __launch_bounds__(BS) k_delta1_flags(int64_t n2, const int64_t* dptr, int64_t* flag) {
  for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n2; r += (int64_t)gridDim.x * BS)
    flag[r] = dptr[r + 1] > dptr[r] ? 1 : 0;
}

__global__ void __launch_bounds__(BS) k_compact_rows(int64_t n2, const int64_t* flag, const int64_t* pos,
                                                     int32_t* rows) {
  for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n2; r += (int64_t)gridDim.x * BS)
    if (flag[r]) rows[pos[r]] = (int32_t)r;
}

__global__ void __launch_bounds__(BS) k_degrees(int64_t n, const int64_t* rp, double* s64, float* s32,
                                                unsigned long long* maxdeg) {
  __shared__ unsigned long long wmax[BS / GREST_WAVE];
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long mx = 0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += stride) {
    const int64_t d = rp[r + 1] - rp[r];
    const double v = d > 0 ? 1.0 / sqrt((double)d) : 0.0;
    if (s64) s64[r] = v;
    if (s32) s32[r] = (float)v;
    if ((unsigned long long)d > mx) mx = (unsigned long long)d;
  }
#pragma unroll
  for (int o = GREST_WAVE / 2; o > 0; o >>= 1) {
    unsigned long long y = __shfl_xor(mx, o, GREST_WAVE);
    mx = y > mx ? y : mx;
  }
  if ((threadIdx.x & (GREST_WAVE - 1)) == 0) wmax[threadIdx.x / GREST_WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {  // one atomic per workgroup
    for (int w = 1; w < BS / GREST_WAVE; ++w) mx = wmax[w] > mx ? wmax[w] : mx;
    atomicMax(maxdeg, mx);
  }
}

}  // namespace

void launch_fill_i64(int64_t* p, int64_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  k_fill_i64<<<grid_for(count), BS, 0, s>>>(p, value, count);
}

void launch_fill_bytes0(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  uintptr_t a = (uintptr_t)p;
  if ((a & 15) == 0 && (bytes & 15) == 0) {
    int64_t cnt = (int64_t)(bytes / 16);
    k_zero16<<<grid_for(cnt), BS, 0, s>>>((uint4*)p, cnt);
  } else {
    k_zero1<<<grid_for((int64_t)bytes), BS, 0, s>>>((uint8_t*)p, (int64_t)bytes);
  }
}

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

void launch_scan_excl(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
  int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
  if (nb < 1) nb = 1;
  k_scan_reduce<<<(unsigned)nb, BS, 0, s>>>(in, n, tmp);
  k_scan_blocks<<<1, BS, 0, s>>>(tmp, nb, out + n);
  k_scan_final<<<(unsigned)nb, BS, 0, s>>>(in, n, tmp, out);
}

int delta_key_shift(int64_t n2) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n2) ++b;
  return b;
}

void launch_delta_keys(const int32_t* ei, const int32_t* ej, const int8_t* sg, int64_t nc, int64_t n_old,
                       int64_t n_new, int shift, uint64_t* keys, int8_t* vals, int64_t* cnt, int32_t* status,
                       hipStream_t s) {
  if (nc <= 0) return;
  k_delta_keys<<<grid_for(nc), BS, 0, s>>>(ei, ej, sg, nc, n_old, n_old + n_new, shift, keys, vals, cnt, status);
}

namespace {

constexpr int SHORT_ROW = 64;      // rows of Delta up to this length are sorted by one thread
constexpr int LONG_BS = 1024;      // threads of the workgroup that sorts one long row

// Every valid key goes to a slot of its row: the row's count is taken down by one per
// key, and the slot is the row offset plus the count left (invalid keys, all ones, were
// never counted and are dropped).  The counts end at zero.
__global__ void k_delta_bucket(const uint64_t* __restrict__ kin, const int8_t* __restrict__ vin, int64_t items,
                               int shift, const int64_t* __restrict__ dptr, int64_t* __restrict__ cnt,
                               uint64_t* __restrict__ kout, int8_t* __restrict__ vout) {
  const int64_t stride = (int64_t)gridDim.x * BS;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < items; t += stride) {
    const uint64_t key = kin[t];
    if (key == ~0ull) continue;
    const int64_t row = (int64_t)(key >> shift);
    const int64_t slot = (int64_t)atomicAdd((unsigned long long*)&cnt[row], (unsigned long long)-1) - 1;
    const int64_t pos = dptr[row] + slot;
    kout[pos] = key;
    vout[pos] = vin[t];
  }
}

// Rows up to SHORT_ROW entries: insertion sort by key in place.  Longer rows go to the
// list (list[0 .. list[n2])) for k_delta_sort_long; rows longer than LONG_MAX are refused.
__global__ void k_delta_sort_short(int64_t n2, const int64_t* __restrict__ dptr, uint64_t* __restrict__ keys,
                                   int8_t* __restrict__ vals, int64_t* __restrict__ list, int32_t* status) {
  const int64_t stride = (int64_t)gridDim.x * BS;
  for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n2; r += stride) {
    const int64_t b = dptr[r], len = dptr[r + 1] - b;
    if (len <= 1) continue;
    if (len > SHORT_ROW) {
      if (len > DELTA_LONG_MAX) {
        atomicOr(status, ST_BAD_FORMAT);
      } else {
        const int64_t q = (int64_t)atomicAdd((unsigned long long*)&list[n2], 1ull);
        list[q] = r;
      }
      continue;
    }
    for (int64_t i = 1; i < len; ++i) {
      const uint64_t k = keys[b + i];
      const int8_t v = vals[b + i];
      int64_t j = i - 1;
      while (j >= 0 && keys[b + j] > k) {
        keys[b + j + 1] = keys[b + j];
        vals[b + j + 1] = vals[b + j];
        --j;
      }
      keys[b + j + 1] = k;
      vals[b + j + 1] = v;
    }
  }
}

// One listed long row per workgroup: bitonic sort of its keys (signs carried) in LDS,
// padded with all-ones keys to a power of two.
__global__ void __launch_bounds__(LONG_BS) k_delta_sort_long(int64_t n2, const int64_t* __restrict__ dptr,
                                                             const int64_t* __restrict__ list,
                                                             uint64_t* __restrict__ keys, int8_t* __restrict__ vals) {
  extern __shared__ char sort_smem[];
  uint64_t* sk = reinterpret_cast<uint64_t*>(sort_smem);
  int8_t* sv = reinterpret_cast<int8_t*>(sk + DELTA_LONG_MAX);
  if ((int64_t)blockIdx.x >= list[n2]) return;
  const int64_t r = list[blockIdx.x];
  const int64_t b = dptr[r];
  const int len = (int)(dptr[r + 1] - b);
  int P = 1;
  while (P < len) P <<= 1;
  for (int i = threadIdx.x; i < P; i += LONG_BS) {
    sk[i] = i < len ? keys[b + i] : ~0ull;
    sv[i] = i < len ? vals[b + i] : (int8_t)0;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += LONG_BS) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const uint64_t a = sk[i], c = sk[ixj];
          if ((a > c) == up) {
            sk[i] = c;
            sk[ixj] = a;
            const int8_t t = sv[i];
            sv[i] = sv[ixj];
            sv[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < len; i += LONG_BS) {
    keys[b + i] = sk[i];
    vals[b + i] = sv[i];
  }
}

}  // namespace

void launch_delta_group(const uint64_t* kin, const int8_t* vin, int64_t items, int shift, int64_t n2,
                        const int64_t* dptr, int64_t* cnt, uint64_t* kout, int8_t* vout, int64_t* list,
                        int32_t* status, hipStream_t s) {
  if (items <= 0 || n2 <= 0) return;
  k_delta_bucket<<<grid_for(items), BS, 0, s>>>(kin, vin, items, shift, dptr, cnt, kout, vout);
  launch_fill_i64(list + n2, 0, 1, s);
  k_delta_sort_short<<<grid_for(n2), BS, 0, s>>>(n2, dptr, kout, vout, list, status);
  // rows longer than SHORT_ROW hold more than SHORT_ROW of the items each
  const int64_t bound = std::min<int64_t>(n2, items / (SHORT_ROW + 1) + 1);
  constexpr size_t lds = (size_t)DELTA_LONG_MAX * (sizeof(uint64_t) + sizeof(int8_t));
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_delta_sort_long, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return true;
  }();
  (void)attr;
  k_delta_sort_long<<<(unsigned)bound, LONG_BS, lds, s>>>(n2, dptr, list, kout, vout);
}

void launch_delta_extract(const uint64_t* keys, int64_t items, const int64_t* total, int shift, int32_t* dcol,
                          hipStream_t s) {
  if (items <= 0) return;
  k_delta_extract<<<grid_for(items), BS, 0, s>>>(keys, items, total, shift, dcol);
}

void launch_delta_rows(int64_t n_old, int64_t n_new, const int64_t* dptr, const int32_t* dcol, const int8_t* dsg,
                       int32_t* dins, const int64_t* rp_old, const int32_t* col_old, int64_t* newlen,
                       int32_t* status, hipStream_t s) {
  int64_t n2 = n_old + n_new;
  if (n2 <= 0) return;
  constexpr int LPR = 8;  // touched rows carry a few changes each
  k_delta_rows<LPR><<<grid_for(n2 * LPR, BS, 1 << 15), BS, 0, s>>>(n_old, n2, dptr, dcol, dsg, dins, rp_old, col_old,
                                                                   newlen, status);
}

void launch_csr_merge(int64_t n_old, int64_t n_new, const int64_t* rp_old, const int32_t* col_old,
                      const int64_t* dptr, const int32_t* dcol, const int8_t* dsg, const int32_t* dins,
                      const int64_t* rp_new, int32_t* col_new, int64_t cap_m, hipStream_t s) {
  int64_t n2 = n_old + n_new;
  if (n2 <= 0) return;
  constexpr int LPR = 16;  // about one pass over a changed row of mean length
  k_csr_merge<LPR><<<grid_for(n2, BS, 1 << 16), BS, 0, s>>>(n_old, n2, rp_old, col_old, dptr, dcol, dsg, dins,
                                                            rp_new, col_new, cap_m);
}

void launch_sketch_rows(int64_t n_old, int64_t n_new, const int64_t* dptr, const int32_t* dcol, int64_t* flag,
                        int64_t* pos, int64_t* scan_tmp, int32_t* rows, hipStream_t s) {
  const int64_t n2 = n_old + n_new;
  if (n2 <= 0) return;
  k_sketch_flags<<<grid_for(n2), BS, 0, s>>>(n_old, n2, dptr, dcol, flag);
  launch_scan_excl(flag, pos, n2, scan_tmp, s);
  k_compact_rows<<<grid_for(n2), BS, 0, s>>>(n2, flag, pos, rows);
}

void launch_delta1_rows(int64_t n_old, int64_t n_new, const int64_t* dptr, const int32_t* dcol, int64_t* flag,
                        int64_t* pos, int64_t* scan_tmp, int32_t* rows, hipStream_t s) {
  const int64_t n2 = n_old + n_new;
  if (n2 <= 0) return;
  (void)dcol;
  k_delta1_flags<<<grid_for(n2), BS, 0, s>>>(n2, dptr, flag);
  launch_scan_excl(flag, pos, n2, scan_tmp, s);
  k_compact_rows<<<grid_for(n2), BS, 0, s>>>(n2, flag, pos, rows);
}

void launch_degrees(int64_t n, const int64_t* rp, double* dinv_sqrt64, float* dinv_sqrt32,
                    int64_t* maxdeg, hipStream_t s) {
  if (n <= 0) return;
  k_degrees<<<grid_for(n, BS, 1024), BS, 0, s>>>(n, rp, dinv_sqrt64, dinv_sqrt32,
                                                 (unsigned long long*)maxdeg);
}

// The rows of Delta Z that the low-rank projected matrix needs, gathered: for the listed
// rows r = rows[i] (slots i < *count), Zg[i] = Z[r] and Dz[i] = (Delta Z)[r], the sum over
// the entries e of row r of Delta of sign_e Z[col_e] (FP64 accumulation); slots from the
// count up to bound get zeros, so that a dense product over bound rows sees only the
// listed ones.  One wave per slot, lanes over the w <= 128 columns.
namespace {
template <typename T>
__global__ void __launch_bounds__(256) k_delta_gather(int64_t bound, const int32_t* __restrict__ rows,
                                                      const int64_t* count, const int64_t* __restrict__ dptr,
                                                      const int32_t* __restrict__ dcol,
                                                      const int8_t* __restrict__ dsg, const T* __restrict__ Z,
                                                      int64_t ldz, int w, T* __restrict__ Zg, T* __restrict__ Dz,
                                                      int lap) {
  const int lane = threadIdx.x & 63;
  const int64_t slot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (slot >= bound) return;
  const int64_t cnt = *count;
  for (int c = lane; c < w; c += 64) {
    T zg = T(0), dz = T(0);
    if (slot < cnt) {
      const int64_t r = rows[slot];
      double acc = 0.0;
      int64_t ssum = 0;
      for (int64_t e = dptr[r]; e < dptr[r + 1]; ++e) {
        acc += (double)dsg[e] * (double)Z[(int64_t)dcol[e] * ldz + c];
        ssum += dsg[e];
      }
      zg = Z[r * ldz + c];
      if (lap) acc = (double)ssum * (double)zg - acc;  // Delta_L = diag(degree changes) - Delta
      dz = (T)acc;
    }
    Zg[slot * w + c] = zg;
    Dz[slot * w + c] = dz;
  }
}
}  // namespace

template <typename T>
void launch_delta_gather(int64_t bound, const int32_t* rows, const int64_t* count, const int64_t* dptr,
                         const int32_t* dcol, const int8_t* dsg, const T* Z, int64_t ldz, int w, T* Zg, T* Dz,
                         hipStream_t s, bool lap) {
  if (bound <= 0 || w <= 0) return;
  k_delta_gather<T><<<(unsigned)((bound + 3) / 4), 256, 0, s>>>(bound, rows, count, dptr, dcol, dsg, Z, ldz, w, Zg,
                                                                 Dz, lap ? 1 : 0);
}

template void launch_delta_gather<float>(int64_t, const int32_t*, const int64_t*, const int64_t*, const int32_t*,
                                        const int8_t*, const float*, int64_t, int, float*, float*, hipStream_t,
                                        bool);
template void launch_delta_gather<double>(int64_t, const int32_t*, const int64_t*, const int64_t*, const int32_t*,
                                         const int8_t*, const double*, int64_t, int, double*, double*, hipStream_t,
                                         bool);
