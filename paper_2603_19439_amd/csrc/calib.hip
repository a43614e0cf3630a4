// Random-gather ceiling of the sparse product: the same launch shape, lane layout, row
// pointers and number of gathered rows as the row-split product (op Z) of a graph, but
// the column of every entry comes from a hash of its index instead of from memory.
// Nothing of the method is computed here; the time of this kernel is the rate at which
// the chip serves gathers of whole dense rows from random places.
#include "grest_calib.h"

#include <cstdio>

#include "rowvec.h"

namespace {

__device__ inline uint32_t mix64(uint64_t x) {  // the splitmix64 finaliser
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ULL;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebULL;
  x ^= x >> 31;
  return (uint32_t)x;
}

__global__ void __launch_bounds__(BS) k_gather_ceiling(int64_t n, const int64_t* __restrict__ rp, uint64_t seed,
                                                       const float* __restrict__ Z, int64_t ldz, int w,
                                                       float* __restrict__ Y, int64_t ldy, int lpr_shift) {
  const int lpr = 1 << lpr_shift;
  const int64_t gid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int gl = (int)(gid & (lpr - 1));
  const int64_t ngroups = ((int64_t)gridDim.x * BS) >> lpr_shift;
  const uint32_t nn = (uint32_t)n;
  for (int64_t r = gid >> lpr_shift; r < n; r += ngroups) {
    const int64_t beg = rp[r], end = rp[r + 1];
    for (int c0 = gl * 4; c0 < w; c0 += lpr * 4) {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      int64_t e = beg;
      for (; e + 4 <= end; e += 4) {
        float z[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) vload<float, 4>(Z + (int64_t)(mix64(seed + e + u) % nn) * ldz + c0, z[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i] += z[u][i];
      }
      for (; e < end; ++e) {
        float z[4];
        vload<float, 4>(Z + (int64_t)(mix64(seed + e) % nn) * ldz + c0, z);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += z[i];
      }
      vstore<float, 4>(Y + r * ldy + c0, acc);
    }
  }
}

}  // namespace

extern "C" grest_status grest_calib_gather(int64_t n, const int64_t* rp, const float* Z, int64_t ldz, int32_t w,
                                           float* Y, int64_t ldy, uint64_t seed, void* stream) {
  if (n <= 0 || n > INT32_MAX || !rp || w <= 0 || w % 4 || ldz < w || ldy < w || ldz % 4 || ldy % 4 || !Z || !Y ||
      ((uintptr_t)Z % 16) || ((uintptr_t)Y % 16))
    return GREST_EINVAL;
  const int lpr = lanes_per_row(w, 4);
  k_gather_ceiling<<<grid_for(n * lpr), BS, 0, (hipStream_t)stream>>>(n, rp, seed, Z, ldz, w, Y, ldy, ilog2(lpr));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fprintf(stderr, "grest_calib_gather: %s\n", hipGetErrorString(e));
    return GREST_EDEVICE;
  }
  return GREST_OK;
}
