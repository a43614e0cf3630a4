/*
 * grest_calib.h -- a measurement aid shipped in libgrest beside the method's entry
 * points (grest.h).  It computes nothing of the method: it times the rate at which the
 * chip serves gathers of whole dense rows from random places, the access that bounds the
 * product of the stored graph with the basis (eq. RR_eigen_graph_upd_main2, the product
 * (op Z)), so that the product's time can be set against the ceiling of its own access
 * pattern as well as against the HBM peak.
 */
#ifndef GREST_CALIB_H
#define GREST_CALIB_H

#include <stdint.h>

#include "grest.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * grest_calib_gather: Y[r, 0:w] = sum over the entries e in [rp[r], rp[r + 1]) of
 * Z[h(seed + e) mod n, 0:w] for r < n, h the low 32 bits of the splitmix64 finaliser;
 * the launch shape, lane layout (four FP32 columns a lane, a power-of-two group of lanes
 * a row) and count of gathered rows are those of the row-split product of a graph with
 * the row pointers rp at width w.
 *   n         rows (1 .. 2^31 - 1);
 *   rp        device, int64, n + 1 nondecreasing entries from 0 (row r gathers
 *             rp[r + 1] - rp[r] rows of Z); read only;
 *   Z         device, FP32, n rows of leading dimension ldz (>= w, a multiple of 4),
 *             16-byte aligned; read only;
 *   w         columns gathered, a positive multiple of 4;
 *   Y         device, FP32, n rows of leading dimension ldy (>= w, a multiple of 4),
 *             16-byte aligned; written (columns 0 .. w - 1);
 *   stream    a hipStream_t, or null for the default stream; the call only enqueues.
 * Returns GREST_EINVAL for arguments outside these ranges (nothing launched) and
 * GREST_EDEVICE if the launch fails.  The caller owns every buffer.
 */
grest_status grest_calib_gather(int64_t n, const int64_t* rp, const float* Z, int64_t ldz, int32_t w, float* Y,
                                int64_t ldy, uint64_t seed, void* stream);

#ifdef __cplusplus
}
#endif

#endif
