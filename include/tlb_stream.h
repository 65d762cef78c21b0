/*
 * tlb_stream.h -- HBM streaming reference kernels of libtlb.so, the measured ceiling against
 * which the stage kernel of tlb.h is judged (it is bound by HBM bandwidth: every Runge-Kutta
 * stage streams the populations once, section II C, eq. boltz_tor).
 *
 * tlb_hbm_stream moves n16 chunks of 16 bytes (one dwordx4 per lane and access) between
 * caller-owned device buffers on the caller's stream, without waiting:
 *   mode 0  copy   z[i] = x[i]                        1 read : 1 write
 *   mode 1  add    z[i] = x[i] + y[i] (as 4 floats)    2 reads : 1 write, the ratio of the
 *                                                      second and third stages (read y_s and
 *                                                      y^n, write one state copy)
 *   mode 2  read   every x[i] is read; per workgroup one 16-byte partial sum goes to z (z must
 *                  hold 8 chunks per compute unit, at most 8192 chunks)
 * Loads and stores are nontemporal (the buffers are far larger than the caches).  The caller
 * times the call (e.g. HIP events on the same stream) and divides the bytes moved by the time.
 * x, y, z must be 16-byte aligned; z must not overlap x or y.  Errors (tlb.h codes):
 * TLB_EINVAL (NULL pointer the mode needs, n16 < 1, unknown mode, misaligned), TLB_EHIP.
 */
#ifndef TLB_STREAM_H
#define TLB_STREAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TLB_STREAM_COPY 0
#define TLB_STREAM_ADD 1
#define TLB_STREAM_READ 2

int32_t tlb_hbm_stream(int32_t mode, const void* x, const void* y, void* z, int64_t n16,
                       void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* TLB_STREAM_H */
