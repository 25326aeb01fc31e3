/*
 * rtf_probe.h -- C ABI of librtf_probe.so, a measurement aid for the
 * sampling kernels of librtforest.so.  It is not part of the method.
 *
 * The sampling step of the radix tree forest (Alg. 2 with the guide table of
 * Sec. 2.5 and the trees of Sec. 3.2) streams its uniforms, makes a few
 * dependent random reads of the auxiliary structure and streams its outputs.
 * On a GPU whose memory system moves whole lines, the number of dependent
 * random reads per sample, not the bytes the search compares, sets the speed
 * (Sec. 2.4 makes the same point about the granularity of memory transfer).
 * The probe reproduces that memory pattern without any search, so that its
 * rate is the ceiling a sampling kernel with the same reads can reach.
 */
#ifndef RTF_PROBE_H
#define RTF_PROBE_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * For s in [0, S): read u[s] (uint64, streamed), read the 64-byte record
 * g = floor(u[s] * m / 2^64) of `table` (m records, 64 bytes each, 64-byte
 * aligned), then depth - 1 further dependent 16-byte reads of `nodes`
 * (n records of 16 bytes, 16-byte aligned) at positions derived from the
 * words read before, and write a value derived from all words read to
 * idx[s] (int32) and x[s] (double, NULL to skip).  The launch shape is the
 * one librtforest's single-distribution sampling kernel uses.
 * All pointers are device pointers owned by the caller; nothing is
 * allocated.  Returns 0, 1 for an invalid argument (null pointer, m < 1,
 * S < 0, depth < 1, depth > 1 with n < 1, misaligned table or nodes), or
 * 4 for a HIP launch error.  S == 0 launches nothing.
 */
int rtf_probe_gather(const void *table, int64_t m, const void *nodes, int64_t n,
                     const uint64_t *u, int64_t S, int32_t depth, int32_t *idx, double *x,
                     hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RTF_PROBE_H */
