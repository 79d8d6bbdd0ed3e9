/*
 * psmprobe.h -- C ABI of libpsmprobe.so, a measurement utility kept apart
 * from the method's library: the attainable streaming bandwidth of the
 * device, stated beside the roofline figures, and the plain copy kernel of
 * known size that calibrates the HBM traffic counters.
 */
#ifndef PSMPROBE_H
#define PSMPROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Streams `bytes` (rounded down to 16-byte elements) through a plain
 * grid-stride kernel of `grid` workgroups of 256 lanes on the null stream:
 * kind 0 copies src to dst, kind 1 reads src (dst: at least 4 bytes; its first
 * float is written only by a lane whose partial sum equals 1234.5), kind 2
 * writes dst.  Two untimed launches, then `reps` timed ones; *ms_per_launch
 * receives their average duration (HIP events).  Device pointers owned by the
 * caller.  Returns 0, -1 on a null or short argument, -5 on a HIP error. */
int32_t psmprobe_stream(int32_t kind, const void* src, void* dst, int64_t bytes, int32_t grid, int32_t reps,
                        double* ms_per_launch);

#ifdef __cplusplus
}
#endif
#endif
