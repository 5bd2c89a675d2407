/*
 * radiotrace -- read-bandwidth probe (measurement plumbing; no counterpart
 * in the paper).
 *
 * States the peak of the memory level that serves a kernel's loads, next to
 * the rate the gridded trace achieves: the gridded field (section 2 lists
 * gridded data among the supported set-ups) is read as eight float4 node
 * gathers per field evaluation, served mostly from each XCD's L2 and the
 * MALL, so HBM's peak alone says little about how close the trace runs to
 * its bound.
 */
#ifndef RADIOTRACE_PROBE_H
#define RADIOTRACE_PROBE_H

#include "radiotrace.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RT_PROBE_STREAM = 0, /* every float4 of the buffer, coalesced, repeated
                          within a pass until the pass has read >= 512 MiB */
  RT_PROBE_GATHER = 1  /* 64 float4 per lane per pass at pseudo-random indices
                          (8 blocks of 256 lanes per CU) */
};

/* Read bandwidth, in GB/s of bytes requested by the lanes, of 'passes'
 * passes of 'pattern' over the caller-owned device buffer of 'bytes' bytes
 * (>= 4096, a multiple of 16; for RT_PROBE_GATHER bytes / 16 a power of
 * two).  The buffer's contents are read, never written.  The size picks the
 * level that serves it: up to a few MiB each XCD's L2, up to ~256 MiB the
 * MALL, beyond that HBM.  One untimed warm-up pass, then the passes are
 * timed with HIP events on 'stream'; the call blocks until they finish and
 * allocates no device memory.  RT_ERR_INVALID_ARG for bad arguments,
 * RT_ERR_DEVICE when a HIP call fails. */
rt_status rt_probe_read_bandwidth(void* buffer, size_t bytes, int32_t pattern, int32_t passes,
                                  void* stream, double* gb_per_s);

#ifdef __cplusplus
}
#endif
#endif /* RADIOTRACE_PROBE_H */
