/*
 * Memory-level probe (measurement support, not part of the method).
 *
 * The advection kernel's cell-cache misses are random record reads from the
 * stored field.  This call measures the rate the memory hierarchy sustains for
 * such reads at a given footprint -- a few hundred KB stays in the L2, ~200 MB
 * in the 256 MB Infinity Cache, gigabytes come from HBM -- so that the
 * kernel's gather rate (streami_stats.gathers x record size / time) can be
 * set against a measured peak of the level that serves it.
 */
#ifndef STREAMI_PROBE_H
#define STREAMI_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random record gathers over `buf` (device memory, 16-byte aligned, `bytes`
 * bytes, contents arbitrary; only read).  Every lane of waves_per_cu waves per
 * CU reads loads_per_lane records of record_bytes (16, 96 or 128) at
 * independent uniformly random record-aligned offsets, in_flight (1, 2, 4 or
 * 8) records at a time.  One untimed launch, then one launch timed with HIP
 * events on hip_stream (NULL = default stream): *ms receives its time and
 * *records_read (nullable) the records it read.  Synchronises the stream
 * before returning.  Errors: E_ARG (NULL buf or ms, record_bytes, in_flight,
 * loads_per_lane not a multiple of in_flight in [in_flight, 2^20],
 * waves_per_cu outside [1, 64], fewer than 1 or 2^32 or more records in
 * `bytes`), E_NOMEM, E_DEVICE. */
int streami_probe_gather(const void* buf, int64_t bytes, int32_t record_bytes, int32_t loads_per_lane,
                         int32_t in_flight, int32_t waves_per_cu, void* hip_stream, float* ms,
                         int64_t* records_read);

/* VALU issue rate: waves_per_cu (a multiple of 4 in [4, 64]) waves per CU
 * each run 8 independent chains of one instruction kind -- kind 0 v_fma_f32
 * (a VOP3 encoding), kind 1 v_add_u32 (VOP2), kind 2 v_exp_f32, kind 3
 * v_rcp_f32 (the two transcendentals of a SiLU) -- 131,072 instructions per wave.
 * One untimed launch, then one timed with HIP events on hip_stream: *ms is
 * its time and *instructions (nullable) the wave-level instructions of the
 * chains, so (4 x CUs) x clock x time / instructions is the cycles a SIMD
 * spends per wave64 instruction of that kind.  Synchronises the stream.  Errors:
 * E_ARG (NULL ms, kind, waves_per_cu), E_NOMEM, E_DEVICE. */
int streami_probe_valu(int32_t kind, int32_t waves_per_cu, void* hip_stream, float* ms, int64_t* instructions);

#ifdef __cplusplus
}
#endif
#endif /* STREAMI_PROBE_H */
