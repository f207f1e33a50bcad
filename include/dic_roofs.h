/*
 * dic_roofs.h -- achievable-rate probes of the device (libdicroofs.so).
 *
 * Not part of the correlation method: these are the measured denominators
 * that the benchmark quotes beside the published peaks (HBM streaming, cache
 * re-reads, LDS reads, FP32 and FP64 fused multiply-adds).  Each call runs on
 * the current HIP device, allocates what it needs and frees it before it
 * returns, times `reps` launches after one warm-up with HIP events on a stream
 * of its own, and returns the best rate.  A negative return means a bad
 * argument or a HIP error (nothing is left allocated).
 */
#ifndef DIC_ROOFS_H
#define DIC_ROOFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* GB/s of float4 loads streamed once over a buffer of `bytes` (>= 1 MiB; use
 * far more than the caches, e.g. 4 GiB). */
double dic_roof_hbm_read(int64_t bytes, int reps);

/* GB/s (read + write bytes) of a device-to-device copy of `bytes`. */
double dic_roof_hbm_copy(int64_t bytes, int reps);

/* GB/s of reads served from a cache: a footprint of `footprint_bytes` read by
 * 2048 workgroups, each `inner` times over `chunk_bytes` (<= footprint) from
 * its own offset.  A footprint within one XCD's L2 (e.g. 2 MiB) measures L2;
 * one within the Infinity Cache (e.g. 64 or 192 MiB) measures that. */
double dic_roof_cache_read(int64_t footprint_bytes, int64_t chunk_bytes, int inner, int reps);

/* GB/s of 128-bit LDS reads (2048 workgroups x 256 threads x iters x 16 reads). */
double dic_roof_lds_read(int iters, int reps);

/* TFLOP/s of independent FMA chains (fp64 = 0: FP32 as the library builds it,
 * one FMA per lane per instruction; fp64 = 1: FP64), 2 flop per FMA. */
double dic_roof_fma(int fp64, int iters, int reps);

#ifdef __cplusplus
}
#endif

#endif
