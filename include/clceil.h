/*
 * clceil.h -- measured memory-system ceilings used by the roofline of the
 * generation kernel (a measurement probe built as libclceil.so beside the
 * generator; a project addition with no counterpart in the paper).
 *
 * The generator reads one float64 weight per visited candidate at a
 * data-dependent position and writes 4-byte slot words; these kernels time
 * the same memory operations alone on the same device:
 *   - clc_gather_uniform: `count` 8-byte loads from w[0 .. n) at positions
 *     floor(mix(seed + i) n / 2^64), i = 0 .. count-1 (mix = splitmix64's
 *     output function), i.e. uniform random positions;
 *   - clc_gather_list: `count` 8-byte loads w[idx[i]] (idx read in order,
 *     coalesced; entries >= n are skipped);
 *   - clc_store: plain coalesced 16-byte stores over buf[0 .. bytes).
 * Pointers are device pointers; out receives one float64 per thread
 * (blocks x 256 entries) so that no load is optimised away; buf must be
 * 16-byte aligned.  Each call only enqueues one kernel on `stream`
 * (a hipStream_t, NULL = the null stream).  Returns 0, -1 for a bad
 * argument, -8 for a launch error.
 */
#ifndef CLCEIL_H_
#define CLCEIL_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int clc_gather_uniform(const double* w, uint64_t n, uint64_t count, uint64_t seed, uint32_t blocks, double* out,
                       void* stream);
int clc_gather_list(const double* w, uint64_t n, const uint32_t* idx, uint64_t count, uint32_t blocks, double* out,
                    void* stream);
int clc_store(void* buf, uint64_t bytes, uint32_t blocks, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CLCEIL_H_ */
