/*
 * sssp_ceilings.h - microbenchmarks of the memory-system rates that bound the
 * Relax phase of the stepping kernel (libsssp_ceilings.so). They measure,
 * with the same launch shape as the stepping kernel (1024 workgroups of 256
 * threads, 4 accesses in flight per thread), how fast MI355X serves the two
 * random accesses of a relaxed arc when nothing else runs:
 *   - a 2-byte gather per arc (the Relax filter reads hint[v] for each arc's
 *     target v; Alg. 1's WriteMin is preceded by this read), and
 *   - a 64-bit atomic minimum per arc at a random address (WriteMin, Sec. 2).
 * Index streams are read coalesced, as Relax reads its packed arcs.
 *
 * Both calls enqueue one kernel on `stream` and return; the caller times
 * them (events on the same stream). Arguments are device pointers:
 *   idx    count int32 indices into the table (each in [0, table size)).
 *   table  the gathered or updated array.
 *   sink   one uint64 that receives an XOR of everything gathered (so the
 *          gathers are not optimised away); its prior value is overwritten.
 * Return 0 on success, or the hipError_t of the launch.
 */
#ifndef SSSP_CEILINGS_H
#define SSSP_CEILINGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int sssp_ceiling_gather16(const int32_t* idx, uint64_t count, const uint16_t* table, uint64_t* sink, void* stream);

/* table[idx[i]] = min(table[idx[i]], value(i)) for every i, value(i) a
 * SplitMix64 mix of i shifted right by 20 (so about half the minima lower
 * the entry early on and few later, as WriteMins do over a solve). */
int sssp_ceiling_atomic_min64(const int32_t* idx, uint64_t count, uint64_t* table, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SSSP_CEILINGS_H */
