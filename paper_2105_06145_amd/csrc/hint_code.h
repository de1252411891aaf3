// 16-bit codes of upper bounds of 64-bit keys: the Relax filter's key bounds
// (hint[v] in the stepping kernel). A code stands for a value at least the
// key it was made from (rounded up), and values grow with codes, so a stale
// code of a key that has only fallen since is still an upper bound.
//
// The code: below 2048 the value itself; above, exponent e (1..31) in the top
// 5 bits and m in the low 11, for the value (2048 + m) << (e - 1). 0xFFFF
// (e = 31, m = 2047) means no bound is known; values above
// (2048 + 2046) << 30 have no code and map to it.
#ifndef SSSP_HINT_CODE_H
#define SSSP_HINT_CODE_H

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sssp_impl {

constexpr uint32_t HINT_NONE = 0xFFFFu;

__host__ __device__ inline uint64_t hint_value(uint32_t c) {
  const uint32_t e = c >> 11, m = c & 2047u;
  return e == 0 ? (uint64_t)m : ((uint64_t)(2048u + m) << (e - 1));
}

// The smallest code whose value is at least d (HINT_NONE beyond the range).
__host__ __device__ inline uint16_t as_hint(uint64_t d) {
  if (d < 2048) return (uint16_t)d;
  const int b = 63 - __builtin_clzll(d);  // d's top bit, at least 11
  uint32_t e = (uint32_t)(b - 10);
  uint64_t mf = d >> (e - 1);  // in [2048, 4095]
  if ((mf << (e - 1)) < d) ++mf;
  if (mf == 4096) {
    ++e;
    mf = 2048;
  }
  const uint32_t c = (e << 11) | (uint32_t)(mf - 2048);
  return (e > 31 || c >= HINT_NONE) ? (uint16_t)HINT_NONE : (uint16_t)c;
}

}  // namespace sssp_impl

#endif  // SSSP_HINT_CODE_H
