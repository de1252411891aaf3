// Memory-system ceilings of the Relax phase (include/sssp_ceilings.h): a
// random 2-byte gather and a random 64-bit atomic minimum per index, read
// from a coalesced index stream, in the stepping kernel's launch shape.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/sssp_ceilings.h"

namespace {

constexpr int WG = 256;
constexpr int GRID = 1024;
constexpr int UNROLL = 4;

typedef unsigned long long ull;

template <class T>
using gptr = __attribute__((address_space(1))) T*;

__global__ __launch_bounds__(WG) void gather16_kernel(const int32_t* idx_, ull count, const uint16_t* table_,
                                                      ull* sink) {
  const gptr<const int32_t> idx = (gptr<const int32_t>)idx_;
  const gptr<const uint16_t> table = (gptr<const uint16_t>)table_;
  const ull stride = (ull)gridDim.x * WG * UNROLL;
  ull acc = 0;
  for (ull base = (ull)blockIdx.x * WG * UNROLL + threadIdx.x; base < count; base += stride) {
    int32_t v[UNROLL];
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const ull i = base + (ull)k * WG;
      v[k] = __builtin_nontemporal_load(&idx[i < count ? i : count - 1]);
    }
    uint32_t h[UNROLL];
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) h[k] = table[v[k]];
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) acc ^= (ull)h[k] << (16 * k);
  }
  for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) atomicXor(sink, acc);
}

__device__ __forceinline__ ull mix(ull i) {
  ull z = (i + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(WG) void atomic_min64_kernel(const int32_t* idx_, ull count, ull* table_) {
  const gptr<const int32_t> idx = (gptr<const int32_t>)idx_;
  const gptr<ull> table = (gptr<ull>)table_;
  const ull stride = (ull)gridDim.x * WG * UNROLL;
  for (ull base = (ull)blockIdx.x * WG * UNROLL + threadIdx.x; base < count; base += stride) {
    int32_t v[UNROLL];
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const ull i = base + (ull)k * WG;
      v[k] = __builtin_nontemporal_load(&idx[i < count ? i : count - 1]);
    }
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const ull i = base + (ull)k * WG;
      if (i < count)
        __hip_atomic_fetch_min(&table[v[k]], mix(i) >> 20, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace

extern "C" {

int sssp_ceiling_gather16(const int32_t* idx, uint64_t count, const uint16_t* table, uint64_t* sink, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemsetAsync(sink, 0, 8, st);
  if (e != hipSuccess) return (int)e;
  if (count == 0) return 0;
  gather16_kernel<<<GRID, WG, 0, st>>>(idx, count, table, (ull*)sink);
  return (int)hipGetLastError();
}

int sssp_ceiling_atomic_min64(const int32_t* idx, uint64_t count, uint64_t* table, void* stream) {
  if (count == 0) return 0;
  atomic_min64_kernel<<<GRID, WG, 0, (hipStream_t)stream>>>(idx, count, (ull*)table);
  return (int)hipGetLastError();
}

}  // extern "C"
