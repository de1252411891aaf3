// Graph creation: validation, upload, packing and the degree-ordered
// internal relabelling (entry points sssp_graph_create / _destroy / _info).
//
// Internal layout: int64 row offsets and one 8-byte word per arc,
// (weight << 32) | target, so Relax reads each arc with one coalesced load.
// Unless SSSP_KEEP_ORDER is given, vertices are renumbered by decreasing
// out-degree (ties by id). On power-law graphs most arcs point at few hub
// vertices; numbering them first packs their tentative distances into a few
// MiB that stay resident in each XCD's L2, so the random distance reads of
// Relax mostly hit cache. The renumbering is internal: sources and distances
// cross the ABI in the caller's ids.

#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <vector>

#include "internal.h"

using namespace sssp_impl;

namespace {

__global__ void pack_edges_kernel(const int32_t* tgt, const uint32_t* w, ull* out, ull m) {
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (ull)gridDim.x * blockDim.x)
    out[i] = ((ull)w[i] << 32) | (uint32_t)tgt[i];
}

__global__ void widen_offsets_kernel(const int32_t* in, int64_t* out, ull count) {
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (ull)gridDim.x * blockDim.x)
    out[i] = in[i];
}

// err occupies the low half of an 8-byte word that is read back whole.
__global__ void reset_flags_kernel(unsigned* err, ull* where) {
  *reinterpret_cast<ull*>(err) = 0;
  *where = INF;
}

// CSR validation on the device. Sets bits in *err: 1 offsets[0] != 0,
// 2 offsets decrease, 4 offsets[n] != m, 8 target out of range; and the
// smallest offending index in *where.
__global__ void validate_kernel(const int64_t* off, const int32_t* tgt, ull n, ull m, unsigned* err, ull* where) {
  const ull stride = (ull)gridDim.x * blockDim.x;
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (off[i + 1] < off[i]) {
      atomicOr(err, 2u);
      atomicMin(where, i);
    }
  }
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int32_t v = tgt[i];
    if (v < 0 || (ull)v >= n) {
      atomicOr(err, 8u);
      atomicMin(where, i);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (off[0] != 0) atomicOr(err, 1u);
    if ((ull)off[n] != m) atomicOr(err, 4u);
  }
}

// Multiset checksums of the arcs (u, v, w) and of their reverses (v, u, w):
// equal for a symmetric graph. Each term is the SplitMix64 finaliser of a
// mix of the three fields; sums are modulo 2^64.
__device__ __forceinline__ ull arc_mix(ull a, ull b, ull w) {
  ull z = a * 0x9e3779b97f4a7c15ull ^ (b + 0x632be59bd9b4e019ull) * 0xd1b54a32d192ed03ull ^ w;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void symmetry_hash_kernel(const int64_t* off, const ull* edges, ull n, ull* sums) {
  ull fwd = 0, rev = 0;
  for (ull u = (ull)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (ull)gridDim.x * blockDim.x)
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const ull v = edges[e] & 0xffffffffull, w = edges[e] >> 32;
      fwd += arc_mix(u, v, w);
      rev += arc_mix(v, u, w);
    }
  for (int o = 32; o > 0; o >>= 1) {
    fwd += __shfl_xor(fwd, o);
    rev += __shfl_xor(rev, o);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&sums[0], fwd);
    atomicAdd(&sums[1], rev);
  }
}

// Sort keys for the relabelling: smaller key = larger out-degree.
__global__ void degree_keys_kernel(const int64_t* off, ull n, uint32_t* keys, int32_t* ids) {
  for (ull v = (ull)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (ull)gridDim.x * blockDim.x) {
    const ull d = (ull)(off[v + 1] - off[v]);
    keys[v] = 0xffffffffu - (uint32_t)(d < 0xffffffffull ? d : 0xffffffffull);
    ids[v] = (int32_t)v;
  }
}

// inv[perm[i]] = i; newdeg[i] = deg(perm[i]).
__global__ void invert_kernel(const int32_t* perm, const int64_t* off, ull n, int32_t* inv, int64_t* newdeg) {
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (ull)gridDim.x * blockDim.x) {
    const int32_t u = perm[i];
    inv[u] = (int32_t)i;
    newdeg[i] = off[u + 1] - off[u];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) newdeg[n] = 0;
}

// Copy row perm[i] to internal row i, renumbering targets. One wavefront per row.
__global__ void relabel_rows_kernel(const int32_t* perm, const int32_t* inv, const int64_t* off,
                                    const int64_t* newoff, const ull* edges, ull* out, ull n) {
  const ull lane = threadIdx.x & 63;
  const ull waves = (ull)gridDim.x * (blockDim.x / 64);
  for (ull i = ((ull)blockIdx.x * blockDim.x + threadIdx.x) / 64; i < n; i += waves) {
    const int32_t u = perm[i];
    const ull src = (ull)off[u], deg = (ull)(off[u + 1] - off[u]), dst = (ull)newoff[i];
    for (ull k = lane; k < deg; k += 64) {
      const ull e = edges[src + k];
      out[dst + k] = (e & 0xffffffff00000000ull) | (uint32_t)inv[(uint32_t)e];
    }
  }
}

// count[k] = the number of vertices of out-degree at least 2^k (k = 0 .. 32),
// on offsets whose degrees do not increase with the id: the first id whose
// degree is below 2^k, by binary search. One thread per k.
__global__ void degree_ranks_kernel(const int64_t* off, ull n, ull* count) {
  const unsigned k = threadIdx.x;
  if (k > 32) return;
  const ull need = 1ull << k;
  ull lo = 0, hi = n;
  while (lo < hi) {
    const ull mid = lo + (hi - lo) / 2;
    if ((ull)(off[mid + 1] - off[mid]) >= need) {
      lo = mid + 1;
    } else {
      hi = mid;
    }
  }
  count[k] = lo;
}

// Swap the 32-bit halves of each packed arc: (weight << 32) | target <->
// (target << 32) | weight, so that a sort on the upper half orders a row by
// target.
__global__ void swap_halves_kernel(ull* e, ull m) {
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (ull)gridDim.x * blockDim.x) {
    const ull x = e[i];
    e[i] = (x << 32) | (x >> 32);
  }
}

// Renumber g's vertices by decreasing degree (see the file comment).
sssp_status relabel_by_degree(sssp_graph* g, hipStream_t st) {
  const ull n = (ull)g->n, m = (ull)g->m;
  DevBuf keys, keys2, ids, newdeg, newoff, newedges, sorted, tmp, ranks;
  auto cleanup = [&]() {
    for (DevBuf* b : {&keys, &keys2, &ids, &newdeg, &newoff, &newedges, &sorted, &tmp, &ranks}) b->release(st);
  };
  hipError_t e;
  do {
    if ((e = keys.alloc(n * 4, st)) != hipSuccess || (e = keys2.alloc(n * 4, st)) != hipSuccess ||
        (e = ids.alloc(n * 4, st)) != hipSuccess || (e = g->perm.alloc(n * 4, st)) != hipSuccess ||
        (e = g->inv.alloc(n * 4, st)) != hipSuccess || (e = newdeg.alloc((n + 1) * 8, st)) != hipSuccess ||
        (e = newoff.alloc((n + 1) * 8, st)) != hipSuccess || (e = newedges.alloc(m * 8, st)) != hipSuccess)
      break;
    degree_keys_kernel<<<1024, 256, 0, st>>>((const int64_t*)g->off.p, n, (uint32_t*)keys.p, (int32_t*)ids.p);
    if ((e = hipGetLastError()) != hipSuccess) break;
    size_t bytes = 0;
    if ((e = rocprim::radix_sort_pairs(nullptr, bytes, (uint32_t*)keys.p, (uint32_t*)keys2.p, (int32_t*)ids.p,
                                       (int32_t*)g->perm.p, (size_t)n, 0, 32, st)) != hipSuccess)
      break;
    if ((e = tmp.alloc(bytes, st)) != hipSuccess) break;
    if ((e = rocprim::radix_sort_pairs(tmp.p, bytes, (uint32_t*)keys.p, (uint32_t*)keys2.p, (int32_t*)ids.p,
                                       (int32_t*)g->perm.p, (size_t)n, 0, 32, st)) != hipSuccess)
      break;
    invert_kernel<<<1024, 256, 0, st>>>((const int32_t*)g->perm.p, (const int64_t*)g->off.p, n,
                                        (int32_t*)g->inv.p, (int64_t*)newdeg.p);
    if ((e = hipGetLastError()) != hipSuccess) break;
    size_t sbytes = 0;
    if ((e = rocprim::exclusive_scan(nullptr, sbytes, (int64_t*)newdeg.p, (int64_t*)newoff.p, (int64_t)0,
                                     (size_t)(n + 1), rocprim::plus<int64_t>(), st)) != hipSuccess)
      break;
    if (sbytes > tmp.bytes && (e = tmp.alloc(sbytes, st)) != hipSuccess) break;
    if ((e = rocprim::exclusive_scan(tmp.p, sbytes, (int64_t*)newdeg.p, (int64_t*)newoff.p, (int64_t)0,
                                     (size_t)(n + 1), rocprim::plus<int64_t>(), st)) != hipSuccess)
      break;
    if (m > 0) {
      relabel_rows_kernel<<<2048, 256, 0, st>>>((const int32_t*)g->perm.p, (const int32_t*)g->inv.p,
                                                (const int64_t*)g->off.p, (const int64_t*)newoff.p,
                                                (const ull*)g->edges.p, (ull*)newedges.p, n);
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    if (m > 0 && m < (1ull << 32) && n < (1ull << 32)) {
      // Each row in increasing target order: the lanes that relax a
      // high-degree row together then read the key bounds of nearby
      // vertices, which share cache lines, so a wave's gather touches fewer
      // lines. (A layout choice; the rows' arc multisets are unchanged.)
      swap_halves_kernel<<<2048, 256, 0, st>>>((ull*)newedges.p, m);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = sorted.alloc(m * 8, st)) != hipSuccess) break;
      size_t qbytes = 0;
      if ((e = rocprim::segmented_radix_sort_keys(nullptr, qbytes, (const ull*)newedges.p, (ull*)sorted.p,
                                                   (unsigned)m, (unsigned)n, (const int64_t*)newoff.p,
                                                   (const int64_t*)newoff.p + 1, 32, 64, st)) != hipSuccess)
        break;
      if (qbytes > tmp.bytes && (e = tmp.alloc(qbytes, st)) != hipSuccess) break;
      if ((e = rocprim::segmented_radix_sort_keys(tmp.p, qbytes, (const ull*)newedges.p, (ull*)sorted.p,
                                                   (unsigned)m, (unsigned)n, (const int64_t*)newoff.p,
                                                   (const int64_t*)newoff.p + 1, 32, 64, st)) != hipSuccess)
        break;
      swap_halves_kernel<<<2048, 256, 0, st>>>((ull*)sorted.p, m);
      if ((e = hipGetLastError()) != hipSuccess) break;
      std::swap(newedges, sorted);
    }
    if ((e = ranks.alloc(33 * 8, st)) != hipSuccess) break;
    degree_ranks_kernel<<<1, 64, 0, st>>>((const int64_t*)newoff.p, n, (ull*)ranks.p);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipMemcpyAsync(g->deg_ge, ranks.p, 33 * 8, hipMemcpyDeviceToHost, st)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) break;
    std::swap(g->off, newoff);
    std::swap(g->edges, newedges);
    g->relabelled = true;
  } while (false);
  cleanup();
  if (e != hipSuccess) {
    g->perm.release(st);
    g->inv.release(st);
    return fail(from_hip(e), std::string("relabel: ") + hipGetErrorString(e));
  }
  return SSSP_OK;
}

}  // namespace

std::string& sssp_impl::last_error() {
  static thread_local std::string s;
  return s;
}

extern "C" {

int sssp_abi_version(void) { return SSSP_ABI_VERSION; }

const char* sssp_status_string(sssp_status s) {
  switch (s) {
    case SSSP_OK: return "ok";
    case SSSP_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SSSP_ERR_INVALID_GRAPH: return "invalid graph";
    case SSSP_ERR_OUT_OF_MEMORY: return "out of device memory";
    case SSSP_ERR_NO_DEVICE: return "no usable HIP device";
    case SSSP_ERR_DEVICE: return "device error";
    case SSSP_ERR_STEP_LIMIT: return "step limit reached";
    case SSSP_ERR_UNSUPPORTED: return "unsupported";
    case SSSP_ERR_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* sssp_last_error(void) { return last_error().c_str(); }

sssp_status sssp_graph_destroy(sssp_graph* g) {
  if (!g) return SSSP_OK;
  if (g->serving) return fail(SSSP_ERR_INVALID_ARGUMENT, "a server is running on this graph; stop it first");
  if (g->pending) return fail(SSSP_ERR_INVALID_ARGUMENT, "an asynchronous solve is pending; sssp_solve_wait first");
  (void)hipSetDevice(g->device);
  g->release_all();
  delete g;
  return SSSP_OK;
}

sssp_status sssp_graph_info(const sssp_graph* g, int64_t* n, int64_t* m, uint64_t* device_bytes) {
  if (!g) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (device_bytes) *device_bytes = g->graph_bytes() + g->workspace_bytes();
  return SSSP_OK;
}

sssp_status sssp_graph_create(int64_t n, int64_t m, sssp_offset_width ow, const void* offsets,
                              const int32_t* targets, const uint32_t* weights, uint32_t flags, void* stream,
                              sssp_graph** out) {
  last_error().clear();
  if (!out) return fail(SSSP_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (n < 1 || n >= ((int64_t)1 << 31)) return fail(SSSP_ERR_INVALID_ARGUMENT, "n must satisfy 1 <= n < 2^31");
  if (m < 0 || m >= ((int64_t)1 << 40)) return fail(SSSP_ERR_INVALID_ARGUMENT, "m must satisfy 0 <= m < 2^40");
  if (ow != SSSP_OFFSETS_I32 && ow != SSSP_OFFSETS_I64) return fail(SSSP_ERR_INVALID_ARGUMENT, "bad offset width");
  if (ow == SSSP_OFFSETS_I32 && m >= ((int64_t)1 << 31))
    return fail(SSSP_ERR_INVALID_ARGUMENT, "int32 offsets need m < 2^31");
  const bool host = (flags & SSSP_INPUT_HOST) != 0, device = (flags & SSSP_INPUT_DEVICE) != 0;
  if (host == device) return fail(SSSP_ERR_INVALID_ARGUMENT, "exactly one of SSSP_INPUT_HOST/DEVICE");
  if (flags & ~(SSSP_INPUT_HOST | SSSP_INPUT_DEVICE | SSSP_TRUST_INPUT | SSSP_KEEP_ORDER | SSSP_UNDIRECTED |
                SSSP_BORROW_DEVICE))
    return fail(SSSP_ERR_INVALID_ARGUMENT, "unknown flag bits");
  const bool borrow = (flags & SSSP_BORROW_DEVICE) != 0;
  if (borrow && !device) return fail(SSSP_ERR_INVALID_ARGUMENT, "SSSP_BORROW_DEVICE needs SSSP_INPUT_DEVICE");
  if (!offsets || (m > 0 && (!targets || !weights))) return fail(SSSP_ERR_INVALID_ARGUMENT, "NULL array");
  const bool trust = (flags & SSSP_TRUST_INPUT) != 0;

  // Host input is validated before any device call.
  if (host && !trust) {
    auto offat = [&](int64_t i) -> int64_t {
      return ow == SSSP_OFFSETS_I64 ? ((const int64_t*)offsets)[i] : (int64_t)((const int32_t*)offsets)[i];
    };
    if (offat(0) != 0) return fail(SSSP_ERR_INVALID_GRAPH, "offsets[0] != 0");
    for (int64_t i = 0; i < n; ++i)
      if (offat(i + 1) < offat(i))
        return fail(SSSP_ERR_INVALID_GRAPH, "offsets decrease at index " + std::to_string(i));
    if (offat(n) != m) return fail(SSSP_ERR_INVALID_GRAPH, "offsets[n] != m");
    for (int64_t i = 0; i < m; ++i)
      if (targets[i] < 0 || targets[i] >= n)
        return fail(SSSP_ERR_INVALID_GRAPH, "target out of range at arc " + std::to_string(i));
  }

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(SSSP_ERR_NO_DEVICE, "no HIP device");
  int dev = 0;
  SSSP_HIP_TRY(hipGetDevice(&dev));
  int coop = 0;
  SSSP_HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return fail(SSSP_ERR_NO_DEVICE, "device lacks cooperative launch");

  sssp_graph* g = new sssp_graph();
  g->device = dev;
  g->n = n;
  g->m = m;
  int cus = 0, khz = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  g->cus = cus > 0 ? cus : 1;
  g->tick_khz = khz > 0 ? (uint64_t)khz : 100000;
  hipStream_t st = (hipStream_t)stream;

  DevBuf t32, w32, o32, flag;
  const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  sssp_status rs = SSSP_OK;
  std::string msg;
  hipError_t e = hipSuccess;
  do {
    if ((e = g->off.alloc((size_t)(n + 1) * 8, st)) != hipSuccess) break;
    if (!borrow && (e = g->edges.alloc((size_t)m * 8, st)) != hipSuccess) break;
    if (ow == SSSP_OFFSETS_I64) {
      if ((e = hipMemcpyAsync(g->off.p, offsets, (size_t)(n + 1) * 8, kind, st)) != hipSuccess) break;
    } else {
      if ((e = o32.alloc((size_t)(n + 1) * 4, st)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(o32.p, offsets, (size_t)(n + 1) * 4, kind, st)) != hipSuccess) break;
      widen_offsets_kernel<<<1024, 256, 0, st>>>((const int32_t*)o32.p, (int64_t*)g->off.p, (ull)(n + 1));
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    const int32_t* tsrc = targets;
    const uint32_t* wsrc = weights;
    if (m > 0 && host) {
      if ((e = t32.alloc((size_t)m * 4, st)) != hipSuccess) break;
      if ((e = w32.alloc((size_t)m * 4, st)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(t32.p, targets, (size_t)m * 4, hipMemcpyHostToDevice, st)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(w32.p, weights, (size_t)m * 4, hipMemcpyHostToDevice, st)) != hipSuccess) break;
      tsrc = (const int32_t*)t32.p;
      wsrc = (const uint32_t*)w32.p;
    }
    if (device && !trust) {
      if ((e = flag.alloc(16, st)) != hipSuccess) break;
      reset_flags_kernel<<<1, 1, 0, st>>>((unsigned*)flag.p, (ull*)flag.p + 1);
      validate_kernel<<<1024, 256, 0, st>>>((const int64_t*)g->off.p, tsrc, (ull)n, (ull)m, (unsigned*)flag.p,
                                            (ull*)flag.p + 1);
      ull back[2] = {0, INF};
      if ((e = hipGetLastError()) == hipSuccess &&
          (e = hipMemcpyAsync(back, flag.p, 16, hipMemcpyDeviceToHost, st)) == hipSuccess)
        e = hipStreamSynchronize(st);
      if (e != hipSuccess) break;
      if ((unsigned)back[0]) {
        rs = SSSP_ERR_INVALID_GRAPH;
        msg = "device CSR validation failed (code " + std::to_string((unsigned)back[0]) + ", index " +
              std::to_string(back[1] == INF ? -1LL : (long long)back[1]) + ")";
        break;
      }
    }
    // Borrowed arrays stay as they are; the symmetry check below reads a
    // packed copy made for it alone.
    DevBuf& packed = borrow ? t32 : g->edges;
    const bool check_sym = (flags & SSSP_UNDIRECTED) && !trust && m > 0;
    if (borrow) {
      g->borrowed = true;
      g->btgt = targets;
      g->bwt = weights;
      if (check_sym && (e = packed.alloc((size_t)m * 8, st)) != hipSuccess) break;
    }
    if (m > 0 && (!borrow || check_sym)) {
      pack_edges_kernel<<<2048, 256, 0, st>>>(tsrc, wsrc, (ull*)packed.p, (ull)m);
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    if (check_sym) {
      if ((e = flag.alloc(16, st)) != hipSuccess) break;
      if ((e = hipMemsetAsync(flag.p, 0, 16, st)) != hipSuccess) break;
      symmetry_hash_kernel<<<1024, 256, 0, st>>>((const int64_t*)g->off.p, (const ull*)packed.p, (ull)n,
                                                 (ull*)flag.p);
      ull sums[2] = {0, 1};
      if ((e = hipGetLastError()) == hipSuccess &&
          (e = hipMemcpyAsync(sums, flag.p, 16, hipMemcpyDeviceToHost, st)) == hipSuccess)
        e = hipStreamSynchronize(st);
      if (e != hipSuccess) break;
      if (sums[0] != sums[1]) {
        rs = SSSP_ERR_INVALID_GRAPH;
        msg = "SSSP_UNDIRECTED: the arcs are not symmetric (some (u, v, w) lacks its reverse (v, u, w))";
        break;
      }
    }
    g->undirected = (flags & SSSP_UNDIRECTED) != 0;
    e = hipStreamSynchronize(st);
  } while (false);
  t32.release(st);
  w32.release(st);
  o32.release(st);
  flag.release(st);
  if (e == hipSuccess && rs == SSSP_OK && !(flags & SSSP_KEEP_ORDER) && !borrow) rs = relabel_by_degree(g, st);
  if (e != hipSuccess) {
    sssp_graph_destroy(g);
    return fail(from_hip(e), std::string("graph upload: ") + hipGetErrorString(e));
  }
  if (rs != SSSP_OK) {
    sssp_graph_destroy(g);
    return msg.empty() ? rs : fail(rs, msg);
  }
  *out = g;
  return SSSP_OK;
}

}  // extern "C"
