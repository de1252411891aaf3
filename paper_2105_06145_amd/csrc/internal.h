// Host-side definitions shared by the library's translation units
// (graph.hip: graph creation; stepping.hip: the solve).
#ifndef SSSP_INTERNAL_H
#define SSSP_INTERNAL_H

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/sssp.h"

namespace sssp_impl {

typedef unsigned long long ull;
constexpr ull INF = ~0ull;

// Thread-local detail string behind sssp_last_error().
std::string& last_error();

inline sssp_status fail(sssp_status s, const std::string& msg) {
  last_error() = msg;
  return s;
}

inline sssp_status from_hip(hipError_t e) {
  return e == hipErrorOutOfMemory ? SSSP_ERR_OUT_OF_MEMORY : SSSP_ERR_DEVICE;
}

#define SSSP_HIP_TRY(expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return ::sssp_impl::fail(::sssp_impl::from_hip(e_),                                    \
                               std::string(#expr) + ": " + hipGetErrorString(e_));           \
  } while (0)

// Owned device allocation, stream-ordered: allocating and freeing wait only
// for work on the given stream (hipFree would wait for the whole device, and
// with it for a persistent serving launch that runs until it is stopped).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t alloc(size_t b, hipStream_t st) {
    release(st);
    bytes = b;
    return hipMallocAsync(&p, b ? b : 8, st);
  }
  void release(hipStream_t st) {
    if (p) (void)hipFreeAsync(p, st);
    p = nullptr;
    bytes = 0;
  }
};

}  // namespace sssp_impl

// The opaque graph handle: the device copy of the graph in the library's own
// layout, plus the solve workspace (allocated on first solve).
struct sssp_graph {
  int device = 0;
  int64_t n = 0, m = 0;
  int cus = 0;
  uint64_t tick_khz = 100000;  // wall-clock counter rate
  // Graph, in internal vertex ids. When `relabelled`, internal id i is the
  // caller's vertex perm[i] and inv[v] is the internal id of caller vertex v.
  sssp_impl::DevBuf off;    // int64[n + 1]
  sssp_impl::DevBuf edges;  // uint64[m]: (weight << 32) | internal target
  sssp_impl::DevBuf perm, inv;
  bool relabelled = false;
  // Relabelled graphs (degrees do not increase with the id): deg_ge[k] is the
  // number of vertices of out-degree at least 2^k, the ids 0 .. deg_ge[k] - 1.
  uint64_t deg_ge[33] = {};
  // SSSP_BORROW_DEVICE: the caller's device targets and weights are used in
  // place (edges is then empty; the caller keeps them alive and unchanged
  // in shape until the graph is destroyed).
  bool borrowed = false;
  const int32_t* btgt = nullptr;
  const uint32_t* bwt = nullptr;
  bool undirected = false;  // every arc (u, v, w) has its reverse (v, u, w)
  bool serving = false;  // a persistent server owns the workspace
  void* pending = nullptr;          // the pending asynchronous solve (owned by stepping.hip)
  uint32_t* cancel_flag = nullptr;  // host (hipHostMalloc): nonzero asks the pending solve to stop
  int32_t* src_host = nullptr;      // host (hipHostMalloc): staged sources of an asynchronous solve
  uint64_t src_host_cap = 0;
  // Workspace.
  bool ws_ready = false;
  uint32_t ws_hub_degree = 0, ws_chunk = 0, ws_probe_cap = 0, ws_G = 0, ws_teams = 0;
  uint64_t ws_src_cap = 0;  // sources the `srcs` buffer holds
  uint64_t ws_segcap = 0;   // F entries per workgroup the workspace was sized for
  uint32_t ws_local_cap = 0;  // local-expansion degree cap of bigmask
  bool ws_repeat = false;     // lastkey / ckey / cbase allocated (repeated-push skip)
  uint64_t nhub = 0;          // hubs numbered first (entries of cbase), with ws_repeat on a relabelled graph
  sssp_impl::DevBuf dist_int, bitmap, hint, tree, hubmask, bigmask, F, FD, H, L, samples, parts, ctl, args, srcs;
  sssp_impl::DevBuf lastkey, ckey, cbase;
  void* hargs = nullptr;  // host staging copy of the kernel arguments (operator new)

  // Local expansion: per arc, the packed row of its target (built on the
  // first launch with local expansion).
  sssp_impl::DevBuf trow;

  uint64_t graph_bytes() const { return off.bytes + edges.bytes + perm.bytes + inv.bytes + trow.bytes; }
  uint64_t workspace_bytes() const {
    return dist_int.bytes + bitmap.bytes + hint.bytes + tree.bytes + hubmask.bytes + bigmask.bytes + F.bytes + FD.bytes + H.bytes + L.bytes + samples.bytes +
           parts.bytes + ctl.bytes + args.bytes + srcs.bytes + lastkey.bytes + ckey.bytes + cbase.bytes;
  }
  void release_ws(hipStream_t st) {
    for (sssp_impl::DevBuf* b : {&dist_int, &bitmap, &hint, &tree, &hubmask, &bigmask, &F, &FD, &H, &L, &samples, &parts, &ctl, &args, &srcs,
                                 &lastkey, &ckey, &cbase})
      b->release(st);
    ws_ready = false;
    ws_repeat = false;
    nhub = 0;
    ws_src_cap = 0;
  }
  void release_all() {
    release_ws(nullptr);
    if (cancel_flag) (void)hipHostFree(cancel_flag);
    if (src_host) (void)hipHostFree(src_host);
    cancel_flag = nullptr;
    src_host = nullptr;
    src_host_cap = 0;
    off.release(nullptr);
    edges.release(nullptr);
    trow.release(nullptr);
    perm.release(nullptr);
    inv.release(nullptr);
    ::operator delete(hargs);
    hargs = nullptr;
  }
};

#endif  // SSSP_INTERNAL_H
