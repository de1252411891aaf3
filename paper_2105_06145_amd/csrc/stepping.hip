// Persistent stepping-loop kernel for single-source shortest paths on
// MI355X (gfx950), and the C ABI declared in include/sssp.h.
//
// One cooperative launch runs Alg. 1 (Sec. 3.2) for one source:
//
//   S0 init      delta[.] = inf, bitmap = 0; delta[s] = 0, Update(s).
//   S1 ExtDist   theta per Table 2: rho-th smallest by sampling (Sec. 6,
//                App. B), i * Delta (Delta*), +inf (Bellman-Ford), min (test).
//   S2 Extract   F = {v in Q : delta[v] <= theta}; their queue flags cleared
//                (Table 1). Q is a bitmap (the flat-array LaB-PQ of Sec. 4.3)
//                plus, while |Q| is small, an explicit list (Sec. 6, sparse
//                mode), so small steps do not scan all n flags.
//   S3 Relax     for u in F, v in N(u): WriteMin(delta[v], delta[u] + w) as a
//                64-bit atomic min (Sec. 2 WriteMin), skipped when a plain read
//                of delta[v] already shows no improvement.
//   S4 Update    a successful WriteMin sets v's flag with an atomic OR; the old
//                word tells whether v is new to Q, so the explicit list gets
//                each new member once, with no hash table or pack pass.
//   S5 loop      until |Q| = 0. Phases are separated by grid barriers, so
//                Extract never overlaps Update (Sec. 3.1).
//
// Work distribution. Each workgroup owns a static slice of the queue: a
// contiguous range of bitmap words (bitmap steps) or of the explicit list
// (list steps). What it extracts goes to its own segment of F, so Extract
// needs no shared counter; in Relax it processes its own segment in tiles of
// 256 vertices, whose (row begin, delta) pairs and degree prefix sums sit in
// LDS, so consecutive lanes read consecutive 8-byte (target, weight) arcs.
// Vertices above hub_degree are cut into fixed-size edge chunks that all
// workgroups share. Counters are per-workgroup partials, summed by the last
// workgroup to reach the step's final barrier.
//
// Memory visibility across the eight XCDs (each with its own L2): the grid
// barrier is hierarchical. Workgroups of one XCD (read from the XCC_ID
// hardware register) meet first; the last of them writes back that XCD's L2
// (agent-scope release) before arriving at the global counter, and after the
// global release invalidates the XCD's L2 (agent-scope acquire) before
// releasing its group. Data other workgroups wrote in earlier phases is read
// with agent-scope loads, which bypass the per-CU L1.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "internal.h"

using namespace sssp_impl;

// Marks device pointers that live in global memory. Expands to nothing: the
// variant that spelled out the global address space here aborted on the GPU
// with no diagnosed cause, so it stays switched off.
#define GPTR

namespace {

constexpr int WG = 256;
constexpr int WAVES = WG / 64;
constexpr int UNROLL = 4;  // arcs / list entries per lane per iteration
constexpr int BATCH = 4;   // queue members per lane per round in bitmap scans
constexpr int MAX_XCC = 16;
constexpr int BLOCK_WORDS = 4;  // bitmap words per ownership block (256 vertices)

// ---------------------------------------------------------------------------
// Device-side control block.

struct alignas(128) StepSlot {
  ull h_count;      // hub chunk tasks in H
  ull list_next;    // entries written to the next explicit list
  ull nsamples;     // accepted threshold samples
  ull x_total;      // vertices extracted (sum of partials)
  ull fresh_total;  // vertices whose flag went 0 -> 1 in Relax
  ull min_next;     // min key over the next queue
  ull edges;        // arcs relaxed
  ull successes;    // successful WriteMins
  ull pad[8];
};

struct alignas(128) Line {
  ull v;
  ull pad[15];
};

struct Control {
  Line arrive_flat;  // first (flat) barrier
  Line gen_flat;
  Line arrive;       // group leaders arriving at the global level
  Line gen;
  Line grp_arrive[MAX_XCC];
  Line grp_gen[MAX_XCC];
  Line grp_size[MAX_XCC];
  alignas(128) unsigned abort_flag;
  unsigned status;  // 0 ok, 1 step limit
  ull theta;
  ull ngroups;
  ull st_steps, st_extracted, st_edges, st_success, st_dense, st_sampled;
  ull phase_ticks[4];  // init, threshold, extract, relax (workgroup 0's view)
  ull relax_busy_max, relax_busy_sum;  // per step: slowest workgroup, sum over workgroups
  alignas(128) StepSlot slot[3];
};

constexpr unsigned ST_OK = 0, ST_STEP_LIMIT = 1;

// Per-workgroup partial counts of one step (written with plain stores, summed
// by the last workgroup at the step's final barrier).
struct alignas(64) Part {
  ull x;        // vertices extracted
  ull minkept;  // min key of members left in Q
  ull edges;    // arcs relaxed
  ull succ;     // successful WriteMins
  ull fresh;    // new queue members
  ull minnew;   // min successful WriteMin value
  ull busy;     // wall-clock ticks this workgroup spent in Relax
  ull pad;
};

struct KArgs {
  int64_t n;
  uint64_t nwords;
  const GPTR int64_t* off;
  const GPTR ull* edges;    // (weight << 32) | target
  const GPTR ull* hubmask;  // bit v set iff deg(v) > hub_degree
  GPTR ull* dist;            // tentative distances, internal ids
  GPTR ull* dist_out;        // the caller's row (caller ids) when the graph is relabelled
  const GPTR int32_t* perm;  // internal id -> caller id (NULL: identity)
  const GPTR int32_t* inv;   // caller id -> internal id (NULL: identity)
  GPTR ull* bitmap;
  GPTR int32_t* F;  // G segments of segcap entries
  GPTR ull* H;      // (vertex << 32) | chunk index
  GPTR int32_t* L0;
  GPTR int32_t* L1;
  GPTR ull* samples;
  GPTR Part* parts;
  GPTR Control* ctl;
  GPTR uint32_t* xcount;
  GPTR sssp_step_record* trace;
  uint64_t trace_cap;
  uint64_t rho, delta, seed, max_steps;
  uint64_t list_threshold;
  uint64_t tlimit;
  uint64_t segcap;
  int32_t source;
  uint32_t rule;
  uint32_t G;
  uint32_t chunk_edges;
  uint32_t sample_cap;
  uint32_t probe_cap;
  uint32_t filter;
};

struct Shared {
  ull beg[WG];
  ull du[WG];
  uint32_t pre[WG + 1];
  uint32_t hist[WG];
  uint32_t wsum[WAVES];
  ull red[WAVES * 4];
  ull bcast[4];
  int last;
  int abort;
};

// Barrier bookkeeping kept in registers by every workgroup.
struct Sync {
  ull epoch = 0;
  unsigned xcc = 0;
  ull gsz = 1;
  ull ngroups = 1;
};

// ---------------------------------------------------------------------------
// Small device helpers.

// Plain load: may hit the per-CU L1. Used for immutable data and for the
// Relax filter, where a stale (never smaller) key is harmless.
template <class P>
__device__ __forceinline__ ull ld_plain(P p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Agent-scope load: bypasses L1; used for data other workgroups wrote.
template <class P>
__device__ __forceinline__ ull ld_agent(P p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ int32_t ld_agent_i32(P p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ ull atom_add(P p, ull v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ ull atom_min(P p, ull v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ ull atom_or(P p, ull v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ ull atom_and(P p, ull v) {
  return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ void st_agent(P p, ull v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output i of the stream
// started at `seed`.
__device__ __forceinline__ ull splitmix(ull seed, ull i) {
  ull z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ ull below(ull r, ull range) { return __umul64hi(r, range); }

__device__ __forceinline__ unsigned lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ ull umin(ull a, ull b) { return a < b ? a : b; }

__device__ __forceinline__ ull wave_sum(ull v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ ull wave_min(ull v) {
  for (int o = 32; o > 0; o >>= 1) v = umin(v, __shfl_xor(v, o));
  return v;
}

// Exclusive prefix sum of one count per thread across the workgroup; every
// thread gets its offset and the total. Whole workgroup, uniform call.
__device__ __forceinline__ uint32_t wg_scan(Shared& sh, uint32_t c, uint32_t& total) {
  const unsigned lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t incl = c;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if ((int)lane >= o) incl += y;
  }
  __syncthreads();
  if (lane == 63) sh.wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (int w = 0; w < WAVES; ++w) {
    const uint32_t s = sh.wsum[w];
    before += (unsigned)w < wave ? s : 0u;
    total += s;
  }
  return before + incl - c;
}

// Reserve c slots per thread in a shared list with one atomic per workgroup.
// Returns each thread's first slot. Whole workgroup, uniform call.
template <class P>
__device__ __forceinline__ ull wg_reserve(Shared& sh, P counter, uint32_t c) {
  uint32_t total;
  const uint32_t off = wg_scan(sh, c, total);
  if (total == 0) return 0;
  if (threadIdx.x == 0) sh.bcast[0] = atom_add(counter, (ull)total);
  __syncthreads();
  const ull base = sh.bcast[0];
  __syncthreads();
  return base + off;
}

// Workgroup reductions of four values (sum, sum, sum, min), broadcast.
__device__ void wg_reduce4(Shared& sh, ull& a, ull& b, ull& c, ull& mn) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  mn = wave_min(mn);
  const unsigned lane = lane_id(), wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh.red[wave * 4 + 0] = a;
    sh.red[wave * 4 + 1] = b;
    sh.red[wave * 4 + 2] = c;
    sh.red[wave * 4 + 3] = mn;
  }
  __syncthreads();
  a = b = c = 0;
  mn = INF;
  for (int w = 0; w < WAVES; ++w) {
    a += sh.red[w * 4 + 0];
    b += sh.red[w * 4 + 1];
    c += sh.red[w * 4 + 2];
    mn = umin(mn, sh.red[w * 4 + 3]);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Grid barriers. Every workgroup calls them in the same order. The last
// workgroup to arrive runs `serial` (whole workgroup) before releasing the
// others, so per-step bookkeeping costs no extra barrier. Every wait is
// bounded: past `tlimit` wall-clock ticks the waiter raises the abort flag and
// all workgroups leave the kernel at their next barrier. Returns false on abort.

template <class P>
__device__ bool spin_until(const GPTR KArgs& a, P flag, ull target) {
  const long long t0 = wall_clock64();
  unsigned spins = 0;
  while (ld_agent(flag) < target) {
    __builtin_amdgcn_s_sleep(1);
    if ((++spins & 63) == 0) {
      if (__hip_atomic_load(&a.ctl->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if ((ull)(wall_clock64() - t0) > a.tlimit) {
        __hip_atomic_store(&a.ctl->abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
  return true;
}

__device__ __forceinline__ bool finish_sync(const GPTR KArgs& a, Shared& sh) {
  if (threadIdx.x == 0)
    sh.abort = __hip_atomic_load(&a.ctl->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  const bool ok = sh.abort == 0;
  __syncthreads();
  return ok;
}

// Flat barrier (every workgroup releases and acquires at agent scope); used
// once, before the XCD groups are known.
template <class Serial>
__device__ bool flat_sync(const GPTR KArgs& a, Shared& sh, Serial serial) {
  GPTR Control* ctl = a.ctl;
  __syncthreads();
  if (threadIdx.x == 0) {
    const ull prev =
        __hip_atomic_fetch_add(&ctl->arrive_flat.v, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    sh.last = prev == (ull)a.G - 1ull;
    if (sh.last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (sh.last) {
    serial();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&ctl->gen_flat.v, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  } else if (threadIdx.x == 0) {
    spin_until(a, &ctl->gen_flat.v, 1ull);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  return finish_sync(a, sh);
}

// Hierarchical barrier (see the file comment).
template <class Serial>
__device__ bool grid_sync(const GPTR KArgs& a, Shared& sh, Sync& sy, Serial serial) {
  GPTR Control* ctl = a.ctl;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
  __syncthreads();
  ++sy.epoch;
  if (threadIdx.x == 0) {
    sh.last = 0;
    const ull prev = atom_add(&ctl->grp_arrive[sy.xcc].v, 1ull);
    if (prev == sy.epoch * sy.gsz - 1ull) {
      // Last of this XCD: publish the XCD's L2 contents, then arrive globally.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const ull p2 = atom_add(&ctl->arrive.v, 1ull);
      if (p2 == sy.epoch * sy.ngroups - 1ull) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        sh.last = 1;
      } else {
        spin_until(a, &ctl->gen.v, sy.epoch);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        st_agent(&ctl->grp_gen[sy.xcc].v, sy.epoch);
      }
    } else {
      spin_until(a, &ctl->grp_gen[sy.xcc].v, sy.epoch);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
  if (sh.last) {
    serial();
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      st_agent(&ctl->gen.v, sy.epoch);
      st_agent(&ctl->grp_gen[sy.xcc].v, sy.epoch);
    }
  }
  return finish_sync(a, sh);
}

struct NoSerial {
  __device__ void operator()() const {}
};

// k-th smallest (1-based) of vals[0..s) by MSD radix selection over the bits
// below the highest bit where min and max differ. Whole workgroup.
template <class P>
__device__ __noinline__ ull wg_select_kth(P vals, ull s, ull k, Shared& sh) {
  const unsigned tid = threadIdx.x;
  ull mn = INF, negmax = INF;  // max(x) = ~min(~x)
  for (ull i = tid; i < s; i += WG) {
    const ull v = ld_agent(&vals[i]);
    mn = umin(mn, v);
    negmax = umin(negmax, ~v);
  }
  {
    ull z0 = 0, z1 = 0, z2 = 0;
    wg_reduce4(sh, z0, z1, z2, mn);
    wg_reduce4(sh, z0, z1, z2, negmax);
  }
  const ull mx = ~negmax;
  if (mn == mx) return mn;
  const int hb = 63 - __clzll((long long)(mn ^ mx));
  int top = hb + 1;
  ull prefix = (top >= 64) ? 0ull : ((mn >> top) << top);
  while (top > 0) {
    const int width = top < 8 ? top : 8;
    const int shift = top - width;
    const ull dmask = (1ull << width) - 1ull;
    sh.hist[tid] = 0;
    __syncthreads();
    for (ull i = tid; i < s; i += WG) {
      const ull v = ld_agent(&vals[i]);
      const bool match = (top >= 64) ? true : ((v >> top) == (prefix >> top));
      if (match) atomicAdd(&sh.hist[(v >> shift) & dmask], 1u);
    }
    __syncthreads();
    if (tid < 64) {
      // Each lane owns 4 consecutive bins; find the bin holding rank k.
      ull c[4], tot = 0;
      for (int j = 0; j < 4; ++j) {
        c[j] = sh.hist[tid * 4 + j];
        tot += c[j];
      }
      ull incl = tot;
      for (int o = 1; o < 64; o <<= 1) {
        const ull y = __shfl_up(incl, o);
        if ((int)tid >= o) incl += y;
      }
      const ull excl = incl - tot;
      const ull hit = __ballot(incl >= k);
      const int owner = __ffsll((long long)hit) - 1;
      if ((int)tid == owner) {
        ull acc = excl;
        int j = 0;
        for (; j < 4; ++j) {
          if (acc + c[j] >= k) break;
          acc += c[j];
        }
        sh.bcast[0] = (ull)(tid * 4 + j);
        sh.bcast[1] = k - acc;
      }
    }
    __syncthreads();
    prefix |= sh.bcast[0] << shift;
    k = sh.bcast[1];
    top = shift;
    __syncthreads();
  }
  return prefix;
}

// ---------------------------------------------------------------------------
// Extract helpers.

// Record one extracted hub vertex: its arcs become chunk tasks shared by all
// workgroups in Relax.
__device__ __noinline__ void push_hub(const GPTR KArgs& a, GPTR StepSlot* S, int32_t v) {
  const ull deg = (ull)(a.off[v + 1] - a.off[v]);
  const ull nch = (deg + a.chunk_edges - 1) / a.chunk_edges;
  const ull base = atom_add(&S->h_count, nch);
  for (ull c = 0; c < nch; ++c) a.H[base + c] = ((ull)(uint32_t)v << 32) | c;
}

// Relax one arc (S3 + S4). Returns true when v became a new queue member.
// Filter: a plain read of delta[v] (possibly stale, but never smaller than
// the current value) showing nd >= delta[v] means the WriteMin cannot succeed,
// so the atomic is skipped.
__device__ __forceinline__ bool relax_arc(const GPTR KArgs& a, ull& succ, ull& minnew, int32_t v, ull nd) {
  if (a.filter && !(nd < ld_plain(&a.dist[v]))) return false;
  const ull old = atom_min(&a.dist[v], nd);
  if (!(nd < old)) return false;
  ++succ;
  minnew = umin(minnew, nd);
  const ull bit = 1ull << (v & 63);
  return !(atom_or(&a.bitmap[v >> 6], bit) & bit);
}

// ---------------------------------------------------------------------------
// Phases. Each is a separate (not inlined) function so that registers are
// allocated per phase rather than for the union of all of them.

__shared__ Shared g_sh;

// Sample size and probe count of a rho step (App. B: s = c (q / rho + log q),
// c = 10, log q = 1 + log2(q + 1)); a bitmap step probes random vertex ids and
// keeps those in Q, so it needs about s * n / q probes.
__device__ __noinline__ ull rho_probes(ull q, ull rho_eff, ull n, bool dense, uint32_t sample_cap,
                                       uint32_t probe_cap) {
  const double lq = 1.0 + log2((double)q + 1.0);
  double st = ceil(10.0 * ((double)q / (double)rho_eff + lq));
  if (st > (double)sample_cap) st = (double)sample_cap;
  if (!dense) return (ull)st;
  double p = ceil(st * (double)n / (double)q * 1.25);
  if (p > (double)probe_cap) p = (double)probe_cap;
  return (ull)p;
}

// S1 for rho-stepping: draw the samples of the queue's keys (App. B). The
// selection itself runs in the following barrier's serial section.
__device__ __noinline__ void phase_sample(const GPTR KArgs* __restrict__ A, GPTR StepSlot* S, const GPTR int32_t* Lcur,
                                          ull q, bool dense, ull probes, ull tseed) {
  Shared& sh = g_sh;
  const ull b = blockIdx.x, G = A->G, nthreads = G * WG, n = (ull)A->n;
  for (ull base = b * WG; base < probes; base += nthreads) {
    const ull j = base + threadIdx.x;
    bool acc = false;
    ull d = 0;
    if (j < probes) {
      const ull r = splitmix(tseed, j);
      if (dense) {
        const ull v = below(r, n);
        if ((ld_agent(&A->bitmap[v >> 6]) >> (v & 63)) & 1ull) {
          acc = true;
          d = ld_agent(&A->dist[v]);
        }
      } else {
        const int32_t v = ld_agent_i32(&Lcur[below(r, q)]);
        acc = true;
        d = ld_agent(&A->dist[v]);
      }
    }
    const ull pos = wg_reserve(sh, &S->nsamples, acc ? 1u : 0u);
    if (acc) A->samples[pos] = d;
  }
}

struct ExtractOut {
  uint32_t fcnt;  // entries written to this workgroup's F segment
  ull x;          // vertices extracted
  ull minkept;    // min key of the members left in Q
};

// S2, bitmap step. Workgroup b owns the blocks of BLOCK_WORDS words
// b, b + G, b + 2G, ... (interleaved, so that the high-degree vertices
// numbered first are spread over all workgroups). Each lane owns one word;
// its members are read in rounds of BATCH keys.
__device__ __noinline__ ExtractOut phase_extract_dense(const GPTR KArgs* __restrict__ A, GPTR StepSlot* S, GPTR int32_t* Fb,
                                                       GPTR int32_t* Lnext, ull theta, bool emit) {
  Shared& sh = g_sh;
  const ull b = blockIdx.x, G = A->G, nw = A->nwords;
  const ull nblocks = (nw + BLOCK_WORDS - 1) / BLOCK_WORDS;
  constexpr ull BLOCKS_PER_ROUND = WG / BLOCK_WORDS;
  ExtractOut o{0, 0, INF};
  for (ull r0 = b; r0 < nblocks; r0 += G * BLOCKS_PER_ROUND) {
    const ull blk = r0 + G * (threadIdx.x / BLOCK_WORDS);
    const ull wi = blk * BLOCK_WORDS + (threadIdx.x % BLOCK_WORDS);
    const ull word = (blk < nblocks && wi < nw) ? ld_agent(&A->bitmap[wi]) : 0ull;
    const ull hubw = word ? ld_plain(&A->hubmask[wi]) : 0ull;
    ull rest = word, clear = 0;
    while (__syncthreads_or(rest != 0)) {
      int32_t v[BATCH];
      ull d[BATCH];
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        v[k] = -1;
        if (rest) {
          const int bit = __ffsll((long long)rest) - 1;
          rest &= rest - 1;
          v[k] = (int32_t)(wi * 64 + bit);
        }
      }
#pragma unroll
      for (int k = 0; k < BATCH; ++k) d[k] = v[k] >= 0 ? ld_agent(&A->dist[v[k]]) : INF;
      uint32_t nsmall = 0, nkeep = 0;
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        if (v[k] < 0) continue;
        const ull bit = 1ull << (v[k] & 63);
        if (d[k] <= theta) {
          clear |= bit;
          ++o.x;
          if (A->xcount) A->xcount[A->perm ? A->perm[v[k]] : v[k]] += 1u;
          if (hubw & bit) {
            push_hub(*A, S, v[k]);
          } else {
            ++nsmall;
          }
        } else {
          o.minkept = umin(o.minkept, d[k]);
          ++nkeep;
        }
      }
      uint32_t total;
      uint32_t fo = o.fcnt + wg_scan(sh, nsmall, total);
      o.fcnt += total;
      ull ko = emit ? wg_reserve(sh, &S->list_next, nkeep) : 0;
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        if (v[k] < 0) continue;
        if (d[k] <= theta) {
          if (!((hubw >> (v[k] & 63)) & 1ull)) Fb[fo++] = v[k];
        } else if (emit) {
          Lnext[ko++] = v[k];
        }
      }
    }
    if (clear) A->bitmap[wi] = word & ~clear;  // this lane owns word wi
  }
  return o;
}

// S2, list step: this workgroup's contiguous slice of the explicit list.
__device__ __noinline__ ExtractOut phase_extract_list(const GPTR KArgs* __restrict__ A, GPTR StepSlot* S, GPTR int32_t* Fb,
                                                      const GPTR int32_t* Lcur, GPTR int32_t* Lnext, ull q, ull theta,
                                                      bool emit) {
  Shared& sh = g_sh;
  const ull b = blockIdx.x, G = A->G;
  const ull lo = b * q / G, hi = (b + 1) * q / G;
  ExtractOut o{0, 0, INF};
  for (ull e0 = lo; e0 < hi; e0 += (ull)WG * UNROLL) {
    int32_t v[UNROLL];
    ull d[UNROLL];
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const ull i = e0 + (ull)k * WG + threadIdx.x;
      v[k] = i < hi ? ld_agent_i32(&Lcur[i]) : -1;
    }
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) d[k] = v[k] >= 0 ? ld_agent(&A->dist[v[k]]) : INF;
    uint32_t nsmall = 0, nkeep = 0;
    unsigned hubs = 0;
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      if (v[k] < 0) continue;
      const ull bit = 1ull << (v[k] & 63);
      if (d[k] <= theta) {
        atom_and(&A->bitmap[v[k] >> 6], ~bit);
        ++o.x;
        if (A->xcount) A->xcount[A->perm ? A->perm[v[k]] : v[k]] += 1u;
        if (ld_plain(&A->hubmask[v[k] >> 6]) & bit) {
          hubs |= 1u << k;
          push_hub(*A, S, v[k]);
        } else {
          ++nsmall;
        }
      } else {
        o.minkept = umin(o.minkept, d[k]);
        ++nkeep;
      }
    }
    uint32_t total;
    uint32_t fo = o.fcnt + wg_scan(sh, nsmall, total);
    o.fcnt += total;
    ull ko = emit ? wg_reserve(sh, &S->list_next, nkeep) : 0;
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      if (v[k] < 0) continue;
      if (d[k] <= theta) {
        if (!((hubs >> k) & 1u)) Fb[fo++] = v[k];
      } else if (emit) {
        Lnext[ko++] = v[k];
      }
    }
  }
  return o;
}

struct RelaxAcc {
  ull edges, succ, fresh, minnew;
};

// Relax UNROLL arcs per lane (ev = packed arc or INF, dd = key of its tail)
// and append new queue members to the next list when it is being built.
__device__ __forceinline__ void relax_batch(const GPTR KArgs* __restrict__ A, GPTR StepSlot* S, GPTR int32_t* Lnext, bool emit,
                                            RelaxAcc& acc, const ull (&ev)[UNROLL], const ull (&dd)[UNROLL]) {
  uint32_t nf = 0;
  int32_t fv[UNROLL];
#pragma unroll
  for (int k = 0; k < UNROLL; ++k) {
    fv[k] = -1;
    if (ev[k] == INF) continue;
    ++acc.edges;
    const int32_t v = (int32_t)(uint32_t)ev[k];
    if (relax_arc(*A, acc.succ, acc.minnew, v, dd[k] + (ev[k] >> 32))) {
      ++acc.fresh;
      fv[k] = v;
      ++nf;
    }
  }
  if (emit) {
    ull o = wg_reserve(g_sh, &S->list_next, nf);
#pragma unroll
    for (int k = 0; k < UNROLL; ++k)
      if (fv[k] >= 0) Lnext[o++] = fv[k];
  }
}

// S3 + S4: the hub chunks (strided over workgroups), then this workgroup's
// own extracted vertices. Writes the workgroup's partial counts.
__device__ __noinline__ void phase_relax(const GPTR KArgs* __restrict__ A, GPTR StepSlot* S, const GPTR int32_t* Fb,
                                         GPTR int32_t* Lnext, bool emit, ExtractOut ex) {
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  const ull b = blockIdx.x, G = A->G;
  const long long t_start = wall_clock64();
  RelaxAcc acc{0, 0, 0, INF};
  const ull nH = ld_agent(&S->h_count);
  const ull CH = A->chunk_edges;
  for (ull item = b; item < nH; item += G) {
    const ull task = ld_agent(&A->H[item]);
    const int32_t u = (int32_t)(task >> 32);
    const ull c = task & 0xffffffffull;
    const ull rb = (ull)A->off[u], re = (ull)A->off[u + 1];
    const ull beg = rb + c * CH;
    const ull end = umin(beg + CH, re);
    const ull du = ld_agent(&A->dist[u]);
    for (ull e0 = beg; e0 < end; e0 += (ull)WG * UNROLL) {
      ull ev[UNROLL], dd[UNROLL];
#pragma unroll
      for (int k = 0; k < UNROLL; ++k) {
        const ull e = e0 + (ull)k * WG + tid;
        ev[k] = e < end ? A->edges[e] : INF;
        dd[k] = du;
      }
      relax_batch(A, S, Lnext, emit, acc, ev, dd);
    }
  }
  for (uint32_t j0 = 0; j0 < ex.fcnt; j0 += WG) {
    const uint32_t j = j0 + tid;
    uint32_t deg = 0;
    ull rb = 0, du = 0;
    if (j < ex.fcnt) {
      const int32_t u = Fb[j];
      rb = (ull)A->off[u];
      deg = (uint32_t)((ull)A->off[u + 1] - rb);
      du = ld_agent(&A->dist[u]);
    }
    uint32_t total;
    const uint32_t excl = wg_scan(sh, deg, total);
    sh.pre[tid] = excl;
    sh.beg[tid] = rb;
    sh.du[tid] = du;
    __syncthreads();
    for (uint32_t e0 = 0; e0 < total; e0 += WG * UNROLL) {
      ull ev[UNROLL], dd[UNROLL];
#pragma unroll
      for (int k = 0; k < UNROLL; ++k) {
        const uint32_t e = e0 + k * WG + tid;
        ev[k] = INF;
        dd[k] = 0;
        if (e < total) {
          int lo = 0;
#pragma unroll
          for (int step = WG / 2; step > 0; step >>= 1)
            if (sh.pre[lo + step] <= e) lo += step;
          ev[k] = A->edges[sh.beg[lo] + (e - sh.pre[lo])];
          dd[k] = sh.du[lo];
        }
      }
      relax_batch(A, S, Lnext, emit, acc, ev, dd);
    }
    __syncthreads();
  }
  ull xs = ex.x, mk = ex.minkept;
  wg_reduce4(sh, acc.edges, acc.succ, acc.fresh, acc.minnew);
  {
    ull z0 = 0, z1 = 0;
    wg_reduce4(sh, xs, z0, z1, mk);
  }
  if (tid == 0) {
    Part p;
    p.x = xs;
    p.minkept = mk;
    p.edges = acc.edges;
    p.succ = acc.succ;
    p.fresh = acc.fresh;
    p.minnew = acc.minnew;
    p.busy = (ull)(wall_clock64() - t_start);
    p.pad = 0;
    A->parts[b] = p;
  }
}

// Serial section of the step's last barrier: sum the partials, publish the
// step totals, clear the slot two steps ahead, update stats and the trace.
__device__ __noinline__ void step_bookkeeping(const GPTR KArgs* __restrict__ A, GPTR StepSlot* S, ull t, ull q, ull theta,
                                              unsigned flags) {
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  GPTR Control* ctl = A->ctl;
  const ull G = A->G;
  ull x = 0, e = 0, s = 0, f = 0, mn = INF, busy = 0, negbusy = INF;
  for (ull i = tid; i < G; i += WG) {
    const ull* p = reinterpret_cast<const ull*>(&A->parts[i]);
    x += ld_agent(p + 0);
    mn = umin(mn, ld_agent(p + 1));
    e += ld_agent(p + 2);
    s += ld_agent(p + 3);
    f += ld_agent(p + 4);
    mn = umin(mn, ld_agent(p + 5));
    const ull bz = ld_agent(p + 6);
    busy += bz;
    negbusy = umin(negbusy, ~bz);
  }
  wg_reduce4(sh, x, e, s, mn);
  {
    ull z0 = 0;
    wg_reduce4(sh, f, busy, z0, negbusy);
  }
  if (tid < 16) {
    ull* z = reinterpret_cast<ull*>(&ctl->slot[(t + 2) % 3]);
    z[tid] = 0ull;
  }
  if (tid == 0) {
    S->x_total = x;
    S->fresh_total = f;
    S->min_next = mn;
    S->edges = e;
    S->successes = s;
    ctl->st_steps += 1;
    ctl->st_extracted += x;
    ctl->st_edges += e;
    ctl->st_success += s;
    ctl->st_dense += (flags & 1u) ? 1 : 0;
    ctl->st_sampled += (flags & 4u) ? 1 : 0;
    ctl->relax_busy_max += ~negbusy;
    ctl->relax_busy_sum += busy;
    if (A->trace && t < A->trace_cap) {
      sssp_step_record r;
      r.theta = theta;
      r.q = q;
      r.extracted = x;
      r.edges = e;
      r.successes = s;
      r.flags = flags;
      r.samples = (flags & 4u) ? (uint32_t)ld_agent(&S->nsamples) : 0u;
      A->trace[t] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// The persistent kernel.

__global__ __launch_bounds__(WG, 4) void stepping_kernel(const GPTR KArgs* __restrict__ A) {
  Shared& sh = g_sh;
  const GPTR KArgs& a = *A;
  const unsigned tid = threadIdx.x;
  const ull b = blockIdx.x;
  const ull G = a.G;
  const ull nthreads = G * WG;
  const ull gtid = b * WG + tid;
  const ull n = (ull)a.n;
  GPTR Control* ctl = a.ctl;
  Sync sy;
  sy.xcc = __builtin_amdgcn_s_getreg(20 | (15 << 11)) & (MAX_XCC - 1);  // hwreg XCC_ID
  GPTR int32_t* Fb = a.F + b * a.segcap;

  // Phase clock: workgroup 0 reads the wall clock as it leaves each barrier.
  ull ph0 = 0, ph1 = 0, ph2 = 0, ph3 = 0;
  long long tmark = wall_clock64();
  auto lap = [&]() {
    const long long now = wall_clock64();
    const ull d = (ull)(now - tmark);
    tmark = now;
    return d;
  };

  // S0: delta = inf, Q empty; then delta[s] = 0 and Update(s).
  if (tid == 0) atom_add(&ctl->grp_size[sy.xcc].v, 1ull);
  for (ull i = gtid; i < n; i += nthreads) a.dist[i] = INF;
  for (ull i = gtid; i < a.nwords; i += nthreads) a.bitmap[i] = 0;
  {
    auto seed_source = [&]() {
      if (tid == 0) {
        const int32_t s = a.inv ? a.inv[a.source] : a.source;
        a.dist[s] = 0;
        a.bitmap[s >> 6] = 1ull << (s & 63);
        a.L0[0] = s;
        ull g = 0;
        for (int x = 0; x < MAX_XCC; ++x) g += ctl->grp_size[x].v ? 1 : 0;
        ctl->ngroups = g;
      }
    };
    if (!flat_sync(a, sh, seed_source)) return;
    sy.gsz = ld_agent(&ctl->grp_size[sy.xcc].v);
    sy.ngroups = ld_agent(&ctl->ngroups);
    ph0 += lap();
  }

  ull q = 1, minq = 0, idelta = 0, dense_steps = 0;
  bool list_valid = true;

  for (ull t = 0;; ++t) {
    if (q == 0) break;
    if (a.max_steps && t >= a.max_steps) {
      if (b == 0 && tid == 0) ctl->status = ST_STEP_LIMIT;
      break;
    }
    GPTR StepSlot* S = &ctl->slot[t % 3];
    GPTR int32_t* Lcur = (t & 1) ? a.L1 : a.L0;
    GPTR int32_t* Lnext = (t & 1) ? a.L0 : a.L1;
    const bool dense = !list_valid;
    const bool emit = q <= a.list_threshold;

    // ---- S1: ExtDist ----
    ull theta = INF;
    bool sampled = false;
    if (a.rule == SSSP_RULE_BF) {
      theta = INF;
    } else if (a.rule == SSSP_RULE_MIN) {
      theta = minq;
    } else if (a.rule == SSSP_RULE_DELTA_STAR) {
      ull i = idelta + 1;
      const ull skip = minq / a.delta + (minq % a.delta != 0);  // ceil(min / Delta)
      if (skip > i) i = skip;
      idelta = i;
      ull prod;
      theta = __builtin_mul_overflow(i, (ull)a.delta, &prod) ? INF : prod;
    } else {
      const ull rho_eff = (dense && dense_steps < 2) ? ((a.rho / 10) > 0 ? a.rho / 10 : 1) : a.rho;
      if (q > rho_eff) {
        sampled = true;
        const ull probes = rho_probes(q, rho_eff, n, dense, a.sample_cap, a.probe_cap);
        phase_sample(A, S, Lcur, q, dense, probes, splitmix(a.seed, t));
        auto choose = [&]() {
          const ull s = ld_agent(&S->nsamples);
          ull th = INF;
          if (s > 0) {
            ull k = (rho_eff * s + q - 1) / q;  // ceil(rho * s / q)
            if (k < 1) k = 1;
            if (k > s) k = s;
            th = wg_select_kth(a.samples, s, k, sh);
          }
          if (tid == 0) ctl->theta = th;
        };
        if (!grid_sync(a, sh, sy, choose)) return;
        ph1 += lap();
        theta = ld_agent(&ctl->theta);
      }
    }

    // ---- S2: Extract(theta) over this workgroup's slice ----
    const ExtractOut ex = dense ? phase_extract_dense(A, S, Fb, Lnext, theta, emit)
                                : phase_extract_list(A, S, Fb, Lcur, Lnext, q, theta, emit);
    if (!grid_sync(a, sh, sy, NoSerial{})) return;
    ph2 += lap();

    // ---- S3/S4: Relax + Update ----
    phase_relax(A, S, Fb, Lnext, emit, ex);
    const unsigned flags = (dense ? 1u : 0u) | (emit ? 2u : 0u) | (sampled ? 4u : 0u);
    auto bookkeeping = [&]() { step_bookkeeping(A, S, t, q, theta, flags); };
    if (!grid_sync(a, sh, sy, bookkeeping)) return;
    ph3 += lap();

    // ---- S5: next queue state, identical in every workgroup ----
    q = q - ld_agent(&S->x_total) + ld_agent(&S->fresh_total);
    minq = ld_agent(&S->min_next);
    list_valid = emit;
    if (dense) ++dense_steps;
  }
  // Distances back in the caller's vertex ids.
  if (a.inv)
    for (ull v = gtid; v < n; v += nthreads) a.dist_out[v] = ld_agent(&a.dist[a.inv[v]]);
  if (b == 0 && tid == 0) {
    ctl->phase_ticks[0] = ph0;
    ctl->phase_ticks[1] = ph1;
    ctl->phase_ticks[2] = ph2;
    ctl->phase_ticks[3] = ph3;
  }
}

// Hub flags: bit v set iff out-degree(v) > hub_degree.
__global__ void hubmask_kernel(const int64_t* off, ull n, ull nwords, uint32_t hub_degree, ull* mask) {
  for (ull w = (ull)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += (ull)gridDim.x * blockDim.x) {
    ull m = 0;
    for (int i = 0; i < 64; ++i) {
      const ull v = w * 64 + i;
      if (v < n && (ull)(off[v + 1] - off[v]) > hub_degree) m |= 1ull << i;
    }
    mask[w] = m;
  }
}

__global__ void reset_control_kernel(Control* ctl) {
  ull* p = reinterpret_cast<ull*>(ctl);
  for (size_t i = threadIdx.x; i < sizeof(Control) / 8; i += blockDim.x) p[i] = 0;
}

}  // namespace

namespace {

sssp_tuning default_tuning() {
  sssp_tuning t;
  std::memset(&t, 0, sizeof(t));
  t.blocks_per_cu = 8;
  t.hub_degree = 1024;
  t.chunk_edges = 4096;
  t.list_divisor = 64;
  t.sample_cap = 4096;
  t.probe_cap = 1u << 16;
  t.no_filter = 0;
  return t;
}

sssp_tuning resolve_tuning(const sssp_tuning* in) {
  sssp_tuning d = default_tuning();
  if (!in) return d;
  sssp_tuning t = *in;
  if (!t.blocks_per_cu) t.blocks_per_cu = d.blocks_per_cu;
  if (!t.hub_degree) t.hub_degree = d.hub_degree;
  if (!t.chunk_edges) t.chunk_edges = d.chunk_edges;
  if (!t.list_divisor) t.list_divisor = d.list_divisor;
  if (!t.sample_cap) t.sample_cap = d.sample_cap;
  if (!t.probe_cap) t.probe_cap = d.probe_cap;
  return t;
}

// F segment size: a workgroup extracts at most the vertices of the blocks it
// owns (bitmap steps) or of its list slice (list steps, at most ceil(n / G)).
uint64_t segment_capacity(uint64_t nwords, uint32_t G) {
  const uint64_t nblocks = (nwords + BLOCK_WORDS - 1) / BLOCK_WORDS;
  return 64ull * BLOCK_WORDS * ((nblocks + G - 1) / G);
}

sssp_status ensure_workspace(sssp_graph* g, const sssp_tuning& tu, uint32_t G, hipStream_t st) {
  if (g->ws_ready && g->ws_hub_degree == tu.hub_degree && g->ws_chunk == tu.chunk_edges &&
      g->ws_probe_cap >= tu.probe_cap && g->ws_G == G)
    return SSSP_OK;
  g->release_ws();
  const uint64_t n = (uint64_t)g->n, m = (uint64_t)g->m;
  const uint64_t nwords = (n + 63) / 64;
  // H capacity: each vertex is extracted at most once per step, and an
  // extracted hub contributes ceil(deg / chunk) tasks, so
  // m / chunk + m / (hub_degree + 1) + 1 bounds the tasks of one step.
  const uint64_t hcap = m / tu.chunk_edges + m / ((uint64_t)tu.hub_degree + 1) + 2;
  if (g->relabelled) SSSP_HIP_TRY(g->dist_int.alloc(n * 8));
  SSSP_HIP_TRY(g->bitmap.alloc(nwords * 8));
  SSSP_HIP_TRY(g->hubmask.alloc(nwords * 8));
  SSSP_HIP_TRY(g->F.alloc((uint64_t)G * segment_capacity(nwords, G) * 4));
  SSSP_HIP_TRY(g->H.alloc(hcap * 8));
  SSSP_HIP_TRY(g->L0.alloc(n * 4));
  SSSP_HIP_TRY(g->L1.alloc(n * 4));
  SSSP_HIP_TRY(g->samples.alloc((uint64_t)tu.probe_cap * 8));
  SSSP_HIP_TRY(g->parts.alloc((uint64_t)G * sizeof(Part)));
  SSSP_HIP_TRY(g->ctl.alloc(sizeof(Control)));
  SSSP_HIP_TRY(g->args.alloc(sizeof(KArgs)));
  SSSP_HIP_TRY(hipHostMalloc(&g->hargs, sizeof(KArgs), hipHostMallocDefault));
  hubmask_kernel<<<1024, 256, 0, st>>>((const int64_t*)g->off.p, n, nwords, tu.hub_degree, (ull*)g->hubmask.p);
  SSSP_HIP_TRY(hipGetLastError());
  g->ws_ready = true;
  g->ws_hub_degree = tu.hub_degree;
  g->ws_chunk = tu.chunk_edges;
  g->ws_probe_cap = tu.probe_cap;
  g->ws_G = G;
  return SSSP_OK;
}

}  // namespace

extern "C" {

void sssp_default_params(sssp_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->rule = SSSP_RULE_RHO;
  p->rho = 1ull << 20;
  p->delta = 1ull << 13;
  p->seed = 1;
}

sssp_status sssp_solve(const sssp_graph* gc, const int32_t* sources, int32_t n_src, const sssp_params* params,
                       uint64_t* dist, void* stream, sssp_stats* stats) {
  last_error().clear();
  if (!gc) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (n_src < 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "n_src < 0");
  if (n_src > 0 && (!sources || !dist)) return fail(SSSP_ERR_INVALID_ARGUMENT, "sources or dist is NULL");
  sssp_params p;
  if (params) {
    p = *params;
  } else {
    sssp_default_params(&p);
  }
  if (p.rule > SSSP_RULE_MIN) return fail(SSSP_ERR_INVALID_ARGUMENT, "unknown rule");
  if (p.rule == SSSP_RULE_RHO && p.rho == 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "rho must be >= 1");
  if (p.rule == SSSP_RULE_DELTA_STAR && p.delta == 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "delta must be >= 1");
  if (p.trace && p.trace_capacity == 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "trace needs trace_capacity > 0");
  for (int32_t i = 0; i < n_src; ++i)
    if (sources[i] < 0 || sources[i] >= gc->n)
      return fail(SSSP_ERR_INVALID_ARGUMENT, "source " + std::to_string(sources[i]) + " out of range");
  sssp_tuning tu = resolve_tuning(p.tuning);
  if (tu.chunk_edges < 64) return fail(SSSP_ERR_INVALID_ARGUMENT, "chunk_edges must be >= 64");
  if (tu.hub_degree > (1u << 22)) return fail(SSSP_ERR_INVALID_ARGUMENT, "hub_degree must be <= 2^22");
  if (tu.sample_cap > tu.probe_cap) return fail(SSSP_ERR_INVALID_ARGUMENT, "sample_cap must be <= probe_cap");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n_src == 0) return SSSP_OK;

  sssp_graph* g = const_cast<sssp_graph*>(gc);
  SSSP_HIP_TRY(hipSetDevice(g->device));
  hipStream_t st = (hipStream_t)stream;
  int occ = 0;
  SSSP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stepping_kernel, WG, 0));
  if (occ < 1) return fail(SSSP_ERR_NO_DEVICE, "stepping kernel cannot be resident");
  const uint32_t bpc = std::min<uint32_t>(tu.blocks_per_cu, (uint32_t)occ);
  const uint32_t G = bpc * (uint32_t)g->cus;
  sssp_status ws = ensure_workspace(g, tu, G, st);
  if (ws != SSSP_OK) return ws;

  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.nwords = ((uint64_t)g->n + 63) / 64;
  a.off = (decltype(a.off))g->off.p;
  a.edges = (decltype(a.edges))g->edges.p;
  a.perm = (decltype(a.perm))(g->relabelled ? g->perm.p : nullptr);
  a.inv = (decltype(a.inv))(g->relabelled ? g->inv.p : nullptr);
  a.hubmask = (decltype(a.hubmask))g->hubmask.p;
  a.parts = (decltype(a.parts))g->parts.p;
  a.segcap = segment_capacity(a.nwords, G);
  a.bitmap = (decltype(a.bitmap))g->bitmap.p;
  a.F = (decltype(a.F))g->F.p;
  a.H = (decltype(a.H))g->H.p;
  a.L0 = (decltype(a.L0))g->L0.p;
  a.L1 = (decltype(a.L1))g->L1.p;
  a.samples = (decltype(a.samples))g->samples.p;
  a.ctl = (decltype(a.ctl))g->ctl.p;
  a.rho = p.rho;
  a.delta = p.delta ? p.delta : 1;
  a.seed = p.seed;
  a.max_steps = p.max_steps;
  a.list_threshold = tu.list_divisor == 0xFFFFFFFFu ? 0 : (uint64_t)g->n / tu.list_divisor;
  if (a.list_threshold < 1) a.list_threshold = 1;
  a.tlimit = g->tick_khz * 1000ull * 20ull;  // 20 s per barrier wait
  a.rule = p.rule;
  a.G = G;
  a.chunk_edges = tu.chunk_edges;
  a.sample_cap = tu.sample_cap;
  a.probe_cap = tu.probe_cap;
  a.filter = tu.no_filter ? 0u : 1u;
  if (tu.list_divisor == 0xFFFFFFFFu) a.list_threshold = 0;

  hipEvent_t ev0, ev1;
  SSSP_HIP_TRY(hipEventCreate(&ev0));
  SSSP_HIP_TRY(hipEventCreate(&ev1));
  sssp_status rc = SSSP_OK;
  std::string msg;
  Control hc;
  double ms_total = 0;
  for (int32_t i = 0; i < n_src && rc == SSSP_OK; ++i) {
    a.source = sources[i];
    a.dist_out = (decltype(a.dist_out))(dist + (size_t)i * (size_t)g->n);
    a.dist = g->relabelled ? (decltype(a.dist))g->dist_int.p : a.dist_out;
    a.xcount = (decltype(a.xcount))(p.extract_counts ? p.extract_counts + (size_t)i * (size_t)g->n : nullptr);
    a.trace = (decltype(a.trace))(i == 0 ? p.trace : nullptr);
    a.trace_cap = i == 0 ? p.trace_capacity : 0;
    reset_control_kernel<<<1, 256, 0, st>>>((Control*)g->ctl.p);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(ev0, st);
    if (e == hipSuccess) {
      std::memcpy(g->hargs, &a, sizeof(KArgs));
      e = hipMemcpyAsync(g->args.p, g->hargs, sizeof(KArgs), hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) {
      const KArgs* dargs = (const KArgs*)g->args.p;
      void* kargs[] = {(void*)&dargs};
      e = hipLaunchCooperativeKernel((const void*)stepping_kernel, dim3(G), dim3(WG), kargs, 0, st);
    }
    if (e == hipSuccess) e = hipEventRecord(ev1, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hc, g->ctl.p, sizeof(Control), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      rc = from_hip(e);
      msg = std::string("solve: ") + hipGetErrorString(e);
      break;
    }
    float ms = 0;
    if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) ms_total += ms;
    if (hc.abort_flag) {
      rc = SSSP_ERR_DEVICE;
      msg = "grid barrier timed out (workgroups not co-resident?)";
      break;
    }
    if (hc.status == ST_STEP_LIMIT) {
      rc = SSSP_ERR_STEP_LIMIT;
      msg = "max_steps reached with a non-empty queue";
    }
    if (stats) {
      stats->steps += hc.st_steps;
      stats->extracted += hc.st_extracted;
      stats->edges_relaxed += hc.st_edges;
      stats->writemin_success += hc.st_success;
      stats->dense_steps += hc.st_dense;
      stats->sampled_steps += hc.st_sampled;
      for (int k = 0; k < 4; ++k) stats->phase_ms[k] += (double)hc.phase_ticks[k] / (double)g->tick_khz;
      stats->relax_wg_ms[0] += (double)hc.relax_busy_max / (double)g->tick_khz;
      stats->relax_wg_ms[1] += (double)hc.relax_busy_sum / (double)G / (double)g->tick_khz;
    }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (stats) stats->device_ms = ms_total;
  if (rc != SSSP_OK) return fail(rc, msg);
  return SSSP_OK;
}

}  // extern "C"
