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
// Work distribution in Relax: extracted vertices of degree <= hub_degree are
// processed in tiles of 256 vertices, whose (begin, delta) pairs and degree
// prefix sums are staged in LDS; each lane maps an edge index to its vertex
// by binary search in LDS, so consecutive lanes read consecutive arcs
// (coalesced 8-byte (target, weight) loads). Larger vertices are cut into
// fixed-size edge chunks appended at Extract time. Tiles and chunks are
// claimed dynamically by workgroups.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sssp.h"

namespace {

constexpr int WG = 256;
constexpr int WAVES = WG / 64;
constexpr int UNROLL = 4;
constexpr uint64_t INF = ~0ull;

typedef unsigned long long ull;

// ---------------------------------------------------------------------------
// Device-side control block.

struct alignas(128) StepSlot {
  ull f_count;       // small-degree extracted vertices in F
  ull h_count;       // hub chunk tasks in H
  ull hub_vertices;  // hub vertices extracted
  ull list_next;     // entries written to the next explicit list
  ull new_members;   // vertices whose flag went 0 -> 1 in Relax
  ull min_next;      // min key over the next queue (kept members, new keys)
  ull work;          // Relax work-item counter
  ull edges;         // arcs relaxed
  ull successes;     // successful WriteMins
  ull nsamples;      // accepted threshold samples
  ull pad[6];
};

struct Control {
  alignas(128) ull bar_arrive;
  alignas(128) ull bar_gen;
  alignas(128) unsigned abort_flag;
  unsigned status;  // 0 ok, 1 step limit, 2 barrier timeout
  ull theta;
  ull st_steps, st_extracted, st_edges, st_success, st_dense, st_sampled;
  ull phase_ticks[4];  // init, threshold, extract, relax (workgroup 0's view)
  alignas(128) StepSlot slot[3];
};

constexpr unsigned ST_OK = 0, ST_STEP_LIMIT = 1, ST_TIMEOUT = 2;

struct KArgs {
  int64_t n;
  uint64_t nwords;
  const int64_t* off;
  const ull* edges;  // (weight << 32) | target
  ull* dist;
  ull* bitmap;
  int32_t* F;
  ull* H;  // (vertex << 32) | chunk index
  int32_t* L0;
  int32_t* L1;
  ull* samples;
  Control* ctl;
  uint32_t* xcount;
  sssp_step_record* trace;
  uint64_t trace_cap;
  uint64_t rho, delta, seed, max_steps;
  uint64_t list_threshold;
  uint64_t tlimit;
  int32_t source;
  uint32_t rule;
  uint32_t G;
  uint32_t hub_degree;
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
  ull red[WAVES * 4];
  ull item;
  ull bcast[4];
  int last;
  int abort;
};

// ---------------------------------------------------------------------------
// Small device helpers.

__device__ __forceinline__ ull ld_wg(const ull* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ ull ld_agent(const ull* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ ull atom_add(ull* p, ull v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ ull atom_min(ull* p, ull v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ ull atom_or(ull* p, ull v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ ull atom_and(ull* p, ull v) {
  return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Append `v` to list[*cnt ...] for every lane with pred set; one atomic per
// wave. Lanes that are inactive in divergent code simply do not take part.
__device__ __forceinline__ void wave_append_i32(int32_t* list, ull* cnt, bool pred, int32_t v) {
  const ull mask = __ballot(pred);
  if (mask == 0) return;
  const unsigned lane = lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  ull base = 0;
  if ((int)lane == leader) base = atom_add(cnt, (ull)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = v;
}

__device__ __forceinline__ void wave_append_u64(ull* list, ull* cnt, bool pred, ull v) {
  const ull mask = __ballot(pred);
  if (mask == 0) return;
  const unsigned lane = lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  ull base = 0;
  if ((int)lane == leader) base = atom_add(cnt, (ull)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = v;
}

__device__ __forceinline__ ull wave_sum(ull v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ ull wave_min(ull v) {
  for (int o = 32; o > 0; o >>= 1) {
    const ull w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ ull wave_max(ull v) {
  for (int o = 32; o > 0; o >>= 1) {
    const ull w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

// Workgroup reductions of up to four values (sum, sum, sum, min), result
// broadcast to all threads through sh.bcast.
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
  if (threadIdx.x == 0) {
    ull s0 = 0, s1 = 0, s2 = 0, m = INF;
    for (int w = 0; w < WAVES; ++w) {
      s0 += sh.red[w * 4 + 0];
      s1 += sh.red[w * 4 + 1];
      s2 += sh.red[w * 4 + 2];
      m = sh.red[w * 4 + 3] < m ? sh.red[w * 4 + 3] : m;
    }
    sh.bcast[0] = s0;
    sh.bcast[1] = s1;
    sh.bcast[2] = s2;
    sh.bcast[3] = m;
  }
  __syncthreads();
  a = sh.bcast[0];
  b = sh.bcast[1];
  c = sh.bcast[2];
  mn = sh.bcast[3];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Grid barrier. Every workgroup calls it the same number of times. The last
// workgroup to arrive runs `serial` (whole workgroup) before releasing the
// others, so a step's bookkeeping costs no extra barrier. Waiting is bounded:
// past `tlimit` wall-clock ticks the waiter raises the abort flag, and every
// workgroup leaves the kernel at its next barrier. Returns false on abort.
template <class Serial>
__device__ bool grid_sync(const KArgs& a, Shared& sh, ull& epoch, Serial serial) {
  Control* ctl = a.ctl;
  __syncthreads();
  ++epoch;
  if (threadIdx.x == 0) {
    const ull prev = __hip_atomic_fetch_add(&ctl->bar_arrive, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    sh.last = prev == epoch * (ull)a.G - 1ull;
    sh.abort = 0;
    if (sh.last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (sh.last) {
    serial();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&ctl->bar_gen, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  } else if (threadIdx.x == 0) {
    const long long t0 = wall_clock64();
    unsigned spins = 0;
    while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 63) == 0) {
        if (__hip_atomic_load(&ctl->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if ((ull)(wall_clock64() - t0) > a.tlimit) {
          __hip_atomic_store(&ctl->abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  if (threadIdx.x == 0)
    sh.abort = __hip_atomic_load(&ctl->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  return sh.abort == 0;
}

struct NoSerial {
  __device__ void operator()() const {}
};

// k-th smallest (1-based) of vals[0..s) by MSD radix selection over the bits
// below the highest bit where min and max differ. Whole workgroup.
__device__ ull wg_select_kth(const ull* vals, ull s, ull k, Shared& sh) {
  const unsigned tid = threadIdx.x;
  ull mn = INF, negmax = INF;  // max(x) = ~min(~x)
  for (ull i = tid; i < s; i += WG) {
    const ull v = vals[i];
    mn = v < mn ? v : mn;
    negmax = ~v < negmax ? ~v : negmax;
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
      const ull v = vals[i];
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
// Relax one arc (S3 + S4). `active` false lanes take part in the wave-level
// list append only.
struct RelaxAcc {
  ull edges = 0, succ = 0, fresh = 0, minv = INF;
};

__device__ __forceinline__ void relax_arc(const KArgs& a, RelaxAcc& acc, int32_t* Lnext, StepSlot* S, bool emit,
                                          bool active, int32_t v, ull nd) {
  bool add = false;
  if (active) {
    ++acc.edges;
    bool go = true;
    if (a.filter) go = nd < ld_wg(&a.dist[v]);
    if (go) {
      const ull old = atom_min(&a.dist[v], nd);
      if (nd < old) {
        ++acc.succ;
        acc.minv = nd < acc.minv ? nd : acc.minv;
        const ull bit = 1ull << (v & 63);
        const ull ow = atom_or(&a.bitmap[v >> 6], bit);
        if (!(ow & bit)) {
          ++acc.fresh;
          add = emit;
        }
      }
    }
  }
  if (emit) wave_append_i32(Lnext, &S->list_next, add, v);
}

// Classify and record an extracted vertex (S2 output).
struct ExtractAcc {
  ull hubs = 0, minkept = INF;
};

__device__ __forceinline__ void emit_extracted(const KArgs& a, ExtractAcc& acc, StepSlot* S, bool ext, int32_t v) {
  bool small = false;
  if (ext) {
    const int64_t b = a.off[v], e = a.off[v + 1];
    const ull deg = (ull)(e - b);
    if (deg > a.hub_degree) {
      const ull nch = (deg + a.chunk_edges - 1) / a.chunk_edges;
      const ull base = atom_add(&S->h_count, nch);
      for (ull c = 0; c < nch; ++c) a.H[base + c] = ((ull)(uint32_t)v << 32) | c;
      ++acc.hubs;
    } else {
      small = true;
    }
    if (a.xcount) a.xcount[v] += 1u;
  }
  wave_append_i32(a.F, &S->f_count, small, v);
}

// ---------------------------------------------------------------------------
// The persistent kernel.

__global__ __launch_bounds__(WG) void stepping_kernel(KArgs a) {
  __shared__ Shared sh;
  const unsigned tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const ull nthreads = (ull)a.G * WG;
  const ull gtid = (ull)blockIdx.x * WG + tid;
  const ull total_waves = (ull)a.G * WAVES;
  const ull gwave = (ull)blockIdx.x * WAVES + wave;
  const ull n = (ull)a.n;
  Control* ctl = a.ctl;
  ull epoch = 0;
  // Phase clock: workgroup 0 reads the wall clock as it leaves each barrier.
  ull ph[4] = {0, 0, 0, 0};
  long long tmark = wall_clock64();
  auto phase_end = [&](int k) {
    const long long now = wall_clock64();
    ph[k] += (ull)(now - tmark);
    tmark = now;
  };

  // S0: delta = inf, Q empty; then delta[s] = 0 and Update(s).
  for (ull i = gtid; i < n; i += nthreads) a.dist[i] = INF;
  for (ull i = gtid; i < a.nwords; i += nthreads) a.bitmap[i] = 0;
  {
    auto seed_source = [&]() {
      if (threadIdx.x < 3) ctl->slot[threadIdx.x].min_next = INF;
      if (threadIdx.x == 0) {
        a.dist[a.source] = 0;
        a.bitmap[a.source >> 6] = 1ull << (a.source & 63);
        a.L0[0] = a.source;
      }
    };
    if (!grid_sync(a, sh, epoch, seed_source)) return;
    phase_end(0);
  }

  ull q = 1, minq = 0, idelta = 0, dense_steps = 0;
  bool list_valid = true;

  for (ull t = 0;; ++t) {
    if (q == 0) break;
    if (a.max_steps && t >= a.max_steps) {
      if (blockIdx.x == 0 && tid == 0) ctl->status = ST_STEP_LIMIT;
      break;
    }
    StepSlot* S = &ctl->slot[t % 3];
    int32_t* Lcur = (t & 1) ? a.L1 : a.L0;
    int32_t* Lnext = (t & 1) ? a.L0 : a.L1;
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
      if (q <= rho_eff) {
        theta = INF;
      } else {
        sampled = true;
        const double lq = 1.0 + log2((double)q + 1.0);
        double st = ceil(10.0 * ((double)q / (double)rho_eff + lq));
        if (st > (double)a.sample_cap) st = (double)a.sample_cap;
        const ull s_target = (ull)st;
        ull probes = s_target;
        if (dense) {
          double p = ceil((double)s_target * (double)n / (double)q * 1.25);
          if (p > (double)a.probe_cap) p = (double)a.probe_cap;
          probes = (ull)p;
        }
        const ull tseed = splitmix(a.seed, t);
        for (ull base = (ull)blockIdx.x * WG; base < probes; base += nthreads) {
          const ull j = base + tid;
          bool acc = false;
          ull d = 0;
          if (j < probes) {
            const ull r = splitmix(tseed, j);
            if (dense) {
              const ull v = below(r, n);
              if ((ld_wg(&a.bitmap[v >> 6]) >> (v & 63)) & 1ull) {
                acc = true;
                d = ld_wg(&a.dist[v]);
              }
            } else {
              const int32_t v = Lcur[below(r, q)];
              acc = true;
              d = ld_wg(&a.dist[v]);
            }
          }
          wave_append_u64(a.samples, &S->nsamples, acc, d);
        }
        auto choose = [&]() {
          const ull s = ld_agent(&S->nsamples);
          ull th = INF;
          if (s > 0) {
            ull k = (rho_eff * s + q - 1) / q;  // ceil(rho * s / q)
            if (k < 1) k = 1;
            if (k > s) k = s;
            th = wg_select_kth(a.samples, s, k, sh);
          }
          if (threadIdx.x == 0) ctl->theta = th;
        };
        if (!grid_sync(a, sh, epoch, choose)) return;
        phase_end(1);
        theta = ld_agent(&ctl->theta);
      }
    }

    // ---- S2: Extract(theta) ----
    {
      ExtractAcc ex;
      if (dense) {
        for (ull w0 = gwave * UNROLL; w0 < a.nwords; w0 += total_waves * UNROLL) {
          ull word[UNROLL], d[UNROLL];
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) word[k] = (w0 + k < a.nwords) ? ld_wg(&a.bitmap[w0 + k]) : 0ull;
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) {
            const ull v = (w0 + k) * 64 + lane;
            d[k] = ((word[k] >> lane) & 1ull) ? ld_wg(&a.dist[v]) : INF;
          }
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) {
            const bool mem = (word[k] >> lane) & 1ull;
            const bool ext = mem && d[k] <= theta;
            const bool keep = mem && !ext;
            const ull em = __ballot(ext);
            if (em != 0 && lane == 0) a.bitmap[w0 + k] = word[k] & ~em;
            if (keep) ex.minkept = d[k] < ex.minkept ? d[k] : ex.minkept;
            const int32_t v = (int32_t)((w0 + k) * 64 + lane);
            if (emit) wave_append_i32(Lnext, &S->list_next, keep, v);
            emit_extracted(a, ex, S, ext, v);
          }
        }
      } else {
        for (ull base = (ull)blockIdx.x * WG * UNROLL; base < q; base += nthreads * UNROLL) {
          int32_t v[UNROLL];
          ull d[UNROLL];
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) {
            const ull i = base + (ull)k * WG + tid;
            v[k] = i < q ? Lcur[i] : -1;
          }
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) d[k] = v[k] >= 0 ? ld_wg(&a.dist[v[k]]) : INF;
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) {
            const bool mem = v[k] >= 0;
            const bool ext = mem && d[k] <= theta;
            const bool keep = mem && !ext;
            if (ext) atom_and(&a.bitmap[v[k] >> 6], ~(1ull << (v[k] & 63)));
            if (keep) ex.minkept = d[k] < ex.minkept ? d[k] : ex.minkept;
            if (emit) wave_append_i32(Lnext, &S->list_next, keep, v[k]);
            emit_extracted(a, ex, S, ext, v[k]);
          }
        }
      }
      ull hubs = ex.hubs, z0 = 0, z1 = 0, mk = ex.minkept;
      wg_reduce4(sh, hubs, z0, z1, mk);
      if (tid == 0) {
        if (hubs) atom_add(&S->hub_vertices, hubs);
        if (mk != INF) atom_min(&S->min_next, mk);
      }
    }
    if (!grid_sync(a, sh, epoch, NoSerial{})) return;
    phase_end(2);

    // ---- S3/S4: Relax + Update ----
    {
      const ull nF = ld_agent(&S->f_count);
      const ull nH = ld_agent(&S->h_count);
      const ull ntiles = (nF + WG - 1) / WG;
      const ull nitems = nH + ntiles;
      const ull CH = a.chunk_edges;
      RelaxAcc acc;
      for (;;) {
        if (tid == 0) sh.item = atom_add(&S->work, 1ull);
        __syncthreads();
        const ull item = sh.item;
        __syncthreads();
        if (item >= nitems) break;
        if (item < nH) {
          // One chunk of a hub vertex's arcs.
          const ull task = a.H[item];
          const int32_t u = (int32_t)(task >> 32);
          const ull c = task & 0xffffffffull;
          const ull rb = (ull)a.off[u], re = (ull)a.off[u + 1];
          const ull beg = rb + c * CH;
          const ull end = (beg + CH < re) ? beg + CH : re;
          const ull du = ld_wg(&a.dist[u]);
          for (ull e0 = beg; e0 < end; e0 += (ull)WG * UNROLL) {
            ull ev[UNROLL];
            bool act[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
              const ull e = e0 + (ull)k * WG + tid;
              act[k] = e < end;
              ev[k] = act[k] ? a.edges[e] : 0ull;
            }
#pragma unroll
            for (int k = 0; k < UNROLL; ++k)
              relax_arc(a, acc, Lnext, S, emit, act[k], (int32_t)(uint32_t)ev[k], du + (ev[k] >> 32));
          }
        } else {
          // A tile of up to WG small-degree vertices.
          const ull idx = (item - nH) * WG + tid;
          uint32_t deg = 0;
          ull b = 0, du = 0;
          if (idx < nF) {
            const int32_t u = a.F[idx];
            b = (ull)a.off[u];
            deg = (uint32_t)((ull)a.off[u + 1] - b);
            du = ld_wg(&a.dist[u]);
          }
          // Exclusive scan of degrees across the workgroup.
          uint32_t incl = deg;
          for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if ((int)lane >= o) incl += y;
          }
          if (lane == 63) sh.hist[wave] = incl;
          __syncthreads();
          uint32_t wbase = 0;
          for (unsigned w = 0; w < wave; ++w) wbase += sh.hist[w];
          uint32_t total = 0;
          for (int w = 0; w < WAVES; ++w) total += sh.hist[w];
          sh.pre[tid] = wbase + incl - deg;
          sh.beg[tid] = b;
          sh.du[tid] = du;
          __syncthreads();
          for (uint32_t e0 = 0; e0 < total; e0 += WG * UNROLL) {
            ull ev[UNROLL], dd[UNROLL];
            bool act[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
              const uint32_t e = e0 + k * WG + tid;
              act[k] = e < total;
              ev[k] = 0;
              dd[k] = 0;
              if (act[k]) {
                int lo = 0;
#pragma unroll
                for (int step = WG / 2; step > 0; step >>= 1)
                  if (sh.pre[lo + step] <= e) lo += step;
                ev[k] = a.edges[sh.beg[lo] + (e - sh.pre[lo])];
                dd[k] = sh.du[lo];
              }
            }
#pragma unroll
            for (int k = 0; k < UNROLL; ++k)
              relax_arc(a, acc, Lnext, S, emit, act[k], (int32_t)(uint32_t)ev[k], dd[k] + (ev[k] >> 32));
          }
          __syncthreads();
        }
      }
      ull e = acc.edges, s = acc.succ, f = acc.fresh, mn = acc.minv;
      wg_reduce4(sh, e, s, f, mn);
      if (tid == 0) {
        if (e) atom_add(&S->edges, e);
        if (s) atom_add(&S->successes, s);
        if (f) atom_add(&S->new_members, f);
        if (mn != INF) atom_min(&S->min_next, mn);
      }
    }

    auto bookkeeping = [&]() {
      if (threadIdx.x < 16) {
        ull* z = reinterpret_cast<ull*>(&ctl->slot[(t + 2) % 3]);
        z[threadIdx.x] = threadIdx.x == 5 ? INF : 0ull;  // field 5 is min_next
      }
      if (threadIdx.x == 0) {
        const ull X = ld_agent(&S->f_count) + ld_agent(&S->hub_vertices);
        const ull E = ld_agent(&S->edges), U = ld_agent(&S->successes);
        ctl->st_steps += 1;
        ctl->st_extracted += X;
        ctl->st_edges += E;
        ctl->st_success += U;
        ctl->st_dense += dense ? 1 : 0;
        ctl->st_sampled += sampled ? 1 : 0;
        if (a.trace && t < a.trace_cap) {
          sssp_step_record r;
          r.theta = theta;
          r.q = q;
          r.extracted = X;
          r.edges = E;
          r.successes = U;
          r.flags = (dense ? 1u : 0u) | (emit ? 2u : 0u) | (sampled ? 4u : 0u);
          r.samples = sampled ? (uint32_t)ld_agent(&S->nsamples) : 0u;
          a.trace[t] = r;
        }
      }
    };
    if (!grid_sync(a, sh, epoch, bookkeeping)) return;
    phase_end(3);

    // ---- S5: next queue state, identical in every workgroup ----
    const ull X = ld_agent(&S->f_count) + ld_agent(&S->hub_vertices);
    q = q - X + ld_agent(&S->new_members);
    minq = ld_agent(&S->min_next);
    list_valid = emit;
    if (dense) ++dense_steps;
  }
  if (blockIdx.x == 0 && tid == 0)
    for (int k = 0; k < 4; ++k) ctl->phase_ticks[k] = ph[k];
}

// Zero the control block before a solve (a kernel rather than a memset, so
// the sequence stays valid under stream capture).
__global__ void reset_control_kernel(Control* ctl) {
  ull* p = reinterpret_cast<ull*>(ctl);
  for (size_t i = threadIdx.x; i < sizeof(Control) / 8; i += blockDim.x) p[i] = 0;
}

// Pack (target, weight) pairs into one 8-byte word per arc.
__global__ void pack_edges_kernel(const int32_t* tgt, const uint32_t* w, ull* out, ull m) {
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (ull)gridDim.x * blockDim.x)
    out[i] = ((ull)w[i] << 32) | (uint32_t)tgt[i];
}

// Widen int32 offsets to int64.
__global__ void widen_offsets_kernel(const int32_t* in, int64_t* out, ull count) {
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (ull)gridDim.x * blockDim.x)
    out[i] = in[i];
}

__global__ void reset_flags_kernel(unsigned* err, ull* where) {
  *err = 0;
  *where = INF;
}

// CSR validation on the device. Sets bits in *err: 1 offsets[0] != 0,
// 2 offsets decrease, 4 offsets[n] != m, 8 target out of range; and the
// smallest offending index in *where (atomic min).
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

// ---------------------------------------------------------------------------
// Host side.

thread_local std::string g_last_error;

sssp_status fail(sssp_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? SSSP_ERR_OUT_OF_MEMORY : SSSP_ERR_DEVICE,        \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                          \
    }                                                                                          \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t alloc(size_t b) {
    bytes = b;
    return hipMalloc(&p, b ? b : 8);
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

}  // namespace

struct sssp_graph {
  int device = 0;
  int64_t n = 0, m = 0;
  int cus = 0;
  uint64_t tick_khz = 100000;
  DevBuf off, edges;
  // Workspace, sized for n and m, allocated on first solve.
  bool ws_ready = false;
  uint32_t ws_hub_degree = 0, ws_chunk = 0, ws_probe_cap = 0;
  DevBuf bitmap, F, H, L0, L1, samples, ctl, trace_dummy;
  uint64_t workspace_bytes() const {
    return bitmap.bytes + F.bytes + H.bytes + L0.bytes + L1.bytes + samples.bytes + ctl.bytes;
  }
  void release_ws() {
    bitmap.release();
    F.release();
    H.release();
    L0.release();
    L1.release();
    samples.release();
    ctl.release();
    ws_ready = false;
  }
};

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

sssp_status ensure_workspace(sssp_graph* g, const sssp_tuning& tu) {
  // H capacity: every extracted hub vertex contributes ceil(deg / chunk)
  // tasks and each vertex is extracted at most once per step, so
  // m / chunk + n / (hub_degree + 1) + 1 bounds the tasks of one step.
  if (g->ws_ready && g->ws_hub_degree == tu.hub_degree && g->ws_chunk == tu.chunk_edges &&
      g->ws_probe_cap >= tu.probe_cap)
    return SSSP_OK;
  g->release_ws();
  const uint64_t n = (uint64_t)g->n, m = (uint64_t)g->m;
  const uint64_t nwords = (n + 63) / 64;
  const uint64_t hcap = m / tu.chunk_edges + m / ((uint64_t)tu.hub_degree + 1) + 2;
  HIP_TRY(g->bitmap.alloc(nwords * 8));
  HIP_TRY(g->F.alloc(n * 4));
  HIP_TRY(g->H.alloc(hcap * 8));
  HIP_TRY(g->L0.alloc(n * 4));
  HIP_TRY(g->L1.alloc(n * 4));
  HIP_TRY(g->samples.alloc((uint64_t)tu.probe_cap * 8));
  HIP_TRY(g->ctl.alloc(sizeof(Control)));
  g->ws_ready = true;
  g->ws_hub_degree = tu.hub_degree;
  g->ws_chunk = tu.chunk_edges;
  g->ws_probe_cap = tu.probe_cap;
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
  }
  return "unknown status";
}

const char* sssp_last_error(void) { return g_last_error.c_str(); }

sssp_status sssp_graph_destroy(sssp_graph* g) {
  if (!g) return SSSP_OK;
  (void)hipSetDevice(g->device);
  g->off.release();
  g->edges.release();
  g->release_ws();
  delete g;
  return SSSP_OK;
}

sssp_status sssp_graph_info(const sssp_graph* g, int64_t* n, int64_t* m, uint64_t* device_bytes) {
  if (!g) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (device_bytes) *device_bytes = g->off.bytes + g->edges.bytes + g->workspace_bytes();
  return SSSP_OK;
}

sssp_status sssp_graph_create(int64_t n, int64_t m, sssp_offset_width ow, const void* offsets,
                              const int32_t* targets, const uint32_t* weights, uint32_t flags, void* stream,
                              sssp_graph** out) {
  g_last_error.clear();
  if (!out) return fail(SSSP_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (n < 1 || n >= ((int64_t)1 << 31)) return fail(SSSP_ERR_INVALID_ARGUMENT, "n must satisfy 1 <= n < 2^31");
  if (m < 0 || m >= ((int64_t)1 << 40)) return fail(SSSP_ERR_INVALID_ARGUMENT, "m must satisfy 0 <= m < 2^40");
  if (ow != SSSP_OFFSETS_I32 && ow != SSSP_OFFSETS_I64) return fail(SSSP_ERR_INVALID_ARGUMENT, "bad offset width");
  if (ow == SSSP_OFFSETS_I32 && m >= ((int64_t)1 << 31))
    return fail(SSSP_ERR_INVALID_ARGUMENT, "int32 offsets need m < 2^31");
  const bool host = (flags & SSSP_INPUT_HOST) != 0, device = (flags & SSSP_INPUT_DEVICE) != 0;
  if (host == device) return fail(SSSP_ERR_INVALID_ARGUMENT, "exactly one of SSSP_INPUT_HOST/DEVICE");
  if (flags & ~(SSSP_INPUT_HOST | SSSP_INPUT_DEVICE | SSSP_TRUST_INPUT))
    return fail(SSSP_ERR_INVALID_ARGUMENT, "unknown flag bits");
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

  int dev = 0;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(SSSP_ERR_NO_DEVICE, "no HIP device");
  HIP_TRY(hipGetDevice(&dev));
  int coop = 0;
  HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
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

  auto cleanup = [&](sssp_status s) {
    sssp_graph_destroy(g);
    return s;
  };
  hipError_t e;
  if ((e = g->off.alloc((size_t)(n + 1) * 8)) != hipSuccess) {
    cleanup(SSSP_OK);
    return fail(SSSP_ERR_OUT_OF_MEMORY, std::string("offsets: ") + hipGetErrorString(e));
  }
  if ((e = g->edges.alloc((size_t)m * 8)) != hipSuccess) {
    cleanup(SSSP_OK);
    return fail(SSSP_ERR_OUT_OF_MEMORY, std::string("edges: ") + hipGetErrorString(e));
  }
  // Stage the caller's arrays on the device, then pack.
  DevBuf t32, w32, o32;
  const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  sssp_status rs = SSSP_OK;
  std::string msg;
  do {
    if (ow == SSSP_OFFSETS_I64) {
      if ((e = hipMemcpyAsync(g->off.p, offsets, (size_t)(n + 1) * 8, kind, st)) != hipSuccess) break;
    } else {
      if ((e = o32.alloc((size_t)(n + 1) * 4)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(o32.p, offsets, (size_t)(n + 1) * 4, kind, st)) != hipSuccess) break;
      widen_offsets_kernel<<<1024, 256, 0, st>>>((const int32_t*)o32.p, (int64_t*)g->off.p, (ull)(n + 1));
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    const int32_t* tsrc = targets;
    const uint32_t* wsrc = weights;
    if (m > 0 && host) {
      if ((e = t32.alloc((size_t)m * 4)) != hipSuccess) break;
      if ((e = w32.alloc((size_t)m * 4)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(t32.p, targets, (size_t)m * 4, hipMemcpyHostToDevice, st)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(w32.p, weights, (size_t)m * 4, hipMemcpyHostToDevice, st)) != hipSuccess) break;
      tsrc = (const int32_t*)t32.p;
      wsrc = (const uint32_t*)w32.p;
    }
    if (device && !trust) {
      DevBuf flag;
      if ((e = flag.alloc(16)) != hipSuccess) break;
      reset_flags_kernel<<<1, 1, 0, st>>>((unsigned*)flag.p, (ull*)flag.p + 1);
      validate_kernel<<<1024, 256, 0, st>>>((const int64_t*)g->off.p, tsrc, (ull)n, (ull)m, (unsigned*)flag.p,
                                            (ull*)flag.p + 1);
      ull back[2] = {0, INF};
      if ((e = hipGetLastError()) == hipSuccess &&
          (e = hipMemcpyAsync(back, flag.p, 16, hipMemcpyDeviceToHost, st)) == hipSuccess)
        e = hipStreamSynchronize(st);
      flag.release();
      if (e != hipSuccess) break;
      const unsigned herr = (unsigned)back[0];
      if (herr) {
        rs = SSSP_ERR_INVALID_GRAPH;
        msg = "device CSR validation failed (code " + std::to_string(herr) + ", index " +
              std::to_string(back[1] == INF ? -1LL : (long long)back[1]) + ")";
        break;
      }
    }
    if (m > 0) {
      pack_edges_kernel<<<2048, 256, 0, st>>>(tsrc, wsrc, (ull*)g->edges.p, (ull)m);
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    e = hipStreamSynchronize(st);
  } while (false);
  t32.release();
  w32.release();
  o32.release();
  if (e != hipSuccess) {
    cleanup(SSSP_OK);
    return fail(e == hipErrorOutOfMemory ? SSSP_ERR_OUT_OF_MEMORY : SSSP_ERR_DEVICE,
                std::string("graph upload: ") + hipGetErrorString(e));
  }
  if (rs != SSSP_OK) {
    cleanup(SSSP_OK);
    return fail(rs, msg);
  }
  *out = g;
  return SSSP_OK;
}

sssp_status sssp_solve(const sssp_graph* gc, const int32_t* sources, int32_t n_src, const sssp_params* params,
                       uint64_t* dist, void* stream, sssp_stats* stats) {
  g_last_error.clear();
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
  HIP_TRY(hipSetDevice(g->device));
  sssp_status ws = ensure_workspace(g, tu);
  if (ws != SSSP_OK) return ws;
  hipStream_t st = (hipStream_t)stream;

  int occ = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stepping_kernel, WG, 0));
  if (occ < 1) return fail(SSSP_ERR_NO_DEVICE, "stepping kernel cannot be resident");
  const uint32_t bpc = std::min<uint32_t>(tu.blocks_per_cu, (uint32_t)occ);
  const uint32_t G = bpc * (uint32_t)g->cus;

  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.nwords = ((uint64_t)g->n + 63) / 64;
  a.off = (const int64_t*)g->off.p;
  a.edges = (const ull*)g->edges.p;
  a.bitmap = (ull*)g->bitmap.p;
  a.F = (int32_t*)g->F.p;
  a.H = (ull*)g->H.p;
  a.L0 = (int32_t*)g->L0.p;
  a.L1 = (int32_t*)g->L1.p;
  a.samples = (ull*)g->samples.p;
  a.ctl = (Control*)g->ctl.p;
  a.rho = p.rho;
  a.delta = p.delta ? p.delta : 1;
  a.seed = p.seed;
  a.max_steps = p.max_steps;
  a.list_threshold = tu.list_divisor == 0xFFFFFFFFu ? 0 : (uint64_t)g->n / tu.list_divisor;
  if (a.list_threshold < 1) a.list_threshold = 1;
  a.tlimit = g->tick_khz * 1000ull * 20ull;  // 20 s per barrier wait
  a.rule = p.rule;
  a.G = G;
  a.hub_degree = tu.hub_degree;
  a.chunk_edges = tu.chunk_edges;
  a.sample_cap = tu.sample_cap;
  a.probe_cap = tu.probe_cap;
  a.filter = tu.no_filter ? 0u : 1u;
  if (tu.list_divisor == 0xFFFFFFFFu) a.list_threshold = 0;

  hipEvent_t ev0, ev1;
  HIP_TRY(hipEventCreate(&ev0));
  HIP_TRY(hipEventCreate(&ev1));
  sssp_status rc = SSSP_OK;
  std::string msg;
  Control hc;
  double ms_total = 0;
  for (int32_t i = 0; i < n_src && rc == SSSP_OK; ++i) {
    a.source = sources[i];
    a.dist = (ull*)(dist + (size_t)i * (size_t)g->n);
    a.xcount = p.extract_counts ? p.extract_counts + (size_t)i * (size_t)g->n : nullptr;
    a.trace = i == 0 ? p.trace : nullptr;
    a.trace_cap = i == 0 ? p.trace_capacity : 0;
    reset_control_kernel<<<1, 256, 0, st>>>(a.ctl);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(ev0, st);
    if (e == hipSuccess) {
      void* kargs[] = {&a};
      e = hipLaunchCooperativeKernel((const void*)stepping_kernel, dim3(G), dim3(WG), kargs, 0, st);
    }
    if (e == hipSuccess) e = hipEventRecord(ev1, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hc, a.ctl, sizeof(Control), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      rc = e == hipErrorOutOfMemory ? SSSP_ERR_OUT_OF_MEMORY : SSSP_ERR_DEVICE;
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
    }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (stats) stats->device_ms = ms_total;
  if (rc != SSSP_OK) return fail(rc, msg);
  return SSSP_OK;
}

}  // extern "C"
