// Persistent stepping-loop kernel for single-source shortest paths on
// MI355X (gfx950), and the solve and serving entry points of the C ABI
// (include/sssp.h).
//
// One persistent launch (cooperative for sssp_solve) runs Alg. 1 (Sec. 3.2)
// for every requested source:
//
//   S0 init      delta[.] = inf, bitmap = 0; delta[s] = 0, Update(s).
//   S1 ExtDist   theta per Table 2: rho-th smallest by sampling (Sec. 6,
//                App. B) or by an exact radix selection, i * Delta (Delta*),
//                +inf (Bellman-Ford), min (test).
//   S2 Extract   F = {v in Q : delta[v] <= theta}; their queue flags cleared
//                (Table 1). Q is a bitmap (the flat-array LaB-PQ of Sec. 4.3)
//                plus, while |Q| is small, an explicit list (Sec. 6, sparse
//                mode), so small steps do not scan all n flags.
//   S3 Relax     for u in F, v in N(u): WriteMin(delta[v], delta[u] + w) as a
//                64-bit atomic min (Sec. 2 WriteMin), skipped when a 16-bit
//                coded upper bound of delta[v] (hint[v]) already shows no
//                improvement. delta[u] is read when u's arcs are relaxed,
//                so a u whose key another WriteMin of the same step has
//                lowered already propagates the lower key.
//                With SSSP_SOLVE_SNAPSHOT_KEYS, delta[u] is instead the key u
//                was extracted with (kept beside u in F): what a step extracts
//                and which vertices it improves then do not depend on the order
//                in which concurrent WriteMins land, so for a fixed theta
//                sequence the run repeats exactly.
//   S4 Update    a successful WriteMin sets v's flag with an atomic OR; the old
//                word tells whether v is new to Q, so the explicit list gets
//                each new member once, with no hash table or pack pass.
//   S5 loop      until |Q| = 0. Phases are separated by barriers, so Extract
//                never overlaps Update (Sec. 3.1).
//
// Sec. 6's road-graph optimisations sit inside S3: local expansion (a
// workgroup relaxes the vertices its WriteMins bring under theta itself, hop
// after hop, in super-sparse steps) and bidirectional relaxation (pull the
// best key from the neighbours before pushing; symmetric graphs only).
//
// Teams. The grid is split into `nteams` teams; team t is the workgroups b
// with b % nteams == t. Each team repeatedly takes the next unsolved source
// and runs the loop above on it with its own queue state, so many small
// queries proceed side by side in one launch (batched solves), while
// nteams = 1 gives one whole-grid solve at a time. With nteams a multiple of
// eight, every team sits on one XCD (workgroups are dealt to the eight XCDs
// round-robin; the kernel checks this against the XCC_ID hardware register).
//
// Work distribution inside a team. Each workgroup owns a slice of the queue:
// interleaved blocks of bitmap words (bitmap steps) or a contiguous slice of
// the explicit list (list steps). What it extracts goes to its own segment
// of F, so Extract needs no shared counter; in Relax it processes its own
// segment in tiles of 256 vertices whose (row begin, delta) pairs and degree
// prefix sums sit in LDS, so consecutive lanes read consecutive 8-byte
// (target, weight) arcs. Vertices above hub_degree are cut into fixed-size
// edge chunks shared by the team. Counters are per-workgroup partials, summed
// by the last workgroup to reach the step's final barrier.
//
// Barriers and memory visibility across XCDs (each has its own L2). A
// whole-grid team meets in two levels: the workgroups of one XCD (grouped by
// XCC_ID) first; the last of them writes back that XCD's L2 (agent-scope
// release) and arrives at the global counter; after the global release each
// XCD leader invalidates (agent-scope acquire) and releases its group. A team
// inside one XCD meets on a single counter whose last arriver does the same.
// Data other workgroups wrote in earlier phases is read with agent-scope
// loads, which bypass the per-CU L1. Every wait is bounded.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "hint_code.h"
#include "internal.h"

using namespace sssp_impl;

namespace {

constexpr int WG = 256;
constexpr int WAVES = WG / 64;
constexpr int UNROLL = 4;       // arcs / list entries per lane per iteration
constexpr int BATCH = 4;        // queue members per lane per round in bitmap scans
constexpr int MAX_XCC = 16;
constexpr int BLOCK_WORDS = 4;  // bitmap words per ownership block (256 vertices)
// The word-per-wave Extract gives wave w word w of each block it owns.
static_assert(BLOCK_WORDS == WAVES, "one wave per bitmap word of a block");
constexpr int LQ = 1024;        // local-expansion list capacity per round (LDS)
constexpr int PEND = 1024;      // Relax's appends to the next explicit list, staged in LDS
constexpr int ROW_SHIFT = 40;   // packed row: (degree << ROW_SHIFT) | row start
constexpr ull ROW_START = (1ull << ROW_SHIFT) - 1;

// ---------------------------------------------------------------------------
// Control blocks.

struct alignas(128) StepSlot {
  ull h_count;      // hub chunk tasks in H
  ull list_next;    // entries reserved in the next explicit list
  ull nsamples;     // accepted threshold samples
  ull x_total;      // vertices extracted (sum of partials)
  ull fresh_total;  // vertices whose flag went 0 -> 1 in Relax
  ull min_next;     // min key over the next queue
  ull edges;        // arcs relaxed
  ull successes;    // successful WriteMins
  ull local_v;      // vertices relaxed by local expansion
  ull pad[7];
};

struct alignas(128) Line {
  ull v;
  ull pad[15];
};

// Per-team state.
struct TeamCtl {
  Line arrive;  // team barrier (teams inside one XCD)
  Line gen;
  alignas(128) ull theta;
  ull theta_h;  // deferred hubs' threshold of the step (rho rule with hub deferral)
  ull query;   // index of the source being solved
  ull status;  // 1: step limit reached on some query
  ull st_steps, st_extracted, st_edges, st_success, st_dense, st_sampled;
  ull st_qdense, st_qlist, st_appends, st_local, st_skipped;
  ull relax_busy_max, relax_busy_sum;
  ull phase_ticks[4];  // init, threshold, extract, relax (the team's first workgroup)
  // Serving: the current request and the one still to be published.
  ull src, out_row;
  ull hash_acc;  // row checksum, summed over the team's workgroups
  // Exact rho-th selection: key bounds, the digit histogram of the current
  // pass, and the selection state (prefix, remaining rank, bits left).
  ull sel_min, sel_max, sel_prefix, sel_k, sel_top;
  ull sel_hist[256];
  ull pending;   // ticket + 1 of a finished request not yet published (0: none)
  // Serving groups. A request is solved by a group of k teams: the group
  // uses its leader's workspace and this block of the leader's, meets on the
  // leader's group barrier (garrive / ggen; counts only grow, so a group
  // starts from the count it finds) and lists its member teams in gteam.
  // The mailbox (mb_*) is this team's assignment, written by whichever team
  // dispatched it; mb_seq grows by one per assignment.
  ull mb_seq, mb_leader, mb_k, mb_idx, mb_base, mb_exit;
  uint32_t gteam[64];
  Line garrive;
  Line ggen;
  alignas(128) StepSlot slot[3];
};

// Whole-grid state.
struct GridCtl {
  Line arrive_flat;  // the first barrier
  Line gen_flat;
  Line arrive;  // global level of the whole-grid barrier
  Line gen;
  Line grp_arrive[MAX_XCC];
  Line grp_gen[MAX_XCC];
  Line grp_size[MAX_XCC];
  Line next_query;
  Line mismatch;  // some workgroup is not on the XCD its index implies
  alignas(128) unsigned abort_flag;
  unsigned cancelled;  // some team saw the host's cancel flag: teams claim no more sources
  ull ngroups;
  // Serving: the dispatcher's lock, the idle teams (bit t = team t) and the
  // closing word (set when a team's idle limit passes: no more assignments).
  alignas(128) unsigned lock;
  ull free_mask;
  ull closing;
};

constexpr unsigned ST_STEP_LIMIT = 1;
constexpr unsigned ST_CANCELLED = 2;

// Per-workgroup partial counts of one step.
struct alignas(64) Part {
  ull x;        // vertices extracted
  ull minkept;  // min key of members left in Q
  ull edges;    // arcs relaxed
  ull succ;     // successful WriteMins
  ull fresh;    // new queue members
  ull minnew;   // min successful WriteMin value
  ull busy;     // wall-clock ticks this workgroup spent in Relax
  ull local;    // vertices relaxed by local expansion
  ull skipped;  // arcs not pushed again: their tail's key had not changed since its last push
};

struct KArgs {
  int64_t n;
  uint64_t m;
  uint64_t nwords;
  const int64_t* off;
  const ull* edges;     // (weight << 32) | target; NULL when the caller's arrays are borrowed:
  const int32_t* tgt;   // borrowed targets and weights (graphs created with SSSP_BORROW_DEVICE)
  const uint32_t* wt;
  const ull* hubmask;   // bit v set iff deg(v) > hub_degree
  const ull* bigmask;   // bit v set iff deg(v) > the local-expansion degree cap
  const int32_t* perm;  // internal id -> caller id (NULL: identity)
  const int32_t* inv;   // caller id -> internal id (NULL: identity)
  const int32_t* srcs;  // n_src sources, caller ids
  ull* dist_out;        // caller's rows, n_src x n, caller ids
  ull* dist_int;        // per-team internal rows (relabelled graphs), else NULL
  ull* bitmap;          // per team, nwords
  uint16_t* hint;       // per team, n: upper bound of each key for the Relax filter (NULL: no filter)
  ull* lastkey;         // per team, n: the key a vertex's arcs were last pushed with (NULL: off)
  ull* ckey;            // per team, hcap: the same per hub chunk (NULL: off)
  const uint32_t* cbase;  // hub u < nhub: index of u's first chunk in ckey (hubs are numbered first)
  uint64_t nhub;
  const ull* trow;      // per arc: (degree << ROW_SHIFT) | row start of its target, for local
                        // expansion (NULL: the next round reads the offsets)
  uint32_t local_cap;   // out-degree above which a vertex is not relaxed by local expansion
  uint64_t ndefer;      // sampled rho steps: vertices below this id (the highest degrees, numbered
                        // first) are extracted only at keys <= theta_h (0: no deferral)
  uint64_t defer_div;   // theta_h is the sampled (rho / defer_div)-th smallest key
  ull* key1;            // tournament-tree queue (NULL: flat array): per team, nwords (one node per bitmap word)
  ull* key2;            // per team, n2 (one node per 64 words)
  uint64_t n2;
  int32_t* F;           // per workgroup, segcap: extracted vertices
  ull* FD;              // per workgroup, segcap: their keys when extracted
  ull* H;               // per team, hcap pairs: ((vertex << 32) | chunk index, key)
  int32_t* L;           // per team, 2 x lcap
  ull* samples;         // per team, probe_cap
  Part* parts;          // per workgroup
  TeamCtl* teams;
  GridCtl* grid;
  uint32_t* xcount;  // n_src x n (caller ids) or NULL
  sssp_step_record* trace;
  uint64_t trace_cap;
  uint64_t rho, delta, seed, max_steps;
  uint64_t list_threshold;
  uint64_t tlimit;
  uint64_t segcap, hcap, lcap;
  int64_t n_src;
  uint32_t rule;
  uint32_t G;       // workgroups in the grid
  uint32_t nteams;  // teams; team size T = G / nteams
  uint32_t chunk_edges;
  uint32_t sample_cap;
  uint32_t probe_cap;
  uint32_t filter;
  uint32_t snapshot;  // relax with the keys at extraction
  uint32_t local_budget;  // vertices a workgroup may relax by local expansion per step (0: off)
  uint32_t ns_per_tick;   // wall-clock counter period
  uint32_t pull;          // bidirectional relaxation (undirected graphs)
  uint32_t super_sparse;  // local expansion in list steps below this average out-degree
  uint64_t sparse_q;      // tournament-tree queue: steps with |Q| at most this count as list steps for local expansion
  // Serving mode: requests come from a ring in host memory instead of srcs.
  uint32_t serve;
  uint32_t hash;               // add each finished row's checksum to its ring entry
  const int32_t* req;          // host: ring_cap x (source, row); ticket t uses entry t % ring_cap
  const uint64_t* posted;      // host: requests posted so far
  const uint32_t* closed;      // host: nonzero once no more requests will come
  uint64_t* ack;               // host: ring_cap entries, ticket + 1 once taken (entry free again)
  uint64_t* done;              // host: per row, ticket + 1 once its request finished
  uint64_t* hashes;            // host: per row, the finished row's checksum
  uint64_t ring_cap;
  uint64_t nrows;              // rows of dist_out
  uint64_t idle_ticks;         // longest wait for a request
  uint32_t* dev_closed;        // host: set to 1 once the launch takes no more requests (idle limit)
  uint32_t group_max;          // serving: most teams that solve one request together (a power of two)
  uint32_t group_min;          // serving: fewest teams a request is dispatched to (a power of two <= group_max)
  const uint32_t* cancel;      // host: nonzero asks the solve to stop (asynchronous solves), or NULL
};

struct Shared {
  ull beg[WG];
  ull du[WG];
  ull pulled[WG];  // bidirectional relaxation: best key each tile vertex can take from its neighbours
  uint32_t pre[WG + 1];
  uint32_t hist[WG];
  uint32_t wsum[WAVES];
  ull red[WAVES * 4];
  ull bcast[4];
  // Local expansion: this round's vertices and the next round's, each with
  // its packed row (or INF: read the offsets).
  int32_t lq[2][LQ];
  ull lqr[2][LQ];
  int32_t uid[WG];  // the tile's vertices (their keys are read per arc in row mode)
  // Relax's new queue members for the next explicit list, written out once
  // per step (pend_flush) instead of with a workgroup reservation per batch.
  int32_t pend[PEND];
  uint32_t npend;
  uint32_t lqn[2];
  uint32_t fcnt;  // F entries reserved by this workgroup in a bitmap step
  ull hub_task, hub_du;  // the hub chunk in hand and the key it is pushed with
  int hub_skip;
  int last;
  int abort;
};

__shared__ Shared g_sh;

// Everything a workgroup needs to know about its team, in registers.
struct Team {
  ull id, rank, T;  // team index, rank in the team, team size
  TeamCtl* ctl;
  ull* bitmap;
  uint16_t* hint;
  ull* lastkey;  // repeated-push skip (NULL: off)
  ull* ckey;
  ull* key1;  // tournament tree (NULL: flat array)
  ull* key2;
  ull* H;
  int32_t* L;
  ull* samples;
  int32_t* Fb;  // this workgroup's F segment: vertices
  ull* FDb;     // and their keys at extraction
  ull k, Tteam;  // teams working on the current source and workgroups per team (T = k * Tteam)
  ull own;       // this workgroup's own team (serving groups: tm.id is the group's leader)
};

// A workgroup's barrier state, the only team state the kernel keeps in
// registers across its phases (the rest is read from the LDS copy g_tm).
struct Bar {
  ull epoch;      // first-level barriers passed
  ull l2_epoch;   // second-level barriers passed since l2_base was taken
  ull l2_base;    // second-level arrival count when the current group formed
  ull* l1_arrive;
  ull* l1_gen;
  ull l1_size;
  ull* l2_arrive;  // NULL: single-level barrier
  ull* l2_gen;
  ull l2_size;
  bool member_release;  // every member releases at agent scope
};

// LDS copy of the workgroup's Team for the out-of-line phase functions (a
// reference to a kernel local would place it in scratch memory).
__shared__ Team g_tm;

// ---------------------------------------------------------------------------
// Small device helpers.

// Global-address-space view of a device pointer. Loads, stores and atomics
// through it compile to global_* instructions, which count only against the
// vector-memory counter; flat_* instructions (what a generic pointer gives)
// count against the LDS counter too, so every wait for an LDS read would also
// wait for every gather in flight. For device buffers only, never LDS.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> glob(T* p) {
  return (gptr<T>)p;
}

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
// Streaming load for the arc array: each arc is read once per relaxation
// pass, so it is marked non-temporal and does not push the keys of
// frequently relaxed targets out of L2.
__device__ __forceinline__ ull ld_stream(const ull* p) { return __builtin_nontemporal_load(glob(p)); }

// Arc e as (weight << 32) | target: one 8-byte load from the library's
// packed arcs, or two 4-byte loads from the caller's borrowed arrays (a
// uniform branch on the launch's layout).
struct ArcSrc {
  const ull* packed;
  const int32_t* tgt;
  const uint32_t* wt;
  __device__ __forceinline__ ull at(ull e) const {
    if (packed) return ld_stream(packed + e);
    const uint32_t w = __builtin_nontemporal_load(glob(wt + e));
    const uint32_t t = (uint32_t)__builtin_nontemporal_load(glob(tgt + e));
    return ((ull)w << 32) | t;
  }
};
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
// Barriers. The last workgroup to arrive runs `serial` (whole workgroup)
// before releasing the others, so per-step bookkeeping costs no extra
// barrier. Every wait is bounded: past `tlimit` wall-clock ticks the waiter
// raises the abort flag and all workgroups leave the kernel at their next
// barrier. Barrier calls return false on abort.

template <class P>
__device__ bool spin_until(const KArgs& a, P flag, ull target) {
  const long long t0 = wall_clock64();
  unsigned spins = 0;
  while (ld_agent(flag) < target) {
    __builtin_amdgcn_s_sleep(1);
    if ((++spins & 63) == 0) {
      if (__hip_atomic_load(&a.grid->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if ((ull)(wall_clock64() - t0) > a.tlimit) {
        __hip_atomic_store(&a.grid->abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
  return true;
}

__device__ __forceinline__ bool finish_sync(const KArgs& a, Shared& sh) {
  if (threadIdx.x == 0)
    sh.abort = __hip_atomic_load(&a.grid->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  const bool ok = sh.abort == 0;
  __syncthreads();
  return ok;
}

// Flat barrier over the whole grid (every workgroup releases and acquires at
// agent scope); used once, before the teams and XCD groups are known.
template <class Serial>
__device__ bool flat_sync(const KArgs& a, Shared& sh, Serial serial) {
  GridCtl* gc = a.grid;
  __syncthreads();
  if (threadIdx.x == 0) {
    const ull prev = __hip_atomic_fetch_add(&gc->arrive_flat.v, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    sh.last = prev == (ull)a.G - 1ull;
    if (sh.last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (sh.last) {
    serial();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&gc->gen_flat.v, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  } else if (threadIdx.x == 0) {
    spin_until(a, &gc->gen_flat.v, 1ull);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  return finish_sync(a, sh);
}

// Team barrier (see the file comment).
template <class Serial>
__device__ bool team_sync(const KArgs& a, Shared& sh, Bar& tm, Serial serial) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
  __syncthreads();
  ++tm.epoch;
  if (tm.l2_arrive) ++tm.l2_epoch;
  // Second-level target: arrivals counted from the group's base; the release
  // publishes the target itself, so the value only grows across groups.
  const ull target2 = tm.l2_base + tm.l2_epoch * tm.l2_size;
  if (threadIdx.x == 0) {
    sh.last = 0;
    if (tm.member_release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const ull prev = atom_add(tm.l1_arrive, 1ull);
    if (prev == tm.epoch * tm.l1_size - 1ull) {
      // Last of the first-level group: publish its L2 contents.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (tm.l2_arrive) {
        const ull p2 = atom_add(tm.l2_arrive, 1ull);
        if (p2 == target2 - 1ull) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          sh.last = 1;
        } else {
          spin_until(a, tm.l2_gen, target2);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          st_agent(tm.l1_gen, tm.epoch);
        }
      } else {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        sh.last = 1;
      }
    } else {
      spin_until(a, tm.l1_gen, tm.epoch);
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
      if (tm.l2_arrive) st_agent(tm.l2_gen, target2);
      st_agent(tm.l1_gen, tm.epoch);
    }
  }
  return finish_sync(a, sh);
}

struct NoSerial {
  __device__ void operator()() const {}
};

// k-th smallest (1-based) of vals[0..s) by MSD radix selection over the bits
// below the highest bit where min and max differ. Whole workgroup.
__device__ __noinline__ ull wg_select_kth(const ull* vals, ull s, ull k) {
  Shared& sh = g_sh;
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
// Phase helpers.

// Record the extracted hub vertices of a wave (lanes with is_hub set): their
// arcs become chunk tasks shared by the team in Relax, each carrying the key
// the vertex was extracted with. The wave reserves its tasks with one atomic
// (hubs are numbered first, so they crowd into the same words and waves, and
// one atomic per hub on the step's single counter would serialise). Whole
// wave, uniform call.
__device__ __noinline__ void wave_push_hubs(const KArgs& a, ull* H, StepSlot* S, bool is_hub, int32_t v, ull d) {
  if (!__ballot(is_hub)) return;
  const unsigned lane = lane_id();
  ull nch = 0;
  if (is_hub) {
    const ull deg = (ull)(a.off[v + 1] - a.off[v]);
    nch = (deg + a.chunk_edges - 1) / a.chunk_edges;
  }
  ull incl = nch;
  for (int o = 1; o < 64; o <<= 1) {
    const ull y = __shfl_up(incl, o);
    if ((int)lane >= o) incl += y;
  }
  ull base = 0;
  if (lane == 63) base = atom_add(&S->h_count, incl);  // lane 63 holds the wave's total
  base = __shfl(base, 63) + incl - nch;
  for (ull c = 0; c < nch; ++c) {
    H[2 * (base + c)] = ((ull)(uint32_t)v << 32) | c;
    H[2 * (base + c) + 1] = d;
  }
}

// WriteMin filter (S3): hint[v] is a 16-bit code of an upper bound of
// delta[v] (HINT_NONE: none known), kept by the successful WriteMins with
// plain stores; a stale hint is still an upper bound, since keys only fall.
// nd >= value(hint[v]) means the WriteMin cannot succeed, so the atomic is
// skipped. This read is the one random read of every arc, and the codes take
// a quarter of the cache lines of the keys; rounding the bound up lets a few
// more arcs through to the atomic.
// The codes and their values: hint_code.h.

// Update(v) (S4): set v's flag; true when v is new to Q.
__device__ __forceinline__ bool mark(ull* bitmap, int32_t v) {
  const ull bit = 1ull << (v & 63);
  return !(__hip_atomic_fetch_or(glob(&bitmap[v >> 6]), bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit);
}

// Tournament-tree queue (Sec. 4.2, Alg. 2), fan-out 64: node key1[w] holds
// the smallest key queued in bitmap word w, key2[j] the smallest over words
// 64j .. 64j + 63 (n2 = ceil(words / 64) of them). A workgroup that extracts
// below a node relaxes what it extracted, and vertices are numbered by
// decreasing degree, so in this mode every vertex above 64 arcs is relaxed
// through the team's shared hub chunks instead (the launch lowers
// hub_degree to 64), which keeps Relax balanced.
//
// Alg. 2's Mark flags the nodes on the path to the root as changed, and its
// Update recomputes the flagged nodes before the next Extract. Here the keys
// that Relax can only lower are lowered at once with an atomic min (the walk
// up stops where a node already holds a smaller key, as Alg. 2's stops at a
// node already flagged), and the nodes that Extract raises are recomputed by
// the workgroup that owns them during that Extract. A node may hold less than
// the minimum below it (a lowered key whose vertex was not queued); Extract
// then finds nothing there and sets the node exact. It never holds more, so
// descending only into nodes with key <= theta finds every such vertex.
//
// A plain read first skips the atomic when the node already holds a key
// <= d (most WriteMins: the node is the minimum of 64 keys, and many
// WriteMins land on the same few words, where atomics would serialise).
// Within Relax the nodes only fall and the per-CU cache was invalidated at
// the phase's barrier, so a stale read is never below the node's key and no
// lowering is lost.
__device__ __forceinline__ void tree_lower(const Team& tm, int32_t v, ull d) {
  if (!tm.key1) return;
  ull* k1 = &tm.key1[v >> 6];
  if (d < ld_plain(k1) && d < atom_min(k1, d)) {
    ull* k2 = &tm.key2[v >> 12];
    if (d < ld_plain(k2)) atom_min(k2, d);
  }
}

// Append the flagged entries of each lane to the next explicit list with one
// atomic per workgroup; entries past the list capacity are dropped (the
// reserved count then exceeds the capacity and the list is not used).
template <int K>
__device__ __forceinline__ void list_append(const KArgs& a, StepSlot* S, int32_t* Lnext, const int32_t (&v)[K],
                                            unsigned mask) {
  ull o = wg_reserve(g_sh, &S->list_next, (uint32_t)__popc(mask));
#pragma unroll
  for (int k = 0; k < K; ++k)
    if ((mask >> k) & 1u) {
      if (o < a.lcap) Lnext[o] = v[k];
      ++o;
    }
}

// Stage v in this workgroup's LDS buffer for the next explicit list (any
// lanes; no barrier); a full buffer sends the entry straight to the list.
__device__ __forceinline__ void pend_push(const KArgs& a, StepSlot* S, int32_t* Lnext, int32_t v) {
  Shared& sh = g_sh;
  const uint32_t slot = atomicAdd(&sh.npend, 1u);
  if (slot < (uint32_t)PEND) {
    sh.pend[slot] = v;
  } else {
    const ull o = atom_add(&S->list_next, 1ull);
    if (o < a.lcap) Lnext[o] = v;
  }
}

// Write the staged entries to the next explicit list with one reservation
// and clear the buffer. Whole workgroup, uniform call.
__device__ __forceinline__ void pend_flush(const KArgs& a, StepSlot* S, int32_t* Lnext) {
  Shared& sh = g_sh;
  __syncthreads();  // every staged entry written
  // Uniform: nothing is staged between the barrier above and the next one.
  const uint32_t n = min(sh.npend, (uint32_t)PEND);
  if (n == 0) return;
  if (threadIdx.x == 0) sh.bcast[0] = atom_add(&S->list_next, (ull)n);
  __syncthreads();
  const ull base = sh.bcast[0];
  for (uint32_t i = threadIdx.x; i < n; i += WG)
    if (base + i < a.lcap) Lnext[base + i] = sh.pend[i];
  __syncthreads();
  if (threadIdx.x == 0) sh.npend = 0;
  __syncthreads();
}

// Between batches of a long tile or hub chunk: flush once the buffer is
// half full (a batch stages at most WG * UNROLL entries, so it rarely
// overflows). Whole workgroup, uniform call.
__device__ __forceinline__ void pend_check(const KArgs& a, StepSlot* S, int32_t* Lnext) {
  Shared& sh = g_sh;
  __syncthreads();
  const bool full = sh.npend > (uint32_t)PEND / 2;
  __syncthreads();  // every thread has read the count before anyone stages more
  if (full) pend_flush(a, S, Lnext);
}

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

// S1 for rho-stepping: draw this workgroup's share of the samples of the
// queue's keys (App. B). The selection runs in the following barrier's serial
// section.
__device__ __noinline__ void phase_sample(const KArgs& a, const ull* dist, StepSlot* S,
                                          const int32_t* Lcur, ull q, bool dense, ull probes, ull tseed) {
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const ull n = (ull)a.n, stride = tm.T * WG;
  for (ull base = tm.rank * WG; base < probes; base += stride) {
    const ull j = base + threadIdx.x;
    bool acc = false;
    ull d = 0;
    if (j < probes) {
      const ull r = splitmix(tseed, j);
      if (dense) {
        const ull v = below(r, n);
        if ((ld_agent(&tm.bitmap[v >> 6]) >> (v & 63)) & 1ull) {
          acc = true;
          d = ld_agent(&dist[v]);
        }
      } else {
        const int32_t v = ld_agent_i32(&Lcur[below(r, q)]);
        acc = true;
        d = ld_agent(&dist[v]);
      }
    }
    const ull pos = wg_reserve(sh, &S->nsamples, acc ? 1u : 0u);
    if (acc) tm.samples[pos] = d;
  }
}

// Extract's thresholds: theta, and theta_h <= theta for the deferred hubs
// (vertex ids below ndefer); ndefer = 0 when no vertex is deferred.
struct Thresh {
  ull theta, theta_h, ndefer;
};
__device__ __forceinline__ ull limit_of(const Thresh& th, int32_t v) {
  return (ull)(uint32_t)v < th.ndefer ? th.theta_h : th.theta;
}

struct ExtractOut {
  uint32_t fcnt;  // entries written to this workgroup's F segment
  ull x;          // vertices extracted
  ull minkept;    // min key of the members left in Q
};

// Extraction decisions of one round: v[k] (or -1), keys d[k], hub flags.
// Small candidates are extracted while the F segment has room; the rest stay
// in Q (a team whose segments cannot hold every candidate of a step extracts
// the first segcap of each segment and leaves the others for the next step).
template <int K>
__device__ __forceinline__ void extract_round(const KArgs& a, const Team& tm, StepSlot* S, int32_t* Lnext,
                                              const Thresh th, bool emit, bool atomic_clear, const int32_t (&v)[K],
                                              const ull (&d)[K], unsigned hubs, ExtractOut& o, ull& clear) {
  Shared& sh = g_sh;
  uint32_t ncand = 0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (v[k] >= 0 && d[k] <= limit_of(th, v[k]) && !((hubs >> k) & 1u)) ++ncand;
  uint32_t total;
  const uint32_t first = o.fcnt + wg_scan(sh, ncand, total);
  const ull room = a.segcap - o.fcnt;
  uint32_t slot = first;
  unsigned keep = 0, hub_taken = 0;
  int32_t ev[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ev[k] = -1;
    if (v[k] < 0) continue;
    const ull bit = 1ull << (v[k] & 63);
    bool ext = d[k] <= limit_of(th, v[k]);
    if (ext && !((hubs >> k) & 1u)) {
      if (slot < a.segcap) {
        tm.Fb[slot] = v[k];
        if (a.snapshot) tm.FDb[slot] = d[k];
      } else {
        ext = false;
      }
      ++slot;
    }
    if (ext) {
      if (atomic_clear) {
        atom_and(&tm.bitmap[v[k] >> 6], ~bit);
      } else {
        clear |= bit;
      }
      ++o.x;
      if (a.xcount) ev[k] = v[k];
      if ((hubs >> k) & 1u) hub_taken |= 1u << k;
    } else {
      o.minkept = umin(o.minkept, d[k]);
      keep |= 1u << k;
    }
  }
  o.fcnt += (uint32_t)umin((ull)total, room);
  if (__ballot(hub_taken != 0)) {
#pragma unroll
    for (int k = 0; k < K; ++k) wave_push_hubs(a, tm.H, S, (hub_taken >> k) & 1u, v[k], d[k]);
  }
  if (emit) list_append(a, S, Lnext, v, keep);
  if (a.xcount) {
    uint32_t* xc = a.xcount + ld_agent(&tm.ctl->query) * (ull)a.n;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (ev[k] >= 0) xc[a.perm ? a.perm[ev[k]] : ev[k]] += 1u;
  }
}

// S2, bitmap step. Within the team, rank r owns the blocks of BLOCK_WORDS
// words r, r + T, r + 2T, ... (interleaved, so that the high-degree vertices
// numbered first are spread over all workgroups). Each lane owns one word;
// its members are read in rounds of BATCH keys.
__device__ __noinline__ ExtractOut phase_extract_dense(const KArgs& a, const ull* dist, StepSlot* S,
                                                       int32_t* Lnext, const Thresh th, bool emit) {
  const Team& tm = g_tm;
  const ull nw = a.nwords, T = tm.T;
  const ull nblocks = (nw + BLOCK_WORDS - 1) / BLOCK_WORDS;
  constexpr ull BLOCKS_PER_ROUND = WG / BLOCK_WORDS;
  ExtractOut o{0, 0, INF};
  for (ull r0 = tm.rank; r0 < nblocks; r0 += T * BLOCKS_PER_ROUND) {
    const ull blk = r0 + T * (threadIdx.x / BLOCK_WORDS);
    const ull wi = blk * BLOCK_WORDS + (threadIdx.x % BLOCK_WORDS);
    const ull word = (blk < nblocks && wi < nw) ? ld_agent(&tm.bitmap[wi]) : 0ull;
    const ull hubw = word ? ld_plain(&a.hubmask[wi]) : 0ull;
    ull rest = word, clear = 0;
    while (__syncthreads_or(rest != 0)) {
      int32_t v[BATCH];
      ull d[BATCH];
      unsigned hubs = 0;
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        v[k] = -1;
        if (rest) {
          const int bit = __ffsll((long long)rest) - 1;
          rest &= rest - 1;
          v[k] = (int32_t)(wi * 64 + bit);
          if ((hubw >> bit) & 1ull) hubs |= 1u << k;
        }
      }
#pragma unroll
      for (int k = 0; k < BATCH; ++k) d[k] = v[k] >= 0 ? ld_agent(&dist[v[k]]) : INF;
      extract_round(a, tm, S, Lnext, th, emit, false, v, d, hubs, o, clear);
    }
    if (clear) tm.bitmap[wi] = word & ~clear;  // this lane owns word wi
  }
  return o;
}

// Position of the n-th (from 0) set bit of w, by halving with popcounts.
__device__ __forceinline__ int select_bit(ull w, uint32_t n) {
  int pos = 0;
#pragma unroll
  for (int h = 32; h > 0; h >>= 1) {
    const uint32_t c = (uint32_t)__popcll(w & ((1ull << h) - 1ull));
    if (n >= c) {
      n -= c;
      w >>= h;
      pos += h;
    }
  }
  return pos;
}

// S2, bitmap step without an explicit list to build. Each thread loads one
// owned word per round (the block layout above); the round's members are
// then dealt out evenly: a prefix sum of the words' member counts in LDS, and
// thread j takes members j, j + WG, ... (its word by binary search, its bit by
// rank), so a round costs the workgroup's member count over WG key reads per
// lane rather than the fullest word's (a lane walking a word of 64 members
// made the whole wave wait for 16 dependent reads). Consecutive threads take
// consecutive members, so the key reads coalesce where words are crowded.
// Extracted bits are collected per word with LDS atomics and written back by
// the word's owner; F slots come from an LDS counter, hubs are recorded with
// one atomic per wave.
__device__ __noinline__ ExtractOut phase_extract_dense_fast(const KArgs& a, const ull* dist, StepSlot* S,
                                                            const Thresh th) {
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  const ull nw = a.nwords, T = tm.T;
  const ull nblocks = (nw + BLOCK_WORDS - 1) / BLOCK_WORDS;
  constexpr ull BLOCKS_PER_ROUND = WG / BLOCK_WORDS;
  ExtractOut o{0, 0, INF};
  if (tid == 0) sh.fcnt = 0;
  __syncthreads();
  uint32_t* xc = a.xcount ? a.xcount + ld_agent(&tm.ctl->query) * (ull)a.n : nullptr;
  // Arguments in registers and global-address-space pointers: a store
  // through a generic pointer might alias the argument block, and the
  // compiler would re-read (and wait for) the arguments after every F store.
  const ull segcap = a.segcap;
  const bool snap = a.snapshot;
  const int32_t* perm = a.perm;
  const gptr<int32_t> Fb = glob(tm.Fb);
  const gptr<ull> FDb = glob(tm.FDb);
  const gptr<ull> bits = glob(tm.bitmap);
  const gptr<const ull> hubmask = glob(a.hubmask);
  const gptr<const ull> gd = glob(dist);
  // The Relax tile arrays are free during Extract: the round's words, their
  // hub flags and the bits extracted from them.
  ull* const wword = sh.beg;
  ull* const whub = sh.du;
  ull* const wclear = sh.pulled;
  for (ull r0 = tm.rank; r0 < nblocks; r0 += T * BLOCKS_PER_ROUND) {
    const ull blk = r0 + T * (tid / BLOCK_WORDS);
    const ull wi = blk * BLOCK_WORDS + (tid % BLOCK_WORDS);
    const ull word =
        (blk < nblocks && wi < nw) ? __hip_atomic_load(&bits[wi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
    const ull hubw = word ? hubmask[wi] : 0ull;
    uint32_t total;
    const uint32_t excl = wg_scan(sh, (uint32_t)__popcll(word), total);
    sh.pre[tid] = excl;
    wword[tid] = word;
    whub[tid] = hubw;
    wclear[tid] = 0;
    __syncthreads();
    for (uint32_t j0 = 0; j0 < total; j0 += WG * BATCH) {
      int32_t v[BATCH];
      int own[BATCH];
      ull d[BATCH];
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        const uint32_t j = j0 + k * WG + tid;
        v[k] = -1;
        own[k] = 0;
        if (j < total) {
          int lo = 0;
#pragma unroll
          for (int step = WG / 2; step > 0; step >>= 1)
            if (sh.pre[lo + step] <= j) lo += step;
          const int bit = select_bit(wword[lo], j - sh.pre[lo]);
          const ull owi = (r0 + T * (ull)(lo / BLOCK_WORDS)) * BLOCK_WORDS + (ull)(lo % BLOCK_WORDS);
          v[k] = (int32_t)(owi * 64 + (ull)bit);
          own[k] = lo;
        }
      }
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        // Unconditional reads (vertex 0 for an empty slot): in flight together.
        d[k] = __hip_atomic_load(&gd[v[k] >= 0 ? v[k] : 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v[k] < 0) d[k] = INF;
      }
      unsigned hub_taken = 0;
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        if (v[k] < 0) continue;
        const ull bit = 1ull << (v[k] & 63);
        bool ext = d[k] <= limit_of(th, v[k]);
        if (ext) {
          if ((whub[own[k]] & bit) != 0) {
            hub_taken |= 1u << k;
          } else {
            const uint32_t slot = atomicAdd(&sh.fcnt, 1u);
            if (slot < segcap) {
              Fb[slot] = v[k];
              if (snap) FDb[slot] = d[k];
            } else {
              ext = false;  // no room: stays queued
            }
          }
        }
        if (ext) {
          atomicOr(&wclear[own[k]], bit);
          ++o.x;
          if (xc) xc[perm ? perm[v[k]] : v[k]] += 1u;
        } else {
          o.minkept = umin(o.minkept, d[k]);
        }
      }
      if (__ballot(hub_taken != 0)) {
#pragma unroll
        for (int k = 0; k < BATCH; ++k) wave_push_hubs(a, tm.H, S, (hub_taken >> k) & 1u, v[k], d[k]);
      }
    }
    __syncthreads();
    const ull clear = wclear[tid];
    if (clear) bits[wi] = word & ~clear;  // this thread owns word wi
    __syncthreads();  // the LDS arrays are refilled next round
  }
  o.fcnt = (uint32_t)umin((ull)sh.fcnt, segcap);
  return o;
}

// S2, bitmap step without an explicit list, when at least a quarter of the
// vertices are queued: a lane walking the members of a crowded word issues
// dozens of dependent loads, so here wave w of the workgroup takes word w of
// each owned block and lane l looks at bit l; the keys of a word's members
// come in one coalesced load. WPI words are in flight per wave. F slots are
// reserved per wave and word with one LDS atomic; the owner wave writes the
// word back without the extracted bits.
constexpr int WPI = 4;

__device__ __noinline__ ExtractOut phase_extract_dense_words(const KArgs& a, const ull* dist, StepSlot* S,
                                                             const Thresh th) {
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const ull nw = a.nwords, T = tm.T;
  const ull nblocks = (nw + BLOCK_WORDS - 1) / BLOCK_WORDS;
  const unsigned lane = lane_id(), wave = threadIdx.x >> 6;
  const ull below_lane = (1ull << lane) - 1ull;
  ExtractOut o{0, 0, INF};
  if (threadIdx.x == 0) sh.fcnt = 0;
  __syncthreads();
  uint32_t* xc = a.xcount ? a.xcount + ld_agent(&tm.ctl->query) * (ull)a.n : nullptr;
  // As in the dealt Extract above: arguments in registers,
  // global-address-space pointers, and unconditional reads.
  const ull segcap = a.segcap;
  const bool snap = a.snapshot;
  const int32_t* perm = a.perm;
  const gptr<int32_t> Fb = glob(tm.Fb);
  const gptr<ull> FDb = glob(tm.FDb);
  const gptr<ull> bits = glob(tm.bitmap);
  const gptr<const ull> hubmask = glob(a.hubmask);
  const gptr<const ull> gd = glob(dist);
  for (ull blk0 = tm.rank; blk0 < nblocks; blk0 += (ull)WPI * T) {
    ull wi[WPI], word[WPI], d[WPI], hubw[WPI];
#pragma unroll
    for (int k = 0; k < WPI; ++k) {
      const ull blk = blk0 + (ull)k * T;
      wi[k] = blk * BLOCK_WORDS + wave;
      const bool in = blk < nblocks && wi[k] < nw;
      word[k] = __hip_atomic_load(&bits[in ? wi[k] : 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!in) word[k] = 0;
    }
#pragma unroll
    for (int k = 0; k < WPI; ++k) {
      const bool member = (word[k] >> lane) & 1ull;
      d[k] = __hip_atomic_load(&gd[member ? wi[k] * 64 + lane : 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!member) d[k] = INF;
      hubw[k] = hubmask[word[k] ? wi[k] : 0];
      if (!word[k]) hubw[k] = 0;
    }
#pragma unroll
    for (int k = 0; k < WPI; ++k) {
      if (!word[k]) continue;  // the same word in every lane
      const int32_t v = (int32_t)(wi[k] * 64 + lane);
      const bool member = (word[k] >> lane) & 1ull;
      const bool hub = (hubw[k] >> lane) & 1ull;
      bool ext = member && d[k] <= limit_of(th, v);
      const ull want = __ballot(ext && !hub);
      if (want) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&sh.fcnt, (uint32_t)__popcll(want));
        base = __shfl(base, 0);
        if (ext && !hub) {
          const uint32_t slot = base + (uint32_t)__popcll(want & below_lane);
          if (slot < segcap) {
            Fb[slot] = v;
            if (snap) FDb[slot] = d[k];
          } else {
            ext = false;  // no room: stays queued
          }
        }
      }
      wave_push_hubs(a, tm.H, S, ext && hub, v, d[k]);
      if (ext) {
        ++o.x;
        if (xc) xc[perm ? perm[v] : v] += 1u;
      } else if (member) {
        o.minkept = umin(o.minkept, d[k]);
      }
      const ull taken = __ballot(ext);
      if (taken && lane == 0) bits[wi[k]] = word[k] & ~taken;  // this wave owns word wi
    }
  }
  __syncthreads();
  o.fcnt = (uint32_t)umin((ull)sh.fcnt, segcap);
  return o;
}

// S2 with the tournament-tree queue: Traverse(theta) of Alg. 2 from the
// second level. Team rank r owns the level-2 nodes r, r + T, ... and the
// words below them; it skips a node whose key is above theta, and below a
// node it visits, wave w takes the children w, w + 4, ... (words 64j + c): a child
// with key above theta is skipped, otherwise the wave extracts its word as in
// phase_extract_dense_words (lane l, bit l) and stores the word's new key
// (the smallest key left in it). The node's key is then recomputed from its
// 64 children. The keys of skipped nodes and of members left bound the keys
// kept in Q.
__device__ __noinline__ ExtractOut phase_extract_tree(const KArgs& a, const ull* dist, StepSlot* S, const Thresh th) {
  const ull theta = th.theta;  // node keys are compared with the larger threshold
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const ull nw = a.nwords;
  const unsigned lane = lane_id(), wave = threadIdx.x >> 6;
  const ull below_lane = (1ull << lane) - 1ull;
  ExtractOut o{0, 0, INF};
  if (threadIdx.x == 0) sh.fcnt = 0;
  __syncthreads();
  uint32_t* xc = a.xcount ? a.xcount + ld_agent(&tm.ctl->query) * (ull)a.n : nullptr;
  for (ull j = tm.rank; j < a.n2; j += tm.T) {
    const ull k2 = ld_agent(&tm.key2[j]);  // the same in every lane
    if (k2 > theta) {
      o.minkept = umin(o.minkept, k2);
      continue;
    }
    // Children c = wave + 4 i; four at a time, their loads issued together.
    for (int i0 = 0; i0 < 64 / WAVES; i0 += 4) {
      ull wi[4], k1[4], word[4], d[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        wi[k] = j * 64 + wave + (ull)WAVES * (i0 + k);
        k1[k] = wi[k] < nw ? ld_agent(&tm.key1[wi[k]]) : INF;  // the same in every lane of the wave
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) word[k] = (wi[k] < nw && k1[k] <= theta) ? ld_agent(&tm.bitmap[wi[k]]) : 0ull;
#pragma unroll
      for (int k = 0; k < 4; ++k) d[k] = ((word[k] >> lane) & 1ull) ? ld_agent(&dist[wi[k] * 64 + lane]) : INF;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (wi[k] >= nw) continue;
        if (k1[k] > theta) {
          o.minkept = umin(o.minkept, k1[k]);
          continue;
        }
        const bool member = (word[k] >> lane) & 1ull;
        const int32_t v = (int32_t)(wi[k] * 64 + lane);
        const bool hub = member && ((ld_plain(&a.hubmask[wi[k]]) >> lane) & 1ull);
        bool ext = member && d[k] <= limit_of(th, v);
        const ull want = __ballot(ext && !hub);
        if (want) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&sh.fcnt, (uint32_t)__popcll(want));
          base = __shfl(base, 0);
          if (ext && !hub) {
            const uint32_t slot = base + (uint32_t)__popcll(want & below_lane);
            if (slot < a.segcap) {
              tm.Fb[slot] = v;
              if (a.snapshot) tm.FDb[slot] = d[k];
            } else {
              ext = false;  // no room: stays queued
            }
          }
        }
        wave_push_hubs(a, tm.H, S, ext && hub, v, d[k]);
        if (ext) {
          ++o.x;
          if (xc) xc[a.perm ? a.perm[v] : v] += 1u;
        }
        const ull left = wave_min(member && !ext ? d[k] : INF);
        o.minkept = umin(o.minkept, left);
        const ull taken = __ballot(ext);
        if (lane == 0) {
          if (taken) tm.bitmap[wi[k]] = word[k] & ~taken;  // this wave owns word wi
          tm.key1[wi[k]] = left;
        }
      }
    }
    __syncthreads();  // the children's new keys are written
    if (wave == 0) {
      const ull wi = j * 64 + lane;
      const ull k = wave_min(wi < nw ? ld_agent(&tm.key1[wi]) : INF);
      if (lane == 0) tm.key2[j] = k;
    }
    __syncthreads();
  }
  __syncthreads();
  o.fcnt = (uint32_t)umin((ull)sh.fcnt, a.segcap);
  return o;
}

// S2, list step: this workgroup's contiguous slice of the explicit list.
__device__ __noinline__ ExtractOut phase_extract_list(const KArgs& a, const ull* dist, StepSlot* S,
                                                      const int32_t* Lcur, int32_t* Lnext, ull q, const Thresh th,
                                                      bool emit) {
  const Team& tm = g_tm;
  const ull lo = tm.rank * q / tm.T, hi = (tm.rank + 1) * q / tm.T;
  ExtractOut o{0, 0, INF};
  ull unused = 0;
  for (ull e0 = lo; e0 < hi; e0 += (ull)WG * UNROLL) {
    int32_t v[UNROLL];
    ull d[UNROLL];
    unsigned hubs = 0;
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const ull i = e0 + (ull)k * WG + threadIdx.x;
      v[k] = i < hi ? ld_agent_i32(&Lcur[i]) : -1;
    }
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      d[k] = INF;
      if (v[k] >= 0) {
        d[k] = ld_agent(&dist[v[k]]);
        if ((ld_plain(&a.hubmask[v[k] >> 6]) >> (v[k] & 63)) & 1ull) hubs |= 1u << k;
      }
    }
    extract_round(a, tm, S, Lnext, th, emit, true, v, d, hubs, o, unused);
  }
  return o;
}

struct RelaxAcc {
  ull edges, succ, fresh, minnew, local, skipped;
};

// Local expansion (the paper's large neighbour sets, Sec. 6): in a sparse
// step, a vertex whose key a WriteMin lowers to at most theta is not put back
// in Q but relaxed by the same workgroup later in the same step, round after
// round from a list in LDS, until the list is empty or the workgroup has
// relaxed `local_budget` vertices this way; what is left then goes to Q. One
// step thus advances several hops without a grid barrier per hop.
struct Local {
  bool on;
  uint32_t nxt;  // LDS list receiving this round's vertices
  ull theta;
};

// Relax UNROLL arcs per lane (ev = packed arc or INF, dd = key of its tail):
// WriteMin, then either the local list or Update, and the new queue members
// to the next explicit list when it is being built.
__device__ __forceinline__ void relax_batch(const KArgs& a, const Team& tm, ull* dist, StepSlot* S, int32_t* Lnext,
                                            bool emit, RelaxAcc& acc, const Local& lx, const ull (&ev)[UNROLL],
                                            const ull (&dd)[UNROLL], const ull (&tr)[UNROLL]) {
  Shared& sh = g_sh;
  int32_t fv[UNROLL];
  uint32_t hv[UNROLL];
  // The batch's key-bound reads first, all in flight together: no branch
  // around a read (an absent arc reads hint[0]), and a wave-uniform switch,
  // because a load under a divergent branch makes the compiler wait for
  // every load in flight where the branch rejoins. Local expansion skips the
  // filter: its vertices' keys were lowered within this step.
  const bool filter = __builtin_amdgcn_readfirstlane((tm.hint != nullptr && !lx.on) ? 1 : 0) != 0;
#pragma unroll
  for (int k = 0; k < UNROLL; ++k) {
    fv[k] = (int32_t)(uint32_t)ev[k];
    hv[k] = HINT_NONE;
  }
  if (filter) {
    const gptr<uint16_t> hint = glob(tm.hint);
#pragma unroll
    for (int k = 0; k < UNROLL; ++k)
      hv[k] = __hip_atomic_load(&hint[ev[k] == INF ? 0 : fv[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  // WriteMin (S3) of every arc that passes the filter, all atomics issued
  // before the first result is used; then the successes.
  ull nd[UNROLL], old[UNROLL];
  unsigned pass = 0;
#pragma unroll
  for (int k = 0; k < UNROLL; ++k) {
    nd[k] = dd[k] + (ev[k] >> 32);
    old[k] = 0;
    if (ev[k] == INF) continue;
    ++acc.edges;
    if (hv[k] == HINT_NONE || nd[k] < hint_value(hv[k])) pass |= 1u << k;
  }
  const gptr<ull> gdist = glob(dist);
#pragma unroll
  for (int k = 0; k < UNROLL; ++k)
    if ((pass >> k) & 1u)
      old[k] = __hip_atomic_fetch_min(&gdist[fv[k]], nd[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned upd = 0;  // successes that go to Q
#pragma unroll
  for (int k = 0; k < UNROLL; ++k) {
    if (!((pass >> k) & 1u) || !(nd[k] < old[k])) continue;
    if (tm.hint) *glob(&tm.hint[fv[k]]) = as_hint(nd[k]);
    ++acc.succ;
    tree_lower(tm, fv[k], nd[k]);
    // Vertices above the local degree cap go to Q, where their arcs are
    // relaxed by the team (local expansion is for small neighbour sets; a
    // high-degree vertex in one workgroup's list would serialise its arcs
    // there).
    if (lx.on && nd[k] <= lx.theta && (ull)(uint32_t)fv[k] >= a.ndefer &&
        (tr[k] != INF ? (tr[k] >> ROW_SHIFT) <= a.local_cap
                      : !((ld_plain(&a.bigmask[fv[k] >> 6]) >> (fv[k] & 63)) & 1ull))) {
      const uint32_t slot = atomicAdd(&sh.lqn[lx.nxt], 1u);
      if (slot < (uint32_t)LQ) {
        sh.lq[lx.nxt][slot] = fv[k];
        sh.lqr[lx.nxt][slot] = tr[k];
        continue;
      }
    }
    acc.minnew = umin(acc.minnew, nd[k]);
    upd |= 1u << k;
  }
  // Update (S4): set the flags, again all atomics before the first result.
  ull ow[UNROLL];
  const gptr<ull> gbits = glob(tm.bitmap);
#pragma unroll
  for (int k = 0; k < UNROLL; ++k) {
    ow[k] = 0;
    if ((upd >> k) & 1u)
      ow[k] = __hip_atomic_fetch_or(&gbits[fv[k] >> 6], 1ull << (fv[k] & 63), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
  }
#pragma unroll
  for (int k = 0; k < UNROLL; ++k)
    if (((upd >> k) & 1u) && !((ow[k] >> (fv[k] & 63)) & 1ull)) {
      ++acc.fresh;
      if (emit) pend_push(a, S, Lnext, fv[k]);
    }
}

// Relax the arcs of up to WG vertices (one per thread; u < 0 for none, du its
// key) as one tile: degree prefix sums and row starts in LDS, then UNROLL
// arcs per lane per round, consecutive lanes on consecutive arcs. Whole
// workgroup, uniform call. Sparse: the graph's tiles hold few arcs (local
// expansion is on), so lanes past the tile's end skip their reads rather
// than repeat the last arc's.
template <bool Sparse>
__device__ __forceinline__ void relax_tile(const KArgs& a, const Team& tm, ull* dist, StepSlot* S, int32_t* Lnext,
                                           bool emit, RelaxAcc& acc, const Local& lx, int32_t u, ull du, ull row,
                                           bool rows, bool sync_after = true) {
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  const ArcSrc arcs{a.edges, a.tgt, a.wt};
  uint32_t deg = 0;
  ull rb = 0;
  if (u >= 0) {
    if (row != INF) {
      // Local expansion: the row came with the arc that queued u.
      rb = row & ROW_START;
      deg = (uint32_t)(row >> ROW_SHIFT);
    } else {
      rb = (ull)*glob(&a.off[u]);
      deg = (uint32_t)((ull)*glob(&a.off[u + 1]) - rb);
    }
    if (tm.lastkey) {
      // u's arcs were already pushed with this very key: every WriteMin
      // would fail, so they are not pushed again.
      const gptr<ull> lk = glob(tm.lastkey);
      if (ld_agent(&lk[u]) == du) {
        acc.skipped += deg;
        deg = 0;
      } else {
        lk[u] = du;
      }
    }
  }
  uint32_t total;
  const uint32_t excl = wg_scan(sh, deg, total);
  sh.pre[tid] = excl;
  sh.beg[tid] = rb;
  sh.du[tid] = du;
  sh.pulled[tid] = du;
  sh.uid[tid] = u;
  __syncthreads();
  if (a.pull) {
    // Bidirectional relaxation (Sec. 6): first lower each vertex's key with
    // its neighbours' keys (the arcs are symmetric), then push with it.
    for (uint32_t e0 = 0; e0 < total; e0 += WG * UNROLL) {
#pragma unroll
      for (int k = 0; k < UNROLL; ++k) {
        const uint32_t e = e0 + k * WG + tid;
        if (e < total) {
          int lo = 0;
#pragma unroll
          for (int step = WG / 2; step > 0; step >>= 1)
            if (sh.pre[lo + step] <= e) lo += step;
          const ull arc = arcs.at(sh.beg[lo] + (e - sh.pre[lo]));
          const ull dv = ld_plain(&dist[(uint32_t)arc]);
          if (dv != INF) {
            const ull cand = dv + (arc >> 32);
            if (cand < sh.pulled[lo]) atomicMin(&sh.pulled[lo], cand);
          }
        }
      }
    }
    __syncthreads();
    if (u >= 0 && sh.pulled[tid] < du) {
      // u's arcs are all pushed below with the lower key, so u need not
      // return to Q (a WriteMin of another workgroup on u still marks it).
      atom_min(&dist[u], sh.pulled[tid]);
      tree_lower(tm, u, sh.pulled[tid]);  // u may have been queued again meanwhile
      sh.du[tid] = sh.pulled[tid];
      ++acc.succ;
    }
    __syncthreads();
  }
  for (uint32_t e0 = 0; e0 < total; e0 += WG * UNROLL) {
    ull ev[UNROLL], dd[UNROLL], tr[UNROLL];
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const uint32_t e = e0 + k * WG + tid;
      tr[k] = INF;
      if constexpr (Sparse) {
        ev[k] = INF;
        dd[k] = 0;
        if (e < total) {
          int lo = 0;
#pragma unroll
          for (int step = WG / 2; step > 0; step >>= 1)
            if (sh.pre[lo + step] <= e) lo += step;
          const ull idx = sh.beg[lo] + (e - sh.pre[lo]);
          ev[k] = arcs.at(idx);
          if (rows) {
            // Row mode: each arc carries its target's row to the LDS list,
            // and its tail's current key is read beside the arc.
            tr[k] = *glob(&a.trow[idx]);
            dd[k] = ld_agent(&dist[sh.uid[lo]]);
          } else {
            dd[k] = sh.du[lo];
          }
        }
      } else {
        // Lanes past the tile's end read its last arc and drop it: the reads
        // stay unconditional, so the batch's reads are in flight together.
        const uint32_t ec = e < total ? e : total - 1;
        int lo = 0;
#pragma unroll
        for (int step = WG / 2; step > 0; step >>= 1)
          if (sh.pre[lo + step] <= ec) lo += step;
        const ull arc = arcs.at(sh.beg[lo] + (ec - sh.pre[lo]));
        ev[k] = e < total ? arc : INF;
        dd[k] = sh.du[lo];
      }
    }
    relax_batch(a, tm, dist, S, Lnext, emit, acc, lx, ev, dd, tr);
    if (emit && e0 + WG * UNROLL < total) pend_check(a, S, Lnext);
  }
  // The tile arrays are reused by the next tile (the caller may end the
  // round with a barrier of its own instead).
  if (sync_after) __syncthreads();
}

// The team's hub chunks, strided over its workgroups. Each chunk is pushed
// with one key, u's current key read once (or its key at extraction with
// snapshot keys); a chunk already pushed with that very key (ckey) is
// skipped, since every WriteMin of it would fail.
__device__ __forceinline__ RelaxAcc relax_hub_chunks(const KArgs& a, ull* dist, StepSlot* S, int32_t* Lnext,
                                                     bool emit, const Local lx) {
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  RelaxAcc acc{0, 0, 0, INF, 0, 0};
  const ArcSrc arcs{a.edges, a.tgt, a.wt};
  const ull nH = ld_agent(&S->h_count);
  const ull CH = a.chunk_edges;
  for (ull item = tm.rank; item < nH; item += tm.T) {
    if (tid == 0) {
      const ull task = ld_agent(&tm.H[2 * item]);
      const int32_t u0 = (int32_t)(task >> 32);
      const ull d0 = a.snapshot ? ld_agent(&tm.H[2 * item + 1]) : ld_agent(&dist[u0]);
      int skip = 0;
      if (tm.ckey && (ull)u0 < a.nhub) {
        ull* ck = &tm.ckey[a.cbase[u0] + (task & 0xffffffffull)];
        if (ld_agent(ck) == d0) {
          skip = 1;
        } else if (!a.pull) {
          *ck = d0;
        }
      }
      sh.hub_task = task;
      sh.hub_du = d0;
      sh.hub_skip = skip;
    }
    __syncthreads();
    const ull task = sh.hub_task;
    ull du = sh.hub_du;
    const bool skip = sh.hub_skip != 0;
    __syncthreads();
    const int32_t u = (int32_t)(task >> 32);
    const ull c = task & 0xffffffffull;
    const ull rb = (ull)a.off[u], re = (ull)a.off[u + 1];
    const ull beg = rb + c * CH;
    const ull end = umin(beg + CH, re);
    if (skip) {
      if (tid == 0) acc.skipped += end - beg;
      continue;
    }
    if (a.pull) {
      // Bidirectional relaxation over this chunk's neighbours. Other chunks
      // of u may already have pushed with the older key, so a lower key
      // also puts u back in Q.
      ull best = du;
      for (ull e = beg + tid; e < end; e += WG) {
        const ull arc = arcs.at(e);
        const ull dv = ld_plain(&dist[(uint32_t)arc]);
        if (dv != INF) best = umin(best, dv + (arc >> 32));
      }
      ull z0 = 0, z1 = 0, z2 = 0;
      wg_reduce4(sh, z0, z1, z2, best);
      if (best < du) {
        int32_t v1[1] = {u};
        unsigned m1 = 0;
        if (tid == 0 && best < atom_min(&dist[u], best)) {
          ++acc.succ;
          tree_lower(tm, u, best);
          acc.minnew = umin(acc.minnew, best);
          if (mark(tm.bitmap, u)) {
            ++acc.fresh;
            m1 = 1;
          }
        }
        if (emit) list_append(a, S, Lnext, v1, m1);
        du = best;
      }
      if (tid == 0 && tm.ckey && (ull)u < a.nhub) tm.ckey[a.cbase[u] + c] = du;
    }
    for (ull e0 = beg; e0 < end; e0 += (ull)WG * UNROLL) {
      ull ev[UNROLL], dd[UNROLL], tr[UNROLL];
#pragma unroll
      for (int k = 0; k < UNROLL; ++k) {
        // A chunk is never empty; lanes past its end read its last arc and
        // drop it (unconditional reads, in flight together).
        const ull e = e0 + (ull)k * WG + tid;
        const ull arc = arcs.at(e < end ? e : end - 1);
        ev[k] = e < end ? arc : INF;
        dd[k] = du;
        tr[k] = INF;
      }
      relax_batch(a, tm, dist, S, Lnext, emit, acc, lx, ev, dd, tr);
      if (emit) pend_check(a, S, Lnext);
    }
  }
  return acc;
}

// S3 + S4: the team's hub chunks (strided over its workgroups), then this
// workgroup's own extracted vertices, then (local expansion) the rounds of
// vertices they improved. Writes the workgroup's partial counts.
__device__ __noinline__ void phase_relax(const KArgs& a, ull* dist, StepSlot* S, int32_t* Lnext, bool emit,
                                         ExtractOut ex, bool local, ull theta) {
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  const long long t_start = wall_clock64();
  RelaxAcc acc{0, 0, 0, INF, 0, 0};
  Local lx{local, 0, theta};
  if (tid < 2) sh.lqn[tid] = 0;
  if (tid == 0) sh.npend = 0;
  __syncthreads();
  {
    const RelaxAcc h = relax_hub_chunks(a, dist, S, Lnext, emit, lx);
    acc.edges += h.edges;
    acc.succ += h.succ;
    acc.fresh += h.fresh;
    acc.minnew = umin(acc.minnew, h.minnew);
    acc.skipped += h.skipped;
  }
  // Round 0: this workgroup's extracted vertices. Later rounds (local
  // expansion): LDS list `cur`, the vertices the previous round improved
  // (capped at LQ; pushes beyond it went to Q).
  uint32_t cnt = ex.fcnt, cur = 1;
  ull done_local = 0;
  const bool sparse_graph = __builtin_amdgcn_readfirstlane(a.local_budget > 0 ? 1 : 0) != 0;
  // Row mode (local expansion with target rows, keys read per arc): a listed
  // vertex needs no offset or key read before its round. Not with the
  // repeated-push skip or bidirectional relaxation, which need u's key
  // up front.
  const bool rows = sparse_graph && local && a.trow != nullptr && tm.lastkey == nullptr && !a.pull;
  for (bool first = true;; first = false) {
    for (uint32_t j0 = 0; j0 < cnt; j0 += WG) {
      const uint32_t j = j0 + tid;
      int32_t u = -1;
      ull du = 0, row = INF;
      if (j < cnt) {
        if (first) {
          u = tm.Fb[j];
          du = a.snapshot ? tm.FDb[j] : ld_agent(&dist[u]);
        } else {
          // A listed vertex's row came with the arc that listed it.
          u = sh.lq[cur][j];
          if (rows) row = sh.lqr[cur][j];
          if (row == INF) du = ld_agent(&dist[u]);
        }
      }
      // A local round's last tile leaves its barrier to the one below.
      const bool sync_after = !(local && j0 + WG >= cnt);
      if (sparse_graph)
        relax_tile<true>(a, tm, dist, S, Lnext, emit, acc, lx, u, du, row, rows, sync_after);
      else
        relax_tile<false>(a, tm, dist, S, Lnext, emit, acc, lx, u, du, row, false, sync_after);
      // Read after the tile's barrier and before the next tile stages
      // anything, so every thread sees the same count.
      if (emit && sync_after && sh.npend > (uint32_t)PEND / 2) pend_flush(a, S, Lnext);
    }
    if (!local) break;
    cur = lx.nxt;
    // The list read in the last round (cur ^ 1) receives the next round's
    // vertices: its count is cleared before the barrier that publishes cur's.
    if (tid == 0) sh.lqn[cur ^ 1u] = 0;
    __syncthreads();
    cnt = min(sh.lqn[cur], (uint32_t)LQ);
    if (emit && sh.npend > (uint32_t)PEND / 2) pend_flush(a, S, Lnext);
    if (cnt == 0) break;
    {
      if (done_local + cnt > a.local_budget) {
        // Out of budget: the rest joins Q.
        for (uint32_t j0 = 0; j0 < cnt; j0 += WG) {
          const uint32_t j = j0 + tid;
          int32_t v[1] = {-1};
          unsigned m = 0;
          if (j < cnt) {
            v[0] = sh.lq[cur][j];
            acc.minnew = umin(acc.minnew, ld_agent(&dist[v[0]]));
            if (mark(tm.bitmap, v[0])) {
              ++acc.fresh;
              m = 1;
            }
          }
          if (emit) list_append(a, S, Lnext, v, m);
        }
        break;
      }
      done_local += cnt;
      lx.nxt = cur ^ 1u;
    }
  }
  acc.local = done_local;
  if (emit) pend_flush(a, S, Lnext);
  ull xs = ex.x, mk = ex.minkept;
  wg_reduce4(sh, acc.edges, acc.succ, acc.fresh, acc.minnew);
  {
    ull z1 = 0;
    wg_reduce4(sh, xs, acc.skipped, z1, mk);
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
    p.local = acc.local;
    p.skipped = acc.skipped;
    a.parts[blockIdx.x] = p;
  }
}

// One pass of the exact rho-th selection over this workgroup's share of Q
// (the same ownership as Extract). With `bounds`: the minimum and maximum
// key. Otherwise: the histogram of the digit (key >> shift) & mask over the
// keys whose bits from `top` up equal those of `prefix`, added to the team's
// histogram.
__device__ __noinline__ void phase_select(const KArgs& a, const ull* dist, const int32_t* Lcur, ull q, bool dense,
                                          bool bounds, int top, int shift, ull mask, ull prefix) {
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  TeamCtl* tc = tm.ctl;
  sh.hist[tid] = 0;
  __syncthreads();
  ull mn = INF, negmx = INF;
  auto visit = [&](ull d) {
    if (bounds) {
      mn = umin(mn, d);
      negmx = umin(negmx, ~d);
    } else if (top >= 64 || (d >> top) == (prefix >> top)) {
      atomicAdd(&sh.hist[(d >> shift) & mask], 1u);
    }
  };
  if (dense) {
    const ull nw = a.nwords, nblocks = (nw + BLOCK_WORDS - 1) / BLOCK_WORDS;
    constexpr ull BLOCKS_PER_ROUND = WG / BLOCK_WORDS;
    for (ull r0 = tm.rank; r0 < nblocks; r0 += tm.T * BLOCKS_PER_ROUND) {
      const ull blk = r0 + tm.T * (tid / BLOCK_WORDS);
      const ull wi = blk * BLOCK_WORDS + (tid % BLOCK_WORDS);
      if (blk >= nblocks || wi >= nw) continue;
      ull rest = ld_agent(&tm.bitmap[wi]);
      while (rest) {
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
        for (int k = 0; k < BATCH; ++k) d[k] = v[k] >= 0 ? ld_agent(&dist[v[k]]) : 0;
#pragma unroll
        for (int k = 0; k < BATCH; ++k)
          if (v[k] >= 0) visit(d[k]);
      }
    }
  } else {
    const ull lo = tm.rank * q / tm.T, hi = (tm.rank + 1) * q / tm.T;
    for (ull i = lo + tid; i < hi; i += WG) visit(ld_agent(&dist[ld_agent_i32(&Lcur[i])]));
  }
  if (bounds) {
    ull z0 = 0, z1 = 0, z2 = 0;
    wg_reduce4(sh, z0, z1, z2, mn);
    wg_reduce4(sh, z0, z1, z2, negmx);
    if (tid == 0) {
      atom_min(&tc->sel_min, mn);
      atom_min(&tc->sel_max, negmx);  // holds ~max
    }
  } else {
    __syncthreads();
    if (sh.hist[tid]) atom_add(&tc->sel_hist[tid], (ull)sh.hist[tid]);
  }
}

// Serial steps of the exact selection (thread 0 of the last workgroup at the
// pass's barrier). After the bounds pass: start from the bits above the
// highest bit where min and max differ. After a digit pass: pick the digit
// whose bin holds the remaining rank.
__device__ __noinline__ void select_serial(TeamCtl* tc, bool after_bounds, int shift, ull rank) {
  if (after_bounds) {
    const ull mn = ld_agent(&tc->sel_min), mx = ~ld_agent(&tc->sel_max);
    const int top = mn == mx ? 0 : 64 - __clzll((long long)(mn ^ mx));
    tc->sel_top = (ull)top;
    tc->sel_prefix = top >= 64 ? 0 : (mn >> top) << top;
    tc->sel_k = rank;
  } else {
    ull k = ld_agent(&tc->sel_k), acc = 0;
    ull digit = 0;
    for (; digit < 256; ++digit) {
      const ull c = ld_agent(&tc->sel_hist[digit]);
      if (acc + c >= k) break;
      acc += c;
    }
    if (digit == 256) digit = 255;  // unreachable when the rank is within the queue
    tc->sel_prefix = ld_agent(&tc->sel_prefix) | (digit << shift);
    tc->sel_k = k - acc;
    tc->sel_top = (ull)shift;
  }
  for (int i = 0; i < 256; ++i) tc->sel_hist[i] = 0;
}

// Serial section of the step's last barrier: sum the partials of the team's
// workgroups, publish the step totals, clear the slot two steps ahead, update
// stats and the trace.
__device__ __noinline__ void step_bookkeeping(const KArgs& a, StepSlot* S, ull t, ull q, ull theta,
                                              unsigned flags, ull extract_ticks, ull relax_start) {
  const Team& tm = g_tm;
  Shared& sh = g_sh;
  const unsigned tid = threadIdx.x;
  TeamCtl* tc = tm.ctl;
  ull x = 0, e = 0, s = 0, f = 0, mn = INF, busy = 0, negbusy = INF, lv = 0, sk = 0;
  for (ull r = tid; r < tm.T; r += WG) {
    // Group rank r is rank r % Tteam of member team r / Tteam.
    const ull team = tm.k > 1 ? (ull)ld_agent_i32(&tc->gteam[r / tm.Tteam]) : tm.id;
    const ull* p = reinterpret_cast<const ull*>(&a.parts[team + (r % tm.Tteam) * a.nteams]);
    x += ld_agent(p + 0);
    mn = umin(mn, ld_agent(p + 1));
    e += ld_agent(p + 2);
    s += ld_agent(p + 3);
    f += ld_agent(p + 4);
    mn = umin(mn, ld_agent(p + 5));
    const ull bz = ld_agent(p + 6);
    lv += ld_agent(p + 7);
    sk += ld_agent(p + 8);
    busy += bz;
    negbusy = umin(negbusy, ~bz);
  }
  wg_reduce4(sh, x, e, s, mn);
  wg_reduce4(sh, f, busy, lv, negbusy);
  {
    ull z0 = 0, z1 = 0, z2 = INF;
    wg_reduce4(sh, sk, z0, z1, z2);
  }
  if (tid < 16) {
    ull* z = reinterpret_cast<ull*>(&tc->slot[(t + 2) % 3]);
    z[tid] = 0ull;
  }
  if (tid == 0) {
    tc->sel_min = INF;  // for the next step's exact selection
    tc->sel_max = INF;
  }
  if (tid == 0) {
    S->x_total = x;
    S->fresh_total = f;
    S->min_next = mn;
    S->edges = e;
    S->successes = s;
    S->local_v = lv;
    tc->st_local += lv;
    tc->st_skipped += sk;
    tc->st_steps += 1;
    tc->st_extracted += x;
    tc->st_edges += e;
    tc->st_success += s;
    tc->st_dense += (flags & 1u) ? 1 : 0;
    tc->st_sampled += (flags & 4u) ? 1 : 0;
    if (flags & 1u) {
      tc->st_qdense += q;
    } else {
      tc->st_qlist += q;
    }
    if (flags & 2u) tc->st_appends += ld_agent(&S->list_next);
    tc->relax_busy_max += ~negbusy;
    tc->relax_busy_sum += busy;
    if (a.trace && tc->query == 0 && t < a.trace_cap) {
      sssp_step_record r;
      r.theta = theta;
      r.q = q;
      r.extracted = x;
      r.edges = e;
      r.successes = s;
      r.flags = flags;
      r.samples = (flags & 4u) ? (uint32_t)ld_agent(&S->nsamples) : 0u;
      r.local = lv;
      r.extract_ns = extract_ticks * a.ns_per_tick;
      r.relax_ns = (ull)(wall_clock64() - (long long)relax_start) * a.ns_per_tick;
      a.trace[t] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// Serving.

// Order-independent checksum of a distance row: the sum over v of a 64-bit
// mix of (v, delta[v]) (the SplitMix64 finaliser), modulo 2^64.
__device__ __forceinline__ ull row_mix(ull v, ull d) {
  ull z = d ^ (v * 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <class T>
__device__ __forceinline__ T ld_system(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Serving: requests are dispatched to groups of idle teams. The dispatcher
// runs under a grid lock, on the thread of whichever idle team holds it: for
// each posted request not yet taken it picks k idle teams, k the largest
// power of two (at most group_max) such that every waiting request still
// finds a team (k = idle teams / waiting requests, rounded down), but at
// least group_min: a request waits while fewer teams are idle (a finished
// group frees its teams soon, and a lone team would take many times longer);
// it copies the request out of the ring into the leader's control block,
// acknowledges the ring entry and writes each member's mailbox. Few requests
// in flight thus get most of the grid each; under load every group solves
// its own. group_min is at most the server's team count, so a request is
// dispatched at the latest once every team is idle.

__device__ bool grid_lock(const KArgs& a, unsigned* lk, bool try_once) {
  const long long t0 = wall_clock64();
  for (;;) {
    unsigned expected = 0u;
    if (__hip_atomic_compare_exchange_strong(lk, &expected, 1u, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return true;
    if (try_once) return false;
    if (__hip_atomic_load(&a.grid->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if ((ull)(wall_clock64() - t0) > a.tlimit) {
      __hip_atomic_store(&a.grid->abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

__device__ void grid_unlock(unsigned* lk) { __hip_atomic_store(lk, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT); }

// Under the lock: assign posted requests to groups of idle teams.
__device__ __noinline__ void serve_dispatch(const KArgs& a, GridCtl* gc) {
  if (ld_agent(&gc->closing)) return;
  ull fm = ld_agent(&gc->free_mask);
  while (fm) {
    const ull nq = ld_agent(&gc->next_query.v);
    const ull posted = ld_system(a.posted);
    if (posted <= nq) break;
    const ull waiting = posted - nq;
    const ull idle = (ull)__popcll(fm);
    ull k = idle / waiting;
    if (k < 1) k = 1;
    k = 1ull << (63 - __clzll((long long)k));  // a power of two
    if (k > a.group_max) k = a.group_max;
    if (k < a.group_min) {
      if (idle < a.group_min) break;  // wait for more idle teams
      k = a.group_min;
    }
    const ull e = nq % a.ring_cap;
    const int32_t src = ld_system(&a.req[2 * e]);
    const uint32_t row = (uint32_t)ld_system(&a.req[2 * e + 1]);
    __hip_atomic_store(&a.ack[e], nq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    st_agent(&gc->next_query.v, nq + 1);
    // A malformed entry (the host checks requests before posting them) is
    // acknowledged and dropped.
    if (src < 0 || src >= a.n || row >= a.nrows) continue;
    const ull leader = (ull)(__ffsll((long long)fm) - 1);
    TeamCtl* lc = a.teams + leader;
    lc->src = (ull)src;
    lc->out_row = row;
    lc->pending = nq + 1;
    lc->query = nq;
    lc->hash_acc = 0;
    const ull base = ld_agent(&lc->garrive.v);
    // Every member's mailbox and the member list first, then the sequence
    // numbers that hand the assignment over.
    for (ull i = 0; i < k; ++i) {
      const ull t = (ull)(__ffsll((long long)fm) - 1);
      fm &= fm - 1;
      lc->gteam[i] = (uint32_t)t;
      TeamCtl* mc = a.teams + t;
      mc->mb_leader = leader;
      mc->mb_k = k;
      mc->mb_idx = i;
      mc->mb_base = base;
      mc->mb_exit = 0;
    }
    for (ull i = 0; i < k; ++i) {
      TeamCtl* mc = a.teams + lc->gteam[i];
      __hip_atomic_store(&mc->mb_seq, ld_agent(&mc->mb_seq) + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  st_agent(&gc->free_mask, fm);
}

// Serial part of a serving team's wait (thread 0 of the last workgroup of
// the team at its own barrier): register the team as idle, dispatch, then
// wait for its mailbox. Leaves mb_exit = 1 when the team is to leave: the
// host closed the ring and every posted request is taken, the team waited
// longer than the idle limit (the launch then takes no more requests: the
// closing word is set here and in host memory), or the abort flag is up.
__device__ __noinline__ void serve_wait(const KArgs& a, GridCtl* gc, ull me) {
  TeamCtl* tc = a.teams + me;
  const ull bit = 1ull << me;
  const ull seq0 = ld_agent(&tc->mb_seq);
  if (!grid_lock(a, &gc->lock, false)) {
    tc->mb_exit = 1;
    return;
  }
  st_agent(&gc->free_mask, ld_agent(&gc->free_mask) | bit);
  serve_dispatch(a, gc);
  grid_unlock(&gc->lock);
  const long long t0 = wall_clock64();
  for (unsigned spin = 0;; ++spin) {
    if (__hip_atomic_load(&tc->mb_seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != seq0) return;
    const bool aborted = __hip_atomic_load(&gc->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const bool idle = (ull)(wall_clock64() - t0) > a.idle_ticks;
    const bool closed = ld_system(a.closed) != 0;
    if (aborted || idle || closed || (spin & 7) == 0) {
      if (grid_lock(a, &gc->lock, !(aborted || idle || closed))) {
        if (__hip_atomic_load(&tc->mb_seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != seq0) {
          grid_unlock(&gc->lock);
          return;
        }
        serve_dispatch(a, gc);
        bool leave = aborted;
        if (__hip_atomic_load(&tc->mb_seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == seq0) {
          // posted is written before closed, so once closed is seen a
          // posted count at or below the next ticket means nothing is left.
          if (closed && ld_system(a.posted) <= ld_agent(&gc->next_query.v)) leave = true;
          if (ld_agent(&gc->closing)) leave = true;
          if (idle) {
            st_agent(&gc->closing, 1ull);
            __hip_atomic_store(a.dev_closed, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            leave = true;
          }
        } else {
          leave = false;  // assigned by the dispatch above
        }
        if (leave) {
          st_agent(&gc->free_mask, ld_agent(&gc->free_mask) & ~bit);
          tc->mb_exit = 1;
        }
        grid_unlock(&gc->lock);
        if (leave || __hip_atomic_load(&tc->mb_seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != seq0) return;
      } else if (aborted || idle || closed) {
        // The lock wait itself gave up (abort): leave without it.
        tc->mb_exit = 1;
        return;
      }
    }
    __builtin_amdgcn_s_sleep(32);
  }
}

// Serial part of a serving group's last barrier for a request: its row (and
// checksum) first, then the row's completion word, in host-visible order.
__device__ __noinline__ void serve_publish(const KArgs& a, TeamCtl* lc) {
  if (!lc->pending) return;
  const ull t = lc->pending - 1, row = lc->out_row;
  const ull h = ld_agent(&lc->hash_acc);
  lc->hash_acc = 0;
  lc->pending = 0;
  __hip_atomic_store(&a.hashes[row], h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&a.done[row], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Point a workgroup's Team at the per-team workspace and control block of
// team `t` (its own, or its group's leader when serving).
__device__ __forceinline__ void bind_workspace(const KArgs& a, Team& tm, ull t) {
  tm.id = t;
  tm.ctl = a.teams + t;
  tm.bitmap = a.bitmap + t * a.nwords;
  tm.hint = a.hint ? a.hint + t * (ull)a.n : nullptr;
  tm.lastkey = a.lastkey ? a.lastkey + t * (ull)a.n : nullptr;
  tm.ckey = a.ckey ? a.ckey + t * a.hcap : nullptr;
  tm.key1 = a.key1 ? a.key1 + t * a.nwords : nullptr;
  tm.key2 = a.key1 ? a.key2 + t * a.n2 : nullptr;
  tm.H = a.H + t * 2 * a.hcap;
  tm.L = a.L + t * 2 * a.lcap;
  tm.samples = a.samples + t * a.probe_cap;
}

// ---------------------------------------------------------------------------
// The persistent kernel.

// S0 over the team's share: delta = inf, key bounds unknown, queue empty.
__device__ __noinline__ void phase_init(const KArgs& a, ull* dist) {
  const Team& tm = g_tm;
  const unsigned tid = threadIdx.x;
  const ull n = (ull)a.n, first = tm.rank * WG + tid, stride = tm.T * WG;
  for (ull i = first; i < n; i += stride) dist[i] = INF;
  if (tm.hint)
    for (ull i = first; i < n; i += stride) tm.hint[i] = HINT_NONE;
  if (tm.lastkey)
    for (ull i = first; i < n; i += stride) tm.lastkey[i] = INF;
  if (tm.ckey)
    for (ull i = first; i < a.hcap; i += stride) tm.ckey[i] = INF;
  if (tm.key1) {
    for (ull i = first; i < a.nwords; i += stride) tm.key1[i] = INF;
    for (ull i = first; i < a.n2; i += stride) tm.key2[i] = INF;
  }
  for (ull i = first; i < a.nwords; i += stride) tm.bitmap[i] = 0;
}

// Serial part of the init barrier: clear the step slots and selection state,
// then delta[s] = 0 and Update(s).
__device__ __noinline__ void seed_source(const KArgs& a, ull* dist, ull qi) {
  const Team& tm = g_tm;
  const unsigned tid = threadIdx.x;
  if (tid < 48) reinterpret_cast<ull*>(&tm.ctl->slot[0])[tid] = 0ull;
  tm.ctl->sel_hist[tid] = 0;
  if (tid == 0) {
    tm.ctl->sel_min = INF;
    tm.ctl->sel_max = INF;
    const int32_t src = a.serve ? (int32_t)tm.ctl->src : a.srcs[qi];
    const int32_t s = a.inv ? a.inv[src] : src;
    dist[s] = 0;
    if (tm.hint) tm.hint[s] = 0;
    if (tm.key1) {
      tm.key1[s >> 6] = 0;
      tm.key2[s >> 12] = 0;
    }
    tm.bitmap[s >> 6] = 1ull << (s & 63);
    tm.L[0] = s;
  }
}

// Distances back in the caller's vertex ids, and the row checksum added to
// the team's accumulator.
__device__ __noinline__ void phase_copyout(const KArgs& a, const ull* dist, ull* out) {
  const Team& tm = g_tm;
  const unsigned tid = threadIdx.x;
  const ull n = (ull)a.n;
  ull h = 0;
  if (a.dist_int) {
    for (ull v = tm.rank * WG + tid; v < n; v += tm.T * WG) {
      const ull d = ld_agent(&dist[a.inv[v]]);
      out[v] = d;
      if (a.hash) h += row_mix(v, d);
    }
  } else if (a.hash) {
    for (ull v = tm.rank * WG + tid; v < n; v += tm.T * WG) h += row_mix(v, ld_agent(&out[v]));
  }
  if (a.hash) {
    h = wave_sum(h);
    if (lane_id() == 0) atom_add(&tm.ctl->hash_acc, h);
  }
}

// Serving: join the group of this team's new assignment (leader's workspace,
// group ranks in g_tm). Whole workgroup. Returns the group barrier's second
// level (by value: a reference to the kernel's barrier state would keep it
// in scratch memory), or ok = false when the team is to leave.
struct Join {
  bool ok;
  ull* l2_arrive;
  ull* l2_gen;
  ull l2_size, l2_base;
};

__device__ __noinline__ Join serve_join(const KArgs& a, bool grouped) {
  Team tm = g_tm;
  const TeamCtl* mine = a.teams + tm.own;
  const bool leave = ld_agent(&mine->mb_exit) != 0;
  Join br{!leave, nullptr, nullptr, 0, 0};
  if (!leave) {
    const ull own_rank = (ull)blockIdx.x / a.nteams;
    const ull leader = ld_agent(&mine->mb_leader);
    tm.k = ld_agent(&mine->mb_k);
    tm.T = tm.k * tm.Tteam;
    tm.rank = ld_agent(&mine->mb_idx) * tm.Tteam + own_rank;
    bind_workspace(a, tm, leader);
    if (grouped && tm.k > 1) {
      br.l2_arrive = &tm.ctl->garrive.v;
      br.l2_gen = &tm.ctl->ggen.v;
      br.l2_size = tm.k;
      br.l2_base = ld_agent(&mine->mb_base);
    }
  }
  __syncthreads();
  if (!leave && threadIdx.x == 0) g_tm = tm;
  __syncthreads();
  return br;
}

__global__ __launch_bounds__(WG, 4) void stepping_kernel(const KArgs* __restrict__ A) {
  Shared& sh = g_sh;
  const KArgs& a = *A;
  const unsigned tid = threadIdx.x;
  const ull b = blockIdx.x;
  const ull n = (ull)a.n;
  GridCtl* gc = a.grid;
  const unsigned xcc = __builtin_amdgcn_s_getreg(20 | (15 << 11)) & (MAX_XCC - 1);  // hwreg XCC_ID
  const ull own_rank = b / a.nteams, own = b % a.nteams;
  // The team's state lives in LDS (g_tm), read where it is needed; only the
  // barrier state stays in registers across the phases.
  const Team& tm = g_tm;
  if (tid == 0) {
    Team t0;
    t0.own = own;
    t0.rank = own_rank;
    t0.Tteam = a.G / a.nteams;
    t0.T = t0.Tteam;
    t0.k = 1;
    bind_workspace(a, t0, own);
    t0.Fb = a.F + b * a.segcap;
    t0.FDb = a.FD + b * a.segcap;
    g_tm = t0;
  }
  Bar br;
  br.epoch = 0;
  br.l2_epoch = 0;
  br.l2_base = 0;
  // Serving with several teams: each request is solved by a group of teams
  // (see serve_dispatch); a team alone meets on its own barrier only.
  const bool grouped = a.serve && a.nteams > 1;

  // Phase clock: the team's first workgroup reads the wall clock as it
  // leaves each barrier.
  ull ph0 = 0, ph1 = 0, ph2 = 0, ph3 = 0;
  long long tmark = wall_clock64();
  auto lap = [&]() {
    const long long now = wall_clock64();
    const ull d = (ull)(now - tmark);
    tmark = now;
    return d;
  };

  // Register the XCD, check the round-robin placement, meet once.
  if (tid == 0) {
    atom_add(&gc->grp_size[xcc].v, 1ull);
    if (xcc != (unsigned)(b % 8)) atom_add(&gc->mismatch.v, 1ull);
  }
  {
    auto count_groups = [&]() {
      if (tid == 0) {
        ull g = 0;
        for (int x = 0; x < MAX_XCC; ++x) g += gc->grp_size[x].v ? 1 : 0;
        gc->ngroups = g;
      }
    };
    if (!flat_sync(a, sh, count_groups)) return;
  }
  if (a.nteams == 1) {
    br.l1_arrive = &gc->grp_arrive[xcc].v;
    br.l1_gen = &gc->grp_gen[xcc].v;
    br.l1_size = ld_agent(&gc->grp_size[xcc].v);
    br.l2_arrive = &gc->arrive.v;
    br.l2_gen = &gc->gen.v;
    br.l2_size = ld_agent(&gc->ngroups);
    br.member_release = false;
  } else {
    TeamCtl* oc = a.teams + own;
    br.l1_arrive = &oc->arrive.v;
    br.l1_gen = &oc->gen.v;
    br.l1_size = a.G / a.nteams;
    br.l2_arrive = nullptr;
    br.l2_gen = nullptr;
    br.l2_size = 0;
    // Teams inside one XCD share an L2 unless the placement is unexpected.
    br.member_release = (a.nteams % 8 != 0) || ld_agent(&gc->mismatch.v) != 0;
  }
  ph0 += lap();

  for (;;) {
    ull qi;
    if (a.serve) {
      // Serving: this team alone becomes idle and waits for its next
      // assignment, then joins its group.
      if (grouped) {
        br.l2_arrive = nullptr;
        br.l2_gen = nullptr;
        br.l2_size = 0;
      }
      auto wait = [&]() {
        if (tid == 0) serve_wait(a, gc, own);
      };
      if (!team_sync(a, sh, br, wait)) return;
      const Join j = serve_join(a, grouped);
      if (!j.ok) break;
      if (j.l2_arrive) {
        br.l2_arrive = j.l2_arrive;
        br.l2_gen = j.l2_gen;
        br.l2_size = j.l2_size;
        br.l2_base = j.l2_base;
        br.l2_epoch = 0;
      }
      qi = ld_agent(&tm.ctl->query);
    } else {
      // Take the next source.
      auto claim = [&]() {
        if (tid == 0)
          tm.ctl->query = (a.cancel && ld_agent(&gc->cancelled)) ? (ull)a.n_src : atom_add(&gc->next_query.v, 1ull);
      };
      if (!team_sync(a, sh, br, claim)) return;
      qi = ld_agent(&tm.ctl->query);
      if (qi >= (ull)a.n_src) break;
    }
    ull* out = a.dist_out + (a.serve ? ld_agent(&tm.ctl->out_row) : qi) * n;
    ull* dist = a.dist_int ? a.dist_int + tm.id * n : out;

    // S0: delta = inf, Q empty; then delta[s] = 0 and Update(s).
    phase_init(a, dist);
    {
      auto seed = [&]() { seed_source(a, dist, qi); };
      if (!team_sync(a, sh, br, seed)) return;
      ph0 += lap();
    }

    ull q = 1, minq = 0, idelta = 0, large_steps = 0;
    // Serving groups: rho and Delta are given per team, so a group of k
    // teams extracts k times as much per step (its work per step grows with
    // its workgroups; a lone team with the group's parameters would take
    // many serial hops per step).
    ull rho = a.rho, delta = a.delta;
    if (a.serve) {
      if (__builtin_mul_overflow(a.rho, tm.k, &rho)) rho = INF;
      if (__builtin_mul_overflow(a.delta, tm.k, &delta)) delta = INF;
    }
    // Vertices relaxed and arcs of the previous step (before the first: the
    // whole graph, so that the first step is super-sparse when the graph is).
    ull prev_x = n, prev_e = a.m;
    bool list_valid = true;

    for (ull t = 0;; ++t) {
      const long long t_step = wall_clock64();
      if (q == 0) break;
      if (a.max_steps && t >= a.max_steps) {
        if (tm.rank == 0 && tid == 0) tm.ctl->status |= ST_STEP_LIMIT;
        break;
      }
      StepSlot* S = &tm.ctl->slot[t % 3];
      int32_t* Lcur = tm.L + ((t & 1) ? a.lcap : 0);
      int32_t* Lnext = tm.L + ((t & 1) ? 0 : a.lcap);
      const bool dense = !list_valid;
      const bool emit = q <= a.list_threshold;

      // ---- S1: ExtDist ----
      ull theta = INF;
      ull theta_h = INF;  // set in sampled rho steps with hub deferral; else theta
      bool sampled = false, exact = false;
      if (a.rule == SSSP_RULE_BF) {
        theta = INF;
      } else if (a.rule == SSSP_RULE_MIN) {
        theta = minq;
      } else if (a.rule == SSSP_RULE_DELTA_STAR) {
        ull i = idelta + 1;
        const ull skip = minq / delta + (minq % delta != 0);  // ceil(min / Delta)
        if (skip > i) i = skip;
        idelta = i;
        ull prod;
        theta = __builtin_mul_overflow(i, delta, &prod) ? INF : prod;
      } else if (a.rule == SSSP_RULE_RHO_EXACT) {
        if (q > rho) {
          // Exact rho-th smallest key: a bounds pass, then 8-bit digit passes.
          exact = true;
          phase_select(a, dist, Lcur, q, dense, true, 64, 0, 0, 0);
          auto start = [&]() {
            if (tid == 0) select_serial(tm.ctl, true, 0, rho);
          };
          if (!team_sync(a, sh, br, start)) return;
          int top = (int)ld_agent(&tm.ctl->sel_top);
          while (top > 0) {
            const int width = top < 8 ? top : 8;
            const int shift = top - width;
            const ull prefix = ld_agent(&tm.ctl->sel_prefix);
            phase_select(a, dist, Lcur, q, dense, false, top, shift, (1ull << width) - 1, prefix);
            auto pick = [&]() {
              if (tid == 0) select_serial(tm.ctl, false, shift, 0);
            };
            if (!team_sync(a, sh, br, pick)) return;
            top = shift;
          }
          theta = ld_agent(&tm.ctl->sel_prefix);
          ph1 += lap();
        }
      } else {
        // The first two steps whose queue exceeds rho / 10 use rho / 10 (Sec. 6
        // lowers rho for the first large steps, whose threshold estimates are
        // the least accurate).
        const ull rho10 = (rho / 10) > 0 ? rho / 10 : 1;
        const ull rho_eff = large_steps < 2 ? rho10 : rho;
        if (q > rho10) ++large_steps;
        if (q > rho_eff) {
          sampled = true;
          const ull probes = rho_probes(q, rho_eff, n, dense, a.sample_cap, a.probe_cap);
          phase_sample(a, dist, S, Lcur, q, dense, probes, splitmix(a.seed ^ qi, t));
          auto choose = [&]() {
            const ull s = ld_agent(&S->nsamples);
            ull th = INF, th_h = INF;
            if (s > 0) {
              ull k = (rho_eff * s + q - 1) / q;  // ceil(rho * s / q)
              if (k < 1) k = 1;
              if (k > s) k = s;
              th = wg_select_kth(tm.samples, s, k);
              th_h = th;
              if (a.ndefer) {
                // Hub deferral: the (rho / defer_div)-th smallest key of the same sample.
                const ull rho_h = rho_eff / a.defer_div > 0 ? rho_eff / a.defer_div : 1;
                ull kh = (rho_h * s + q - 1) / q;
                if (kh < 1) kh = 1;
                if (kh < k) th_h = wg_select_kth(tm.samples, s, kh);
              }
            }
            if (tid == 0) {
              tm.ctl->theta = th;
              tm.ctl->theta_h = th_h;
            }
          };
          if (!team_sync(a, sh, br, choose)) return;
          ph1 += lap();
          theta = ld_agent(&tm.ctl->theta);
          theta_h = ld_agent(&tm.ctl->theta_h);
        }
      }

      // ---- S2: Extract(theta) over this workgroup's slice ----
      const bool tree = tm.key1 != nullptr;
      const Thresh th{theta, sampled ? umin(theta_h, theta) : theta, sampled ? a.ndefer : 0};
      const ExtractOut ex = tree          ? phase_extract_tree(a, dist, S, th)
                            : !dense       ? phase_extract_list(a, dist, S, Lcur, Lnext, q, th, emit)
                            : emit        ? phase_extract_dense(a, dist, S, Lnext, th, emit)
                            : q * 4 >= n  ? phase_extract_dense_words(a, dist, S, th)
                                          : phase_extract_dense_fast(a, dist, S, th);
      if (!team_sync(a, sh, br, NoSerial{})) return;
      ph2 += lap();
      const long long t_relax = wall_clock64();

      // ---- S3/S4: Relax + Update ----
      // Local expansion in super-sparse steps: list steps whose previous
      // step relaxed fewer than super_sparse arcs per vertex on average.
      const bool sparse = tree ? q <= a.sparse_q : !dense;
      const bool local = a.local_budget && sparse && prev_e < (ull)a.super_sparse * umin(prev_x, INF / 64);
      phase_relax(a, dist, S, Lnext, emit, ex, local, theta);
      const unsigned flags = (dense ? 1u : 0u) | (emit ? 2u : 0u) | (sampled ? 4u : 0u) | (exact ? 8u : 0u);
      auto bookkeeping = [&]() {
        step_bookkeeping(a, S, t, q, theta, flags, (ull)(t_relax - t_step), (ull)t_relax);
        if (a.cancel && tid == 0 && ld_system(a.cancel) != 0u) {
          tm.ctl->status |= ST_CANCELLED;
          __hip_atomic_store(&gc->cancelled, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      };
      if (!team_sync(a, sh, br, bookkeeping)) return;
      ph3 += lap();
      if (a.cancel && (ld_agent(&tm.ctl->status) & ST_CANCELLED)) break;

      // ---- S5: next queue state, identical in every workgroup of the team ----
      q = q - ld_agent(&S->x_total) + ld_agent(&S->fresh_total);
      minq = ld_agent(&S->min_next);
      prev_x = ld_agent(&S->x_total) + ld_agent(&S->local_v);
      prev_e = ld_agent(&S->edges);
      list_valid = emit && ld_agent(&S->list_next) <= a.lcap;
    }
    phase_copyout(a, dist, out);
    if (a.serve) {
      // The group's last barrier for this request publishes it; the row must
      // be visible outside the device (system scope) first.
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      auto publish = [&]() {
        if (tid == 0) serve_publish(a, tm.ctl);
      };
      if (!team_sync(a, sh, br, publish)) return;
    }
  }
  if (own_rank == 0 && tid == 0) {
    TeamCtl* pc = a.teams + own;
    pc->phase_ticks[0] += ph0;
    pc->phase_ticks[1] += ph1;
    pc->phase_ticks[2] += ph2;
    pc->phase_ticks[3] += ph3;
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

// First chunk index of every hub (out-degree above hub_degree) in the
// per-chunk key array: an exclusive prefix sum of ceil(degree / chunk) over
// the hubs, which a graph numbered by decreasing degree holds first. One
// workgroup of 1024 threads; stops at the first block holding a vertex that
// is not a hub, and writes the hub count to *nhub.
__global__ __launch_bounds__(1024) void chunk_base_kernel(const int64_t* off, ull n, uint32_t hub_degree,
                                                         uint32_t chunk, uint32_t* cbase, ull* nhub) {
  __shared__ uint32_t wsum[16];
  __shared__ int any_small;
  const unsigned tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t base = 0;
  ull hubs = 0;
  for (ull b0 = 0; b0 < n; b0 += 1024) {
    const ull v = b0 + tid;
    const ull deg = v < n ? (ull)(off[v + 1] - off[v]) : 0;
    const bool is_hub = v < n && deg > hub_degree;
    const uint32_t c = is_hub ? (uint32_t)((deg + chunk - 1) / chunk) : 0u;
    uint32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if ((int)lane >= o) incl += y;
    }
    if (tid == 0) any_small = 0;
    __syncthreads();
    if (lane == 63) wsum[wave] = incl;
    if (v < n && !is_hub) any_small = 1;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (unsigned w = 0; w < 16; ++w) {
      before += w < wave ? wsum[w] : 0u;
      total += wsum[w];
    }
    if (is_hub) cbase[v] = base + before + incl - c;
    base += total;
    const int stop = any_small;
    ull cnt = is_hub ? 1 : 0;
    hubs += (ull)__syncthreads_count((int)cnt);
    if (stop) break;
  }
  if (tid == 0) *nhub = hubs;
}

// Zero the control blocks before a solve (a kernel rather than a memset, so
// the sequence stays valid under stream capture).
__global__ void reset_control_kernel(ull* p, ull words) {
  for (ull i = (ull)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (ull)gridDim.x * blockDim.x) p[i] = 0;
}

sssp_tuning default_tuning() {
  sssp_tuning t;
  std::memset(&t, 0, sizeof(t));
  t.blocks_per_cu = 4;
  t.hub_degree = 1024;
  t.chunk_edges = 4096;
  t.list_divisor = 64;
  t.sample_cap = 1u << 16;
  t.probe_cap = 1u << 16;
  t.no_filter = 0;
  t.teams = 0;
  t.local_budget = 4096;
  t.super_sparse_degree = 10;
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
  if (!t.local_budget) t.local_budget = d.local_budget;
  if (!t.super_sparse_degree) t.super_sparse_degree = d.super_sparse_degree;
  return t;
}

// Out-degree above which a vertex is not relaxed by local expansion (eight
// times the super-sparse average degree, at most the hub degree).
uint32_t local_degree_cap(const sssp_tuning& tu) {
  return std::min<uint32_t>(tu.hub_degree, 8u * std::min<uint32_t>(tu.super_sparse_degree, 1u << 20));
}

// Workspace geometry of one solve.
struct Geometry {
  uint32_t G, nteams, T;
  uint64_t nwords, segcap, hcap, lcap;
};

constexpr uint64_t TEAM_SEGMENT_CAP = 1ull << 16;  // F entries per workgroup when teams share the grid
constexpr uint64_t TEAM_LIST_CAP = 1ull << 20;     // explicit-list entries per team when teams share the grid

Geometry make_geometry(const sssp_graph* g, const sssp_tuning& tu, uint32_t G, uint32_t nteams) {
  Geometry geo;
  geo.G = G;
  geo.nteams = nteams;
  geo.T = G / nteams;
  const uint64_t n = (uint64_t)g->n, m = (uint64_t)g->m;
  geo.nwords = (n + 63) / 64;
  // A workgroup extracts at most the vertices of the blocks it owns (bitmap
  // steps) or of its list slice (list steps, at most ceil(n / T)).
  const uint64_t nblocks = (geo.nwords + BLOCK_WORDS - 1) / BLOCK_WORDS;
  geo.segcap = 64ull * BLOCK_WORDS * ((nblocks + geo.T - 1) / geo.T);
  if (tu.queue == 1) {
    // Tournament tree: a workgroup owns whole level-2 nodes of 4096 vertices.
    const uint64_t n2 = (geo.nwords + 63) / 64;
    geo.segcap = std::max<uint64_t>(geo.segcap, 4096ull * ((n2 + geo.T - 1) / geo.T));
  }
  // Each vertex is extracted at most once per step and an extracted hub
  // contributes ceil(deg / chunk) tasks: m / chunk + m / (hub_degree + 1) + 1
  // bounds the tasks of one step.
  geo.hcap = m / tu.chunk_edges + m / ((uint64_t)tu.hub_degree + 1) + 2;
  geo.lcap = n;
  if (nteams > 1) {
    geo.segcap = std::min<uint64_t>(geo.segcap, TEAM_SEGMENT_CAP);
    geo.lcap = std::min<uint64_t>(n, TEAM_LIST_CAP);
  }
  return geo;
}

uint64_t control_words(uint32_t nteams) { return (sizeof(GridCtl) + (uint64_t)nteams * sizeof(TeamCtl)) / 8; }

// Device addresses of one launch's workspace: the graph's own buffers
// (ensure_workspace) or slices of the static scratch array (carve_scratch).
struct WsView {
  void *dist_int, *bitmap, *hint, *tree, *hubmask, *bigmask, *F, *FD, *H, *L, *samples, *parts, *ctl, *args, *srcs;
};

WsView graph_view(const sssp_graph* g) {
  return WsView{g->dist_int.p, g->bitmap.p, g->hint.p, g->tree.p, g->hubmask.p, g->bigmask.p, g->F.p, g->FD.p,
                g->H.p,        g->L.p,      g->samples.p, g->parts.p, g->ctl.p,  g->args.p, g->srcs.p};
}

// Sizes in bytes of the workspace arrays of a launch, in WsView order.
void workspace_sizes(const sssp_graph* g, const sssp_tuning& tu, const Geometry& geo, uint64_t n_src,
                     uint64_t (&sz)[15]) {
  const uint64_t n = (uint64_t)g->n, nt = geo.nteams;
  sz[0] = g->relabelled ? nt * n * 8 : 0;                            // dist_int
  sz[1] = nt * geo.nwords * 8;                                       // bitmap
  sz[2] = nt * n * 2;                                                // hint
  sz[3] = nt * (geo.nwords + (geo.nwords + 63) / 64) * 8;            // tree
  sz[4] = geo.nwords * 8;                                            // hubmask
  sz[5] = geo.nwords * 8;                                            // bigmask
  sz[6] = (uint64_t)geo.G * geo.segcap * 4;                          // F
  sz[7] = (uint64_t)geo.G * geo.segcap * 8;                          // FD
  sz[8] = nt * geo.hcap * 16;                                        // H
  sz[9] = nt * 2 * geo.lcap * 4;                                     // L
  sz[10] = nt * (uint64_t)tu.probe_cap * 8;                          // samples
  sz[11] = (uint64_t)geo.G * sizeof(Part);                           // parts
  sz[12] = control_words(geo.nteams) * 8;                            // ctl
  sz[13] = sizeof(KArgs);                                            // args
  sz[14] = n_src * 4;                                                // srcs
}

// Hub flags (out-degree above hub_degree) and local-expansion flags (above
// the local degree cap), one bit per vertex.
hipError_t build_masks(const sssp_graph* g, const sssp_tuning& tu, const Geometry& geo, void* hubmask,
                       void* bigmask, hipStream_t st) {
  const uint64_t n = (uint64_t)g->n;
  hubmask_kernel<<<1024, 256, 0, st>>>((const int64_t*)g->off.p, n, geo.nwords, tu.hub_degree, (ull*)hubmask);
  hubmask_kernel<<<1024, 256, 0, st>>>((const int64_t*)g->off.p, n, geo.nwords, local_degree_cap(tu),
                                       (ull*)bigmask);
  return hipGetLastError();
}

sssp_status ensure_workspace(sssp_graph* g, const sssp_tuning& tu, const Geometry& geo, bool repeat,
                             hipStream_t st) {
  if (g->ws_ready && g->ws_hub_degree == tu.hub_degree && g->ws_chunk == tu.chunk_edges &&
      g->ws_probe_cap >= tu.probe_cap && g->ws_G == geo.G && g->ws_teams == geo.nteams && g->ws_segcap == geo.segcap &&
      g->ws_local_cap == local_degree_cap(tu) && g->ws_repeat == repeat)
    return SSSP_OK;
  g->release_ws(st);
  const uint64_t n = (uint64_t)g->n, nt = geo.nteams;
  if (g->relabelled) SSSP_HIP_TRY(g->dist_int.alloc(nt * n * 8, st));
  SSSP_HIP_TRY(g->bitmap.alloc(nt * geo.nwords * 8, st));
  SSSP_HIP_TRY(g->hint.alloc(nt * n * 2, st));
  SSSP_HIP_TRY(g->tree.alloc(nt * (geo.nwords + (geo.nwords + 63) / 64) * 8, st));
  SSSP_HIP_TRY(g->hubmask.alloc(geo.nwords * 8, st));
  SSSP_HIP_TRY(g->bigmask.alloc(geo.nwords * 8, st));
  SSSP_HIP_TRY(g->F.alloc((uint64_t)geo.G * geo.segcap * 4, st));
  SSSP_HIP_TRY(g->FD.alloc((uint64_t)geo.G * geo.segcap * 8, st));
  SSSP_HIP_TRY(g->H.alloc(nt * geo.hcap * 16, st));
  SSSP_HIP_TRY(g->L.alloc(nt * 2 * geo.lcap * 4, st));
  SSSP_HIP_TRY(g->samples.alloc(nt * (uint64_t)tu.probe_cap * 8, st));
  SSSP_HIP_TRY(g->parts.alloc((uint64_t)geo.G * sizeof(Part), st));
  SSSP_HIP_TRY(g->ctl.alloc(control_words(geo.nteams) * 8, st));
  SSSP_HIP_TRY(g->args.alloc(sizeof(KArgs), st));
  if (!g->hargs) {
    g->hargs = ::operator new(sizeof(KArgs), std::nothrow);
    if (!g->hargs) return fail(SSSP_ERR_OUT_OF_MEMORY, "kernel argument staging");
  }
  SSSP_HIP_TRY(build_masks(g, tu, geo, g->hubmask.p, g->bigmask.p, st));
  if (repeat) {
    SSSP_HIP_TRY(g->lastkey.alloc(nt * n * 8, st));
    if (g->relabelled) {
      // Hub chunks have keys of their own; hubs are numbered first.
      SSSP_HIP_TRY(g->ckey.alloc(nt * geo.hcap * 8, st));
      // nhub <= m / (hub_degree + 1) entries, then the hub count (8-byte aligned).
      const uint64_t cb_bytes = ((uint64_t)g->m / ((uint64_t)tu.hub_degree + 1) + 2) * 4;
      const uint64_t cnt_off = (cb_bytes + 7) / 8 * 8;
      SSSP_HIP_TRY(g->cbase.alloc(cnt_off + 8, st));
      uint64_t* cnt = reinterpret_cast<uint64_t*>((char*)g->cbase.p + cnt_off);
      chunk_base_kernel<<<1, 1024, 0, st>>>((const int64_t*)g->off.p, n, tu.hub_degree, tu.chunk_edges,
                                            (uint32_t*)g->cbase.p, (ull*)cnt);
      SSSP_HIP_TRY(hipGetLastError());
      uint64_t nh = 0;
      SSSP_HIP_TRY(hipMemcpyAsync(&nh, cnt, 8, hipMemcpyDeviceToHost, st));
      SSSP_HIP_TRY(hipStreamSynchronize(st));
      g->nhub = nh;
    }
  }
  g->ws_repeat = repeat;
  g->ws_ready = true;
  g->ws_hub_degree = tu.hub_degree;
  g->ws_chunk = tu.chunk_edges;
  g->ws_probe_cap = tu.probe_cap;
  g->ws_G = geo.G;
  g->ws_teams = geo.nteams;
  g->ws_segcap = geo.segcap;
  g->ws_local_cap = local_degree_cap(tu);
  return SSSP_OK;
}

// Teams for n_src sources when the caller leaves it to the library: one
// whole-grid team for a single source, otherwise the smallest power of two
// >= 8 (so that each team sits on one XCD) that covers the sources, as long
// as it divides the grid.
uint32_t auto_teams(int32_t n_src, uint32_t G) {
  if (n_src <= 1 || G % 8 != 0) return 1;
  uint32_t t = 8;
  while (t < (uint32_t)n_src && G % (2 * t) == 0) t <<= 1;
  return t;
}


// Shared set-up of a launch: parameter checks, grid, teams, workspace and the
// kernel arguments (everything but the source list and the serving ring).
struct Launch {
  sssp_params p;
  sssp_tuning tu;
  uint32_t G = 0, nteams = 0;
  Geometry geo;
  KArgs a;
};

sssp_status check_params(const sssp_params* params, sssp_params& p, sssp_tuning& tu) {
  if (params) {
    p = *params;
  } else {
    sssp_default_params(&p);
  }
  if (p.rule > SSSP_RULE_RHO_EXACT) return fail(SSSP_ERR_INVALID_ARGUMENT, "unknown rule");
  if (p.flags & ~SSSP_SOLVE_SNAPSHOT_KEYS) return fail(SSSP_ERR_INVALID_ARGUMENT, "unknown flags");
  if ((p.rule == SSSP_RULE_RHO || p.rule == SSSP_RULE_RHO_EXACT) && p.rho == 0)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "rho must be >= 1");
  if (p.rule == SSSP_RULE_DELTA_STAR && p.delta == 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "delta must be >= 1");
  if (p.trace && p.trace_capacity == 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "trace needs trace_capacity > 0");
  tu = resolve_tuning(p.tuning);
  if (tu.chunk_edges < 64) return fail(SSSP_ERR_INVALID_ARGUMENT, "chunk_edges must be >= 64");
  if (tu.hub_degree > (1u << 22)) return fail(SSSP_ERR_INVALID_ARGUMENT, "hub_degree must be <= 2^22");
  if (tu.sample_cap > tu.probe_cap) return fail(SSSP_ERR_INVALID_ARGUMENT, "sample_cap must be <= probe_cap");
  if (tu.queue > 1) return fail(SSSP_ERR_INVALID_ARGUMENT, "queue must be 0 (flat array) or 1 (tournament tree)");
  // Tournament tree: vertices above 64 arcs are relaxed as shared hub chunks
  // (a workgroup extracts 4096 consecutive, similar-degree vertices).
  if (tu.queue == 1) tu.hub_degree = std::min(tu.hub_degree, 64u);
  return SSSP_OK;
}

// Grid, teams and workspace geometry of a launch.
sssp_status plan_launch(sssp_graph* g, Launch& L, uint32_t default_teams) {
  SSSP_HIP_TRY(hipSetDevice(g->device));
  int occ = 0;
  SSSP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stepping_kernel, WG, 0));
  if (occ < 1) return fail(SSSP_ERR_NO_DEVICE, "stepping kernel cannot be resident");
  const uint32_t bpc = std::min<uint32_t>(L.tu.blocks_per_cu, (uint32_t)occ);
  L.G = bpc * (uint32_t)g->cus;
  L.nteams = L.tu.teams ? L.tu.teams : default_teams;
  if (L.nteams > L.G || L.G % L.nteams != 0)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "teams must divide the grid of " + std::to_string(L.G) + " workgroups");
  L.geo = make_geometry(g, L.tu, L.G, L.nteams);
  if (L.tu.pull == 1 && !g->undirected)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "pull = 1 needs a graph created with SSSP_UNDIRECTED");
  return SSSP_OK;
}

// Kernel arguments of a planned launch over workspace `w`.
void fill_args(const sssp_graph* g, Launch& L, const WsView& w, uint64_t* dist) {
  const sssp_params& p = L.p;
  const sssp_tuning& tu = L.tu;
  const Geometry& geo = L.geo;
  KArgs& a = L.a;
  std::memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.m = (uint64_t)g->m;
  a.nwords = geo.nwords;
  a.off = (const int64_t*)g->off.p;
  a.edges = g->borrowed ? nullptr : (const ull*)g->edges.p;
  a.tgt = g->btgt;
  a.wt = g->bwt;
  a.perm = g->relabelled ? (const int32_t*)g->perm.p : nullptr;
  a.inv = g->relabelled ? (const int32_t*)g->inv.p : nullptr;
  a.dist_out = (ull*)dist;
  a.dist_int = g->relabelled ? (ull*)w.dist_int : nullptr;
  a.bitmap = (ull*)w.bitmap;
  a.hubmask = (const ull*)w.hubmask;
  a.bigmask = (const ull*)w.bigmask;
  a.F = (int32_t*)w.F;
  a.FD = (ull*)w.FD;
  a.H = (ull*)w.H;
  a.L = (int32_t*)w.L;
  a.samples = (ull*)w.samples;
  a.parts = (Part*)w.parts;
  a.grid = (GridCtl*)w.ctl;
  a.teams = (TeamCtl*)((char*)w.ctl + sizeof(GridCtl));
  a.srcs = (const int32_t*)w.srcs;
  a.xcount = p.extract_counts;
  a.trace = p.trace;
  a.trace_cap = p.trace ? p.trace_capacity : 0;
  a.rho = p.rho;
  a.delta = p.delta ? p.delta : 1;
  a.seed = p.seed;
  a.max_steps = p.max_steps;
  a.list_threshold = tu.list_divisor == 0xFFFFFFFFu ? 0 : std::max<uint64_t>(1, (uint64_t)g->n / tu.list_divisor);
  a.list_threshold = std::min<uint64_t>(a.list_threshold, geo.lcap);
  if (tu.queue == 1) {
    // The tournament tree replaces the explicit list as well as the scan;
    // local expansion keeps the list's notion of a small queue.
    a.sparse_q = a.list_threshold;
    a.list_threshold = 0;
    a.n2 = (geo.nwords + 63) / 64;
    a.key1 = (ull*)w.tree;
    a.key2 = a.key1 + (uint64_t)L.nteams * geo.nwords;
  }
  a.tlimit = g->tick_khz * 1000ull * 20ull;  // 20 s per barrier wait
  a.ns_per_tick = (uint32_t)std::max<uint64_t>(1, 1000000ull / g->tick_khz);
  a.segcap = geo.segcap;
  a.hcap = geo.hcap;
  a.lcap = geo.lcap;
  a.rule = p.rule;
  a.G = L.G;
  a.nteams = L.nteams;
  a.chunk_edges = tu.chunk_edges;
  a.sample_cap = tu.sample_cap;
  a.probe_cap = tu.probe_cap;
  a.filter = tu.no_filter ? 0u : 1u;
  a.hint = tu.no_filter ? nullptr : (uint16_t*)w.hint;
  a.snapshot = (p.flags & SSSP_SOLVE_SNAPSHOT_KEYS) ? 1u : 0u;
  // Local expansion reads current keys, so snapshot-key runs go without it.
  a.local_budget = (a.snapshot || tu.local_budget == 0xFFFFFFFFu) ? 0u : tu.local_budget;
  a.super_sparse = tu.super_sparse_degree;
  // Local expansion serves graphs of small degree (the paper's road graphs):
  // on a graph whose average out-degree is not below the super-sparse
  // threshold, a step after a low-degree source only looks super-sparse.
  if ((uint64_t)g->m >= (uint64_t)tu.super_sparse_degree * (uint64_t)g->n) a.local_budget = 0;
  // Bidirectional relaxation reads current keys too; it needs symmetric arcs.
  a.pull = (!a.snapshot && g->undirected && tu.pull != 0xFFFFFFFFu && tu.pull != 0) ? 1u : 0u;
  // Local expansion admits vertices up to this out-degree (the packed rows
  // hold degrees below 2^24 - 1).
  a.local_cap = std::min<uint32_t>(local_degree_cap(tu), (1u << 24) - 2u);
  // Hub deferral (rho rule): on a graph numbered by degree the vertices of
  // out-degree at least 2^k are the ids below deg_ge[k].
  a.defer_div = tu.hub_defer_div ? tu.hub_defer_div : 10u;
  if (p.rule == SSSP_RULE_RHO && g->relabelled && tu.hub_defer_degree != 0 && tu.hub_defer_degree != 0xFFFFFFFFu)
    a.ndefer = g->deg_ge[31 - __builtin_clz(tu.hub_defer_degree)];
}

// trow[e] = (degree << ROW_SHIFT) | row start of arc e's target, degree
// saturated at 2^24 - 1.
__global__ void target_rows_kernel(const int64_t* off, const ull* edges, const int32_t* tgt, ull m, ull* trow) {
  for (ull e = (ull)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (ull)gridDim.x * blockDim.x) {
    const uint32_t t = edges ? (uint32_t)edges[e] : (uint32_t)tgt[e];
    const ull rb = (ull)off[t], deg = (ull)off[t + 1] - rb;
    trow[e] = (umin(deg, (1ull << 24) - 1) << ROW_SHIFT) | rb;
  }
}

// The graph's target rows for local expansion (8 bytes per arc), built on
// the first launch that can use them. Not for borrowed arrays (the caller
// may rewrite them between solves), nor beyond 2^40 arcs, nor when the
// device has no room for them; the kernel then reads the offsets.
sssp_status ensure_target_rows(sssp_graph* g, hipStream_t st) {
  const ull m = (ull)g->m;
  if (g->trow.p || g->borrowed || m == 0 || m > ROW_START) return SSSP_OK;
  const hipError_t e = g->trow.alloc(m * 8, st);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();  // not kept: an optional array
    g->trow.p = nullptr;
    g->trow.bytes = 0;
    return SSSP_OK;
  }
  SSSP_HIP_TRY(e);
  target_rows_kernel<<<2048, 256, 0, st>>>((const int64_t*)g->off.p, g->borrowed ? nullptr : (const ull*)g->edges.p,
                                          g->btgt, m, (ull*)g->trow.p);
  SSSP_HIP_TRY(hipGetLastError());
  return SSSP_OK;
}

// Plan the launch, make sure the graph's workspace fits it, and fill the
// kernel arguments.
sssp_status prepare_launch(sssp_graph* g, Launch& L, uint32_t default_teams, uint64_t* dist, hipStream_t st) {
  sssp_status s = plan_launch(g, L, default_teams);
  if (s != SSSP_OK) return s;
  // Repeated-push skip: by default for launches of one team (its arrays
  // cost 8 bytes per vertex and per hub chunk for every team) on graphs
  // without local expansion (average out-degree at least the super-sparse
  // threshold): there, repeated pushes of high-degree vertices are common;
  // on sparse graphs the extra read per vertex cost more than it saved.
  const bool dense_graph = (uint64_t)g->m >= (uint64_t)L.tu.super_sparse_degree * (uint64_t)g->n;
  const bool repeat = L.tu.repeat_skip != 0xFFFFFFFFu &&
                      (L.tu.repeat_skip == 1 || (L.nteams == 1 && dense_graph));
  s = ensure_workspace(g, L.tu, L.geo, repeat, st);
  if (s != SSSP_OK) return s;
  fill_args(g, L, graph_view(g), dist);
  if (L.a.local_budget > 0) {
    s = ensure_target_rows(g, st);
    if (s != SSSP_OK) return s;
    L.a.trow = (const ull*)g->trow.p;
  }
  if (repeat) {
    L.a.lastkey = (ull*)g->lastkey.p;
    if (g->relabelled && g->nhub > 0) {
      L.a.ckey = (ull*)g->ckey.p;
      L.a.cbase = (const uint32_t*)g->cbase.p;
      L.a.nhub = g->nhub;
    }
  }
  return SSSP_OK;
}

// Copy the kernel arguments (staged in `hargs`, host memory that stays valid
// until the copy has run) to `args_dev` and clear the control blocks.
hipError_t stage_launch(const Launch& L, void* hargs, void* args_dev, void* ctl_dev, hipStream_t st) {
  std::memcpy(hargs, &L.a, sizeof(KArgs));
  hipError_t e = hipMemcpyAsync(args_dev, hargs, sizeof(KArgs), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  reset_control_kernel<<<64, 256, 0, st>>>((ull*)ctl_dev, control_words(L.nteams));
  return hipGetLastError();
}

hipError_t stage_launch(sssp_graph* g, const Launch& L, hipStream_t st) {
  return stage_launch(L, g->hargs, g->args.p, g->ctl.p, st);
}

// Read the control blocks at `ctl_dev` back (after the kernel finished) into
// stats, a few team blocks at a time through a host buffer on the stack.
// Returns the abort and step-limit indications.
sssp_status collect_stats(sssp_graph* g, const Launch& L, const void* ctl_dev, hipStream_t st, sssp_stats* stats,
                          bool& aborted, bool& step_limit, bool& cancelled) {
  constexpr uint32_t CHUNK = 8;
  GridCtl hg;
  TeamCtl hteams[CHUNK];
  SSSP_HIP_TRY(hipMemcpyAsync(&hg, ctl_dev, sizeof(GridCtl), hipMemcpyDeviceToHost, st));
  SSSP_HIP_TRY(hipStreamSynchronize(st));
  aborted = hg.abort_flag != 0;
  step_limit = false;
  cancelled = false;
  for (uint32_t t = 0; t < L.nteams; ++t) {
    if (t % CHUNK == 0) {
      const uint32_t k = std::min(CHUNK, L.nteams - t);
      SSSP_HIP_TRY(hipMemcpyAsync(hteams, (const char*)ctl_dev + sizeof(GridCtl) + (size_t)t * sizeof(TeamCtl),
                                  (size_t)k * sizeof(TeamCtl), hipMemcpyDeviceToHost, st));
      SSSP_HIP_TRY(hipStreamSynchronize(st));
    }
    const TeamCtl& tc = hteams[t % CHUNK];
    step_limit |= (tc.status & ST_STEP_LIMIT) != 0;
    cancelled |= (tc.status & ST_CANCELLED) != 0;
    if (!stats) continue;
    stats->steps += tc.st_steps;
    stats->extracted += tc.st_extracted;
    stats->edges_relaxed += tc.st_edges;
    stats->writemin_success += tc.st_success;
    stats->dense_steps += tc.st_dense;
    stats->sampled_steps += tc.st_sampled;
    stats->queue_dense += tc.st_qdense;
    stats->queue_list += tc.st_qlist;
    stats->list_appends += tc.st_appends;
    stats->local_vertices += tc.st_local;
    stats->repeat_skipped += tc.st_skipped;
    if (t == 0) {
      for (int k = 0; k < 4; ++k) stats->phase_ms[k] = (double)tc.phase_ticks[k] / (double)g->tick_khz;
      stats->relax_wg_ms[0] = (double)tc.relax_busy_max / (double)g->tick_khz;
      stats->relax_wg_ms[1] = (double)tc.relax_busy_sum / (double)L.geo.T / (double)g->tick_khz;
    }
  }
  if (stats) stats->teams = L.nteams;
  return SSSP_OK;
}

sssp_status collect_stats(sssp_graph* g, const Launch& L, hipStream_t st, sssp_stats* stats, bool& aborted,
                          bool& step_limit, bool& cancelled) {
  return collect_stats(g, L, g->ctl.p, st, stats, aborted, step_limit, cancelled);
}

// Checksum of one distance row (the same mix as the serving kernel's).
__global__ void row_hash_kernel(const ull* dist, ull n, ull* out) {
  ull h = 0;
  for (ull v = (ull)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (ull)gridDim.x * blockDim.x)
    h += row_mix(v, dist[v]);
  h = wave_sum(h);
  if (lane_id() == 0) atom_add(out, h);
}

// Checks, workspace and the kernel launch of a solve (shared by the
// synchronous and the asynchronous entry points). `src_stage` is a host copy
// of the sources that stays valid until the copy has run (the caller's array
// for a synchronous solve, the graph's pinned staging array otherwise).
sssp_status enqueue_solve(sssp_graph* g, const int32_t* sources, int32_t n_src,
                          uint64_t* dist, hipStream_t st, const uint32_t* cancel, Launch& L, hipEvent_t ev0,
                          hipEvent_t ev1) {
  {
    // The default team count needs the grid size, which prepare_launch
    // computes; resolve it there through a provisional value.
    int occ = 0;
    SSSP_HIP_TRY(hipSetDevice(g->device));
    SSSP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stepping_kernel, WG, 0));
    const uint32_t G = std::max(1u, std::min<uint32_t>(L.tu.blocks_per_cu, (uint32_t)std::max(occ, 1))) *
                       (uint32_t)g->cus;
    sssp_status s = prepare_launch(g, L, auto_teams(n_src, G), dist, st);
    if (s != SSSP_OK) return s;
  }
  if ((uint64_t)n_src > g->ws_src_cap) {
    SSSP_HIP_TRY(g->srcs.alloc((uint64_t)n_src * 4, st));
    g->ws_src_cap = (uint64_t)n_src;
  }
  L.a.srcs = (const int32_t*)g->srcs.p;
  L.a.n_src = n_src;
  L.a.cancel = cancel;
  hipError_t e = hipMemcpyAsync(g->srcs.p, sources, (size_t)n_src * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = stage_launch(g, L, st);
  if (e == hipSuccess) e = hipEventRecord(ev0, st);
  if (e == hipSuccess) {
    const KArgs* dargs = (const KArgs*)g->args.p;
    void* kargs[] = {(void*)&dargs};
    e = hipLaunchCooperativeKernel((const void*)stepping_kernel, dim3(L.G), dim3(WG), kargs, 0, st);
  }
  if (e == hipSuccess) e = hipEventRecord(ev1, st);
  if (e != hipSuccess) return fail(from_hip(e), std::string("solve: ") + hipGetErrorString(e));
  return SSSP_OK;
}

// After the launch has finished: stats and the run's status.
sssp_status finish_solve(sssp_graph* g, const Launch& L, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                         sssp_stats* stats) {
  float ms = 0;
  (void)hipEventElapsedTime(&ms, ev0, ev1);
  bool aborted = false, step_limit = false, cancelled = false;
  sssp_status cs = collect_stats(g, L, st, stats, aborted, step_limit, cancelled);
  if (cs != SSSP_OK) return cs;
  if (stats) stats->device_ms = ms;
  if (aborted) return fail(SSSP_ERR_DEVICE, "grid barrier timed out (workgroups not co-resident?)");
  if (cancelled) return fail(SSSP_ERR_CANCELLED, "solve cancelled");
  if (step_limit) return fail(SSSP_ERR_STEP_LIMIT, "max_steps reached with a non-empty queue");
  return SSSP_OK;
}

sssp_status check_solve_args(const sssp_graph* gc, const int32_t* sources, int32_t n_src, uint64_t* dist) {
  if (!gc) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (gc->serving) return fail(SSSP_ERR_INVALID_ARGUMENT, "a server is running on this graph");
  if (gc->pending) return fail(SSSP_ERR_INVALID_ARGUMENT, "an asynchronous solve is pending on this graph");
  if (n_src < 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "n_src < 0");
  if (n_src > 0 && (!sources || !dist)) return fail(SSSP_ERR_INVALID_ARGUMENT, "sources or dist is NULL");
  for (int32_t i = 0; i < n_src; ++i)
    if (sources[i] < 0 || sources[i] >= gc->n)
      return fail(SSSP_ERR_INVALID_ARGUMENT, "source " + std::to_string(sources[i]) + " out of range");
  return SSSP_OK;
}

// ---------------------------------------------------------------------------
// Workspace without allocation (sssp_solve_noalloc): a static device array.
// In host code `scratch` names a host-side stand-in, not device memory; its
// device address is looked up once per device (scratch_address) and only
// that address is ever handed to kernels or copies.

static __device__ __align__(256) unsigned char scratch[SSSP_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu[NOALLOC_MAX_DEVICES];     // one call at a time per device
void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};    // device address of `scratch` per device

// Device address of this device's copy of `scratch` (the device must be
// current; the caller holds g_scratch_mu[dev]).
sssp_status scratch_address(int dev, char** out) {
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SSSP_ERR_DEVICE, std::string("scratch array address: ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = (char*)g_scratch_dev[dev];
  return SSSP_OK;
}

// Lay the launch's workspace out in the scratch array at `base` (256-byte
// aligned slices, in WsView order).
sssp_status carve_scratch(const sssp_graph* g, const Launch& L, uint64_t n_src, char* base, WsView& w) {
  uint64_t sz[15];
  workspace_sizes(g, L.tu, L.geo, n_src, sz);
  void** slot[15] = {&w.dist_int, &w.bitmap, &w.hint, &w.tree, &w.hubmask, &w.bigmask, &w.F,  &w.FD,
                     &w.H,        &w.L,      &w.samples, &w.parts, &w.ctl, &w.args, &w.srcs};
  uint64_t off = 0;
  for (int i = 0; i < 15; ++i) {
    *slot[i] = base + off;
    off += (std::max<uint64_t>(sz[i], 8) + 255) / 256 * 256;
  }
  if (off > SSSP_NOALLOC_SCRATCH_BYTES)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "the solve needs " + std::to_string(off) +
                                               " bytes of workspace; the scratch array holds " +
                                               std::to_string((uint64_t)SSSP_NOALLOC_SCRATCH_BYTES));
  return SSSP_OK;
}

// An asynchronous solve between sssp_solve_async and sssp_solve_wait.
struct PendingSolve {
  Launch L;
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

}  // namespace

// A persistent serving launch on one graph (include/sssp.h).
struct sssp_server {
  sssp_graph* g = nullptr;
  hipStream_t caller = nullptr;  // orders the start after the caller's queued work
  hipStream_t st = nullptr;      // the server's own stream (a hardware queue of its own)
  Launch L;
  uint64_t n = 0, rows = 0, cap = 0;
  // Ring and completion words in pinned, coherent host memory, shared with
  // the kernel: req[cap] pairs, then posted, closed | dev_closed, ack[cap],
  // done[rows], hashes[rows].
  int32_t* req = nullptr;
  uint64_t* words = nullptr;
  uint64_t* posted = nullptr;
  uint32_t* closed = nullptr;
  uint32_t* dev_closed = nullptr;  // set by the kernel once it takes no more requests
  uint64_t* ack = nullptr;
  uint64_t* done = nullptr;
  uint64_t* hashes = nullptr;
  uint64_t next_ticket = 0;
  std::vector<uint64_t> row_ticket;  // per row: ticket + 1 of its unfinished request, or 0
  std::vector<uint32_t> busy_rows;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool stopped = false;
  sssp_status stop_status = SSSP_OK;
  sssp_stats final_stats{};
  // Admission by memory budget (sssp_server_start_budget): the result rows
  // are the library's, drawn from the budget; requests wait in `waitq` until
  // a row is free, and a finished request holds its row until released.
  bool budget = false;
  DevBuf own_rows;
  uint64_t budget_bytes = 0;
  uint64_t ws_bytes = 0;                // workspace counted in the budget
  std::deque<int32_t> waitq;            // sources of requests not yet admitted, in ticket order
  uint64_t next_enqueue = 0;            // ticket of the next enqueued request
  std::vector<uint32_t> free_rows;
  std::unordered_map<uint64_t, uint32_t> held;  // finished, not yet released: ticket -> row
  std::unordered_map<uint64_t, uint32_t> admitted_row;  // admitted, not finished: ticket -> row
};

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
  sssp_status as = check_solve_args(gc, sources, n_src, dist);
  if (as != SSSP_OK) return as;
  Launch L;
  sssp_status ps = check_params(params, L.p, L.tu);
  if (ps != SSSP_OK) return ps;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n_src == 0) return SSSP_OK;

  sssp_graph* g = const_cast<sssp_graph*>(gc);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev0, ev1;
  SSSP_HIP_TRY(hipEventCreate(&ev0));
  SSSP_HIP_TRY(hipEventCreate(&ev1));
  sssp_status s = enqueue_solve(g, sources, n_src, dist, st, nullptr, L, ev0, ev1);
  if (s == SSSP_OK) {
    const hipError_t e = hipStreamSynchronize(st);
    s = e == hipSuccess ? finish_solve(g, L, st, ev0, ev1, stats)
                        : fail(from_hip(e), std::string("solve: ") + hipGetErrorString(e));
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  return s;
}

sssp_status sssp_solve_noalloc(const sssp_graph* gc, const int32_t* sources, int32_t n_src,
                               const sssp_params* params, uint64_t* dist, void* stream, sssp_stats* stats) {
  last_error().clear();
  sssp_status as = check_solve_args(gc, sources, n_src, dist);
  if (as != SSSP_OK) return as;
  Launch L;
  sssp_status ps = check_params(params, L.p, L.tu);
  if (ps != SSSP_OK) return ps;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n_src == 0) return SSSP_OK;
  sssp_graph* g = const_cast<sssp_graph*>(gc);
  if (g->device < 0 || g->device >= NOALLOC_MAX_DEVICES)
    return fail(SSSP_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu[g->device]);
  SSSP_HIP_TRY(hipSetDevice(g->device));
  char* base = nullptr;
  sssp_status s = scratch_address(g->device, &base);
  if (s != SSSP_OK) return s;
  {
    int occ = 0;
    SSSP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stepping_kernel, WG, 0));
    const uint32_t G = std::max(1u, std::min<uint32_t>(L.tu.blocks_per_cu, (uint32_t)std::max(occ, 1))) *
                       (uint32_t)g->cus;
    s = plan_launch(g, L, auto_teams(n_src, G));
    if (s != SSSP_OK) return s;
  }
  WsView w;
  s = carve_scratch(g, L, (uint64_t)n_src, base, w);
  if (s != SSSP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  fill_args(g, L, w, dist);
  L.a.n_src = n_src;
  L.a.cancel = nullptr;
  // Host staging of the arguments: this frame outlives the copy, since the
  // call waits for the stream before returning.
  KArgs staged;
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e = build_masks(g, L.tu, L.geo, w.hubmask, w.bigmask, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w.srcs, sources, (size_t)n_src * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = stage_launch(L, &staged, w.args, w.ctl, st);
  if (e == hipSuccess) {
    const KArgs* dargs = (const KArgs*)w.args;
    void* kargs[] = {(void*)&dargs};
    e = hipLaunchCooperativeKernel((const void*)stepping_kernel, dim3(L.G), dim3(WG), kargs, 0, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    return fail(from_hip(e), std::string("solve_noalloc: ") + hipGetErrorString(e));
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool aborted = false, step_limit = false, cancelled = false;
  s = collect_stats(g, L, w.ctl, st, stats, aborted, step_limit, cancelled);
  if (s != SSSP_OK) return s;
  if (stats) stats->device_ms = ms;
  if (aborted) return fail(SSSP_ERR_DEVICE, "grid barrier timed out (workgroups not co-resident?)");
  if (step_limit) return fail(SSSP_ERR_STEP_LIMIT, "max_steps reached with a non-empty queue");
  return SSSP_OK;
}

sssp_status sssp_solve_async(const sssp_graph* gc, const int32_t* sources, int32_t n_src,
                             const sssp_params* params, uint64_t* dist, void* stream) {
  last_error().clear();
  sssp_status as = check_solve_args(gc, sources, n_src, dist);
  if (as != SSSP_OK) return as;
  if (n_src == 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "an asynchronous solve needs at least one source");
  auto* P = new (std::nothrow) PendingSolve;
  if (!P) return fail(SSSP_ERR_OUT_OF_MEMORY, "pending-solve record");
  sssp_status ps = check_params(params, P->L.p, P->L.tu);
  if (ps != SSSP_OK) {
    delete P;
    return ps;
  }
  sssp_graph* g = const_cast<sssp_graph*>(gc);
  hipError_t e = hipSetDevice(g->device);
  // Pinned staging for the sources and the cancel flag: the caller may
  // reuse its array once this call returns.
  if (e == hipSuccess && !g->cancel_flag) e = hipHostMalloc((void**)&g->cancel_flag, 64, hipHostMallocCoherent);
  if (e == hipSuccess && (uint64_t)n_src > g->src_host_cap) {
    if (g->src_host) (void)hipHostFree(g->src_host);
    g->src_host = nullptr;
    g->src_host_cap = 0;
    e = hipHostMalloc((void**)&g->src_host, (size_t)n_src * 4, hipHostMallocDefault);
    if (e == hipSuccess) g->src_host_cap = (uint64_t)n_src;
  }
  if (e == hipSuccess) e = hipEventCreate(&P->ev0);
  if (e == hipSuccess) e = hipEventCreate(&P->ev1);
  if (e != hipSuccess) {
    if (P->ev0) (void)hipEventDestroy(P->ev0);
    if (P->ev1) (void)hipEventDestroy(P->ev1);
    delete P;
    return fail(from_hip(e), std::string("solve_async: ") + hipGetErrorString(e));
  }
  std::memcpy(g->src_host, sources, (size_t)n_src * 4);
  __atomic_store_n(g->cancel_flag, 0u, __ATOMIC_SEQ_CST);
  P->st = (hipStream_t)stream;
  sssp_status s = enqueue_solve(g, g->src_host, n_src, dist, P->st, g->cancel_flag, P->L, P->ev0, P->ev1);
  if (s != SSSP_OK) {
    // Whatever was enqueued must finish before the staging memory is reused.
    (void)hipStreamSynchronize(P->st);
    (void)hipEventDestroy(P->ev0);
    (void)hipEventDestroy(P->ev1);
    delete P;
    return s;
  }
  g->pending = P;
  return SSSP_OK;
}

sssp_status sssp_solve_query(const sssp_graph* gc, int* done) {
  last_error().clear();
  if (!gc || !done) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph or done is NULL");
  if (!gc->pending) return fail(SSSP_ERR_INVALID_ARGUMENT, "no asynchronous solve is pending");
  const auto* P = static_cast<const PendingSolve*>(gc->pending);
  const hipError_t e = hipEventQuery(P->ev1);
  if (e == hipSuccess) {
    *done = 1;
  } else if (e == hipErrorNotReady) {
    *done = 0;
  } else {
    return fail(from_hip(e), std::string("solve_query: ") + hipGetErrorString(e));
  }
  return SSSP_OK;
}

sssp_status sssp_solve_wait(const sssp_graph* gc, sssp_stats* stats) {
  last_error().clear();
  if (!gc) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (!gc->pending) return fail(SSSP_ERR_INVALID_ARGUMENT, "no asynchronous solve is pending");
  sssp_graph* g = const_cast<sssp_graph*>(gc);
  auto* P = static_cast<PendingSolve*>(g->pending);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  (void)hipSetDevice(g->device);
  const hipError_t e = hipEventSynchronize(P->ev1);
  sssp_status s = e == hipSuccess ? finish_solve(g, P->L, P->st, P->ev0, P->ev1, stats)
                                  : fail(from_hip(e), std::string("solve_wait: ") + hipGetErrorString(e));
  (void)hipEventDestroy(P->ev0);
  (void)hipEventDestroy(P->ev1);
  delete P;
  g->pending = nullptr;
  return s;
}

sssp_status sssp_solve_cancel(const sssp_graph* gc) {
  last_error().clear();
  if (!gc) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (!gc->pending || !gc->cancel_flag) return fail(SSSP_ERR_INVALID_ARGUMENT, "no asynchronous solve is pending");
  __atomic_store_n(gc->cancel_flag, 1u, __ATOMIC_SEQ_CST);
  return SSSP_OK;
}

sssp_status sssp_row_hash(const uint64_t* dist, int64_t n, void* stream, uint64_t* hash) {
  last_error().clear();
  if (!dist || !hash || n < 0) return fail(SSSP_ERR_INVALID_ARGUMENT, "dist or hash is NULL, or n < 0");
  hipStream_t st = (hipStream_t)stream;
  DevBuf acc;
  SSSP_HIP_TRY(acc.alloc(8, st));
  hipError_t e = hipMemsetAsync(acc.p, 0, 8, st);
  if (e == hipSuccess && n > 0) {
    row_hash_kernel<<<1024, 256, 0, st>>>((const ull*)dist, (ull)n, (ull*)acc.p);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hash, acc.p, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  acc.release(st);
  if (e != hipSuccess) return fail(from_hip(e), std::string("row hash: ") + hipGetErrorString(e));
  return SSSP_OK;
}

}  // extern "C"

namespace {

// Start a serving launch into `dist_rows` (rows x n); `s` is filled in and
// owned by the caller of this helper (freed with destroy_server on error).
sssp_status launch_server(sssp_graph* g, sssp_server* s, uint64_t* dist_rows, uint32_t rows, uint32_t ring_capacity,
                          uint32_t flags, uint32_t idle_ms) {
  // Half the co-resident slots by default, leaving room for other kernels
  // (copies, checksums, a second server).
  if (!s->L.p.tuning || s->L.p.tuning->blocks_per_cu == 0) s->L.tu.blocks_per_cu = 2;
  if (s->L.p.trace || s->L.p.extract_counts || s->L.p.max_steps)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "trace, extract_counts and max_steps are not available when serving");
  s->g = g;
  s->n = (uint64_t)g->n;
  s->rows = rows;
  s->cap = ring_capacity;
  s->row_ticket.assign(rows, 0);
  {
    int occ = 0;
    hipError_t e = hipSetDevice(g->device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stepping_kernel, WG, 0);
    if (e != hipSuccess) return fail(from_hip(e), hipGetErrorString(e));
    const uint32_t G = std::max(1u, std::min<uint32_t>(s->L.tu.blocks_per_cu, (uint32_t)std::max(occ, 1))) *
                       (uint32_t)g->cus;
    // Default: teams of 16 workgroups (a power of two count, at least 8),
    // at most 64 (the dispatcher's idle-team mask).
    uint32_t t = 8;
    while (t * 2 <= G / 16 && t * 2 <= 64 && G % (t * 2) == 0) t *= 2;
    sssp_status ls = prepare_launch(g, s->L, G % 8 == 0 ? t : 1, dist_rows, s->caller);
    if (ls != SSSP_OK) return ls;
    if (s->L.nteams > 64) return fail(SSSP_ERR_INVALID_ARGUMENT, "a server runs at most 64 teams");
  }
  {
    // HIP spreads streams over a few shared hardware queues, and a queue runs
    // its kernels one after another: a persistent launch would hold back
    // whatever shares its queue (another server, a copy of a finished row).
    // A stream with a CU mask gets a queue of its own; the mask keeps every
    // compute unit.
    std::vector<uint32_t> mask(((size_t)g->cus + 31) / 32, 0xffffffffu);
    hipError_t e = hipExtStreamCreateWithCUMask(&s->st, (uint32_t)mask.size(), mask.data());
    hipEvent_t ready = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ready, s->caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->st, ready, 0);
    if (ready) (void)hipEventDestroy(ready);
    if (e != hipSuccess) return fail(from_hip(e), std::string("server stream: ") + hipGetErrorString(e));
  }
  // Host ring: requests, then the control words, in one coherent pinned
  // allocation (device loads and stores reach it directly).
  const size_t req_bytes = (size_t)s->cap * 8, words = 2 + (size_t)s->cap + 2 * (size_t)rows;
  {
    hipError_t e = hipHostMalloc((void**)&s->req, req_bytes, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->words, words * 8, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipEventCreate(&s->ev0);
    if (e == hipSuccess) e = hipEventCreate(&s->ev1);
    if (e != hipSuccess) return fail(from_hip(e), std::string("server ring: ") + hipGetErrorString(e));
  }
  std::memset(s->req, 0, req_bytes);
  std::memset(s->words, 0, words * 8);
  s->posted = s->words;
  s->closed = reinterpret_cast<uint32_t*>(s->words + 1);
  s->dev_closed = s->closed + 1;
  s->ack = s->words + 2;
  s->done = s->ack + s->cap;
  s->hashes = s->done + rows;

  KArgs& a = s->L.a;
  a.n_src = 0;
  a.serve = 1;
  a.hash = (flags & SSSP_SERVE_HASH) ? 1u : 0u;
  a.req = s->req;
  a.posted = s->posted;
  a.closed = s->closed;
  a.dev_closed = s->dev_closed;
  a.ack = s->ack;
  a.done = s->done;
  a.hashes = s->hashes;
  a.ring_cap = s->cap;
  a.nrows = rows;
  {
    uint32_t gm = s->L.tu.group_max ? std::min(s->L.tu.group_max, s->L.nteams) : s->L.nteams;
    uint32_t p2 = 1;
    while (p2 * 2 <= gm) p2 *= 2;
    a.group_max = p2;
    // group_min: a power of two, at most group_max (hence at most the team count).
    const uint32_t gn = s->L.tu.group_min ? std::min(s->L.tu.group_min, p2) : 1u;
    uint32_t q2 = 1;
    while (q2 * 2 <= gn) q2 *= 2;
    a.group_min = q2;
  }
  a.idle_ticks = g->tick_khz * (uint64_t)(idle_ms ? idle_ms : 60000);
  a.tlimit += a.idle_ticks;  // team members wait at their barrier while a request is awaited
  hipError_t e = stage_launch(g, s->L, s->st);
  if (e == hipSuccess) e = hipEventRecord(s->ev0, s->st);
  if (e == hipSuccess) {
    // A plain launch: a cooperative one may wait for other cooperative
    // launches, and servers on several graphs run side by side. The grid fits
    // when the servers' blocks_per_cu sum to at most the occupancy; otherwise
    // the first barrier times out and the server stops with an error.
    const KArgs* dargs = (const KArgs*)g->args.p;
    hipLaunchKernelGGL(stepping_kernel, dim3(s->L.G), dim3(WG), 0, s->st, dargs);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(s->ev1, s->st);
  if (e != hipSuccess) return fail(from_hip(e), std::string("server launch: ") + hipGetErrorString(e));
  g->serving = true;
  return SSSP_OK;
}

// Release what launch_server (or the budget start) acquired; the launch must
// have ended or never started.
void free_server(sssp_server* s) {
  if (s->req) (void)hipHostFree(s->req);
  if (s->words) (void)hipHostFree(s->words);
  if (s->st) (void)hipStreamDestroy(s->st);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  s->own_rows.release(nullptr);
  delete s;
}

sssp_status start_checks(const sssp_graph* gc, uint32_t flags) {
  if (flags & ~SSSP_SERVE_HASH) return fail(SSSP_ERR_INVALID_ARGUMENT, "unknown server flags");
  if (gc->serving) return fail(SSSP_ERR_INVALID_ARGUMENT, "a server is already running on this graph");
  if (gc->pending) return fail(SSSP_ERR_INVALID_ARGUMENT, "an asynchronous solve is pending on this graph");
  return SSSP_OK;
}

// Post one request into the ring (the caller has checked source and row).
sssp_status post_request(sssp_server* s, int32_t source, uint32_t row, uint64_t* ticket) {
  const uint64_t t = s->next_ticket;
  const uint64_t e = t % s->cap;
  // The entry is free once the kernel has taken the request that held it.
  if (t >= s->cap && __atomic_load_n(&s->ack[e], __ATOMIC_ACQUIRE) != t - s->cap + 1)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "ring full");
  if (__atomic_load_n(s->dev_closed, __ATOMIC_ACQUIRE) || hipEventQuery(s->ev1) == hipSuccess)
    return fail(SSSP_ERR_DEVICE, "the server launch takes no more requests (idle limit reached or an error)");
  ++s->next_ticket;
  s->req[2 * e] = source;
  s->req[2 * e + 1] = (int32_t)row;
  __atomic_store_n(s->posted, t + 1, __ATOMIC_RELEASE);
  s->row_ticket[row] = t + 1;
  s->busy_rows.push_back(row);
  if (ticket) *ticket = t;
  return SSSP_OK;
}

// Budget servers: admit waiting requests while rows are free.
sssp_status admit_waiting(sssp_server* s) {
  while (!s->waitq.empty() && !s->free_rows.empty()) {
    const uint32_t row = s->free_rows.back();
    uint64_t t = 0;
    sssp_status st = post_request(s, s->waitq.front(), row, &t);
    if (st != SSSP_OK) return st;
    s->free_rows.pop_back();
    s->waitq.pop_front();
    s->admitted_row[t] = row;
  }
  return SSSP_OK;
}

}  // namespace

extern "C" {

sssp_status sssp_server_start(const sssp_graph* gc, const sssp_params* params, uint64_t* dist_rows, uint32_t rows,
                              uint32_t ring_capacity, uint32_t flags, uint32_t idle_ms, void* stream,
                              sssp_server** out) {
  last_error().clear();
  if (!out) return fail(SSSP_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!gc || !dist_rows || rows == 0 || ring_capacity == 0)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "graph or dist_rows is NULL, or rows / ring_capacity is 0");
  sssp_status cs = start_checks(gc, flags);
  if (cs != SSSP_OK) return cs;
  sssp_server* s = new (std::nothrow) sssp_server;
  if (!s) return fail(SSSP_ERR_OUT_OF_MEMORY, "server");
  sssp_status ps = check_params(params, s->L.p, s->L.tu);
  if (ps == SSSP_OK) {
    s->caller = (hipStream_t)stream;
    ps = launch_server(const_cast<sssp_graph*>(gc), s, dist_rows, rows, ring_capacity, flags, idle_ms);
  }
  if (ps != SSSP_OK) {
    free_server(s);
    return ps;
  }
  *out = s;
  return SSSP_OK;
}

sssp_status sssp_server_start_budget(const sssp_graph* gc, const sssp_params* params, uint64_t budget_bytes,
                                     uint32_t flags, uint32_t idle_ms, void* stream, sssp_server** out) {
  last_error().clear();
  if (!out) return fail(SSSP_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!gc) return fail(SSSP_ERR_INVALID_ARGUMENT, "graph is NULL");
  sssp_status cs = start_checks(gc, flags);
  if (cs != SSSP_OK) return cs;
  sssp_graph* g = const_cast<sssp_graph*>(gc);
  sssp_server* s = new (std::nothrow) sssp_server;
  if (!s) return fail(SSSP_ERR_OUT_OF_MEMORY, "server");
  s->budget = true;
  s->budget_bytes = budget_bytes;
  s->caller = (hipStream_t)stream;
  sssp_status ps = check_params(params, s->L.p, s->L.tu);
  if (ps == SSSP_OK && (!s->L.p.tuning || s->L.p.tuning->blocks_per_cu == 0)) s->L.tu.blocks_per_cu = 2;
  uint64_t rows = 0;
  if (ps == SSSP_OK) {
    // The workspace of the launch comes out of the budget first; the rest is
    // result rows of 8 n bytes.
    Launch probe;
    probe.p = s->L.p;
    probe.tu = s->L.tu;
    int occ = 0;
    hipError_t e = hipSetDevice(g->device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stepping_kernel, WG, 0);
    if (e != hipSuccess) {
      ps = fail(from_hip(e), hipGetErrorString(e));
    } else {
      const uint32_t G = std::max(1u, std::min<uint32_t>(probe.tu.blocks_per_cu, (uint32_t)std::max(occ, 1))) *
                         (uint32_t)g->cus;
      uint32_t t = 8;
      while (t * 2 <= G / 16 && t * 2 <= 64 && G % (t * 2) == 0) t *= 2;
      ps = plan_launch(g, probe, G % 8 == 0 ? t : 1);
      if (ps == SSSP_OK) {
        uint64_t sz[15], ws = 0;
        workspace_sizes(g, probe.tu, probe.geo, 0, sz);
        for (uint64_t b : sz) ws += b;
        s->ws_bytes = ws;
        const uint64_t row_bytes = 8ull * (uint64_t)g->n;
        rows = budget_bytes > ws ? (budget_bytes - ws) / row_bytes : 0;
        if (rows == 0)
          ps = fail(SSSP_ERR_OUT_OF_MEMORY, "budget of " + std::to_string(budget_bytes) +
                                                " bytes holds no result row: the workspace takes " +
                                                std::to_string(ws) + " and a row " + std::to_string(row_bytes));
        rows = std::min<uint64_t>(rows, 1u << 16);
      }
    }
  }
  if (ps == SSSP_OK) {
    const hipError_t e = s->own_rows.alloc(rows * 8ull * (uint64_t)g->n, s->caller);
    if (e != hipSuccess) ps = fail(from_hip(e), std::string("server rows: ") + hipGetErrorString(e));
  }
  if (ps == SSSP_OK)
    ps = launch_server(g, s, (uint64_t*)s->own_rows.p, (uint32_t)rows, (uint32_t)rows, flags, idle_ms);
  if (ps != SSSP_OK) {
    if (s->st) (void)hipStreamSynchronize(s->st);
    free_server(s);
    return ps;
  }
  for (uint32_t r = (uint32_t)rows; r > 0; --r) s->free_rows.push_back(r - 1);
  *out = s;
  return SSSP_OK;
}

sssp_status sssp_server_submit(sssp_server* s, int32_t source, uint32_t row, uint64_t* ticket) {
  last_error().clear();
  if (!s) return fail(SSSP_ERR_INVALID_ARGUMENT, "server is NULL");
  if (s->budget) return fail(SSSP_ERR_INVALID_ARGUMENT, "a budget server takes requests by sssp_server_enqueue");
  if (s->stopped) return fail(SSSP_ERR_INVALID_ARGUMENT, "server is stopped");
  if (source < 0 || (uint64_t)source >= s->n)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "source " + std::to_string(source) + " out of range");
  if (row >= s->rows) return fail(SSSP_ERR_INVALID_ARGUMENT, "row " + std::to_string(row) + " out of range");
  if (s->row_ticket[row]) return fail(SSSP_ERR_INVALID_ARGUMENT, "row " + std::to_string(row) + " is busy");
  return post_request(s, source, row, ticket);
}

sssp_status sssp_server_enqueue(sssp_server* s, int32_t source, uint64_t* ticket) {
  last_error().clear();
  if (!s) return fail(SSSP_ERR_INVALID_ARGUMENT, "server is NULL");
  if (!s->budget) return fail(SSSP_ERR_INVALID_ARGUMENT, "sssp_server_enqueue needs a budget server");
  if (s->stopped) return fail(SSSP_ERR_INVALID_ARGUMENT, "server is stopped");
  if (source < 0 || (uint64_t)source >= s->n)
    return fail(SSSP_ERR_INVALID_ARGUMENT, "source " + std::to_string(source) + " out of range");
  if (__atomic_load_n(s->dev_closed, __ATOMIC_ACQUIRE) || hipEventQuery(s->ev1) == hipSuccess)
    return fail(SSSP_ERR_DEVICE, "the server launch takes no more requests (idle limit reached or an error)");
  s->waitq.push_back(source);
  if (ticket) *ticket = s->next_enqueue;
  ++s->next_enqueue;
  return admit_waiting(s);
}

sssp_status sssp_server_poll(sssp_server* s, uint64_t* tickets, uint64_t* hashes, uint32_t max, uint32_t* count) {
  last_error().clear();
  if (!s || !count || (max && !tickets)) return fail(SSSP_ERR_INVALID_ARGUMENT, "server, tickets or count is NULL");
  uint32_t c = 0;
  for (size_t i = 0; i < s->busy_rows.size() && c < max;) {
    const uint32_t row = s->busy_rows[i];
    const uint64_t t1 = s->row_ticket[row];
    if (__atomic_load_n(&s->done[row], __ATOMIC_ACQUIRE) == t1) {
      tickets[c] = t1 - 1;
      if (hashes) hashes[c] = __atomic_load_n(&s->hashes[row], __ATOMIC_RELAXED);
      ++c;
      s->row_ticket[row] = 0;
      s->busy_rows[i] = s->busy_rows.back();
      s->busy_rows.pop_back();
      if (s->budget) {
        s->admitted_row.erase(t1 - 1);
        s->held[t1 - 1] = row;
      }
    } else {
      ++i;
    }
  }
  *count = c;
  // Requests can no longer finish once the launch has ended: say so rather
  // than leave the caller waiting.
  if (c == 0 && (!s->busy_rows.empty() || !s->waitq.empty()) && !s->stopped &&
      hipEventQuery(s->ev1) == hipSuccess) {
    // Completion words written just before the end are read once more.
    for (uint32_t row : s->busy_rows)
      if (__atomic_load_n(&s->done[row], __ATOMIC_ACQUIRE) == s->row_ticket[row])
        return SSSP_OK;
    return fail(SSSP_ERR_DEVICE, "the server launch has ended with " +
                                     std::to_string(s->busy_rows.size() + s->waitq.size()) +
                                     " requests unfinished (idle limit reached or an error)");
  }
  return SSSP_OK;
}

sssp_status sssp_server_result(sssp_server* s, uint64_t ticket, const uint64_t** row) {
  last_error().clear();
  if (!s || !row) return fail(SSSP_ERR_INVALID_ARGUMENT, "server or row is NULL");
  if (!s->budget) return fail(SSSP_ERR_INVALID_ARGUMENT, "sssp_server_result needs a budget server");
  auto it = s->held.find(ticket);
  if (it == s->held.end())
    return fail(SSSP_ERR_INVALID_ARGUMENT, "ticket " + std::to_string(ticket) + " is not finished and held");
  *row = (const uint64_t*)s->own_rows.p + (uint64_t)it->second * s->n;
  return SSSP_OK;
}

sssp_status sssp_server_release(sssp_server* s, uint64_t ticket) {
  last_error().clear();
  if (!s) return fail(SSSP_ERR_INVALID_ARGUMENT, "server is NULL");
  if (!s->budget) return fail(SSSP_ERR_INVALID_ARGUMENT, "sssp_server_release needs a budget server");
  auto it = s->held.find(ticket);
  if (it == s->held.end())
    return fail(SSSP_ERR_INVALID_ARGUMENT, "ticket " + std::to_string(ticket) + " is not finished and held");
  s->free_rows.push_back(it->second);
  s->held.erase(it);
  if (s->stopped) return SSSP_OK;
  return admit_waiting(s);
}

sssp_status sssp_server_take(sssp_server* s, uint64_t ticket, uint64_t* dst, void* stream) {
  last_error().clear();
  if (!dst) return fail(SSSP_ERR_INVALID_ARGUMENT, "dst is NULL");
  const uint64_t* row = nullptr;
  sssp_status rs = sssp_server_result(s, ticket, &row);
  if (rs != SSSP_OK) return rs;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(dst, row, 8ull * s->n, hipMemcpyDefault, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(from_hip(e), std::string("server take: ") + hipGetErrorString(e));
  return sssp_server_release(s, ticket);
}

sssp_status sssp_server_counts(const sssp_server* s, sssp_server_load* load) {
  last_error().clear();
  if (!s || !load) return fail(SSSP_ERR_INVALID_ARGUMENT, "server or load is NULL");
  std::memset(load, 0, sizeof(*load));
  load->rows = s->rows;
  load->row_bytes = 8ull * s->n;
  load->budget_bytes = s->budget_bytes;
  load->teams = s->L.nteams;
  load->waiting = s->waitq.size();
  load->admitted = s->busy_rows.size();
  load->held = s->budget ? s->held.size() : 0;
  load->free_rows = s->budget ? s->free_rows.size() : s->rows - s->busy_rows.size();
  load->workspace_bytes = s->budget ? s->ws_bytes : (s->g ? s->g->workspace_bytes() : 0);
  return SSSP_OK;
}

sssp_status sssp_server_stop(sssp_server* s, sssp_stats* stats) {
  last_error().clear();
  if (!s) return fail(SSSP_ERR_INVALID_ARGUMENT, "server is NULL");
  if (!s->stopped) {
    s->stopped = true;
    __atomic_store_n(s->closed, 1u, __ATOMIC_RELEASE);
    hipError_t e = hipStreamSynchronize(s->st);
    std::memset(&s->final_stats, 0, sizeof(s->final_stats));
    if (e != hipSuccess) {
      s->stop_status = fail(from_hip(e), std::string("server: ") + hipGetErrorString(e));
    } else {
      bool aborted = false, step_limit = false;
      bool cancelled = false;  // servers have no cancel flag
      s->stop_status = collect_stats(s->g, s->L, s->st, &s->final_stats, aborted, step_limit, cancelled);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, s->ev0, s->ev1);
      s->final_stats.device_ms = ms;
      if (s->stop_status == SSSP_OK && aborted)
        s->stop_status = fail(SSSP_ERR_DEVICE, "server barrier or request wait timed out");
    }
    // Requests never admitted are dropped.
    s->waitq.clear();
    s->g->serving = false;
  }
  if (stats) *stats = s->final_stats;
  return s->stop_status;
}

sssp_status sssp_server_destroy(sssp_server* s) {
  if (!s) return SSSP_OK;
  sssp_status st = SSSP_OK;
  if (!s->stopped) st = sssp_server_stop(s, nullptr);
  free_server(s);
  return st;
}

}  // extern "C"
