// Seeded synthetic graph generators for the stepping-SSSP workloads.
//
// This module produces inputs only: CSR graphs (int64 offsets, int32 targets,
// uint32 weights) and source vertices. It holds none of the shortest-path
// arithmetic, and it is shared by the CPU oracle and the GPU path, which both
// consume the bytes it writes.
//
// Randomness: every draw is the i-th output of a SplitMix64 stream (Steele,
// Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
// 2014): out(seed, i) = mix(seed + (i + 1) * 0x9e3779b97f4a7c15), where mix is
// the published 64-bit finaliser. Because each draw is a pure function of
// (seed, counter), results do not depend on the number of threads.
//
// Graph shapes (stand-ins for the paper's datasets, Sec. 7 "Graphs"):
//   grid2d : 4-neighbour W x H grid, one uniform weight per undirected edge.
//   rmat   : R-MAT power-law sampler (quadrant probabilities a, b, c, d),
//            optional seeded relabelling, symmetrised, self-loops and
//            duplicate pairs removed, one uniform weight per undirected pair.
//   road   : jittered W x H grid, a fraction of grid edges deleted, extra
//            short-range edges added, weight = round(1000 * Euclidean length).
//   knn    : Gaussian-mixture point cloud in the unit cube, exact k nearest
//            neighbours, union-symmetrised, weight = round(scale * distance).
//
// Every graph is symmetric (each undirected pair appears as two arcs with the
// same weight) and rows are sorted by target id, so a graph is a deterministic
// function of its parameters.

#include <omp.h>
#include <parallel/algorithm>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// i-th output of a SplitMix64 stream started at `seed`.
inline uint64_t draw(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * kGamma); }

// Derive an independent stream seed for a named purpose.
inline uint64_t substream(uint64_t seed, uint64_t tag) { return draw(seed ^ 0x5eed5eed5eed5eedULL, tag); }

// Uniform integer in [0, range) by the multiply-high method.
inline uint64_t below(uint64_t r, uint64_t range) {
  return (uint64_t)(((unsigned __int128)r * range) >> 64);
}

// Uniform double in [0, 1) from the top 53 bits.
inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

// Weight of the undirected pair {u, v}, uniform in [lo, hi).
inline uint32_t pair_weight(uint64_t wseed, int64_t u, int64_t v, uint32_t lo, uint32_t hi) {
  uint64_t a = (uint64_t)std::min(u, v), b = (uint64_t)std::max(u, v);
  uint64_t key = (a << 32) ^ b;
  return lo + (uint32_t)below(mix64(wseed ^ mix64(key + kGamma)), (uint64_t)(hi - lo));
}

struct Arc {
  int32_t u, v;
};

}  // namespace

extern "C" {

typedef struct {
  int64_t n;
  int64_t m;
  int64_t* offsets;   // n + 1
  int32_t* targets;   // m
  uint32_t* weights;  // m
} gg_csr;

void gg_free(gg_csr* g) {
  if (!g) return;
  std::free(g->offsets);
  std::free(g->targets);
  std::free(g->weights);
  g->offsets = nullptr;
  g->targets = nullptr;
  g->weights = nullptr;
  g->n = g->m = 0;
}

}  // extern "C"

namespace {

// Build a symmetric, deduplicated CSR from a list of undirected pairs.
// `weight_of(u, v)` must be symmetric. Self-loops are dropped.
//
// Arcs are first distributed into vertex-range buckets with per-thread
// histograms (no shared counters, so hub vertices cause no contention), then
// each bucket is counting-sorted by source, and each row is sorted by target
// and deduplicated.
template <class WeightFn>
int build_symmetric_csr(int64_t n, const std::vector<Arc>& pairs, WeightFn weight_of, gg_csr* out) {
  const int64_t np = (int64_t)pairs.size();
  const int nthreads = omp_get_max_threads();
  const int64_t width = std::max<int64_t>(1, (n + 8191) / 8192);
  const int64_t nb = (n + width - 1) / width;
  std::vector<int64_t> hist((size_t)nthreads * nb, 0);
  auto chunk = [&](int t, int64_t& lo, int64_t& hi) {
    lo = np * t / nthreads;
    hi = np * (t + 1) / nthreads;
  };
#pragma omp parallel num_threads(nthreads)
  {
    const int t = omp_get_thread_num();
    int64_t lo, hi;
    chunk(t, lo, hi);
    int64_t* h = hist.data() + (size_t)t * nb;
    for (int64_t i = lo; i < hi; ++i) {
      const Arc a = pairs[i];
      if (a.u == a.v) continue;
      ++h[a.u / width];
      ++h[a.v / width];
    }
  }
  // Exclusive prefix in (bucket, thread) order.
  std::vector<int64_t> bstart(nb + 1, 0);
  {
    int64_t acc = 0;
    for (int64_t b = 0; b < nb; ++b) {
      bstart[b] = acc;
      for (int t = 0; t < nthreads; ++t) {
        const int64_t c = hist[(size_t)t * nb + b];
        hist[(size_t)t * nb + b] = acc;
        acc += c;
      }
    }
    bstart[nb] = acc;
  }
  const int64_t m_raw = bstart[nb];
  uint64_t* packed = (uint64_t*)std::malloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(m_raw, 1));
  if (!packed) return 2;
#pragma omp parallel num_threads(nthreads)
  {
    const int t = omp_get_thread_num();
    int64_t lo, hi;
    chunk(t, lo, hi);
    int64_t* h = hist.data() + (size_t)t * nb;
    for (int64_t i = lo; i < hi; ++i) {
      const Arc a = pairs[i];
      if (a.u == a.v) continue;
      packed[h[a.u / width]++] = ((uint64_t)(uint32_t)a.u << 32) | (uint32_t)a.v;
      packed[h[a.v / width]++] = ((uint64_t)(uint32_t)a.v << 32) | (uint32_t)a.u;
    }
  }
  // Per-vertex raw degrees from each bucket (disjoint vertex ranges).
  std::vector<int64_t> off(n + 1, 0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < nb; ++b)
    for (int64_t i = bstart[b]; i < bstart[b + 1]; ++i) ++off[(int64_t)(packed[i] >> 32) + 1];
  for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
  int32_t* tmp = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m_raw, 1));
  if (!tmp) {
    std::free(packed);
    return 2;
  }
#pragma omp parallel
  {
    std::vector<int64_t> cur;
#pragma omp for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t v0 = b * width, v1 = std::min(n, v0 + width);
      cur.assign(off.begin() + v0, off.begin() + v1);
      for (int64_t i = bstart[b]; i < bstart[b + 1]; ++i) {
        const int64_t u = (int64_t)(packed[i] >> 32);
        tmp[cur[u - v0]++] = (int32_t)(uint32_t)packed[i];
      }
    }
  }
  std::free(packed);
  // Sort each row and drop repeated targets.
  std::vector<int64_t> ndeg(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* b = tmp + off[i];
    int32_t* e = tmp + off[i + 1];
    std::sort(b, e);
    ndeg[i] = std::unique(b, e) - b;
  }
  int64_t* o = (int64_t*)std::malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!o) {
    std::free(tmp);
    return 2;
  }
  o[0] = 0;
  for (int64_t i = 0; i < n; ++i) o[i + 1] = o[i] + ndeg[i];
  const int64_t m = o[n];
  int32_t* t = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
  uint32_t* w = (uint32_t*)std::malloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(m, 1));
  if (!t || !w) {
    std::free(tmp);
    std::free(o);
    std::free(t);
    std::free(w);
    return 2;
  }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t src = off[i], dst = o[i], d = ndeg[i];
    for (int64_t k = 0; k < d; ++k) {
      const int32_t v = tmp[src + k];
      t[dst + k] = v;
      w[dst + k] = weight_of(i, (int64_t)v);
    }
  }
  std::free(tmp);
  out->n = n;
  out->m = m;
  out->offsets = o;
  out->targets = t;
  out->weights = w;
  return 0;
}

}  // namespace

extern "C" {

// 4-neighbour W x H grid; vertex id = y * W + x. Each undirected edge gets a
// weight uniform in [wlo, whi), identical on both arcs.
int gg_grid2d(int64_t W, int64_t H, uint32_t wlo, uint32_t whi, uint64_t seed, gg_csr* out) {
  if (W <= 0 || H <= 0 || W * H >= (int64_t)1 << 31 || whi <= wlo || !out) return 1;
  const int64_t n = W * H;
  std::vector<Arc> pairs;
  pairs.reserve((size_t)(2 * n));
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) {
      const int32_t u = (int32_t)(y * W + x);
      if (x + 1 < W) pairs.push_back({u, (int32_t)(u + 1)});
      if (y + 1 < H) pairs.push_back({u, (int32_t)(u + W)});
    }
  const uint64_t ws = substream(seed, 1);
  return build_symmetric_csr(n, pairs, [&](int64_t a, int64_t b) { return pair_weight(ws, a, b, wlo, whi); }, out);
}

// R-MAT sampler with 2^scale vertices and edge_factor * 2^scale samples. Each
// sample descends `scale` levels, choosing quadrant (0,0), (0,1), (1,0), (1,1)
// with probabilities a, b, c, 1-a-b-c (each rounded to a multiple of 2^-21). With relabel != 0 the vertex ids are
// passed through a seeded uniform permutation. Weight per pair ~ U[wlo, whi).
int gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint32_t wlo, uint32_t whi,
            uint64_t seed, int relabel, gg_csr* out) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || whi <= wlo || !out) return 1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return 1;
  const int64_t n = (int64_t)1 << scale;
  const int64_t ns = edge_factor * n;
  // Quadrant thresholds at 21-bit resolution; one 64-bit draw serves three levels.
  const double two21 = 2097152.0;
  const uint64_t ta = (uint64_t)std::llround(a * two21), tab = (uint64_t)std::llround((a + b) * two21),
                 tabc = (uint64_t)std::llround((a + b + c) * two21);
  const uint64_t es = substream(seed, 2);
  std::vector<int32_t> perm;
  if (relabel) {
    // Seeded permutation: sort vertex ids by a per-vertex random key.
    const uint64_t ps = substream(seed, 3);
    std::vector<std::pair<uint64_t, int32_t>> key(n);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) key[v] = {draw(ps, (uint64_t)v), (int32_t)v};
    __gnu_parallel::sort(key.begin(), key.end());
    perm.resize(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) perm[key[i].second] = (int32_t)i;
  }
  std::vector<Arc> pairs;
  try {
    pairs.resize((size_t)ns);
  } catch (const std::bad_alloc&) {
    return 2;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ns; ++i) {
    uint64_t u = 0, v = 0, r = 0;
    const uint64_t per = (uint64_t)(scale + 2) / 3;
    for (int l = 0; l < scale; ++l) {
      if (l % 3 == 0) r = draw(es, (uint64_t)i * per + (uint64_t)(l / 3));
      const uint64_t x = (r >> (21 * (l % 3))) & 0x1fffff;
      const uint64_t q = (uint64_t)(x >= ta) + (uint64_t)(x >= tab) + (uint64_t)(x >= tabc);
      u = (u << 1) | (q >> 1);
      v = (v << 1) | (q & 1);
    }
    if (relabel) {
      u = (uint64_t)perm[u];
      v = (uint64_t)perm[v];
    }
    pairs[i] = {(int32_t)u, (int32_t)v};
  }
  const uint64_t ws = substream(seed, 4);
  return build_symmetric_csr(n, pairs, [&](int64_t x, int64_t y) { return pair_weight(ws, x, y, wlo, whi); }, out);
}

// Road-like graph. Point (x, y) sits at (x + jx, y + jy), jx, jy ~ U[-jitter, jitter].
// Each 4-neighbour grid edge is deleted with probability del_frac. Then
// round(extra_frac * #grid edges) extra candidates are drawn: a uniform vertex
// u and a uniform offset in [-reach, reach]^2 \ {(0,0)}; out-of-range candidates
// are skipped and repeated pairs collapse. Weight = max(1, llround(wscale * |p_u - p_v|)).
int gg_road(int64_t W, int64_t H, double jitter, double del_frac, double extra_frac, int reach, double wscale,
            uint64_t seed, gg_csr* out) {
  if (W <= 0 || H <= 0 || W * H >= (int64_t)1 << 31 || reach < 1 || !out) return 1;
  const int64_t n = W * H;
  const uint64_t js = substream(seed, 5), ds = substream(seed, 6), xs = substream(seed, 7);
  std::vector<double> px(n), py(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t x = i % W, y = i / W;
    px[i] = (double)x + (2.0 * unit(draw(js, 2 * (uint64_t)i)) - 1.0) * jitter;
    py[i] = (double)y + (2.0 * unit(draw(js, 2 * (uint64_t)i + 1)) - 1.0) * jitter;
  }
  const int64_t n_grid = 2 * W * H - W - H;
  const int64_t n_extra = (int64_t)std::llround(extra_frac * (double)n_grid);
  std::vector<Arc> pairs;
  pairs.reserve((size_t)(n_grid + n_extra));
  // Grid edges in a fixed order; edge id e indexes the deletion draw.
  int64_t e = 0;
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) {
      const int32_t u = (int32_t)(y * W + x);
      if (x + 1 < W) {
        if (unit(draw(ds, (uint64_t)e)) >= del_frac) pairs.push_back({u, (int32_t)(u + 1)});
        ++e;
      }
      if (y + 1 < H) {
        if (unit(draw(ds, (uint64_t)e)) >= del_frac) pairs.push_back({u, (int32_t)(u + W)});
        ++e;
      }
    }
  const int side = 2 * reach + 1;
  const uint64_t n_off = (uint64_t)side * side - 1;
  for (int64_t j = 0; j < n_extra; ++j) {
    const int64_t u = (int64_t)below(draw(xs, 2 * (uint64_t)j), (uint64_t)n);
    uint64_t k = below(draw(xs, 2 * (uint64_t)j + 1), n_off);
    if (k >= n_off / 2) ++k;  // skip the centre cell
    const int64_t dx = (int64_t)(k % side) - reach, dy = (int64_t)(k / side) - reach;
    const int64_t x = u % W + dx, y = u / W + dy;
    if (x < 0 || x >= W || y < 0 || y >= H) continue;
    pairs.push_back({(int32_t)u, (int32_t)(y * W + x)});
  }
  auto wfn = [&](int64_t a, int64_t b) {
    const double ddx = px[a] - px[b], ddy = py[a] - py[b];
    const long long r = std::llround(wscale * std::sqrt(ddx * ddx + ddy * ddy));
    return (uint32_t)std::max<long long>(1, std::min<long long>(r, 0xffffffffLL));
  };
  return build_symmetric_csr(n, pairs, wfn, out);
}

// Connected components of a symmetric CSR graph (label = smallest vertex id in
// the component is NOT guaranteed; labels are 0..k-1 in order of discovery by
// increasing start vertex). Returns the number of components.
int64_t gg_components(const gg_csr* g, int32_t* label) {
  const int64_t n = g->n;
  for (int64_t i = 0; i < n; ++i) label[i] = -1;
  std::vector<int32_t> stack;
  int64_t k = 0;
  for (int64_t s = 0; s < n; ++s) {
    if (label[s] >= 0) continue;
    label[s] = (int32_t)k;
    stack.push_back((int32_t)s);
    while (!stack.empty()) {
      const int32_t u = stack.back();
      stack.pop_back();
      for (int64_t e = g->offsets[u]; e < g->offsets[u + 1]; ++e) {
        const int32_t v = g->targets[e];
        if (label[v] < 0) {
          label[v] = (int32_t)k;
          stack.push_back(v);
        }
      }
    }
    ++k;
  }
  return k;
}

// Membership of the largest connected component (undirected graphs). Uses a
// parallel breadth-first search from the highest-degree vertex; if that
// component holds more than half the vertices it is the largest, otherwise a
// full labelling decides. Writes 1/0 into `in_lcc` and returns its size.
int64_t gg_largest_component(const gg_csr* g, uint8_t* in_lcc) {
  const int64_t n = g->n;
  int64_t best = 0, bestdeg = -1;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = g->offsets[v + 1] - g->offsets[v];
    if (d > bestdeg) {
      bestdeg = d;
      best = v;
    }
  }
  std::vector<std::atomic<uint8_t>> seen(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) seen[i].store(0, std::memory_order_relaxed);
  std::vector<int32_t> frontier{(int32_t)best}, next;
  seen[best].store(1);
  int64_t size = 1;
  while (!frontier.empty()) {
    next.clear();
    const int64_t fs = (int64_t)frontier.size();
#pragma omp parallel
    {
      std::vector<int32_t> local;
#pragma omp for schedule(dynamic, 256) nowait
      for (int64_t i = 0; i < fs; ++i) {
        const int32_t u = frontier[i];
        for (int64_t e = g->offsets[u]; e < g->offsets[u + 1]; ++e) {
          const int32_t v = g->targets[e];
          if (seen[v].load(std::memory_order_relaxed)) continue;
          uint8_t z = 0;
          if (seen[v].compare_exchange_strong(z, 1)) local.push_back(v);
        }
      }
#pragma omp critical
      next.insert(next.end(), local.begin(), local.end());
    }
    size += (int64_t)next.size();
    frontier.swap(next);
  }
  if (2 * size > n) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) in_lcc[i] = seen[i].load(std::memory_order_relaxed);
    return size;
  }
  std::vector<int32_t> label(n);
  const int64_t k = gg_components(g, label.data());
  std::vector<int64_t> cnt(k, 0);
  for (int64_t i = 0; i < n; ++i) ++cnt[label[i]];
  const int64_t big = std::max_element(cnt.begin(), cnt.end()) - cnt.begin();
  for (int64_t i = 0; i < n; ++i) in_lcc[i] = label[i] == big;
  return cnt[big];
}

// `count` seeded uniform picks (with replacement) among vertices whose mask
// byte is nonzero (or among all vertices if mask is NULL), in increasing-id
// rank order.
int gg_pick_sources(int64_t n, const uint8_t* mask, uint64_t seed, int32_t count, int32_t* out) {
  std::vector<int32_t> pool;
  if (mask) {
    for (int64_t i = 0; i < n; ++i)
      if (mask[i]) pool.push_back((int32_t)i);
  }
  const int64_t size = mask ? (int64_t)pool.size() : n;
  if (size == 0) return 1;
  const uint64_t ss = substream(seed, 8);
  for (int32_t j = 0; j < count; ++j) {
    const int64_t r = (int64_t)below(draw(ss, (uint64_t)j), (uint64_t)size);
    out[j] = mask ? pool[r] : (int32_t)r;
  }
  return 0;
}

// Gaussian-mixture point cloud: `clusters` centres ~ U[0,1]^3, `per_cluster`
// points each ~ N(centre, sigma^2 I) (Box-Muller), not clipped. Exact k nearest
// neighbours (Euclidean, self excluded, ties broken by smaller index) via a
// k-d tree search, union-symmetrised; weight = max(1, llround(wscale * d)).
int gg_knn(int64_t clusters, int64_t per_cluster, double sigma, int k, double wscale, uint64_t seed, gg_csr* out) {
  if (clusters < 1 || per_cluster < 1 || k < 1 || !out) return 1;
  const int64_t n = clusters * per_cluster;
  if (n >= ((int64_t)1 << 31) || k >= n) return 1;
  const uint64_t cs = substream(seed, 9), ps = substream(seed, 10);
  std::vector<double> cx(clusters * 3);
  for (int64_t i = 0; i < clusters * 3; ++i) cx[i] = unit(draw(cs, (uint64_t)i));
  std::vector<double> P((size_t)n * 3);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t cl = i / per_cluster;
    for (int d = 0; d < 3; ++d) {
      // Box-Muller: two uniforms -> one normal deviate per coordinate.
      const double u1 = 1.0 - unit(draw(ps, 6 * (uint64_t)i + 2 * d));
      const double u2 = unit(draw(ps, 6 * (uint64_t)i + 2 * d + 1));
      const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
      P[3 * i + d] = cx[3 * cl + d] + sigma * z;
    }
  }
  // k-d tree over the points: node j (root 1, children 2j and 2j+1) covers
  // tree positions [lo, hi) and splits them at mid = (lo + hi) / 2 on the axis
  // of widest extent; positions below mid hold keys <= the split key, those
  // from mid on hold keys >= it (key = (coordinate, point index)).
  constexpr int64_t LEAF = 16;
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  int64_t nodes = 1;
  while (n / nodes > LEAF) nodes *= 2;
  std::vector<int8_t> axis_of(2 * nodes, -1);
  std::vector<double> split_of(2 * nodes, 0.0);
  struct Range {
    int64_t node, lo, hi;
  };
  std::vector<Range> level{{1, 0, n}};
  while (!level.empty()) {
    std::vector<Range> next;
    std::vector<std::array<Range, 2>> kids(level.size());
    std::vector<char> split(level.size(), 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < (int64_t)level.size(); ++r) {
      const Range R = level[r];
      if (R.hi - R.lo <= LEAF || 2 * R.node + 1 >= 2 * nodes) continue;
      double lo3[3] = {1e300, 1e300, 1e300}, hi3[3] = {-1e300, -1e300, -1e300};
      for (int64_t q = R.lo; q < R.hi; ++q)
        for (int d = 0; d < 3; ++d) {
          lo3[d] = std::min(lo3[d], P[3 * (int64_t)order[q] + d]);
          hi3[d] = std::max(hi3[d], P[3 * (int64_t)order[q] + d]);
        }
      int ax = 0;
      for (int d = 1; d < 3; ++d)
        if (hi3[d] - lo3[d] > hi3[ax] - lo3[ax]) ax = d;
      const int64_t mid = (R.lo + R.hi) / 2;
      std::nth_element(order.begin() + R.lo, order.begin() + mid, order.begin() + R.hi, [&](int32_t a, int32_t b) {
        const double pa = P[3 * (int64_t)a + ax], pb = P[3 * (int64_t)b + ax];
        return pa < pb || (pa == pb && a < b);
      });
      axis_of[R.node] = (int8_t)ax;
      split_of[R.node] = P[3 * (int64_t)order[mid] + ax];
      kids[r] = {Range{2 * R.node, R.lo, mid}, Range{2 * R.node + 1, mid, R.hi}};
      split[r] = 1;
    }
    for (size_t r = 0; r < level.size(); ++r)
      if (split[r]) {
        next.push_back(kids[r][0]);
        next.push_back(kids[r][1]);
      }
    level.swap(next);
  }
  // Points in tree order, for locality of the leaf scans.
  std::vector<double> T((size_t)n * 3);
  for (int64_t q = 0; q < n; ++q)
    for (int d = 0; d < 3; ++d) T[3 * q + d] = P[3 * (int64_t)order[q] + d];

  std::vector<int32_t> nbr((size_t)n * k);
#pragma omp parallel
  {
    // The k best (squared distance, index) pairs so far, ascending.
    std::vector<std::pair<double, int32_t>> best;
    struct Frame {
      int64_t node, lo, hi;
      double bound;  // lower bound on the squared distance to any point in the node
    };
    std::vector<Frame> stack;
#pragma omp for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      const double* pi = &P[3 * i];
      best.clear();
      stack.clear();
      stack.push_back({1, 0, n, 0.0});
      while (!stack.empty()) {
        const Frame f = stack.back();
        stack.pop_back();
        // Prune only on a strictly larger bound, so that points at the k-th
        // distance are still seen and the smaller index wins the tie.
        if ((int64_t)best.size() == k && f.bound > best.back().first) continue;
        const int ax = f.node < 2 * nodes ? axis_of[f.node] : -1;
        if (ax < 0) {
          for (int64_t q = f.lo; q < f.hi; ++q) {
            const int32_t j = order[q];
            if (j == i) continue;
            double s = 0;
            for (int d = 0; d < 3; ++d) {
              const double t = pi[d] - T[3 * q + d];
              s += t * t;
            }
            const std::pair<double, int32_t> c{s, j};
            if ((int64_t)best.size() == k) {
              if (!(c < best.back())) continue;
              best.pop_back();
            }
            best.insert(std::upper_bound(best.begin(), best.end(), c), c);
          }
          continue;
        }
        const int64_t mid = (f.lo + f.hi) / 2;
        const double sp = split_of[f.node];
        // The far side's points lie beyond the split plane: its squared
        // distance from the query bounds theirs from below (rounding is
        // monotone, so the bound also holds for the computed distances).
        const double gap = pi[ax] < sp ? sp - pi[ax] : pi[ax] - sp;
        const Frame lo_f{2 * f.node, f.lo, mid, pi[ax] < sp ? f.bound : std::max(f.bound, gap * gap)};
        const Frame hi_f{2 * f.node + 1, mid, f.hi, pi[ax] < sp ? std::max(f.bound, gap * gap) : f.bound};
        if (pi[ax] < sp) {
          stack.push_back(hi_f);
          stack.push_back(lo_f);
        } else {
          stack.push_back(lo_f);
          stack.push_back(hi_f);
        }
      }
      for (int q = 0; q < k; ++q) nbr[(size_t)i * k + q] = best[q].second;
    }
  }
  std::vector<Arc> pairs((size_t)n * k);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int q = 0; q < k; ++q) pairs[(size_t)i * k + q] = {(int32_t)i, nbr[(size_t)i * k + q]};
  auto wfn = [&](int64_t a, int64_t b) {
    double s = 0;
    for (int d = 0; d < 3; ++d) {
      const double t = P[3 * a + d] - P[3 * b + d];
      s += t * t;
    }
    const long long r = std::llround(wscale * std::sqrt(s));
    return (uint32_t)std::max<long long>(1, std::min<long long>(r, 0xffffffffLL));
  };
  return build_symmetric_csr(n, pairs, wfn, out);
}

// Raw SplitMix64 outputs, exposed so tests can pin the generator against the
// published reference sequence.
void gg_splitmix64(uint64_t seed, uint64_t count, uint64_t* out) {
  for (uint64_t i = 0; i < count; ++i) out[i] = draw(seed, i);
}

}  // extern "C"
