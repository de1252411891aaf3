/*
 * CPU oracle for single-source shortest paths on non-negatively weighted
 * directed graphs in CSR form. TEST INFRASTRUCTURE ONLY: the GPU library never
 * links, loads or calls this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it.
 *
 * What it computes (Sec. 2, problem statement and graph notation): for a
 * source s, d(s, v) = the minimum over directed paths s ~> v of the sum of the
 * arc weights, computed exactly in unsigned 64-bit integers; d(s, v) =
 * UINT64_MAX when v is unreachable, d(s, s) = 0. Every stepping algorithm of
 * the framework (Sec. 3.2, Alg. 1 and Table 2) reaches exactly this array; only
 * the number of steps and the work differ, so the oracle is the definition
 * itself, computed by textbook algorithms:
 *
 *   oracle_dijkstra       binary-heap Dijkstra with lazy deletion (the theta =
 *                         min rule of Table 2 run one vertex at a time).
 *   oracle_bellman_ford   rounds over all arcs until nothing changes (at most
 *                         n - 1 rounds); brute force for tiny graphs.
 *   oracle_floyd_warshall all pairs over an n x n matrix; brute force.
 *   oracle_certificate    linear-time check that an array IS the distance
 *                         array: d[s] = 0, no tense arc, and every finite vertex
 *                         reachable from s over tight arcs.
 *   oracle_hop_depth      fewest arcs on a shortest path to each vertex (the
 *                         hop distance of Sec. 2; k_n is its maximum).
 *
 * No distance sum can overflow: n < 2^31 and weights < 2^32 keep every simple
 * path below 2^63; sums are only formed from finite tentative distances.
 *
 * Graph arrays: offsets int64[n+1] (offsets[0] = 0, non-decreasing,
 * offsets[n] = m), targets int32[m] in [0, n), weights uint32[m].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define INF UINT64_MAX

/* ---------------------------------------------------------------------- */
/* Binary min-heap of (key, vertex) pairs; duplicates allowed (lazy deletion). */

typedef struct {
  uint64_t key;
  int32_t v;
} hitem;

typedef struct {
  hitem* a;
  int64_t size, cap;
} heap;

static int heap_push(heap* h, uint64_t key, int32_t v) {
  if (h->size == h->cap) {
    int64_t nc = h->cap ? 2 * h->cap : 1024;
    hitem* na = (hitem*)realloc(h->a, (size_t)nc * sizeof(hitem));
    if (!na) return 1;
    h->a = na;
    h->cap = nc;
  }
  int64_t i = h->size++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->a[p].key <= key) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i].key = key;
  h->a[i].v = v;
  return 0;
}

static hitem heap_pop(heap* h) {
  hitem top = h->a[0];
  hitem last = h->a[--h->size];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->size) break;
    if (c + 1 < h->size && h->a[c + 1].key < h->a[c].key) ++c;
    if (last.key <= h->a[c].key) break;
    h->a[i] = h->a[c];
    i = c;
  }
  if (h->size > 0) h->a[i] = last;
  return top;
}

/* ---------------------------------------------------------------------- */

/*
 * Dijkstra from `src`. Writes dist[0..n). If `max_settled` > 0 the search
 * stops after that many vertices are settled (dist then holds tentative values
 * for the rest); `settled_out` / `scanned_out` (nullable) receive the number of
 * settled vertices and the number of arcs scanned out of them.
 * Returns 0, or 1 on bad arguments / allocation failure.
 */
int oracle_dijkstra(int64_t n, const int64_t* off, const int32_t* tgt, const uint32_t* w, int32_t src,
                    uint64_t* dist, int64_t max_settled, int64_t* settled_out, int64_t* scanned_out) {
  if (n <= 0 || src < 0 || src >= n || !off || !dist) return 1;
  for (int64_t v = 0; v < n; ++v) dist[v] = INF;
  unsigned char* done = (unsigned char*)calloc((size_t)n, 1);
  if (!done) return 1;
  heap h = {0, 0, 0};
  dist[src] = 0;
  if (heap_push(&h, 0, src)) {
    free(done);
    return 1;
  }
  int64_t settled = 0, scanned = 0;
  int rc = 0;
  while (h.size > 0) {
    hitem it = heap_pop(&h);
    int32_t u = it.v;
    if (done[u] || it.key != dist[u]) continue; /* stale entry */
    done[u] = 1;
    ++settled;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = tgt[e];
      uint64_t nd = dist[u] + (uint64_t)w[e];
      ++scanned;
      if (nd < dist[v]) {
        dist[v] = nd;
        if (heap_push(&h, nd, v)) {
          rc = 1;
          break;
        }
      }
    }
    if (rc || (max_settled > 0 && settled >= max_settled)) break;
  }
  free(h.a);
  free(done);
  if (settled_out) *settled_out = settled;
  if (scanned_out) *scanned_out = scanned;
  return rc;
}

/*
 * Bellman-Ford: repeat a pass that relaxes every arc (u, v) with d[u] finite,
 * until a pass changes nothing. With non-negative weights this ends after at
 * most n passes. Returns the number of passes that changed something, or -1.
 */
int64_t oracle_bellman_ford(int64_t n, const int64_t* off, const int32_t* tgt, const uint32_t* w, int32_t src,
                            uint64_t* dist) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  for (int64_t v = 0; v < n; ++v) dist[v] = INF;
  dist[src] = 0;
  int64_t rounds = 0;
  for (int64_t r = 0; r < n; ++r) {
    int changed = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (dist[u] == INF) continue;
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        uint64_t nd = dist[u] + (uint64_t)w[e];
        if (nd < dist[tgt[e]]) {
          dist[tgt[e]] = nd;
          changed = 1;
        }
      }
    }
    if (!changed) break;
    ++rounds;
  }
  return rounds;
}

/*
 * Floyd-Warshall over all pairs: D[i*n + j] = d(i, j). Parallel arcs take the
 * smallest weight; self-loops never beat d(i, i) = 0. Intended for n <= ~512.
 */
int oracle_floyd_warshall(int64_t n, const int64_t* off, const int32_t* tgt, const uint32_t* w, uint64_t* D) {
  if (n <= 0) return 1;
  for (int64_t i = 0; i < n * n; ++i) D[i] = INF;
  for (int64_t i = 0; i < n; ++i) D[i * n + i] = 0;
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int64_t v = tgt[e];
      if ((uint64_t)w[e] < D[u * n + v]) D[u * n + v] = w[e];
    }
  for (int64_t k = 0; k < n; ++k)
    for (int64_t i = 0; i < n; ++i) {
      uint64_t dik = D[i * n + k];
      if (dik == INF) continue;
      for (int64_t j = 0; j < n; ++j) {
        uint64_t dkj = D[k * n + j];
        if (dkj == INF) continue;
        if (dik + dkj < D[i * n + j]) D[i * n + j] = dik + dkj;
      }
    }
  return 0;
}

/*
 * Certificate that `dist` is the exact distance array from `src`
 * (non-negative weights):
 *   (i)   dist[src] == 0;
 *   (ii)  no tense arc: for every arc (u, v, w) with dist[u] finite,
 *         dist[v] <= dist[u] + w;
 *   (iii) a search from src over tight arcs (dist[u] + w == dist[v]) reaches
 *         every vertex whose dist is finite.
 * (iii) shows each finite dist[v] is the length of a real path, hence
 * dist >= d; (ii) by induction along a shortest path shows dist <= d.
 * Returns 0 if valid, else the number of the failed condition (1, 2, 3);
 * *bad receives a witness vertex. Returns 4 on allocation failure.
 */
int oracle_certificate(int64_t n, const int64_t* off, const int32_t* tgt, const uint32_t* w, int32_t src,
                       const uint64_t* dist, int64_t* bad) {
  *bad = -1;
  if (dist[src] != 0) {
    *bad = src;
    return 1;
  }
  for (int64_t u = 0; u < n; ++u) {
    if (dist[u] == INF) continue;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      if (dist[tgt[e]] > dist[u] + (uint64_t)w[e]) {
        *bad = tgt[e];
        return 2;
      }
    }
  }
  unsigned char* seen = (unsigned char*)calloc((size_t)n, 1);
  int32_t* stack = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!seen || !stack) {
    free(seen);
    free(stack);
    return 4;
  }
  int64_t top = 0;
  seen[src] = 1;
  stack[top++] = src;
  while (top > 0) {
    int32_t u = stack[--top];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = tgt[e];
      if (!seen[v] && dist[u] + (uint64_t)w[e] == dist[v]) {
        seen[v] = 1;
        stack[top++] = v;
      }
    }
  }
  int rc = 0;
  for (int64_t v = 0; v < n; ++v)
    if (dist[v] != INF && !seen[v]) {
      *bad = v;
      rc = 3;
      break;
    }
  free(seen);
  free(stack);
  return rc;
}

/*
 * Hop depth: hop[v] = the fewest arcs on any shortest s ~> v path, -1 if v is
 * unreachable. Every path made of tight arcs from s is a shortest path, so
 * this is the breadth-first level of v in the tight-arc subgraph. `dist` must
 * be the exact distance array. Returns max hop (k_n) or -1 on error.
 */
int64_t oracle_hop_depth(int64_t n, const int64_t* off, const int32_t* tgt, const uint32_t* w, int32_t src,
                         const uint64_t* dist, int32_t* hop) {
  int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!queue) return -1;
  for (int64_t v = 0; v < n; ++v) hop[v] = -1;
  int64_t head = 0, tail = 0, kmax = 0;
  hop[src] = 0;
  queue[tail++] = src;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = tgt[e];
      if (hop[v] < 0 && dist[u] + (uint64_t)w[e] == dist[v]) {
        hop[v] = hop[u] + 1;
        if (hop[v] > kmax) kmax = hop[v];
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return kmax;
}

/* Monotonic wall-clock seconds, for the CPU-baseline timing. */
double oracle_now(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}
