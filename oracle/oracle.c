/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, single-threaded CPU implementation of what the GPU library
 * computes, written from the GraphIt paper (Zhang et al., "GraphIt: A
 * High-Performance Graph DSL", OOPSLA 2018).  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU library
 * neither links nor calls it, and it shares no code with the library.
 *
 * Floating point is IEEE double throughout.  Every function states the
 * passage it follows.  The exhaustive and closed-form pins that tie it to
 * the mathematics live in tests/test_oracle_pins.py.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* Adjacency build.                                                          */
/* The edgeset of the algorithm language (section 3, data model) is a set of */
/* directed (src, dst) pairs.  Reading: self-loops are dropped and repeated  */
/* pairs collapse to one edge; when weights are given the smallest weight of */
/* a repeated pair is kept.  Rows are sorted by neighbour id.               */
/* Returns the number of edges kept, or -1 on bad input, -2 on no memory.   */
/* Build a CSC by passing (dst, src) in place of (src, dst).                */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t v; uint32_t w; } or_pair;

static int pair_cmp(const void* a, const void* b) {
  const or_pair* x = (const or_pair*)a;
  const or_pair* y = (const or_pair*)b;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  if (x->w != y->w) return x->w < y->w ? -1 : 1;
  return 0;
}

int64_t or_build_adj(int32_t n, int64_t m_raw, const int32_t* src, const int32_t* dst,
                     const uint32_t* w, int32_t* off, int32_t* idx, uint32_t* wout) {
  if (n < 0 || m_raw < 0) return -1;
  for (int64_t e = 0; e < m_raw; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  or_pair* tmp = (or_pair*)malloc(sizeof(or_pair) * (size_t)(m_raw > 0 ? m_raw : 1));
  if (!cnt || !tmp) { free(cnt); free(tmp); return -2; }
  for (int64_t e = 0; e < m_raw; ++e)
    if (src[e] != dst[e]) cnt[src[e] + 1]++;
  for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  /* bucket the kept records by source */
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!cur) { free(cnt); free(tmp); return -2; }
  memcpy(cur, cnt, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t e = 0; e < m_raw; ++e) {
    if (src[e] == dst[e]) continue;
    or_pair p;
    p.v = dst[e];
    p.w = w ? w[e] : 0u;
    tmp[cur[src[e]]++] = p;
  }
  free(cur);
  /* sort each row, keep the first record of each neighbour */
  int64_t m = 0;
  off[0] = 0;
  for (int32_t u = 0; u < n; ++u) {
    int64_t b = cnt[u], e = cnt[u + 1];
    if (e - b > 1) qsort(tmp + b, (size_t)(e - b), sizeof(or_pair), pair_cmp);
    for (int64_t k = b; k < e; ++k) {
      if (k > b && tmp[k].v == tmp[k - 1].v) continue;
      idx[m] = tmp[k].v;
      if (wout) wout[m] = tmp[k].w;
      ++m;
    }
    if (m > INT32_MAX) { free(cnt); free(tmp); return -1; }
    off[u + 1] = (int32_t)m;
  }
  free(cnt);
  free(tmp);
  return m;
}

/* ------------------------------------------------------------------------ */
/* PageRank (evaluation section: 20 iterations; damping 0.85 as in the      */
/* PageRankDelta program of section 3).  The paper prints no PageRank       */
/* formula; this is the power iteration that its PageRankDelta computes     */
/* when every vertex stays active:                                           */
/*   x_0[v] = 1/n,                                                           */
/*   x_{k+1}[v] = (1-alpha)/n + alpha * sum_{u -> v} x_k[u] / outdeg(u).     */
/* Rank only flows along out-edges, so vertices without out-edges pass      */
/* nothing on.  Pull form over the in-adjacency, as in the DensePull figure.*/
/* ------------------------------------------------------------------------ */
int or_pagerank(int32_t n, const int32_t* out_off, const int32_t* in_off,
                const int32_t* in_idx, int32_t iters, double alpha, double* x) {
  if (n <= 0 || iters < 0) return -1;
  double* contrib = (double*)malloc(sizeof(double) * (size_t)n);
  if (!contrib) return -2;
  for (int32_t v = 0; v < n; ++v) x[v] = 1.0 / (double)n;
  for (int32_t k = 0; k < iters; ++k) {
    for (int32_t u = 0; u < n; ++u) {
      int32_t d = out_off[u + 1] - out_off[u];
      contrib[u] = d > 0 ? x[u] / (double)d : 0.0;
    }
    for (int32_t v = 0; v < n; ++v) {
      double s = 0.0;
      for (int32_t e = in_off[v]; e < in_off[v + 1]; ++e) s += contrib[in_idx[e]];
      x[v] = (1.0 - alpha) / (double)n + alpha * s;
    }
  }
  free(contrib);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* PageRankDelta, following the GraphIt program for it (section 3 figure)   */
/* in SparsePush order (section 2 figure): active vertices push             */
/* Delta/OutDegree into DeltaSum of their out-neighbours, then every vertex */
/* updates.  First round: Delta = alpha*DeltaSum + (1-alpha)/n, Rank +=     */
/* Delta, then Delta -= 1/n (the GraphIt program's order).  Later rounds:   */
/* Delta = alpha*DeltaSum, Rank += Delta.  A vertex is active next round    */
/* when |Delta| > eps * Rank.  `active` (may be NULL) receives the frontier */
/* size after each round.                                                   */
/* ------------------------------------------------------------------------ */
int or_prdelta(int32_t n, const int32_t* out_off, const int32_t* out_idx, int32_t iters,
               double alpha, double eps, double* rank, int64_t* active) {
  if (n <= 0 || iters < 0) return -1;
  double* delta = (double*)malloc(sizeof(double) * (size_t)n);
  double* dsum = (double*)calloc((size_t)n, sizeof(double));
  uint8_t* in_f = (uint8_t*)malloc((size_t)n);
  if (!delta || !dsum || !in_f) { free(delta); free(dsum); free(in_f); return -2; }
  const double inv_n = 1.0 / (double)n;
  for (int32_t v = 0; v < n; ++v) {
    rank[v] = 0.0;
    delta[v] = inv_n;
    in_f[v] = 1;
  }
  for (int32_t round = 1; round <= iters; ++round) {
    for (int32_t u = 0; u < n; ++u) {
      if (!in_f[u]) continue;
      int32_t d = out_off[u + 1] - out_off[u];
      for (int32_t e = out_off[u]; e < out_off[u + 1]; ++e) dsum[out_idx[e]] += delta[u] / (double)d;
    }
    int64_t cnt = 0;
    for (int32_t v = 0; v < n; ++v) {
      if (round == 1) {
        delta[v] = alpha * dsum[v] + (1.0 - alpha) * inv_n;
        rank[v] += delta[v];
        delta[v] -= inv_n;
      } else {
        delta[v] = alpha * dsum[v];
        rank[v] += delta[v];
      }
      dsum[v] = 0.0;
      double ad = delta[v] < 0 ? -delta[v] : delta[v];
      in_f[v] = ad > eps * rank[v];
      cnt += in_f[v];
    }
    if (active) active[round - 1] = cnt;
  }
  free(delta);
  free(dsum);
  free(in_f);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* BFS (evaluation section, algorithms paragraph): level[v] = fewest edges  */
/* on a path s -> v along out-edges, -1 when unreachable.  Plain FIFO queue */
/* over the out-adjacency; parent[v] = the vertex that first discovered v,  */
/* parent[s] = s, -1 when unreachable.  Returns the number of levels.       */
/* ------------------------------------------------------------------------ */
int32_t or_bfs(int32_t n, const int32_t* off, const int32_t* idx, int32_t s, int32_t* level,
               int32_t* parent) {
  if (n <= 0 || s < 0 || s >= n) return -1;
  int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!q) return -2;
  for (int32_t v = 0; v < n; ++v) {
    level[v] = -1;
    if (parent) parent[v] = -1;
  }
  int64_t head = 0, tail = 0;
  level[s] = 0;
  if (parent) parent[s] = s;
  q[tail++] = s;
  int32_t depth = 0;
  while (head < tail) {
    int32_t u = q[head++];
    if (level[u] + 1 > depth) depth = level[u] + 1;
    for (int32_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = idx[e];
      if (level[v] == -1) {
        level[v] = level[u] + 1;
        if (parent) parent[v] = u;
        q[tail++] = v;
      }
    }
  }
  free(q);
  return depth;
}

/* ------------------------------------------------------------------------ */
/* Connected components by synchronous label propagation (evaluation        */
/* section, algorithms paragraph).  Edges are taken in both directions      */
/* (weak components: the paper runs CC on directed inputs too).             */
/*   L_0 = id, F_0 = V;  per round, L_new = L_old, and for every edge {u,v} */
/*   with u in F: L_new[v] = min(L_new[v], L_old[u]) (and symmetrically);   */
/*   F_next = {v : L_new[v] < L_old[v]}; stop when F is empty.             */
/* Returns the number of rounds executed (the last one yields empty F).     */
/* ------------------------------------------------------------------------ */
int32_t or_cc(int32_t n, const int32_t* off, const int32_t* idx, int32_t* label) {
  if (n <= 0) return -1;
  int32_t* old = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t* in_f = (uint8_t*)malloc((size_t)n);
  if (!old || !in_f) { free(old); free(in_f); return -2; }
  for (int32_t v = 0; v < n; ++v) {
    label[v] = v;
    in_f[v] = 1;
  }
  int32_t rounds = 0;
  int64_t fsize = n;
  while (fsize > 0) {
    memcpy(old, label, sizeof(int32_t) * (size_t)n);
    for (int32_t u = 0; u < n; ++u) {
      for (int32_t e = off[u]; e < off[u + 1]; ++e) {
        int32_t v = idx[e];
        if (in_f[u] && old[u] < label[v]) label[v] = old[u];
        if (in_f[v] && old[v] < label[u]) label[u] = old[v];
      }
    }
    fsize = 0;
    for (int32_t v = 0; v < n; ++v) {
      in_f[v] = label[v] < old[v];
      fsize += in_f[v];
    }
    ++rounds;
  }
  free(old);
  free(in_f);
  return rounds;
}

/* ------------------------------------------------------------------------ */
/* Connected components by union-find over the raw edge records: the        */
/* alternative algorithm the paper names for CC, with the same unique       */
/* result as or_cc (weak components, label = least vertex id of the         */
/* component).  Every record {u, v} joins the sets of u and v.  A set's     */
/* root is kept at its least id (the larger root is linked under the        */
/* smaller), and path halving only moves a parent pointer to a smaller id,  */
/* so every parent id is at most the vertex's own: one pass in increasing   */
/* id then sets each label from its parent's final label.  Needs no         */
/* adjacency, so it also serves graphs too large for the CSR oracles.       */
/* Returns the number of components, -1 on bad input.                       */
/* ------------------------------------------------------------------------ */
static int32_t uf_find(int32_t* p, int32_t x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

int64_t or_cc_union_find(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         int32_t* label) {
  if (n <= 0 || m < 0) return -1;
  for (int32_t v = 0; v < n; ++v) label[v] = v;
  for (int64_t e = 0; e < m; ++e) {
    const int32_t u = src[e], v = dst[e];
    if (u < 0 || u >= n || v < 0 || v >= n) return -1;
    const int32_t ru = uf_find(label, u), rv = uf_find(label, v);
    if (ru < rv) label[rv] = ru;
    else if (rv < ru) label[ru] = rv;
  }
  int64_t comps = 0;
  for (int32_t v = 0; v < n; ++v) {
    label[v] = label[label[v]];
    comps += label[v] == v;
  }
  return comps;
}

/* ------------------------------------------------------------------------ */
/* SSSP reference: Dijkstra with a binary heap and 64-bit tentative         */
/* distances.  dist[v] = least total weight of an s -> v path, UINT32_MAX   */
/* when unreachable.  Returns 0, or -5 when a finite distance does not fit  */
/* below UINT32_MAX.                                                        */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t d; int32_t v; } or_item;

static void heap_push(or_item* h, int64_t* size, or_item it) {
  int64_t i = (*size)++;
  h[i] = it;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= h[i].d) break;
    or_item t = h[p]; h[p] = h[i]; h[i] = t;
    i = p;
  }
}

static or_item heap_pop(or_item* h, int64_t* size) {
  or_item top = h[0];
  h[0] = h[--(*size)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, b = i;
    if (l < *size && h[l].d < h[b].d) b = l;
    if (r < *size && h[r].d < h[b].d) b = r;
    if (b == i) break;
    or_item t = h[b]; h[b] = h[i]; h[i] = t;
    i = b;
  }
  return top;
}

int or_dijkstra(int32_t n, const int32_t* off, const int32_t* idx, const uint32_t* w, int32_t s,
                uint32_t* dist) {
  if (n <= 0 || s < 0 || s >= n) return -1;
  int64_t m = off[n];
  uint64_t* d = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  or_item* h = (or_item*)malloc(sizeof(or_item) * (size_t)(m + 1));
  uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
  if (!d || !h || !done) { free(d); free(h); free(done); return -2; }
  for (int32_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
  int64_t hs = 0;
  d[s] = 0;
  or_item it0 = {0, s};
  heap_push(h, &hs, it0);
  while (hs > 0) {
    or_item it = heap_pop(h, &hs);
    if (done[it.v]) continue;
    done[it.v] = 1;
    for (int32_t e = off[it.v]; e < off[it.v + 1]; ++e) {
      int32_t v = idx[e];
      uint64_t nd = it.d + (uint64_t)w[e];
      if (nd < d[v]) {
        d[v] = nd;
        or_item x = {nd, v};
        heap_push(h, &hs, x);
      }
    }
  }
  int rc = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (d[v] == UINT64_MAX) dist[v] = UINT32_MAX;
    else if (d[v] >= (uint64_t)UINT32_MAX) { dist[v] = UINT32_MAX; rc = -5; }
    else dist[v] = (uint32_t)d[v];
  }
  free(d);
  free(h);
  free(done);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* SSSP as the paper's evaluation runs it: frontier-based Bellman-Ford with */
/* a min reduction (evaluation section; the asyncMin reduction of the       */
/* compiler section).  Synchronous rounds: D_new = D_old; for u in F and    */
/* u -> v: D_new[v] = min(D_new[v], D_old[u] + w); F = {v: D_new < D_old}. */
/* Returns the number of rounds, or -5 on distance overflow.                */
/* ------------------------------------------------------------------------ */
int32_t or_bellman_ford(int32_t n, const int32_t* off, const int32_t* idx, const uint32_t* w,
                        int32_t s, uint32_t* dist) {
  if (n <= 0 || s < 0 || s >= n) return -1;
  uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  uint64_t* nxt = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  uint8_t* in_f = (uint8_t*)calloc((size_t)n, 1);
  if (!cur || !nxt || !in_f) { free(cur); free(nxt); free(in_f); return -2; }
  for (int32_t v = 0; v < n; ++v) cur[v] = UINT64_MAX;
  cur[s] = 0;
  in_f[s] = 1;
  int64_t fsize = 1;
  int32_t rounds = 0;
  while (fsize > 0) {
    memcpy(nxt, cur, sizeof(uint64_t) * (size_t)n);
    for (int32_t u = 0; u < n; ++u) {
      if (!in_f[u]) continue;
      for (int32_t e = off[u]; e < off[u + 1]; ++e) {
        uint64_t nd = cur[u] + (uint64_t)w[e];
        if (nd < nxt[idx[e]]) nxt[idx[e]] = nd;
      }
    }
    fsize = 0;
    for (int32_t v = 0; v < n; ++v) {
      in_f[v] = nxt[v] < cur[v];
      fsize += in_f[v];
    }
    uint64_t* t = cur; cur = nxt; nxt = t;
    ++rounds;
  }
  int32_t rc = rounds;
  for (int32_t v = 0; v < n; ++v) {
    if (cur[v] == UINT64_MAX) dist[v] = UINT32_MAX;
    else if (cur[v] >= (uint64_t)UINT32_MAX) { dist[v] = UINT32_MAX; rc = -5; }
    else dist[v] = (uint32_t)cur[v];
  }
  free(cur);
  free(nxt);
  free(in_f);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Betweenness centrality, one source (the paper's BC, two labelled applies: */
/* a forward BFS that counts shortest paths, then a backward sweep of the   */
/* dependencies), as defined by Brandes ("A faster algorithm for            */
/* betweenness centrality", J. Math. Sociol. 2001):                         */
/*   sigma[s] = 1; sigma[w] = sum of sigma[v] over v -> w with              */
/*   level[v] = level[w] - 1;                                                */
/*   delta[v] = sum over v -> w with level[w] = level[v] + 1 of             */
/*              sigma[v] / sigma[w] * (1 + delta[w]);                       */
/* delta[s] = 0 and 0 for unreachable vertices.  FIFO order, fp64.          */
/* ------------------------------------------------------------------------ */
int or_bc(int32_t n, const int32_t* off, const int32_t* idx, int32_t s, double* delta,
          double* sigma_out) {
  if (n <= 0 || s < 0 || s >= n) return -1;
  int32_t* level = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  double* sigma = (double*)calloc((size_t)n, sizeof(double));
  if (!level || !order || !sigma) { free(level); free(order); free(sigma); return -2; }
  for (int32_t v = 0; v < n; ++v) { level[v] = -1; delta[v] = 0.0; }
  level[s] = 0;
  sigma[s] = 1.0;
  int32_t head = 0, tail = 0;
  order[tail++] = s;
  while (head < tail) {
    const int32_t v = order[head++];
    for (int32_t e = off[v]; e < off[v + 1]; ++e) {
      const int32_t w = idx[e];
      if (level[w] < 0) { level[w] = level[v] + 1; order[tail++] = w; }
      if (level[w] == level[v] + 1) sigma[w] += sigma[v];
    }
  }
  for (int32_t i = tail - 1; i >= 0; --i) {
    const int32_t v = order[i];
    double acc = 0.0;
    for (int32_t e = off[v]; e < off[v + 1]; ++e) {
      const int32_t w = idx[e];
      if (level[w] == level[v] + 1) acc += sigma[v] / sigma[w] * (1.0 + delta[w]);
    }
    delta[v] = v == s ? 0.0 : acc;
  }
  if (sigma_out) memcpy(sigma_out, sigma, sizeof(double) * (size_t)n);
  free(level);
  free(order);
  free(sigma);
  return tail;
}

/* ------------------------------------------------------------------------ */
/* Eigenvector centrality by power iteration (the kernel the paper fuses    */
/* with PageRank in its program-structure optimizations; the paper gives no */
/* formula, this is the textbook one):                                      */
/*   x_0[v] = 1/n;  y[v] = sum_{u -> v} x_k[u];  x_{k+1} = y / ||y||_2,     */
/* and x_{k+1} = 0 when ||y|| = 0.  Pull order over the in-adjacency, fp64. */
/* ------------------------------------------------------------------------ */
int or_eigenvector(int32_t n, const int32_t* in_off, const int32_t* in_idx, int32_t iters,
                   double* x) {
  if (n <= 0 || iters < 0) return -1;
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  if (!y) return -2;
  for (int32_t v = 0; v < n; ++v) x[v] = 1.0 / (double)n;
  for (int32_t k = 0; k < iters; ++k) {
    double ss = 0.0;
    for (int32_t v = 0; v < n; ++v) {
      double s = 0.0;
      for (int32_t e = in_off[v]; e < in_off[v + 1]; ++e) s += x[in_idx[e]];
      y[v] = s;
      ss += s * s;
    }
    const double norm = sqrt(ss);
    for (int32_t v = 0; v < n; ++v) x[v] = norm > 0.0 ? y[v] / norm : 0.0;
  }
  free(y);
  return 0;
}
