/*
 * Seeded synthetic input generators (raw edge lists).
 *
 * This module produces the inputs that both the CPU oracle and the GPU
 * library consume.  It holds none of the graph method's arithmetic: no
 * adjacency build, no de-duplication, no traversal.  Every random number is
 * drawn from a counter-based generator keyed by (seed, stream, index), so a
 * result does not depend on the number of threads that produced it.
 *
 * Counter-based generator: the SplitMix64 output function (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * applied to a Weyl sequence of the index under a per-(seed, stream) key.
 *
 * Generators:
 *   - R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): recursive quadrant
 *     choice per level, followed by a seeded random relabelling of vertices.
 *   - 2-D grid with 4-neighbour undirected edges and uniformly random
 *     long-range shortcut pairs; one uniform integer weight per undirected
 *     edge, emitted identically in both directions.
 *   - Chung-Lu power-law graph: expected degree w_i = c (i + i0)^(-1/(gamma-1)),
 *     endpoints sampled independently from the weight distribution with
 *     Walker/Vose alias tables, followed by a seeded random relabelling.
 *
 * Outputs may contain self-loops and duplicate pairs; removing them is the
 * consumer's job.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t gg_u64(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t key = mix64(seed + GOLDEN * (stream + 1));
  return mix64(key + GOLDEN * (idx + 1));
}

static inline double unif01(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(gg_u64(seed, stream, idx) >> 11) * (1.0 / 9007199254740992.0);
}

/* integer in [0, range) by the multiply-shift reduction of a 32-bit draw */
static inline uint32_t below(uint64_t r, uint32_t range) {
  return (uint32_t)(((r >> 32) * (uint64_t)range) >> 32);
}

/* Random permutation of [0, n) by Fisher-Yates (Durstenfeld) driven by the
 * counter generator on `stream`. */
static void permutation(int32_t n, uint64_t seed, uint64_t stream, int32_t* perm) {
  for (int32_t i = 0; i < n; ++i) perm[i] = i;
  for (int32_t i = n - 1; i > 0; --i) {
    uint32_t j = below(gg_u64(seed, stream, (uint64_t)i), (uint32_t)i + 1u);
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

void gg_permutation(int32_t n, uint64_t seed, uint64_t stream, int32_t* perm) {
  permutation(n, seed, stream, perm);
}

/* R-MAT: nsamp samples over 2^scale vertices. */
int gg_rmat(int scale, int64_t nsamp, double a, double b, double c, uint64_t seed,
            int permute, int32_t* src, int32_t* dst) {
  if (scale < 1 || scale > 30 || nsamp < 0) return -1;
  const double ab = a + b, abc = a + b + c;
  #pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nsamp; ++k) {
    int32_t s = 0, d = 0;
    for (int l = 0; l < scale; ++l) {
      double u = unif01(seed, 0, (uint64_t)k * (uint64_t)scale + (uint64_t)l);
      int32_t bit = 1 << (scale - 1 - l);
      if (u < a) {
      } else if (u < ab) {
        d |= bit;
      } else if (u < abc) {
        s |= bit;
      } else {
        s |= bit;
        d |= bit;
      }
    }
    src[k] = s;
    dst[k] = d;
  }
  if (permute) {
    int32_t n = 1 << scale;
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!perm) return -2;
    permutation(n, seed, 1, perm);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nsamp; ++k) {
      src[k] = perm[src[k]];
      dst[k] = perm[dst[k]];
    }
    free(perm);
  }
  return 0;
}

/* Number of directed edge records gg_grid emits. */
int64_t gg_grid_count(int32_t rows, int32_t cols, int64_t nshort) {
  int64_t und = (int64_t)rows * (cols - 1) + (int64_t)cols * (rows - 1) + nshort;
  return 2 * und;
}

/* 2-D grid, vertex id r*cols + c.  Undirected edge e (horizontal edges first,
 * then vertical, then shortcuts) is emitted as records 2e (u->v) and 2e+1
 * (v->u) with the same weight, uniform in [wlo, whi] when w != NULL. */
int gg_grid(int32_t rows, int32_t cols, int64_t nshort, uint32_t wlo, uint32_t whi,
            uint64_t seed, int32_t* src, int32_t* dst, uint32_t* w) {
  if (rows < 1 || cols < 1 || nshort < 0 || whi < wlo) return -1;
  const int64_t nh = (int64_t)rows * (cols - 1);
  const int64_t nv = (int64_t)cols * (rows - 1);
  const int64_t n = (int64_t)rows * cols;
  const uint32_t range = whi - wlo + 1u;
  const int64_t und = nh + nv + nshort;
  #pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < und; ++e) {
    int64_t u, v;
    if (e < nh) {
      int64_t r = e / (cols - 1), c = e % (cols - 1);
      u = r * cols + c;
      v = u + 1;
    } else if (e < nh + nv) {
      int64_t f = e - nh;
      int64_t r = f / cols, c = f % cols;
      u = r * cols + c;
      v = u + cols;
    } else {
      int64_t j = e - nh - nv;
      u = (int64_t)below(gg_u64(seed, 3, 2 * (uint64_t)j), (uint32_t)n);
      v = (int64_t)below(gg_u64(seed, 3, 2 * (uint64_t)j + 1), (uint32_t)n);
    }
    src[2 * e] = (int32_t)u;
    dst[2 * e] = (int32_t)v;
    src[2 * e + 1] = (int32_t)v;
    dst[2 * e + 1] = (int32_t)u;
    if (w) {
      uint32_t x = wlo + below(gg_u64(seed, 2, (uint64_t)e), range);
      w[2 * e] = x;
      w[2 * e + 1] = x;
    }
  }
  return 0;
}

/* Uniform integer weights in [lo, hi], one per record. */
int gg_uniform_weights(int64_t m, uint32_t lo, uint32_t hi, uint64_t seed, uint32_t* w) {
  if (hi < lo || m < 0) return -1;
  const uint32_t range = hi - lo + 1u;
  #pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) w[k] = lo + below(gg_u64(seed, 8, (uint64_t)k), range);
  return 0;
}

/* Sum of (i + i0)^(-beta) over [0, n), in fixed chunks combined in order so
 * the value does not depend on the thread count. */
static double powsum(int64_t n, double i0, double beta) {
  enum { CH = 1024 };
  double part[CH];
  int64_t step = (n + CH - 1) / CH;
  #pragma omp parallel for schedule(static)
  for (int k = 0; k < CH; ++k) {
    double s = 0.0;
    int64_t lo = (int64_t)k * step, hi = lo + step;
    if (hi > n) hi = n;
    for (int64_t i = hi - 1; i >= lo; --i) s += pow((double)i + i0, -beta);
    part[k] = s;
  }
  double t = 0.0;
  for (int k = 0; k < CH; ++k) t += part[k];
  return t;
}

/* Chung-Lu weights: w_i = dmax * (i0 / (i + i0))^beta with beta = 1/(gamma-1)
 * and i0 chosen by bisection so that sum_i w_i = wsum.  Returns i0. */
double gg_chunglu_weights(int32_t n, double gamma, double dmax, double wsum, double* w) {
  const double beta = 1.0 / (gamma - 1.0);
  double lo = 1e-9, hi = (double)n;
  for (int it = 0; it < 32; ++it) {
    double mid = sqrt(lo * hi);
    double s = dmax * pow(mid, beta) * powsum(n, mid, beta);
    if (s < wsum) lo = mid; else hi = mid;
  }
  double i0 = sqrt(lo * hi);
  double c = dmax * pow(i0, beta);
  if (w) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) w[i] = c * pow((double)i + i0, -beta);
  }
  return i0;
}

/* Walker/Vose alias table over n non-negative weights. */
static int alias_build(int32_t n, const double* w, double* prob, int32_t* alias) {
  double total = 0.0;
  for (int32_t i = 0; i < n; ++i) total += w[i];
  int32_t* small = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* large = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!small || !large) { free(small); free(large); return -2; }
  int32_t ns = 0, nl = 0;
  for (int32_t i = 0; i < n; ++i) {
    prob[i] = w[i] * (double)n / total;
    alias[i] = i;
    if (prob[i] < 1.0) small[ns++] = i; else large[nl++] = i;
  }
  while (ns > 0 && nl > 0) {
    int32_t s = small[--ns], l = large[nl - 1];
    alias[s] = l;
    prob[l] = (prob[l] + prob[s]) - 1.0;
    if (prob[l] < 1.0) { --nl; small[ns++] = l; }
  }
  while (nl > 0) prob[large[--nl]] = 1.0;
  while (ns > 0) prob[small[--ns]] = 1.0;
  free(small);
  free(large);
  return 0;
}

/* Chung-Lu: nsamp records, both endpoints drawn from the weights, then ids
 * relabelled by a random permutation (stream 6). */
int gg_chunglu(int32_t n, int64_t nsamp, double gamma, double dmax, double wsum,
               uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 1 || nsamp < 0 || gamma <= 1.0) return -1;
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  double* prob = (double*)malloc(sizeof(double) * (size_t)n);
  int32_t* alias = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!w || !prob || !alias || !perm) { free(w); free(prob); free(alias); free(perm); return -2; }
  gg_chunglu_weights(n, gamma, dmax, wsum, w);
  int rc = alias_build(n, w, prob, alias);
  if (rc == 0) {
    permutation(n, seed, 6, perm);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nsamp; ++k) {
      for (int side = 0; side < 2; ++side) {
        uint64_t r = gg_u64(seed, 5, 2 * (uint64_t)k + (uint64_t)side);
        uint32_t col = below(r, (uint32_t)n);
        double coin = (double)(r & 0xffffffffULL) * (1.0 / 4294967296.0);
        int32_t v = coin < prob[col] ? (int32_t)col : alias[col];
        if (side == 0) src[k] = perm[v]; else dst[k] = perm[v];
      }
    }
  }
  free(w);
  free(prob);
  free(alias);
  free(perm);
  return rc;
}

/* Erdos-Renyi style multigraph: nsamp records with uniform endpoints. */
int gg_uniform(int32_t n, int64_t nsamp, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 1 || nsamp < 0) return -1;
  #pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nsamp; ++k) {
    src[k] = (int32_t)below(gg_u64(seed, 9, 2 * (uint64_t)k), (uint32_t)n);
    dst[k] = (int32_t)below(gg_u64(seed, 9, 2 * (uint64_t)k + 1), (uint32_t)n);
  }
  return 0;
}

/* k distinct sources chosen uniformly without replacement among vertices that
 * have at least one record to a different vertex (stream 7).  Returns the
 * number chosen (< k when fewer candidates exist). */
int64_t gg_pick_sources(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        int64_t k, uint64_t seed, int32_t* out) {
  uint8_t* has = (uint8_t*)calloc((size_t)n, 1);
  if (!has) return -2;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] != dst[e] && src[e] >= 0 && src[e] < n) has[src[e]] = 1;
  int64_t nc = 0;
  for (int32_t v = 0; v < n; ++v) nc += has[v];
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  if (!cand) { free(has); return -2; }
  nc = 0;
  for (int32_t v = 0; v < n; ++v)
    if (has[v]) cand[nc++] = v;
  free(has);
  if (k > nc) k = nc;
  for (int64_t i = 0; i < k; ++i) {
    uint32_t j = (uint32_t)i + below(gg_u64(seed, 7, (uint64_t)i), (uint32_t)(nc - i));
    int32_t t = cand[i];
    cand[i] = cand[j];
    cand[j] = t;
    out[i] = cand[i];
  }
  free(cand);
  return k;
}
