// BFS device routines shared by the frontier engine (algos.hip) and the
// batched persistent kernel (batch.hip).
#pragma once

#include "kernels.h"

namespace gi {

struct BfsVisit {
  const int32_t* idx;
  int32_t* level;
  int32_t* parent;
  int l1;
  DenseSet next;
  uint64_t* vis;
  const int32_t* deg = nullptr;  // when set: count the claimed vertices and their degrees
  long long work = 0, found = 0, found_deg = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    if (!valid) return;
    const int v = idx[e];
    ++work;
    if (level[v] >= 0) return;
    if (atomicCAS(&level[v], -1, l1) != -1) return;
    if (parent) parent[v] = u;
    next.insert(v);
    atomicOr((unsigned long long*)&vis[v >> 6], 1ull << (v & 63));
    if (deg) {
      ++found;
      found_deg += deg[v];
    }
  }
};

// DensePull: a wave owns 64-vertex words and takes G of them at a time, so
// the dependent load chains of G words (visited word -> in-row bounds ->
// in-neighbour ids -> frontier bits) overlap instead of running one after
// another.  Each unvisited lane first tests its in-neighbour of largest
// out-degree (`in_probe`, a coalesced load): an unvisited vertex's
// in-neighbours are all either in the frontier or unvisited, and hubs are
// reached early, so in the large pull levels this test usually succeeds
// and the in-row, whose first line would otherwise be fetched for just one
// or two ids, is never read.  Lanes still open test their first in-edges
// in two batches of four independent loads; the rows still open are then
// concatenated and walked 64 edges per round across the wave.  A row stops
// at its first source in the frontier (the probe, else in in-edge order).  The next frontier word and the
// visited word are written whole, without atomics.
// Words [wbeg, wend) are covered by waves wave0, wave0 + nwaves, ...; with
// `deg` set, the claimed vertices and their degrees are accumulated
// degrees (*nfound, *nfound_deg).
template <int BT, int G = 4>
__device__ long long bfs_pull_range(const BfsArgs& b, int l1, int wbeg, int wend, int wave0,
                                    int nwaves, const int32_t* deg, long long* nfound,
                                    long long* nfound_deg) {
  const DevGraph& g = b.g;
  const int n = g.n, W = wend, lane = __lane_id();
  const DenseSet cur = b.cur, nxt = b.next;
  long long work = 0;
  for (int wb = wbeg + wave0; wb < W; wb += G * nwaves) {
    uint64_t vw[G];
    bool cand[G], found[G];
    int j[G], e[G], par[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int w = wb + q * nwaves;  // wave-uniform
      const int v = (w << 6) + lane;
      vw[q] = w < W ? b.vis[w] : ~0ull;
      cand[q] = w < W && v < n && !((vw[q] >> lane) & 1ull);
      found[q] = false;
      par[q] = -1;
      j[q] = 0;
      e[q] = 0;
    }
    int pb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      pb[q] = -1;
      if (cand[q]) {
        const int v = ((wb + q * nwaves) << 6) + lane;
        if (g.in_probe) pb[q] = g.in_probe[v];
        j[q] = g.in_off[v];
        e[q] = g.in_off[v + 1];
      }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      if (pb[q] >= 0) {
        ++work;
        if (cur.test(pb[q])) {
          found[q] = true;
          par[q] = pb[q];
        }
      }
    }
#pragma unroll
    for (int batch = 0; batch < 2; ++batch) {
      int u[G][4];
#pragma unroll
      for (int q = 0; q < G; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          u[q][r] = (cand[q] && !found[q] && j[q] + r < e[q]) ? g.in_idx[j[q] + r] : -1;
      bool h[G][4];
#pragma unroll
      for (int q = 0; q < G; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) h[q][r] = u[q][r] >= 0 && cur.test(u[q][r]);
#pragma unroll
      for (int q = 0; q < G; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!found[q] && u[q][r] >= 0) {
            ++work;
            if (h[q][r]) {
              found[q] = true;
              par[q] = u[q][r];
            }
          }
        }
        if (!found[q]) j[q] = min(e[q], j[q] + 4);
      }
    }
    // Rows still open are walked as one concatenated edge list per word,
    // 64 edges per round spread over the lanes; a row leaves the list at
    // its first frontier hit.
    for (;;) {
      int rem[G], ex[G], tot[G];
      bool more = false;
#pragma unroll
      for (int q = 0; q < G; ++q) {
        rem[q] = (cand[q] && !found[q]) ? e[q] - j[q] : 0;
        ex[q] = wave_excl_scan(rem[q], &tot[q]);
        more |= tot[q] > 0;
      }
      if (!more) break;  // wave-uniform
      int uu[G];
      bool hit[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        // owner of list position `lane`: the last lane whose list starts at
        // or before it (later lanes with empty rows start after it)
        int own = 0;
#pragma unroll
        for (int st = 32; st > 0; st >>= 1) {
          const int c = own + st;
          const int exc = __shfl(ex[q], c < kWave ? c : kWave - 1, kWave);
          if (c < kWave && exc <= lane) own = c;
        }
        const int jo = __shfl(j[q], own, kWave);
        const int eo = __shfl(ex[q], own, kWave);
        const bool act = lane < tot[q];
        uu[q] = act ? g.in_idx[jo + (lane - eo)] : 0;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) hit[q] = lane < tot[q] && cur.test(uu[q]);
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const unsigned long long hm = __ballot(hit[q]);
        // this lane's positions in the round: [a, b)
        const int a = ex[q], b = min(kWave, ex[q] + rem[q]);
        const bool mine = rem[q] > 0 && a < kWave;
        unsigned long long span = 0ull;
        if (mine) {
          const unsigned long long hi = b >= kWave ? ~0ull : ((1ull << b) - 1ull);
          span = hi & ~((1ull << a) - 1ull);
        }
        const unsigned long long mh = hm & span;
        const int first = mh ? __ffsll((long long)mh) - 1 : 0;
        const int pu = __shfl(uu[q], first, kWave);
        if (mine) {
          if (mh) {
            found[q] = true;
            par[q] = pu;
            work += first - a + 1;
          } else {
            work += b - a;
            j[q] += b - a;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int w = wb + q * nwaves;
      if (w >= W) break;  // wave-uniform
      const int v = (w << 6) + lane;
      const unsigned long long fm = __ballot(found[q]);
      if (found[q]) {
        b.level[v] = l1;
        if (b.parent) b.parent[v] = par[q];
        if (deg) {
          ++*nfound;
          *nfound_deg += deg[v];
        }
      }
      if (nxt.bm) {
        nxt.bm[v] = found[q] ? 1 : 0;  // the bool map is padded to whole words
      } else if (lane == 0) {
        nxt.bv[w] = fm;
      }
      if (lane == 0) b.vis[w] = vw[q] | fm;
    }
  }
  return work;
}

}  // namespace gi
