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
    visit(u, idx[e]);
  }
  // The visited bitvector (n/8 bytes, cache resident) filters targets
  // before the level array (4n bytes, a line per random access) is touched;
  // a bit still clear from a stale copy only costs the CAS, which decides.
  __device__ __forceinline__ void visit(int u, int v) {
    ++work;
    if ((vis[v >> 6] >> (v & 63)) & 1ull) return;
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

// Push of the frontier's hubs (rows longer than kHubDeg, listed per graph)
// by all k workgroups of a batch task, workgroup r taking the r-th of k
// equal slices of each row, four edges in flight per thread.  Without it a
// hub's whole row falls to the one workgroup that owns its frontier word.
template <int BT>
__device__ void push_hubs(const int32_t* hubs, int nhubs, const DenseSet& cur,
                          const int32_t* off, const int32_t* idx, int r, int k, BfsVisit& vis) {
  __shared__ int s_h[BT];
  __shared__ int s_cnt;
  const int tid = threadIdx.x;
  for (int h0 = 0; h0 < nhubs; h0 += BT) {
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    const int h = h0 + tid;
    if (h < nhubs && cur.test(hubs[h])) s_h[atomicAdd(&s_cnt, 1)] = hubs[h];
    __syncthreads();
    const int cnt = s_cnt;
    for (int i = 0; i < cnt; ++i) {
      const int u = s_h[i];
      const long long beg = off[u], len = (long long)off[u + 1] - beg;
      const int s0 = (int)(beg + len * r / k), s1 = (int)(beg + len * (r + 1) / k);
      for (int e = s0 + tid; e < s1; e += 4 * BT) {
        int v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = e + q * BT < s1 ? idx[e + q * BT] : -1;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (v[q] >= 0) vis.visit(u, v[q]);
      }
    }
    __syncthreads();
  }
}

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
// at its first source in the frontier (the probe, else in scan order).
// The scan order is the graph's BFS copy of the in-rows when it has one:
// sources by decreasing out-degree, so a row begins with its probe (skipped)
// and goes on with the sources most likely to be on the frontier; on R-MAT
// 22 that halves the edges scanned after a probe miss and the rows that
// need the round loop.  The next frontier word and the visited word are
// written whole, without atomics.
// Words [wbeg, wend) are covered by waves wave0, wave0 + nwaves, ...; with
// `deg` set, the claimed vertices and their degrees are accumulated
// degrees (*nfound, *nfound_deg).
template <int BT, int G = 4>
__device__ long long bfs_pull_range(const BfsArgs& b, int l1, int wbeg, int wend, int wave0,
                                    int nwaves, const int32_t* deg, long long* nfound,
                                    long long* nfound_deg) {
  const DevGraph& g = b.g;
  const int n = g.n, W = wend, lane = __lane_id();
  // rows led by their probe: the scan starts after it
  const int32_t* in_idx = g.bfs_idx ? g.bfs_idx : g.in_idx;
  const int skip = g.bfs_idx ? 1 : 0;
  const DenseSet cur = b.cur, nxt = b.next;
  long long work = 0;
  // visited words of the next group are loaded one group ahead (only this
  // wave writes them in this step)
  uint64_t vn[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int w = wbeg + wave0 + q * nwaves;
    vn[q] = w < W ? b.vis[w] : ~0ull;
  }
  for (int wb = wbeg + wave0; wb < W; wb += G * nwaves) {
    uint64_t vw[G];
    bool cand[G], found[G];
    int j[G], e[G], par[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      vw[q] = vn[q];
      const int wn = wb + G * nwaves + q * nwaves;
      vn[q] = wn < W ? b.vis[wn] : ~0ull;
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int w = wb + q * nwaves;  // wave-uniform
      const int v = (w << 6) + lane;
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
        if (pb[q] >= 0) j[q] += skip;
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
          u[q][r] = (cand[q] && !found[q] && j[q] + r < e[q]) ? in_idx[j[q] + r] : -1;
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
        uu[q] = act ? in_idx[jo + (lane - eo)] : 0;
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
