#!/usr/bin/env python3
"""Benchmark of the traversal hot path on one MI355X.

Default workload (one "step"): direction-optimizing BFS (DensePull-SparsePush,
bitvector frontier, hybrid divisor 20) from 64 seeded sources with out-degree
>= 1, plus connected components by label propagation, on an R-MAT graph of
scale 22 and edge factor 16 ((a,b,c,d) = (.57,.19,.19,.05), seed 2, vertex
ids randomly relabelled, self-loops and repeated pairs removed).  The 64
BFS run as one batched persistent launch (--bfs-path batched, the default:
levels and parents of every source, workgroups per source autotuned) or as
64 plain calls (--bfs-path plain); both are reported.

value = GTEPS = (sum over sources of m_reach(s) + m) / step time, where
m_reach(s) is the number of out-edges of the vertices BFS reaches from s
(Graph500 convention on a directed graph) and CC counts each edge once.

roofline: the dominant kernel is whichever of the BFS kernel (k_batch, or
k_bfs_step on the plain path) and the CC step kernel k_cc_step has the larger
summed GPU time.  Launches are timed with HIP events on the stream they run
on: the batch's graph launch, or per step around the step kernel (per-step
timing; every launch counts, including no-op steps after the frontier
emptied).  Algorithmic bytes come from the per-step byte models below
(bfs_step_bytes, cc_step_bytes) applied to each step's trace entry (|F|,
D_F, edges examined); for k_batch, the sum over the 64 sources' BFS (the
frontiers, and so the bytes, are those of the plain path's traces);
achieved = bytes per launch / mean launch time.

Other workloads (--workload): pr_rmat16 (20-iteration DensePull PageRank on
R-MAT scale 16, the PageRank configuration), pr_rmat22, sssp_grid
(delta-stepping on the 4096x4096 grid with 1% shortcuts, or with none:
--grid-shortcuts 0), selector (learned schedule selector against the hybrid
rule on a held-out Chung-Lu graph), batched (256 BFS/PageRank instances over
14 graphs, one persistent launch against 256 plain calls), prdelta_rmat22,
prec_rmat22 (PageRank fused with eigenvector centrality), bc_rmat22
(betweenness from 8 sources).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS + % HBM peak (PageRank, BFS); learned vs heuristic schedule speedup"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bfs_cc_rmat22",
                    choices=["bfs_cc_rmat22", "pr_rmat16", "pr_rmat22", "sssp_grid", "selector",
                             "batched", "prdelta_rmat22", "prec_rmat22", "bc_rmat22"])
    ap.add_argument("--heldout", default="small", choices=["small", "full"],
                    help="selector workload: held-out Chung-Lu graph with 4M vertices (small) "
                         "or 41M vertices and ~1.4B edges (full)")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--selector-dump", default="",
                    help="selector workload: write the training records, the trained "
                         "parameters and the held-out per-step timings to this .npz")
    ap.add_argument("--grid-shortcuts", type=float, default=0.01,
                    help="sssp_grid: shortcut pairs as a fraction of the vertices (0: the "
                         "plain grid, diameter 8190, the many-phase regime of road graphs)")
    ap.add_argument("--delta-sweep", default="",
                    help="sssp_grid: comma-separated bucket widths for the engine's sweep "
                         "(default: 2^5 ... 2^14 and 1000)")
    ap.add_argument("--sssp-path", default="batched", choices=["batched", "plain"],
                    help="sssp_grid: the 4 sources as one batched launch, or 4 engine runs")
    ap.add_argument("--overlap", type=int, default=1, choices=[0, 1],
                    help="default workload, batched path: run CC on a second stream while "
                         "the BFS batch runs (1) or after it (0)")
    ap.add_argument("--bfs-path", default="batched", choices=["batched", "plain"],
                    help="BFS part of the default workload: the 64 sources as one batched "
                         "persistent launch, or one plain call per source")
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--batch-barrier", default="xcd", choices=["xcd", "agent"],
                    help="barrier of batched tasks: one-XCD tasks only invalidate L1 (xcd, "
                         "the default) or every barrier writes back and invalidates L2 (agent)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-threads", type=int, default=0, choices=[0, 256, 512, 1024],
                    help="default and sssp_grid workloads: pin the batch's workgroup size "
                         "(0: autotuned)")
    ap.add_argument("--batch-workgroups", type=int, default=0,
                    help="default and sssp_grid workloads: pin each task's workgroups "
                         "(0: autotuned)")
    ap.add_argument("--sssp-batch-delta", type=int, default=0,
                    help="sssp_grid: the batched path's bucket width (0: swept)")
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload: skip the batched, road-like SSSP and persistent "
                         "PageRank legs (which launch their own k_batch before this workload's)")
    ap.add_argument("--schedule", default="", help="k=v,... overrides of the schedule")
    ap.add_argument("--json-out", default="")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="first run one elementwise copy of this many MiB (read once, written "
                         "once), a reference dispatch for hardware byte counters")
    return ap.parse_args()


def barrier_scope(args):
    import paper_1805_00923_amd as gi
    return gi.BARRIER_XCD if args.batch_barrier == "xcd" else gi.BARRIER_AGENT


def sched_overrides(text):
    kw = {}
    for part in filter(None, text.split(",")):
        k, v = part.split("=")
        kw[k.strip()] = int(v)
    return kw


# ------------------------------------------------------------- byte model --
# Algorithmic bytes of one launch of a step (edge-traversal) kernel, from the
# step's trace entry.  Compulsory traffic only: every array element the step
# must touch is counted once, random gathers of vertex data at their
# compulsory size.

def bfs_step_bytes(n, dirs, fs, ds, es):
    """Per-step bytes of the BFS step kernel.
      SparsePush/DensePush  12|F| + 8 D_F + 8|F'|   (ids+offsets, index stream +
                                                    level CAS, level+parent of F')
      DensePull             3n/8 + 8U + 4E + 4|F'|  (visited, frontier and next
                                                    bitvectors; offsets of the U
                                                    unvisited rows; E in-edges
                                                    scanned up to the first hit)"""
    out = []
    visited = 0
    k = len(fs)
    for i in range(k):
        f, d, e = int(fs[i]), int(ds[i]), int(es[i])
        fnext = int(fs[i + 1]) if i + 1 < k else 0
        visited += f
        if dirs[i] == 2:
            out.append(3 * n // 8 + 8 * (n - visited) + 4 * e + 4 * fnext)
        else:
            out.append(12 * f + 8 * d + 8 * fnext)
    return out


class PullScanReplay:
    """E_scan of BFS DensePull steps by a host replay in CSC order: at step k
    (frontier: the vertices of level k) every vertex not yet visited scans
    its in-edges in CSC order up to and including the first whose source is
    in the frontier, or all of them when none is.  From the final levels:
    a vertex of level k + 1 stops at its first in-edge from level k; one of
    a later level, or unreached, finds none (an in-neighbour of level k
    would have put it at level k + 1) and scans its whole row."""

    def __init__(self, in_off, in_idx):
        import numpy as np
        self.n = len(in_off) - 1
        self.m = int(in_off[-1])
        self.idx = np.ascontiguousarray(in_idx[:self.m], np.int32)
        self.deg = np.diff(np.asarray(in_off, np.int64))
        self.row = np.repeat(np.arange(self.n, dtype=np.int32), self.deg)
        self.pos = (np.arange(self.m, dtype=np.int64) -
                    np.repeat(np.asarray(in_off[:-1], np.int64), self.deg)).astype(np.int32)
        self.starts = np.minimum(np.asarray(in_off[:-1], np.int64), max(self.m - 1, 0))

    def step_edges(self, level, dirs):
        """{k: E_scan} for the steps k with dirs[k] == 2 (DensePull)."""
        import numpy as np
        level = np.asarray(level, np.int32)
        pulls = [k for k, d in enumerate(dirs) if int(d) == 2]
        if not pulls or self.m == 0:
            return {k: 0 for k in pulls}
        lv_dst = level[self.row]
        hit = (level[self.idx] == lv_dst - 1) & (lv_dst > 0)
        first = np.minimum.reduceat(np.where(hit, self.pos, np.int32(2**31 - 1)), self.starts)
        first = np.where(self.deg > 0, first, 0).astype(np.int64)
        top = int(level.max()) + 2
        lv = np.where(level < 0, top, level)          # unreached: after every level
        stop = np.bincount(lv, weights=np.minimum(first + 1, self.deg), minlength=top + 1)
        full = np.bincount(lv, weights=self.deg, minlength=top + 1)
        later = np.cumsum(full[::-1])[::-1]           # later[L] = rows of level >= L
        return {k: int(stop[k + 1] + later[k + 2]) for k in pulls}


def cc_step_bytes(n, dirs, fs, ds, es):
    """Per-step bytes of the CC step kernel (symmetric adjacency, E = edges
    examined, both directions of every edge).
      push  16|F| + 8E + 8|F'|        (ids+offsets+own label, index stream +
                                       atomic-min target, changed labels)
      pull  4(n+1) + 4E + 12n + n/4   (offsets, index stream, label gather
                                       (compulsory 4n), own label, new label,
                                       frontier in and out)"""
    out = []
    k = len(fs)
    for i in range(k):
        f, e = int(fs[i]), int(es[i])
        fnext = int(fs[i + 1]) if i + 1 < k else 0
        if dirs[i] == 2:
            out.append(4 * (n + 1) + 4 * e + 12 * n + n // 4)
        else:
            out.append(16 * f + 8 * e + 8 * fnext)
    return out


def prdelta_round_bytes(n, m, dirs, fs, ds):
    """Per-round bytes of PageRankDelta (fp64 vertex data).
      DensePull   4(n+1) + 4m + 8n + 8n   (offsets, index stream, each source's
                                          contribution once, DeltaSum written)
      SparsePush  12|F| + 12 D_F + n/8    (ids, offsets and contributions of
                                          the active sources, index stream and
                                          fp64 atomic add per edge, frontier)
      vertex update, every round: 52n + n/8 (DeltaSum, Rank and out-degree
                                          read; DeltaSum cleared, Delta, Rank
                                          and the next contribution written;
                                          next frontier)"""
    out = []
    for i in range(len(fs)):
        f, d = int(fs[i]), int(ds[i])
        if dirs[i] == 2:
            step = 4 * (n + 1) + 4 * m + 16 * n
        else:
            step = 12 * f + 12 * d + n // 8
        out.append(step + 52 * n + n // 8)
    return out


def sssp_label_setting_bytes(m_reach, n_reach):
    """Algorithmic bytes of one SSSP run: the label-setting minimum, which
    relaxes every edge out of a reached vertex once (index, weight, target
    distance: 12 m_reach) and reads each reached vertex's offsets and
    distance once (12 n_reach).  Work beyond it is the re-relaxation factor,
    reported apart."""
    return 12 * int(m_reach) + 12 * int(n_reach)


SCHED_KEY_FIELDS = ("vertex_order", "num_segments", "segments_concurrent", "block_threads",
                    "pull_items_per_thread", "pull_hot_sources", "pull_block_edges")


def sched_key(sched):
    """The schedule fields that change a PageRank kernel's traffic, as text."""
    return ",".join("%s=%d" % (k, int(sched.get(k, 0))) for k in SCHED_KEY_FIELDS)


def profile_traffic(kernel, workload=None, schedule=None, plan=None):
    """HBM bytes per launch of `kernel` from the hardware-counter figures
    committed under profiles/, or None when there are none for this kernel
    (and workload, schedule and batch plan, where the figures name them) or
    the kernel's sources changed since the counters were taken (sha256
    mismatch)."""
    import glob
    import hashlib
    import re
    blocks = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        blocks += re.findall(r"<!-- figures.*?-->", open(path).read(), re.S)
    for b in blocks:
        kv = dict(re.findall(r"^(\w+): (.+)$", b, re.M))
        if kv.get("kernel") != kernel:
            continue
        if "workload" in kv and kv["workload"] != workload:
            continue
        if "schedule" in kv and (schedule is None or kv["schedule"] != sched_key(schedule)):
            continue
        if "plan" in kv and kv["plan"] != plan:
            continue
        h = hashlib.sha256()
        for f in kv.get("sources", "").split():
            with open(os.path.join(ROOT, "paper_1805_00923_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() == kv.get("source_sha256"):
            return int(kv["traffic_bytes_per_launch"])
    return None


class KernelTally:
    """Launch count, summed HIP-event duration and algorithmic bytes of one
    step kernel over the timed region."""

    def __init__(self, name):
        self.name, self.launches, self.ms, self.bytes = name, 0, 0.0, 0

    def add(self, main_ms, step_bytes):
        self.launches += len(main_ms)
        self.ms += float(sum(main_ms))
        self.bytes += int(sum(step_bytes))

    def roofline(self):
        avg = self.ms / max(self.launches, 1)
        bpl = self.bytes / max(self.launches, 1)
        achieved = bpl / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        return {"bound": "hbm", "kernel": self.name, "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": None, "avg_launch_ms": round(avg, 5),
                "bytes_per_launch": int(bpl), "launches": self.launches}


class one_core:
    """Pin this process to one host core (the first it may run on) while the
    oracle is timed, as `taskset -c <core>` would; the previous affinity is
    restored afterwards."""

    def __enter__(self):
        self.prev = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(self.prev)})
        return self

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.prev)
        return False


def copy_peak_gbs(torch, dev, mib=1024, reps=10):
    """Practical HBM peak: a device-to-device copy of `mib` MiB (read once and
    written once), timed with HIP events; bytes moved = 2 x size."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return round(2 * (mib << 20) / (ms * 1e-3) / 1e9, 1)


# ------------------------------------------------------------- workloads --

def make_rmat_graph(scale, seed, weighted=False):
    import graphgen as gg
    import paper_1805_00923_amd as gi
    t0 = time.time()
    el = gg.rmat(scale, 16, seed=seed)
    if weighted:
        el.w = gg.uniform_weights(el.m, seed + 1000, 1, 1000)
    t1 = time.time()
    g = gi.Graph.from_edges(el.n, el.src, el.dst, el.w)
    log("rmat%d: generated in %.1fs, ingested in %.1fs, n=%d m=%d" %
        (scale, t1 - t0, time.time() - t1, g.n, g.m))
    return el, g


def run_bfs_cc(args, torch, dev):
    import numpy as np

    import graphgen as gg
    import paper_1805_00923_amd as gi
    # the batched and road-like SSSP configurations, each a launch of its own,
    # measured first so that the last batch launches are this workload's
    legs, persistent = {}, None
    if not args.no_legs:
        legs["batched"] = batched_pool_leg(torch, dev)
        legs["sssp_road"] = sssp_road_leg(torch, dev)
        _, g16 = make_rmat_graph(16, 1)
        persistent = persistent_pagerank(torch, dev, g16)
        g16.close()
    el, g = make_rmat_graph(22, 2)
    kw = dict(direction=gi.DENSE_PULL_SPARSE_PUSH, dense_frontier=gi.BITVECTOR, hybrid_divisor=20)
    kw.update(sched_overrides(args.schedule))
    g.set_schedule(**kw)
    srcs = gg.pick_sources(el, args.sources, 3)
    n, m = g.n, g.m
    level = torch.empty(n, dtype=torch.int32, device=dev)
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    label = torch.empty(n, dtype=torch.int32, device=dev)

    # per-source reach and algorithmic bytes from the plain path's traces
    # (levels, and so frontiers and directions, are the same on every path);
    # the pull steps' E_scan comes from a host replay in CSC order
    odeg = np.diff(g.out_off).astype(np.int64)
    m_reach, runs, ref_levels = [], [], []
    for s in srcs:
        g.bfs(int(s), level)
        lv = level.cpu().numpy()
        m_reach.append(int(odeg[lv >= 0].sum()))
        st = g.stats()
        dirs, fs, ds = st.trace()
        runs.append((lv, dirs, fs, ds, list(st.step_edges_examined())))
        if len(ref_levels) < 4:
            ref_levels.append(level.clone())
    t0 = time.time()
    ioff, iidx, _ = gi.build_adjacency(el.n, el.dst, el.src)
    replay = PullScanReplay(ioff, iidx)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        scans = list(ex.map(lambda r: replay.step_edges(r[0], r[1]), runs))
    bfs_bytes, kernel_e, replay_e = [], 0, 0
    for (lv, dirs, fs, ds, es), sc in zip(runs, scans):
        for k, e in sc.items():
            kernel_e += int(es[k])
            replay_e += e
            es[k] = e
        bfs_bytes.append(sum(bfs_step_bytes(n, dirs, fs, ds, es)))
    del replay, ioff, iidx, runs
    log("pull E_scan replayed in CSC order (%.1fs): %d edges, kernel count %d" %
        (time.time() - t0, replay_e, kernel_e))
    teps_edges = sum(m_reach) + m

    # plain path: one call per source (reported beside the batched path)
    for s in srcs:
        g.bfs(int(s), level, parent)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_ms = []
    for s in srcs:
        g.bfs(int(s), level, parent)
        plain_ms.append(g.stats().kernel_ms)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0

    batched = args.bfs_path == "batched"
    if batched:
        outs = [(torch.empty(n, dtype=torch.int32, device=dev),
                 torch.empty(n, dtype=torch.int32, device=dev)) for _ in srcs]
        batch = gi.Batch([g], [dict(graph=0, algorithm=gi.ALG_BFS, src=int(s), out=o, parent=p,
                                    workgroups=args.batch_workgroups)
                               for s, (o, p) in zip(srcs, outs)])
        batch.set_barrier_scope(barrier_scope(args))
        if args.batch_threads:
            batch.set_threads(args.batch_threads)
        t0 = time.perf_counter()
        batch.autotune(reps=3)
        t_tune = time.perf_counter() - t0

    # CC schedule: the hybrid divisor is tuned once (untimed), the way the
    # paper's autotuner tunes a schedule per algorithm and graph
    bfs_sched = g.schedule().as_dict()
    cc_div, cc_seg, cc_best, cc_sweep = 20, {}, None, {}
    for seg in ({}, *({"num_segments": p, "segment_strategy": 1} for p in (4, 8, 16))):
        for div in (2, 4, 8, 20, 50):
            g.set_schedule(**dict(bfs_sched, hybrid_divisor=div, **seg))
            g.cc(label)
            g.cc(label)
            ms = g.stats().kernel_ms
            cc_sweep["div%d%s" % (div, "_seg%d" % seg["num_segments"] if seg else "")] = round(ms, 3)
            if cc_best is None or ms < cc_best:
                cc_div, cc_seg, cc_best = div, seg, ms
    cc_sched = dict(bfs_sched, hybrid_divisor=cc_div, **cc_seg)
    g.set_schedule(**cc_sched)
    log("cc schedule sweep (ms): %s -> divisor %d %s (%.3f ms)" % (cc_sweep, cc_div, cc_seg, cc_best))

    cc_k = KernelTally("k_cc_step + k_cc_seg_merge" if cc_seg else "k_cc_step")
    batch_k = KernelTally("k_batch")
    bfs_k = KernelTally("k_bfs_step")

    overlap = batched and bool(args.overlap)
    cc_stream = torch.cuda.Stream() if overlap else None

    def one_step(record):
        cc_info = None
        if overlap:
            # the BFS batch and CC are independent: CC runs on its own stream
            # in the compute units the persistent batch leaves free
            batch.launch(use_graph=True)
            g.cc(label, stream=cc_stream)
            batch.wait()
            if record:
                batch_k.add([batch.info()["ms"]], [sum(bfs_bytes)])
        elif batched:
            batch.run(use_graph=True)
            if record:
                batch_k.add([batch.info()["ms"]], [sum(bfs_bytes)])
        else:
            g.set_schedule(**bfs_sched)
            for s in srcs:
                g.bfs(int(s), level, parent)
                if record:
                    st = g.stats()
                    dirs, fs, ds = st.trace()
                    _, mm = g.step_times()
                    bfs_k.add(mm, bfs_step_bytes(n, dirs, fs, ds, st.step_edges_examined()))
            g.set_schedule(**cc_sched)
        if not overlap:
            g.cc(label)
        if record:
            st = g.stats()
            dirs, fs, ds = st.trace()
            _, mm = g.step_times()
            cc_k.add(mm, cc_step_bytes(n, dirs, fs, ds, st.step_edges_examined()))
            cc_info = (st.kernel_ms, st.steps, st.dense_steps)
        return cc_info

    g.set_step_timing(True)
    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    cc_all = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cc_all.append(one_step(True))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    value = teps_edges * args.steps / dt / 1e9
    if batched:
        ok = all(torch.equal(outs[i][0], ref_levels[i]) for i in range(len(ref_levels)))
        if not ok:
            raise RuntimeError("batched BFS levels differ from the plain path")
    bfs_tally = batch_k if batched else bfs_k
    dominant = bfs_tally if bfs_tally.ms >= cc_k.ms else cc_k
    other = cc_k if dominant is bfs_tally else bfs_tally
    per_src_gteps = np.array([mr / (t * 1e-3) / 1e9 for mr, t in zip(m_reach, plain_ms)])
    # sources whose BFS reaches under 1% of the edges finish in a few steps
    # of fixed cost: their TEPS say nothing about traversal speed, so the
    # distribution is reported with them counted apart
    big = np.array(m_reach) >= 0.01 * m
    extra = {
        "n": n, "m": m, "sources": int(len(srcs)), "bfs_path": args.bfs_path,
        "plain_bfs_ms_total": round(t_plain * 1e3, 3),
        "plain_bfs_ms_median": round(float(np.median(plain_ms)), 4),
        "plain_bfs_gteps_per_source": {
            "min": round(float(per_src_gteps.min()), 3),
            "p10": round(float(np.percentile(per_src_gteps, 10)), 3),
            "median": round(float(np.median(per_src_gteps)), 3),
            "p90": round(float(np.percentile(per_src_gteps, 90)), 3),
            "max": round(float(per_src_gteps.max()), 3),
            "harmonic_mean_reach_ge_1pct": round(float(big.sum() / (1.0 / per_src_gteps[big]).sum()), 3)
            if big.any() else None,
            "sources_reach_under_1pct_of_m": int((~big).sum())},
        "cc_ms": round(float(np.median([c[0] for c in cc_all])), 4),
        "cc_rounds": int(cc_all[0][1]), "cc_dense_rounds": int(cc_all[0][2]),
        "cc_hybrid_divisor": cc_div, "cc_schedule": cc_sched, "cc_schedule_sweep_ms": cc_sweep,
        "other_kernel": other.roofline(),
        "pull_escan": {"replayed_csc_order": replay_e, "kernel_count": kernel_e},
    }
    if batched:
        info = batch.info()
        extra.update({"batched_bfs_ms": round(batch_k.ms / max(batch_k.launches, 1), 3),
                      "batch_grid": info["grid"], "batch_threads": batch.threads(),
                      "batch_xcd_local": batch.placement(),
                      "batch_barrier": args.batch_barrier,
                      "batch_workgroups_per_source": int(np.median(info["workgroups"])),
                      "autotune_s": round(t_tune, 2),
                      "speedup_batched_vs_plain_bfs": round(
                          t_plain * 1e3 / (batch_k.ms / max(batch_k.launches, 1)), 3)})
    config = {"workload": "rmat22_ef16_bfs64_plus_cc", "graph": "rmat scale 22 edge factor 16 "
              "abcd=.57/.19/.19/.05 seed 2, relabelled, dedup", "n": n, "m": m,
              "bfs_sources": int(len(srcs)), "bfs_path": args.bfs_path,
              "cc_overlaps_bfs_batch": overlap,
              "schedule": bfs_sched, "cc_hybrid_divisor": cc_div}
    if batched:
        # the batch plan the traffic figures are keyed by
        config["batch_plan"] = "threads=%d,workgroups=%d" % (
            batch.threads(), int(np.median(batch.info()["workgroups"])))
    # PageRank legs (the PageRank configuration on R-MAT 16, and R-MAT 22 on
    # this graph), each tuned and timed on its own with its own roofline
    extra["pagerank"] = pagerank_legs(torch, dev, g, persistent=persistent)
    extra.update(legs)
    extra["hbm_copy_gbs"] = copy_peak_gbs(torch, dev)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_bfs_cc(el, srcs, m_reach)
    return value, "GTEPS", ms_step, "int32", config, dominant.roofline(), cpu, extra


def pagerank_legs(torch, dev, g22, steps=5, persistent=None):
    """20-iteration PageRank on R-MAT 16 (seed 1) and on the R-MAT 22 graph of
    the default workload: tuned schedule, GTEPS and roofline of each."""
    import numpy as np
    legs = {}
    el16, g16 = make_rmat_graph(16, 1)
    for name, g in (("rmat16", g16), ("rmat22", g22)):
        ranks = torch.empty(g.n, dtype=torch.float32, device=dev)
        kw, tuned, kms, dt, tally = pr_tune_and_time(g, torch, ranks, steps, 1)
        kmed = float(np.median(kms))
        roof = tally.roofline()
        roof["traffic"] = profile_traffic(roof["kernel"], "pagerank20_%s_ef16" % name,
                                          g.schedule().as_dict())
        legs[name] = {"n": g.n, "m": g.m, "schedule": kw, "run_ms_median": round(kmed, 4),
                      "gteps": round(20.0 * g.m / (kmed * 1e-3) / 1e9, 3),
                      "roofline": roof, "schedule_sweep_ms": tuned}
        log("pagerank %s: %s, %.3f ms per 20 iterations" % (name, kw, kmed))
        if name == "rmat16" and persistent is not None:
            legs[name]["persistent"] = persistent
    g16.close()
    return legs


POOL_KERNEL = "k_batch (128 BFS + 128 PageRank tasks)"


def pool_launch_bytes(gi, graphs, els, tasks, outs):
    """Algorithmic bytes of one launch of the 256-instance pool: each BFS
    task's levels (from its output; BFS levels are unique) under the hybrid
    rule at divisor 20, the pull levels' scans by a host replay in CSC order
    (bfs_step_bytes); 20 iterations of 4m + 16n per PageRank task."""
    import numpy as np
    replays, total = {}, 0
    for t, r in zip(tasks, outs):
        gx = t["graph"]
        g, el = graphs[gx], els[gx]
        if t["algorithm"] != gi.ALG_BFS:
            total += 20 * (4 * g.m + 16 * g.n)
            continue
        if gx not in replays:
            ioff, iidx, _ = gi.build_adjacency(el.n, el.dst, el.src)
            replays[gx] = PullScanReplay(ioff, iidx)
        lv = r.cpu().numpy()
        odeg = np.diff(g.out_off).astype(np.int64)
        nl = int(lv.max()) + 1
        fs = np.bincount(lv[lv >= 0], minlength=nl).astype(np.int64)
        ds = np.bincount(lv[lv >= 0], weights=odeg[lv >= 0], minlength=nl).astype(np.int64)
        dirs = [2 if (int(fs[k]) + int(ds[k])) * 20 > g.m else 0 for k in range(nl)]
        es = [0] * nl
        for k, e in replays[gx].step_edges(lv, dirs).items():
            es[k] = e
        total += sum(bfs_step_bytes(g.n, dirs, fs, ds, es))
    return total


def batched_pool_leg(torch, dev, steps=3, warmup=1):
    """The batched workload's launch alone (256 BFS / PageRank instances over
    the 14-graph pool, autotuned, replayed from a HIP graph): time, aggregate
    GTEPS over the launch's own outputs, overhead fractions.  The comparison
    with 256 plain calls is the batched workload's own (`--workload
    batched`)."""
    import numpy as np

    import graphgen as gg
    import paper_1805_00923_amd as gi
    t_all = time.time()
    els = [gg.rmat(s, 16, seed=100 + s) for s in range(10, 19)]
    els += [gg.grid(d, d, 0.0, weighted=False) for d in (64, 128, 256, 512, 1024)]
    graphs = [gi.Graph.from_edges(el.n, el.src, el.dst) for el in els]
    tasks = []
    for i in range(256):
        gidx = i % len(graphs)
        g, el = graphs[gidx], els[gidx]
        if i % 2 == 0:
            tasks.append(dict(graph=gidx, algorithm=gi.ALG_BFS,
                              src=int(gg.pick_sources(el, 1, 200 + i)[0]),
                              out=torch.empty(g.n, dtype=torch.int32, device=dev)))
        else:
            tasks.append(dict(graph=gidx, algorithm=gi.ALG_PAGERANK, iters=20, damping=0.85,
                              out=torch.empty(g.n, dtype=torch.float32, device=dev)))
    b = gi.Batch(graphs, tasks)
    b.autotune(reps=3)
    for _ in range(warmup):
        b.run(use_graph=True)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run(use_graph=True)
        kms.append(b.info()["ms"])
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    edges = 0
    for t in tasks:
        g = graphs[t["graph"]]
        if t["algorithm"] == gi.ALG_BFS:
            edges += int(np.diff(g.out_off)[t["out"].cpu().numpy() >= 0].sum())
        else:
            edges += 20 * g.m
    info = b.info()
    bar = b.barrier_ms().astype(np.float64)
    wgs = info["workgroups"].astype(np.float64)
    tally = KernelTally(POOL_KERNEL)
    tally.add(kms, [pool_launch_bytes(gi, graphs, els, tasks, [t["out"] for t in tasks])] * len(kms))
    leg = {"workload": "batched256_bfs_pr20_rmat10-18_grid64-1024", "ms_per_launch": round(t_batch * 1e3, 3),
           "kernel_ms_median": round(float(np.median(kms)), 3),
           "gteps": round(edges / t_batch / 1e9, 3), "roofline": tally.roofline(),
           "threads": b.threads(), "grid": info["grid"],
           "pr_block_edges_per_graph": {els[i].name: int(c) for i, c in enumerate(b.pr_block_edges()) if c},
           "barrier_fraction_of_workgroup_time": round(float(
               (bar * wgs).sum() / max(float((info["task_ms"] * wgs).sum()), 1e-9)), 4),
           "launch_overhead_fraction": round(max(0.0, 1.0 - float(np.median(kms)) / (t_batch * 1e3)), 4),
           "wall_s": round(time.time() - t_all, 1)}
    b.close()
    for g in graphs:
        g.close()
    log("batched leg: %.3f ms per launch, %.1f GTEPS" % (leg["ms_per_launch"], leg["gteps"]))
    return leg


def sssp_road_leg(torch, dev, delta=4096, steps=3, warmup=1):
    """Delta-stepping from the 4 benchmark sources on the 4096 x 4096 grid
    without shortcuts (the road-like regime) as 4 SSSP tasks of one batched
    launch at bucket width 4096 (the width the SSSP workload's sweep picks),
    autotuned: time, GTEPS, label-setting roofline, re-relaxation.  The
    distances are checked against Dijkstra in the tests and against the
    engine in the SSSP workload."""
    import numpy as np

    import graphgen as gg
    import paper_1805_00923_amd as gi
    t_all = time.time()
    el = gg.grid(4096, 4096, 0.0, seed=4)
    g = gi.Graph.from_edges(el.n, el.src, el.dst, el.w)
    srcs = gg.pick_sources(el, 4, 5)
    del el
    outs = [torch.empty(g.n, dtype=torch.int32, device=dev) for _ in srcs]
    b = gi.Batch([g], [dict(graph=0, algorithm=gi.ALG_SSSP, src=int(s), sssp_delta=delta, out=o)
                       for s, o in zip(srcs, outs)])
    b.autotune(reps=1)
    for _ in range(warmup):
        b.run()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
        kms.append(b.info()["ms"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    odeg = np.diff(g.out_off).astype(np.int64)
    m_reach, n_reach = [], []
    for o in outs:
        reached = o.cpu().numpy().view(np.uint32) != 0xFFFFFFFF
        m_reach.append(int(odeg[reached].sum()))
        n_reach.append(int(reached.sum()))
    tally = KernelTally("k_batch (4 SSSP tasks)")
    tally.add(kms, [sum(sssp_label_setting_bytes(mr, nr) for mr, nr in zip(m_reach, n_reach))] * len(kms))
    info = b.info()
    roof = tally.roofline()
    roof["traffic"] = profile_traffic(roof["kernel"], "sssp_grid4096_noshortcut", None,
                                      sssp_batch_plan(b, delta))
    leg = {"workload": "sssp_grid4096_noshortcut", "delta": delta, "ms_per_launch": round(dt * 1e3, 3),
           "gteps": round(sum(m_reach) / dt / 1e9, 3), "roofline": roof,
           "rerelaxation": round(float(b.edges().sum()) / sum(m_reach), 4),
           "phases": [int(x) for x in info["levels"]], "threads": b.threads(),
           "workgroups": [int(x) for x in info["workgroups"]], "wall_s": round(time.time() - t_all, 1)}
    b.close()
    g.close()
    log("sssp road leg: %.3f ms per launch, %.2f GTEPS" % (leg["ms_per_launch"], leg["gteps"]))
    return leg


def persistent_pagerank(torch, dev, g, steps=5, scope=None):
    """The same 20 iterations as one persistent launch (a single batched
    PageRank task, workgroups and block size autotuned): its time and the
    split between work and the task barriers between iterations."""
    import numpy as np

    import paper_1805_00923_amd as gi
    out = torch.empty(g.n, dtype=torch.float32, device=dev)
    b = gi.Batch([g], [dict(graph=0, algorithm=gi.ALG_PAGERANK, iters=20, damping=0.85, out=out)])
    if scope is not None:
        b.set_barrier_scope(scope)
    b.autotune(reps=3)
    b.run()
    ms, bar = [], []
    for _ in range(steps):
        b.run()
        ms.append(b.info()["ms"])
        bar.append(float(b.barrier_ms()[0]))
    info = b.info()
    res = {"ms_per_20_iterations": round(float(np.median(ms)), 4),
           "barrier_ms": round(float(np.median(bar)), 4),
           "barrier_fraction": round(float(np.median(bar)) / max(float(info["task_ms"][0]), 1e-9), 3),
           "workgroups": int(info["workgroups"][0]), "threads": b.threads(),
           "pr_block_edges": int(b.pr_block_edges()[0])}
    b.close()
    return res


def cpu_baseline_bfs_cc(el, srcs, m_reach, budget_s=12.0):
    """The oracle, single-threaded, on a bounded sample of the same workload:
    BFS from the sources in order until the budget is spent (at least 2),
    then one CC.  TEPS counted as for the GPU line."""
    import oracle
    log("cpu baseline: building the oracle graph (not timed)")
    t0 = time.time()
    og = oracle.Graph(el)
    log("oracle graph built in %.1fs" % (time.time() - t0))
    with one_core():
        t0 = time.perf_counter()
        done = 0
        for s in srcs:
            oracle.bfs(og, int(s))
            done += 1
            if done >= 2 and time.perf_counter() - t0 > budget_s:
                break
        oracle.cc(og)
        dt = time.perf_counter() - t0
    edges = sum(m_reach[:done]) + og.m
    return {"value": round(edges / dt / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "oracle FIFO BFS from the first %d of the 64 sources + one label-"
                      "propagation CC on the same RMAT-22 graph, one thread pinned to one core, "
                      "%.1f s" % (done, dt)}


# PageRank schedules the autotuner tries (untimed), as the paper's autotuner
# does per algorithm and graph: id-order block size and id-range segments
# (sequential or concurrent), and the degree-ordered pull with its tile shape
# and LDS source count.
PR_CANDIDATES = [
    dict(), dict(pull_block_edges=512), dict(pull_block_edges=1024), dict(num_segments=4),
    dict(num_segments=8, segments_concurrent=1), dict(num_segments=16, segments_concurrent=1),
    dict(vertex_order=1, block_threads=1024, pull_items_per_thread=4, pull_hot_sources=-1),
    dict(vertex_order=1, block_threads=1024, pull_items_per_thread=8, pull_hot_sources=-1),
    dict(vertex_order=1, block_threads=1024, pull_items_per_thread=4, pull_hot_sources=0),
    dict(vertex_order=1, block_threads=512, pull_items_per_thread=4, pull_hot_sources=0),
    dict(vertex_order=1, block_threads=512, pull_items_per_thread=8, pull_hot_sources=-1),
]


def pr_kernel_name(sch):
    if sch.vertex_order == 1:
        return "k_pr_ord + k_pr_ord_split"
    if sch.num_segments <= 1:
        return "k_pr_rows"
    return ("k_pr_seg_concurrent + k_pr_seg_final_multi" if sch.segments_concurrent
            else "k_pr_rows per segment + k_pr_seg_final")


def pr_tune_and_time(g, torch, ranks, steps, warmup, overrides=None, cands=PR_CANDIDATES):
    """Tune the PageRank schedule of `g` over `cands` (two 20-iteration runs
    each, the second timed), then time `steps` runs with per-iteration HIP
    events (the kernels' times, for the roofline) and `steps` whole runs
    (the run's time: repeated arguments, so the degree-ordered run replays
    from a HIP graph).  Returns (schedule, sweep, run ms list, wall seconds
    of the whole runs, tally)."""
    n, m = g.n, g.m
    tuned = {}
    for c in cands:
        g.set_schedule(**c)
        g.pagerank(ranks, 20, 0.85)
        g.pagerank(ranks, 20, 0.85)
        tuned[json.dumps(c)] = round(g.stats().kernel_ms, 4)
    kw = dict(json.loads(min(tuned, key=tuned.get)))
    kw.update(overrides or {})
    g.set_schedule(**kw)
    g.set_step_timing(True)
    for _ in range(warmup):
        g.pagerank(ranks, 20, 0.85)
    torch.cuda.synchronize()
    tally = KernelTally(pr_kernel_name(g.schedule()))
    for _ in range(steps):
        g.pagerank(ranks, 20, 0.85)
        _, mm = g.step_times()
        tally.add(mm, [4 * m + 16 * n] * len(mm))
    g.set_step_timing(False)
    for _ in range(max(warmup, 1)):
        g.pagerank(ranks, 20, 0.85)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        g.pagerank(ranks, 20, 0.85)
        kms.append(g.stats().kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return kw, tuned, kms, dt, tally


def run_pr(args, torch, dev, scale):
    import numpy as np
    el, g = make_rmat_graph(scale, 1 if scale == 16 else 2)
    n, m = g.n, g.m
    ranks = torch.empty(n, dtype=torch.float32, device=dev)
    kw, tuned, kms, dt, tally = pr_tune_and_time(g, torch, ranks, args.steps, args.warmup,
                                                 sched_overrides(args.schedule))
    log("pagerank schedule sweep (ms per 20 iterations): %s -> %s" % (tuned, kw))
    ms_step = dt * 1e3 / args.steps
    value = 20.0 * m * args.steps / dt / 1e9
    kmed = float(np.median(kms))
    config = {"workload": "pagerank20_rmat%d_ef16" % scale, "n": n, "m": m,
              "schedule": g.schedule().as_dict()}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph(el)
        # whole runs until about 10 s are spent (at least one)
        reps = 0
        with one_core():
            t0 = time.perf_counter()
            while reps < 1 or time.perf_counter() - t0 < 10.0:
                oracle.pagerank(og, 20, 0.85)
                reps += 1
            dt_c = (time.perf_counter() - t0) / reps
        cpu = {"value": round(20.0 * og.m / dt_c / 1e9, 5), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", "sample": "FP64 pull PageRank, 20 iterations, full graph, "
                                           "one thread pinned to one core, %d runs, %.3f s per "
                                           "run" % (reps, dt_c)}
    extra = {"schedule_sweep_ms": tuned,
             "run_ms_median": round(kmed, 4),
             "gteps_kernel": round(20.0 * m / (kmed * 1e-3) / 1e9, 3),
             "bytes_per_run": 20 * (4 * m + 16 * n) + 4 * n}
    if scale == 16:
        extra["persistent"] = persistent_pagerank(torch, dev, g, scope=barrier_scope(args))
    return value, "GTEPS", ms_step, "f32 storage / f64 accumulate", config, tally.roofline(), cpu, extra


SSSP_BATCH_DELTAS = (1000, 1 << 10, 1 << 11, 1 << 12, 1 << 13, 1 << 14)


def sssp_batch_plan(b, delta):
    """Key of a batched SSSP launch's plan in the committed counter figures:
    workgroup size, each task's workgroups, bucket width."""
    wg = "/".join(str(int(x)) for x in b.info()["workgroups"])
    return "threads=%d,workgroups=%s,delta=%d" % (b.threads(), wg, delta)


def run_sssp(args, torch, dev):
    """Delta-stepping SSSP from 4 sources on the 4096 x 4096 grid: the
    engine's per-phase launches (delta swept over {2^k, 5 <= k <= 14} and
    1000), and the 4 sources as SSSP tasks of one persistent launch (delta
    swept over the upper part of the same set).  Bytes are the label-setting
    minimum; the re-relaxation factor (edges relaxed / m_reach) is reported
    beside it, as are the phases and the time per delta-stepping phase of
    the engine at the same delta."""
    import numpy as np

    import graphgen as gg
    import paper_1805_00923_amd as gi
    t0 = time.time()
    el = gg.grid(4096, 4096, args.grid_shortcuts, seed=4)
    g = gi.Graph.from_edges(el.n, el.src, el.dst, el.w)
    log("grid: built in %.1fs n=%d m=%d" % (time.time() - t0, g.n, g.m))
    srcs = gg.pick_sources(el, 4, 5)
    dist = torch.empty(g.n, dtype=torch.int32, device=dev)
    # delta swept (untimed) on the first source: {2^k, 5 <= k <= 14} and 1000
    sweep = {}
    deltas = ([int(x) for x in args.delta_sweep.split(",")] if args.delta_sweep else
              [1 << k for k in range(5, 15)] + [1000])
    for delta in deltas:
        g.set_schedule(sssp_delta=delta)
        g.sssp(int(srcs[0]), dist)
        g.sssp(int(srcs[0]), dist)
        sweep[delta] = round(g.stats().kernel_ms, 3)
    best_delta = min(sweep, key=sweep.get)
    log("sssp delta sweep (ms): %s -> %d" % (sweep, best_delta))
    kw = dict(sssp_delta=best_delta)
    kw.update(sched_overrides(args.schedule))
    g.set_schedule(**kw)
    odeg = np.diff(g.out_off).astype(np.int64)
    m_reach, n_reach, refs = [], [], []
    for s in srcs:
        g.sssp(int(s), dist)
        refs.append(dist.clone())
        d = dist.cpu().numpy().view(np.uint32)
        reached = d != 0xFFFFFFFF
        m_reach.append(int(odeg[reached].sum()))
        n_reach.append(int(reached.sum()))
    run_bytes = [sssp_label_setting_bytes(mr, nr) for mr, nr in zip(m_reach, n_reach)]
    for _ in range(args.warmup):
        for s in srcs:
            g.sssp(int(s), dist)
    torch.cuda.synchronize()
    phases, relaxed = [], 0
    tally = KernelTally("sssp engine (all kernels of a run)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for i, s in enumerate(srcs):
            g.sssp(int(s), dist)
            st = g.stats()
            phases.append(st.steps)
            relaxed += int(sum(st.step_edges_examined()))
            tally.add([st.kernel_ms], [run_bytes[i]])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = sum(m_reach) * args.steps / dt / 1e9
    roof = tally.roofline()
    wname = ("sssp_grid4096_noshortcut" if args.grid_shortcuts == 0 else
             "sssp_grid4096_shortcut%gpct" % (100 * args.grid_shortcuts))
    config = {"workload": wname, "n": g.n, "m": g.m, "sources": 4,
              "schedule": g.schedule().as_dict(), "sssp_path": args.sssp_path}
    plain_ms = dt * 1e3 / args.steps
    extra = {"phases_median": int(np.median(phases)), "delta_sweep_ms": sweep,
             "delta": best_delta, "plain_ms": round(plain_ms, 3),
             "plain_gteps": round(value, 3),
             "plain_us_per_phase": round(plain_ms * 1e3 / (sum(phases) / args.steps), 3),
             "plain_rerelaxation": round(relaxed / (args.steps * sum(m_reach)), 4),
             "plain_roofline": roof, "m_reach": m_reach, "n_reach": n_reach,
             "label_setting_bytes_per_step": int(sum(run_bytes))}
    ms_step = plain_ms
    if args.sssp_path == "batched":
        # the 4 sources as SSSP tasks of one persistent launch (task barriers
        # instead of per-phase kernel launches); bucket width swept untimed
        outs = [torch.empty(g.n, dtype=torch.int32, device=dev) for _ in srcs]
        bsweep, best = {}, None
        for delta in ((args.sssp_batch_delta,) if args.sssp_batch_delta else SSSP_BATCH_DELTAS):
            b = gi.Batch([g], [dict(graph=0, algorithm=gi.ALG_SSSP, src=int(s_), sssp_delta=delta,
                                    out=o, workgroups=args.batch_workgroups)
                               for s_, o in zip(srcs, outs)])
            b.set_barrier_scope(barrier_scope(args))
            if args.batch_threads:
                b.set_threads(args.batch_threads)
            b.autotune(reps=1)
            b.run()
            b.run()
            bsweep[delta] = round(b.info()["ms"], 3)
            log("batched sssp delta %d: %.3f ms (%d threads)" % (delta, bsweep[delta], b.threads()))
            if best is None or bsweep[delta] < bsweep[best[0]]:
                if best is not None:
                    best[1].close()
                best = (delta, b)
            else:
                b.close()
        bdelta, b = best
        log("batched sssp delta sweep (ms): %s -> %d" % (bsweep, bdelta))
        # the engine's phases at the same delta: the rounds a delta-stepping
        # schedule needs, against which the launch's time per phase is taken
        g.set_schedule(**dict(kw, sssp_delta=bdelta))
        eng_phases = []
        for s_ in srcs:
            g.sssp(int(s_), dist)
            eng_phases.append(int(g.stats().steps))
        g.set_schedule(**kw)
        for _ in range(args.warmup):
            b.run()
        torch.cuda.synchronize()
        btally = KernelTally("k_batch (4 SSSP tasks)")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.run()
            btally.add([b.info()["ms"]], [sum(run_bytes)])
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        bad = sum(int(not torch.equal(o, r)) for o, r in zip(outs, refs))
        if bad:
            raise RuntimeError("batched SSSP distances differ from the plain path")
        value = sum(m_reach) * args.steps / dtb / 1e9
        ms_step = dtb * 1e3 / args.steps
        extra["batched_roofline"] = roof = btally.roofline()
        info = b.info()
        bedges = b.edges()
        task_us = [float(x) * 1e3 for x in info["task_ms"]]
        extra.update({"batched_ms": round(ms_step, 3), "batched_delta": bdelta,
                      "batched_delta_sweep_ms": bsweep, "batch_threads": b.threads(),
                      "batch_workgroups": [int(x) for x in info["workgroups"]],
                      "batch_phases": [int(x) for x in info["levels"]],
                      "engine_phases_at_batched_delta": eng_phases,
                      "batched_us_per_engine_phase": [round(t / p, 3) for t, p in
                                                      zip(task_us, eng_phases)],
                      "batched_rerelaxation": round(float(bedges.sum()) / sum(m_reach), 4),
                      "speedup_vs_plain": round(dt / dtb, 3)})
        config["batched_delta"] = bdelta
        config["batch_plan"] = sssp_batch_plan(b, bdelta)
        b.close()
    return value, "GTEPS", ms_step, "uint32", config, roof, None, extra


def selector_records(g, gi, alg, src=0):
    f, t, v = g.trace_exhaustive(alg, src)
    import numpy as np
    y = np.where(v > 0, np.log(np.maximum(t, 1e-6)), 0.0).astype(np.float32)
    return f, y, v, t


# fixed schedules the selector is compared against (direction 0 SparsePush,
# 2 DensePull, 3 the hybrid rule DensePull/SparsePush, 4 DensePush/SparsePush)
SEL_FIXED_BFS = ([dict(direction=3, hybrid_divisor=d) for d in (5, 10, 20, 40)] +
                 [dict(direction=0), dict(direction=2), dict(direction=4)])
SEL_FIXED_CC = ([dict(direction=0), dict(direction=2)] +
                [dict(direction=3, hybrid_divisor=d, **seg)
                 for seg in ({}, dict(num_segments=4, segment_strategy=1),
                             dict(num_segments=16, segment_strategy=1))
                 for d in (2, 8, 20)])   # one segment layout after another
SEL_FIXED_PR = PR_CANDIDATES + [dict(num_segments=p) for p in (32, 64, 128)]


def bf16_fp32_regret(sel, feats, times, valid):
    """Per-step schedule choices (least predicted time among the valid
    schedules) with BF16 and with FP32 inference on the same records: the
    records where they differ and the time the BF16 choices cost beyond the
    FP32 ones, in % of the FP32 choices' time."""
    import numpy as np
    ok = valid > 0
    pb = np.where(ok, sel.predict(feats, bf16=True), np.inf)
    pf = np.where(ok, sel.predict(feats, bf16=False), np.inf)
    cb, cf = pb.argmin(1), pf.argmin(1)
    r = np.arange(len(cb))
    tb, tf = times[r, cb], times[r, cf]
    return int(len(cb)), int((cb != cf).sum()), float(tb.sum()), float(tf.sum())


def run_selector(args, torch, dev):
    """Train the selector on exhaustive per-step timings of training graphs,
    then compare, on a held-out Chung-Lu graph (exponent 2.0), per algorithm:
    the hybrid heuristic, the best fixed schedule (autotuned on the held-out
    graph itself), the learned selector and the per-step best schedule; and
    check that BF16 inference chooses within 5% of FP32's choices."""
    import numpy as np

    import graphgen as gg
    import paper_1805_00923_amd as gi
    t_all = time.time()
    # training graphs: R-MAT and Chung-Lu graphs with degree exponents 2.2,
    # 2.5 and 3.0 and 20-34 edges per vertex; the held-out exponent (2.0)
    # is not among them
    train = [("rmat", 16, 316), ("rmat", 18, 318), ("rmat", 20, 320), ("rmat", 22, 322),
             ("chunglu", 1 << 20, 2.2, 401), ("chunglu", 1 << 20, 2.5, 402),
             ("chunglu", 1 << 21, 3.0, 403), ("chunglu", 1 << 22, 2.2, 404),
             ("chunglu34", 1 << 20, 2.2, 405), ("chunglu34", 1 << 21, 2.5, 406),
             ("rmat", 24, 324), ("chunglu34", 1 << 24, 2.2, 407)]
    F, Y, V = [], [], []
    for spec in train:
        if spec[0] == "rmat":
            el = gg.rmat(spec[1], 16, seed=spec[2])
        else:
            n = spec[1]
            per = 34 if spec[0] == "chunglu34" else 20
            el = gg.chung_lu(n, per * n, spec[2], min(1e5, n / 8), seed=spec[3])
        g = gi.Graph.from_edges(el.n, el.src, el.dst)
        g.set_schedule(direction=gi.DENSE_PULL_SPARSE_PUSH)
        for s in gg.pick_sources(el, 24, spec[-1]):
            f, y, v, _ = selector_records(g, gi, gi.ALG_BFS, int(s))
            F.append(f), Y.append(y), V.append(v)
        for alg in (gi.ALG_CC, gi.ALG_PAGERANK):
            f, y, v, _ = selector_records(g, gi, alg)
            F.append(f), Y.append(y), V.append(v)
        log("training graph %s: n=%d m=%d, %d records so far" % (el.name, g.n, g.m,
                                                                sum(len(x) for x in F)))
        g.close()
    X, Yl, Vm = np.concatenate(F), np.concatenate(Y), np.concatenate(V)
    sel = gi.Selector(seed=1)
    t0 = time.time()
    loss = sel.train(X, Yl, Vm, epochs=args.epochs, lr=1e-3, seed=7)
    t_train = time.time() - t0
    log("trained on %d records, %d epochs in %.1fs: loss %.4f -> %.4f" %
        (len(X), args.epochs, t_train, loss[0], loss[-1]))

    # held-out graph
    if args.heldout == "full":
        n_h, samples, dmax = 41_000_000, 1_500_000_000, 1e6
    else:
        n_h, samples, dmax = 1 << 22, 34 * (1 << 22), 1e6 * (1 << 22) / 41e6
    t0 = time.time()
    el = gg.chung_lu(n_h, samples, 2.0, dmax, seed=999)
    log("held-out records generated in %.1fs" % (time.time() - t0))
    off, idx, _ = gi.build_adjacency(el.n, el.src, el.dst)
    log("held-out out-adjacency built (%.1fs)" % (time.time() - t0))
    ioff, iidx, _ = gi.build_adjacency(el.n, el.dst, el.src)
    log("held-out in-adjacency built (%.1fs)" % (time.time() - t0))
    g = gi.Graph(el.n, off, idx, None, ioff, iidx, None)
    del off, idx, ioff, iidx
    log("held-out %s: n=%d m=%d built in %.1fs" % (el.name, g.n, g.m, time.time() - t0))
    srcs = gg.pick_sources(el, 16, 1000)
    del el
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ranks = torch.empty(g.n, dtype=torch.float32, device=dev)
    g.attach_selector(sel)

    def timed(alg, direction, src=0, reps=3):
        g.set_schedule(direction=direction)
        ms, dirs = [], None
        for _ in range(reps):
            if alg == gi.ALG_BFS:
                g.bfs(int(src), out)
            elif alg == gi.ALG_CC:
                g.cc(out)
            else:
                g.pagerank(ranks, 20, 0.85)
            ms.append(g.stats().kernel_ms)
            dirs = g.stats().step_schedules()
        return float(np.median(ms)), dirs

    rows = []
    cases = [(gi.ALG_BFS, int(s)) for s in srcs] + [(gi.ALG_CC, 0), (gi.ALG_PAGERANK, 0)]
    regret_l, regret_h, best_steps = [], [], []
    prec = [0, 0, 0.0, 0.0]  # records, BF16/FP32 disagreements, BF16 and FP32 choice times
    t_heur = t_learn = t_best = 0.0
    dump = {}
    for alg, s in cases:
        g.set_schedule(direction=gi.DENSE_PULL_SPARSE_PUSH)
        hf, _, v, tt = selector_records(g, gi, alg, s)
        dump["case_%d_%d" % (alg, s)] = np.concatenate([hf, tt, v.astype(np.float32)], 1)
        rec, dis, tb, tf = bf16_fp32_regret(sel, hf, np.where(v > 0, tt, 0.0), v)
        prec = [prec[0] + rec, prec[1] + dis, prec[2] + tb, prec[3] + tf]
        tt = np.where(v > 0, tt, np.inf)
        best = tt.min(1)
        if alg == gi.ALG_PAGERANK:
            heur_ms, _ = timed(alg, gi.DENSE_PULL)          # the plain schedule: unsegmented
            learn_ms, _ = timed(alg, gi.LEARNED)
            pred = sel.predict(g.trace_exhaustive(alg)[0][:1], bf16=True)[0]
            pick = 3 if pred[2] - pred[3] > 0.14 else 2   # the library's margin
            lchoice = np.full(len(best), pick)
            hchoice = np.full(len(best), 2)
        else:
            heur_ms, hd = timed(alg, gi.DENSE_PULL_SPARSE_PUSH, s)
            learn_ms, ld = timed(alg, gi.LEARNED, s)
            hchoice, lchoice = hd.astype(int), ld.astype(int)
        k = len(best)
        rl = tt[np.arange(k), lchoice[:k]] - best
        rh = tt[np.arange(k), hchoice[:k]] - best
        regret_l += list(rl)
        regret_h += list(rh)
        best_steps += list(best)
        log("held-out %s src=%d: heuristic %.3f ms, learned %.3f ms, per-step best %.3f ms" %
            ({0: "pagerank", 1: "bfs", 2: "cc"}[alg], s, heur_ms, learn_ms, float(best.sum())))
        t_heur += heur_ms
        t_learn += learn_ms
        t_best += float(best.sum())
        rows.append({"alg": {0: "pagerank", 1: "bfs", 2: "cc"}[alg], "src": s,
                     "heuristic_ms": round(heur_ms, 4), "learned_ms": round(learn_ms, 4),
                     "best_steps_ms": round(float(best.sum()), 4), "steps": k,
                     "choices": {"heuristic": "".join(str(int(x)) for x in hchoice[:k]),
                                 "learned": "".join(str(int(x)) for x in lchoice[:k]),
                                 "best": "".join(str(int(x)) for x in tt.argmin(1))}})
    # the best fixed schedule per algorithm, autotuned on the held-out graph:
    # every candidate run once over the algorithm's cases (after one
    # untimed run), the fastest then timed like the other columns
    g.attach_selector(None)
    names = {0: "pagerank", 1: "bfs", 2: "cc"}
    fixed = {}
    for alg, cands in ((gi.ALG_BFS, SEL_FIXED_BFS), (gi.ALG_CC, SEL_FIXED_CC),
                       (gi.ALG_PAGERANK, SEL_FIXED_PR)):
        acase = [s for a, s in cases if a == alg]
        sweep = {}
        for c in cands:
            g.set_schedule(**c)
            tot = 0.0
            for i, s in enumerate(acase):
                if alg == gi.ALG_BFS:
                    if i == 0:
                        g.bfs(int(s), out)
                    g.bfs(int(s), out)
                elif alg == gi.ALG_CC:
                    g.cc(out)
                    g.cc(out)
                else:
                    g.pagerank(ranks, 20, 0.85)
                    g.pagerank(ranks, 20, 0.85)
                tot += g.stats().kernel_ms
            sweep[json.dumps(c)] = round(tot, 3)
            log("held-out fixed %s %s: %.3f ms" % (names[alg], c, tot))
        bc = json.loads(min(sweep, key=sweep.get))
        tot = 0.0
        for s in acase:
            g.set_schedule(**bc)
            ms = []
            for _ in range(3):
                if alg == gi.ALG_BFS:
                    g.bfs(int(s), out)
                elif alg == gi.ALG_CC:
                    g.cc(out)
                else:
                    g.pagerank(ranks, 20, 0.85)
                ms.append(g.stats().kernel_ms)
            tot += float(np.median(ms))
        fixed[names[alg]] = {"schedule": bc, "ms": round(tot, 3), "sweep_ms": sweep}
        log("held-out best fixed %s: %s %.3f ms" % (names[alg], bc, tot))
    # the learned direction on the autotuned layout: the best fixed schedule's
    # layout fields (segments, vertex order, pull shape) with the learned
    # per-step choice in place of its direction rule
    g.attach_selector(sel)
    layout_keys = ("num_segments", "segment_strategy", "segments_concurrent", "vertex_order",
                   "block_threads", "pull_items_per_thread", "pull_hot_sources",
                   "pull_block_edges")
    for alg in (gi.ALG_BFS, gi.ALG_CC, gi.ALG_PAGERANK):
        lay = {k: v for k, v in fixed[names[alg]]["schedule"].items() if k in layout_keys}
        tot = 0.0
        for s in [s for a, s in cases if a == alg]:
            g.set_schedule(direction=gi.LEARNED, **lay)
            ms = []
            for _ in range(4):
                if alg == gi.ALG_BFS:
                    g.bfs(int(s), out)
                elif alg == gi.ALG_CC:
                    g.cc(out)
                else:
                    g.pagerank(ranks, 20, 0.85)
                ms.append(g.stats().kernel_ms)
            tot += float(np.median(ms[1:]))
        fixed[names[alg]]["learned_on_layout_ms"] = round(tot, 3)
        fixed[names[alg]]["layout"] = lay
        log("held-out learned on the tuned layout %s %s: %.3f ms" % (names[alg], lay, tot))
    per_alg = {}
    for alg in ("bfs", "cc", "pagerank"):
        rs = [r for r in rows if r["alg"] == alg]
        h = sum(r["heuristic_ms"] for r in rs)
        le = sum(r["learned_ms"] for r in rs)
        b = sum(r["best_steps_ms"] for r in rs)
        f = fixed[alg]["ms"]
        per_alg[alg] = {"cases": len(rs), "heuristic_ms": round(h, 3),
                        "best_fixed_ms": f, "best_fixed": fixed[alg]["schedule"],
                        "learned_ms": round(le, 3), "per_step_best_ms": round(b, 3),
                        "learned_vs_heuristic": round(h / le, 3),
                        "learned_vs_best_fixed": round(f / le, 3),
                        "tuned_layout": fixed[alg]["layout"],
                        "learned_on_tuned_layout_ms": fixed[alg]["learned_on_layout_ms"],
                        "learned_on_tuned_layout_vs_best_fixed":
                            round(f / fixed[alg]["learned_on_layout_ms"], 3)}
    t_fixed = sum(fixed[a]["ms"] for a in fixed)
    t_learn_lay = sum(fixed[a]["learned_on_layout_ms"] for a in fixed)
    if args.selector_dump:
        p, mu, sd = sel.params()
        np.savez_compressed(args.selector_dump, X=X, Y=Yl, V=Vm, params=p, mu=mu, sd=sd, **dump)
    regret_l, regret_h = np.array(regret_l), np.array(regret_h)
    speedup = t_fixed / t_learn
    prec_pct = 100.0 * (prec[2] - prec[3]) / prec[3] if prec[3] > 0 else 0.0
    detail = {
        "learned_vs_heuristic": round(t_heur / t_learn, 3),
        "learned_vs_best_fixed": round(t_fixed / t_learn, 3),
        "learned_on_tuned_layout_vs_best_fixed": round(t_fixed / t_learn_lay, 3),
        "per_algorithm": per_alg,
        "best_fixed_sweeps_ms": {a: fixed[a]["sweep_ms"] for a in fixed},
        "bf16_vs_fp32": {"records": prec[0], "disagree": prec[1],
                         "regret_pct": round(prec_pct, 3), "bound_pct": 5.0,
                         "within_bound": bool(prec_pct <= 5.0)},
        "train_records": int(len(X)), "epochs": args.epochs, "train_s": round(t_train, 2),
        "loss_first_last": [round(float(loss[0]), 4), round(float(loss[-1]), 4)],
        "heldout": {"n": g.n, "m": g.m, "gamma": 2.0, "bfs_sources": int(len(srcs))},
        "total_ms": {"heuristic": round(t_heur, 3), "best_fixed": round(t_fixed, 3),
                     "learned": round(t_learn, 3), "learned_on_tuned_layout": round(t_learn_lay, 3),
                     "per_step_best": round(t_best, 3)},
        "regret_learned_us": {"mean": round(1e3 * regret_l.mean(), 3),
                              "p50": round(1e3 * float(np.percentile(regret_l, 50)), 3),
                              "p95": round(1e3 * float(np.percentile(regret_l, 95)), 3),
                              "total_pct": round(100 * regret_l.sum() / sum(best_steps), 2)},
        "regret_heuristic_us": {"mean": round(1e3 * regret_h.mean(), 3),
                                "p50": round(1e3 * float(np.percentile(regret_h, 50)), 3),
                                "p95": round(1e3 * float(np.percentile(regret_h, 95)), 3),
                                "total_pct": round(100 * regret_h.sum() / sum(best_steps), 2)},
        "per_case": rows, "wall_s": round(time.time() - t_all, 1),
    }
    config = {"workload": "selector_chunglu_g2.0_%s" % args.heldout, "n": g.n, "m": g.m,
              "train_graphs": ["rmat16", "rmat18", "rmat20", "rmat22", "chunglu1M_g2.2",
                               "chunglu1M_g2.5", "chunglu2M_g3.0", "chunglu4M_g2.2",
                               "chunglu1M_g2.2_x34", "chunglu2M_g2.5_x34", "rmat24",
                               "chunglu16M_g2.2_x34"]}
    roof = None
    return speedup, "x (best fixed schedule time / learned time)", t_learn, \
        "f32 train / bf16 infer", \
        config, roof, None, detail


def run_batched(args, torch, dev):
    """256 instances (even: BFS, odd: 20-iteration PageRank) over a pool of 14
    graphs: R-MAT scales 10..18 (seeds 100 + scale) and 4-neighbour grids
    64^2 .. 1024^2; BFS sources seeded per instance (seed 200 + i).  One
    persistent launch replayed from a HIP graph, workgroups autotuned, against
    256 sequential calls of the plain entry points on the same stream."""
    import numpy as np

    import graphgen as gg
    import paper_1805_00923_amd as gi
    els = [gg.rmat(s, 16, seed=100 + s) for s in range(10, 19)]
    els += [gg.grid(d, d, 0.0, weighted=False) for d in (64, 128, 256, 512, 1024)]
    graphs = [gi.Graph.from_edges(el.n, el.src, el.dst) for el in els]
    tasks, edges = [], 0
    for i in range(256):
        gidx = i % len(graphs)
        g, el = graphs[gidx], els[gidx]
        if i % 2 == 0:
            src = int(gg.pick_sources(el, 1, 200 + i)[0])
            out = torch.empty(g.n, dtype=torch.int32, device=dev)
            tasks.append(dict(graph=gidx, algorithm=gi.ALG_BFS, src=src, out=out))
        else:
            out = torch.empty(g.n, dtype=torch.float32, device=dev)
            tasks.append(dict(graph=gidx, algorithm=gi.ALG_PAGERANK, iters=20, damping=0.85,
                              out=out))
    # plain path: one call per instance, same stream
    ref = [torch.empty_like(t["out"]) for t in tasks]

    def plain():
        for t, r in zip(tasks, ref):
            g = graphs[t["graph"]]
            if t["algorithm"] == gi.ALG_BFS:
                g.bfs(t["src"], r)
            else:
                g.pagerank(r, 20, 0.85)
        torch.cuda.synchronize()
    # edges traversed per pass (TEPS convention: BFS m_reach, PageRank 20 m)
    plain()
    for t, r in zip(tasks, ref):
        g = graphs[t["graph"]]
        if t["algorithm"] == gi.ALG_BFS:
            lv = r.cpu().numpy()
            odeg = np.diff(g.out_off)
            edges += int(odeg[lv >= 0].sum())
        else:
            edges += 20 * g.m
    for _ in range(args.warmup):
        plain()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain()
    t_plain = (time.perf_counter() - t0) / args.steps
    b = gi.Batch(graphs, tasks)
    b.set_barrier_scope(barrier_scope(args))
    t0 = time.perf_counter()
    b.autotune(reps=3)
    t_tune = time.perf_counter() - t0
    for _ in range(args.warmup):
        b.run(use_graph=True)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run(use_graph=True)
        kms.append(b.info()["ms"])
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    # outputs agree with the plain path
    bad = 0
    for t, r in zip(tasks, ref):
        if t["algorithm"] == gi.ALG_BFS:
            bad += int(not torch.equal(t["out"], r))
        else:
            x, y = t["out"].double(), r.double()
            bad += int(((x - y).abs() / y).max().item() > 1e-6)
    info = b.info()
    bar = b.barrier_ms().astype(np.float64)
    wgs = info["workgroups"].astype(np.float64)
    is_bfs = np.array([t["algorithm"] == gi.ALG_BFS for t in tasks])
    value = edges / t_batch / 1e9
    tally = KernelTally(POOL_KERNEL)
    tally.add(kms, [pool_launch_bytes(gi, graphs, els, tasks, ref)] * len(kms))
    roof = tally.roofline()
    slow = np.argsort(-info["task_ms"])[:5]
    detail = {"plain_ms": round(t_plain * 1e3, 3), "batched_ms": round(t_batch * 1e3, 3),
              "batched_kernel_ms_median": round(float(np.median(kms)), 3),
              "speedup_vs_plain": round(t_plain / t_batch, 3),
              "plain_gteps": round(edges / t_plain / 1e9, 3),
              "autotune_s": round(t_tune, 2), "grid": info["grid"], "threads": b.threads(),
              "xcd_local": b.placement(),
              "workgroups_per_graph": {els[i].name: sorted(set(int(info["workgroups"][j])
                                                             for j in range(256)
                                                             if tasks[j]["graph"] == i))
                                       for i in range(len(els))},
              "mismatches_vs_plain": bad, "edges_per_pass": edges,
              "pr_block_edges_per_graph": {els[i].name: int(c)
                                           for i, c in enumerate(b.pr_block_edges()) if c},
              "slowest_tasks": [{"graph": els[tasks[j]["graph"]].name,
                                 "alg": "bfs" if tasks[j]["algorithm"] == gi.ALG_BFS else "pr",
                                 "ms": round(float(info["task_ms"][j]), 3),
                                 "levels": int(info["levels"][j]),
                                 "workgroups": int(info["workgroups"][j]),
                                 "barrier_ms": round(float(bar[j]), 3),
                                 "barrier_fraction": round(float(bar[j] / max(info["task_ms"][j], 1e-9)), 3)}
                                for j in slow],
              # synchronisation in place of the plain path's launches: the
              # workgroup-time the tasks spent in their barriers, and the
              # launch's host-side overhead beyond the kernel's own time
              "barrier_fraction_of_workgroup_time": round(float(
                  (bar * wgs).sum() / max(float((info["task_ms"] * wgs).sum()), 1e-9)), 4),
              "barrier_fraction_by_algorithm": {
                  a: round(float((bar * wgs)[sel].sum() / max(float((info["task_ms"] * wgs)[sel].sum()), 1e-9)), 4)
                  for a, sel in (("bfs", is_bfs), ("pagerank", ~is_bfs))},
              "launch_overhead_fraction": round(max(0.0, 1.0 - float(np.median(kms)) / (t_batch * 1e3)), 4)}
    config = {"workload": "batched256_bfs_pr20_rmat10-18_grid64-1024", "instances": 256,
              "graphs": [el.name for el in els]}
    return value, "GTEPS", t_batch * 1e3, "int32 / f32+f64", config, roof, None, detail


def run_prdelta(args, torch, dev):
    """PageRankDelta, 10 rounds, epsilon 0.1, damping 0.85, DensePull-SparsePush
    with a bitvector frontier, on R-MAT scale 22 (seed 2).  GTEPS counts the
    edges the rounds examined (push: out-edges of the active vertices; pull:
    every in-edge)."""
    import numpy as np
    import paper_1805_00923_amd as gi
    el, g = make_rmat_graph(22, 2)
    g.set_schedule(direction=gi.DENSE_PULL_SPARSE_PUSH, dense_frontier=gi.BITVECTOR,
                   **sched_overrides(args.schedule))
    ranks = torch.empty(g.n, dtype=torch.float64, device=dev)
    g.set_step_timing(True)
    for _ in range(args.warmup):
        g.prdelta(ranks, 10, 0.85, 0.1)
    torch.cuda.synchronize()
    edges, kms = 0, []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.prdelta(ranks, 10, 0.85, 0.1)
        st = g.stats()
        edges += int(st.edges_examined)
        kms.append(st.kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = g.stats()
    dirs, fs, ds = st.trace()
    value = edges / dt / 1e9
    # roofline per run: every kernel of the 10 rounds (frontier bookkeeping
    # included) against the rounds' algorithmic bytes
    tally = KernelTally("prdelta run (all kernels of its rounds)")
    tally.add(kms, [sum(prdelta_round_bytes(g.n, g.m, dirs, fs, ds))] * len(kms))
    roof = tally.roofline()
    detail = {"rounds": int(st.steps), "directions": [int(x) for x in dirs],
              "frontiers": [int(x) for x in fs], "run_ms_median": round(float(np.median(kms)), 3)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph(el)
        t0 = time.perf_counter()
        oracle.prdelta(og, 10, 0.85, 0.1)
        dtc = time.perf_counter() - t0
        cpu = {"value": round(edges / args.steps / dtc / 1e9, 5), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", "sample": "fp64 PageRankDelta, 10 rounds, full graph, one "
                                           "thread, %.2f s (edges counted as on the GPU)" % dtc}
    config = {"workload": "prdelta10_eps0.1_rmat22_ef16", "n": g.n, "m": g.m,
              "schedule": g.schedule().as_dict()}
    return value, "GTEPS", dt * 1e3 / args.steps, "f64", config, roof, cpu, detail


def run_bc(args, torch, dev):
    """Single-source betweenness dependencies (Brandes: forward path counts,
    backward dependencies) from 8 sources on R-MAT scale 22 (seed 2).  GTEPS
    counts each reached edge twice per source (forward and backward sweep).
    Algorithmic bytes per source: 16 n_r + 36 m_r (n_r, m_r: reached vertices
    and their out-edges; forward 8 n_r + 16 m_r: offsets, ids, level test,
    fp64 path-count add; backward 8 n_r + 20 m_r: offsets, ids, level test,
    fp64 path count and dependency), over the GPU span of the run measured
    with HIP events on its stream."""
    import numpy as np

    import graphgen as gg
    el, g = make_rmat_graph(22, 2)
    n = g.n
    srcs = [int(x) for x in gg.pick_sources(el, 8, 9)]
    dep = torch.empty(n, dtype=torch.float64, device=dev)
    sig = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    odeg = np.diff(g.out_off).astype(np.int64)
    reach = []
    for s_ in srcs:
        g.bc(s_, dep, sig)
        sg = sig.cpu().numpy()
        r = sg > 0
        reach.append((int(r.sum()), int(odeg[r].sum())))
    for _ in range(args.warmup):
        for s_ in srcs:
            g.bc(s_, dep, sig)
    torch.cuda.synchronize()
    tally = KernelTally("k_bc_forward + k_bc_advance + k_bc_backward (one source)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for s_, (nr, mr) in zip(srcs, reach):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.bc(s_, dep, sig)
            e1.record(stream)
            e1.synchronize()
            tally.add([e0.elapsed_time(e1)], [16 * nr + 36 * mr])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    edges = 2 * sum(mr for _, mr in reach)
    value = edges / dt / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph(el)
        t0 = time.perf_counter()
        oracle.bc(og, srcs[0])
        dtc = time.perf_counter() - t0
        cpu = {"value": round(2 * reach[0][1] / dtc / 1e9, 5), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", "sample": "fp64 Brandes dependencies from the first source, "
                                           "full graph, one thread, %.2f s" % dtc}
    detail = {"sources": srcs, "reached_vertices": [nr for nr, _ in reach],
              "reached_edges": [mr for _, mr in reach],
              "ms_per_source": round(dt * 1e3 / len(srcs), 3)}
    config = {"workload": "bc8_rmat22_ef16", "n": n, "m": g.m}
    return value, "GTEPS", dt * 1e3, "f64", config, tally.roofline(), cpu, detail


def run_prec(args, torch, dev):
    """PageRank and eigenvector centrality, 20 iterations each, on R-MAT scale
    22 (seed 2): the fused pass (one traversal, (contribution, x) pairs)
    timed against the two separate passes.  GTEPS counts the edges of both
    kernels, 2 * 20 * m per run, either way."""
    import numpy as np
    import paper_1805_00923_amd as gi
    el, g = make_rmat_graph(22, 2)
    n, m = g.n, g.m
    ranks = torch.empty(n, dtype=torch.float32, device=dev)
    eigen = torch.empty(n, dtype=torch.float32, device=dev)
    base_sched = sched_overrides(args.schedule)
    res = {}
    outs = {}
    # unfused, fused over the id-order rows, fused over the degree-ordered rows
    for fused in (False, True, "ordered"):
        g.set_schedule(**dict(base_sched, vertex_order=1 if fused == "ordered" else 0))
        g.set_step_timing(True)
        for _ in range(max(1, args.warmup)):
            g.pagerank_eigenvector(ranks, eigen, 20, 0.85, bool(fused))
        torch.cuda.synchronize()
        tally = KernelTally("k_prec_rows<fused> (degree-ordered)" if fused == "ordered" else
                            "k_prec_rows<fused>" if fused else "k_pr_rows + k_prec_rows<unfused>")
        kms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.pagerank_eigenvector(ranks, eigen, 20, 0.85, bool(fused))
            kms.append(g.stats().kernel_ms)
            _, mm = g.step_times()
            per = 4 * m + 24 * n if fused else 8 * m + 28 * n
            tally.add(mm, [per] * len(mm))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[fused] = (dt, float(np.median(kms)), tally)
        outs[fused] = (ranks.clone(), eigen.clone())
    g.set_step_timing(False)
    # the headline fused figure is the faster layout's
    best = "ordered" if res["ordered"][1] < res[True][1] else True
    g.set_schedule(**dict(base_sched, vertex_order=1 if best == "ordered" else 0))
    dt, kmed, tally = res[best]
    dtu, kmedu, tallyu = res[False]
    dti, kmedi, tallyi = res[True]
    dto, kmedo, tallyo = res["ordered"]
    (rf, ef), (ru, eu) = outs[best], outs[False]
    ro, eo = outs["ordered"]
    ri, ei = outs[True]
    agree = {"pr_max_rel": float(((rf.double() - ru.double()).abs() / ru.double()).max().item()),
             "ec_max_abs_over_max": float((ef.double() - eu.double()).abs().max().item()
                                          / max(eu.double().abs().max().item(), 1e-30))}
    value = 40.0 * m / dt / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph(el)
        t0 = time.perf_counter()
        oracle.pagerank(og, 3, 0.85)
        oracle.eigenvector(og, 3)
        dtc = time.perf_counter() - t0
        cpu = {"value": round(6.0 * m / dtc / 1e9, 5), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", "sample": "fp64 pull PageRank and power-iteration eigenvector "
                                           "centrality, 3 iterations each on the full graph, "
                                           "one thread, %.2f s" % dtc}
    uroof = tallyu.roofline()
    detail = {"fused_ms": round(dt * 1e3, 3), "unfused_ms": round(dtu * 1e3, 3),
              "fused_kernel_ms_median": round(kmed, 3),
              "unfused_kernel_ms_median": round(kmedu, 3),
              # fusion on the same (id-order) layout, and the degree order on
              # top of fusion, apart
              "fusion_speedup": round(kmedu / kmedi, 3),
              "degree_order_speedup_fused": round(kmedi / kmedo, 3),
              "unfused_gteps": round(40.0 * m / dtu / 1e9, 3),
              "unfused_roofline": uroof, "fused_vs_unfused": agree,
              "fused_layout": "degree-ordered" if best == "ordered" else "id order",
              "fused_id_order_kernel_ms_median": round(kmedi, 3),
              "fused_degree_ordered_kernel_ms_median": round(kmedo, 3),
              "fused_id_order_roofline": tallyi.roofline(),
              "fused_degree_ordered_roofline": tallyo.roofline(),
              "degree_ordered_vs_id_order": {
                  "pr_max_rel": float(((ro.double() - ri.double()).abs() / ri.double()).max().item()),
                  "ec_max_abs_over_max": float((eo.double() - ei.double()).abs().max().item()
                                               / max(ei.double().abs().max().item(), 1e-30))},
              "bytes_per_iteration": {"fused": 4 * m + 24 * n, "unfused": 8 * m + 28 * n}}
    config = {"workload": "pagerank20+eigenvector20_fused_rmat22_ef16", "n": n, "m": m,
              "schedule": g.schedule().as_dict()}
    return value, "GTEPS", dt * 1e3, "f32 storage / f64 accumulate", config, tally.roofline(), \
        cpu, detail


def gpu_clocks():
    """Current shader and memory clock levels as rocm-smi reports them (clocks
    are not pinned).  Read in a child process before this process touches
    the GPU; any failure is reported as text."""
    import shutil
    import subprocess
    # under rocprofv3 (which sets ROCPROF* variables) a child would inherit
    # the profiler's preloaded library
    if any(k.startswith("ROCPROF") for k in os.environ):
        return {"skipped": "running under a profiler"}
    exe = shutil.which("rocm-smi") or "/opt/rocm/bin/rocm-smi"
    try:
        r = subprocess.run([exe, "--showclocks", "--json"], capture_output=True,
                           text=True, timeout=30)
        data = json.loads(r.stdout)
    except Exception as e:  # noqa: BLE001 - the reading is informational
        return {"error": str(e)[:200]}
    out = {}
    for card, kv in data.items():
        if isinstance(kv, dict):
            out[card] = {k: v for k, v in kv.items() if "sclk" in k or "mclk" in k}
    return out or {"error": (r.stderr or r.stdout)[:200]}


def host_info():
    """Logical core count, CPU model and memory of the host (the oracle's
    baseline uses one thread of it)."""
    model, mem_gb = "unknown CPU", 0.0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    mem_gb = int(line.split()[1]) / 1024.0 / 1024.0
                    break
    except OSError:
        pass
    return "%d logical cores, %s, %.0f GiB RAM" % (os.cpu_count() or 0, model, mem_gb)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the library is a "
              "single-device build)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    clocks = gpu_clocks()
    import torch
    dev = torch.device("cuda:0")
    if args.copy_calib_mb > 0:
        src = torch.ones(args.copy_calib_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "bfs_cc_rmat22":
        res = run_bfs_cc(args, torch, dev)
    elif args.workload == "pr_rmat16":
        res = run_pr(args, torch, dev, 16)
    elif args.workload == "pr_rmat22":
        res = run_pr(args, torch, dev, 22)
    elif args.workload == "prdelta_rmat22":
        res = run_prdelta(args, torch, dev)
    elif args.workload == "prec_rmat22":
        res = run_prec(args, torch, dev)
    elif args.workload == "bc_rmat22":
        res = run_bc(args, torch, dev)
    elif args.workload == "batched":
        res = run_batched(args, torch, dev)
    elif args.workload == "selector":
        res = run_selector(args, torch, dev)
    else:
        res = run_sssp(args, torch, dev)
    value, unit, ms_step, dtype, config, roof, cpu, extra = res
    extra = dict(extra or {}, gpu_clocks_at_start=clocks)
    if cpu:
        cpu = dict(cpu, sample=cpu["sample"] + "; host: " + host_info())
    if roof and roof.get("traffic") is None:
        roof["traffic"] = profile_traffic(roof["kernel"], config.get("workload"),
                                          config.get("schedule"), config.get("batch_plan"))
    line = {"metric": METRIC, "value": round(value, 4), "unit": unit, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config, "roofline": roof, "cpu_baseline": cpu,
            "detail": extra}
    s = json.dumps(line, default=lambda o: o.item() if hasattr(o, "item") else str(o))
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(s + "\n")
    print(s, flush=True)


if __name__ == "__main__":
    main()
