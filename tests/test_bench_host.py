"""Host-side logic of bench.py: the algorithmic byte counts per step (the
formulas of the measurement plan, checked on hand-made traces), the lookup
of committed hardware-counter figures (valid only while the kernel sources
hash to the recorded value), the clock reading's failure path, and the
single-GPU contract."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bfs_step_bytes_push_and_pull():
    n = 1024
    # step 0 push: |F| = 1, D_F = 10, |F'| = 10
    # step 1 pull: |F| = 10, so 11 vertices are visited and U = n - 11;
    #   E = 300 in-edges scanned, |F'| = 500
    # step 2 push: |F| = 500, D_F = 40, |F'| = 0 (last step)
    dirs, fs, ds, es = [0, 2, 0], [1, 10, 500], [10, 4000, 40], [10, 300, 40]
    got = bench.bfs_step_bytes(n, dirs, fs, ds, es)
    assert got[0] == 12 * 1 + 8 * 10 + 8 * 10
    assert got[1] == 3 * n // 8 + 8 * (n - 11) + 4 * 300 + 4 * 500
    assert got[2] == 12 * 500 + 8 * 40 + 0


def test_cc_step_bytes_push_and_pull():
    n = 4096
    dirs, fs, ds, es = [2, 0], [n, 7], [0, 0], [50000, 30]
    got = bench.cc_step_bytes(n, dirs, fs, ds, es)
    assert got[0] == 4 * (n + 1) + 4 * 50000 + 12 * n + n // 4
    assert got[1] == 16 * 7 + 8 * 30 + 0


def test_sssp_label_setting_bytes():
    # a run that reaches 3 vertices with 5 edges out of them: each edge's
    # index, weight and target distance, each vertex's offsets and distance
    assert bench.sssp_label_setting_bytes(5, 3) == 12 * 5 + 12 * 3
    assert bench.sssp_label_setting_bytes(0, 1) == 12


def test_profile_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    """A committed figure is read only for its kernel, workload and (where
    named) schedule, and only while the kernel's sources hash to the value
    recorded with it."""
    import hashlib
    csrc = tmp_path / "paper_1805_00923_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text("kernel a\n")
    (csrc / "b.h").write_text("header b\n")
    sha = hashlib.sha256(b"kernel a\nheader b\n").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    sched = dict(vertex_order=1, num_segments=1, block_threads=1024, pull_items_per_thread=4,
                 pull_hot_sources=-1)
    (prof / "x.md").write_text(
        "text\n<!-- figures\nkernel: kx\nworkload: w1\nschedule: %s\nsource_sha256: %s\n"
        "sources: a.hip b.h\ntraffic_bytes_per_launch: 1234\n-->\n" % (bench.sched_key(sched), sha))
    (prof / "y.md").write_text(
        "<!-- figures\nkernel: ky\nsource_sha256: %s\nsources: a.hip b.h\n"
        "traffic_bytes_per_launch: 99\n-->\n" % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_traffic("kx", "w1", sched) == 1234
    assert bench.profile_traffic("kx", "w2", sched) is None          # other workload
    assert bench.profile_traffic("kx", "w1", dict(sched, block_threads=512)) is None
    assert bench.profile_traffic("kx", "w1", None) is None           # schedule required
    assert bench.profile_traffic("ky", "anything") == 99             # names neither
    assert bench.profile_traffic("kz") is None
    (prof / "z.md").write_text(
        "<!-- figures\nkernel: kp\nplan: threads=512,workgroups=32\nsource_sha256: %s\n"
        "sources: a.hip b.h\ntraffic_bytes_per_launch: 7\n-->\n"
        "<!-- figures\nkernel: kp\nplan: threads=256,workgroups=32\nsource_sha256: %s\n"
        "sources: a.hip b.h\ntraffic_bytes_per_launch: 8\n-->\n" % (sha, sha))
    assert bench.profile_traffic("kp", plan="threads=512,workgroups=32") == 7
    assert bench.profile_traffic("kp", plan="threads=256,workgroups=32") == 8   # second block
    assert bench.profile_traffic("kp", plan="threads=1024,workgroups=16") is None
    (csrc / "b.h").write_text("header b, changed\n")
    assert bench.profile_traffic("kx", "w1", sched) is None          # sources changed
    assert bench.profile_traffic("ky") is None


def test_gpu_clocks_reports_failure_as_text():
    c = bench.gpu_clocks()
    assert isinstance(c, dict) and c
    if "error" in c:
        assert isinstance(c["error"], str)


def test_gpu_clocks_skipped_under_a_profiler(monkeypatch):
    monkeypatch.setenv("ROCPROF_OUTPUT_PATH", "/tmp/x")
    assert bench.gpu_clocks() == {"skipped": "running under a profiler"}


def test_host_info_names_cores_and_memory():
    h = bench.host_info()
    assert "logical cores" in h and "GiB RAM" in h


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_oracle_timing_pins_one_core_and_restores():
    before = os.sched_getaffinity(0)
    with bench.one_core():
        inside = os.sched_getaffinity(0)
        assert len(inside) == 1 and inside <= before
    assert os.sched_getaffinity(0) == before


def test_pagerank_kernel_names_follow_the_schedule():
    class S:
        vertex_order, num_segments, segments_concurrent = 0, 1, 0
    s = S()
    assert bench.pr_kernel_name(s) == "k_pr_rows"
    s.num_segments = 4
    assert bench.pr_kernel_name(s) == "k_pr_rows per segment + k_pr_seg_final"
    s.segments_concurrent = 1
    assert bench.pr_kernel_name(s) == "k_pr_seg_concurrent + k_pr_seg_final_multi"
    s.vertex_order = 1
    assert bench.pr_kernel_name(s) == "k_pr_ord + k_pr_ord_split"
    # every candidate the autotuner tries is a dict of known schedule fields
    import paper_1805_00923_amd as gi
    names = {f for f, _ in gi.Schedule._fields_}
    for c in bench.PR_CANDIDATES:
        assert set(c) <= names, c


def _brute_pull_scan(in_off, in_idx, level, k):
    e = 0
    for v in range(len(in_off) - 1):
        if 0 <= level[v] <= k:
            continue                      # visited before step k
        for j in range(in_off[v], in_off[v + 1]):
            e += 1
            if level[in_idx[j]] == k:     # first in-edge from the frontier
                break
    return e


def test_pull_scan_replay_matches_brute_force():
    """The host replay of E_scan (in-edges scanned in CSC order up to the
    first frontier member) equals a literal scan, for every step taken as a
    pull, on an R-MAT graph and a grid from several sources."""
    import numpy as np
    import graphgen as gg
    import oracle
    for el in (gg.rmat(9, seed=21), gg.grid(9, 13, 0.05, seed=3, weighted=False)):
        og = oracle.Graph(el)
        rep = bench.PullScanReplay(og.inc.off, og.inc.idx)
        for s in gg.pick_sources(el, 3, 5):
            level = oracle.bfs(og, int(s))[0]
            steps = int(level.max()) + 1
            got = rep.step_edges(level, [2] * steps)
            for k in range(steps):
                assert got[k] == _brute_pull_scan(og.inc.off, og.inc.idx, level, k), (el.name, s, k)
            # only the steps marked as pulls are replayed
            assert set(rep.step_edges(level, [0, 2] + [0] * (steps - 2))) == {1}


def test_pool_launch_bytes_bfs_and_pagerank():
    """The pool's launch bytes: a BFS task's levels under the hybrid rule at
    divisor 20 with CSC-order pull scans, plus 20 (4m + 16n) per PageRank
    task, on a path (push only) and a star (one pull level)."""
    import types
    import numpy as np
    import graphgen as gg
    import paper_1805_00923_amd as gi
    path, star = gg.path(6), gg.star(9)
    els = [path, star]

    def host_graph(el):
        off, idx, _ = gi.build_adjacency(el.n, el.src, el.dst)
        return types.SimpleNamespace(n=el.n, m=int(off[-1]), out_off=off)
    graphs = [host_graph(el) for el in els]
    Out = types.SimpleNamespace
    arr = lambda a: Out(cpu=lambda: Out(numpy=lambda: np.asarray(a, np.int32)))
    tasks = [dict(graph=0, algorithm=gi.ALG_BFS), dict(graph=1, algorithm=gi.ALG_BFS),
             dict(graph=0, algorithm=gi.ALG_PAGERANK)]
    outs = [arr([0, 1, 2, 3, 4, 5]), arr([0] + [1] * 8), None]
    got = bench.pool_launch_bytes(gi, graphs, els, tasks, outs)
    # path 0->1->...->5, m = 5: level k holds one vertex of out-degree 1 (the
    # last none); (1 + 1) * 20 > 5 pulls every level but the last
    n0, m0 = 6, 5
    lv0 = np.arange(6)
    fs0 = np.ones(6, np.int64)
    ds0 = np.array([1, 1, 1, 1, 1, 0])
    dirs0 = [2 if (fs0[k] + ds0[k]) * 20 > m0 else 0 for k in range(6)]
    ioff0, iidx0, _ = gi.build_adjacency(path.n, path.dst, path.src)
    es0 = [0] * 6
    for k, e in bench.PullScanReplay(ioff0, iidx0).step_edges(lv0, dirs0).items():
        es0[k] = e
    want = sum(bench.bfs_step_bytes(n0, dirs0, fs0, ds0, es0))
    # star 0 -> 1..8, m = 8: level 0 has degree 8, (1 + 8) * 20 > 8 pulls;
    # level 1 has no out-edges and 8 * 20 > 8 pulls too
    lv1 = np.array([0] + [1] * 8)
    fs1 = np.array([1, 8])
    ds1 = np.array([8, 0])
    dirs1 = [2, 2]
    ioff1, iidx1, _ = gi.build_adjacency(star.n, star.dst, star.src)
    es1 = [0, 0]
    for k, e in bench.PullScanReplay(ioff1, iidx1).step_edges(lv1, dirs1).items():
        es1[k] = e
    assert es1 == [8, 0]  # each leaf stops at its only in-edge; nothing left after
    want += sum(bench.bfs_step_bytes(9, dirs1, fs1, ds1, es1))
    want += 20 * (4 * m0 + 16 * n0)
    assert got == want


def test_prdelta_round_bytes_by_hand():
    """PageRankDelta's round bytes on n = 64, m = 100: a pull round and a
    push round of 3 active vertices with 7 out-edges, each with the vertex
    update of every round."""
    n, m = 64, 100
    got = bench.prdelta_round_bytes(n, m, [2, 0], [64, 3], [100, 7])
    update = 52 * 64 + 8
    assert got == [4 * 65 + 400 + 16 * 64 + update, 36 + 84 + 8 + update]


def test_profile_figures_match_the_kernel_sources():
    """Every counter figure committed under profiles/ was taken on the kernel
    sources as they are: the sha256 of the sources a block lists equals the
    one it records (a kernel changed since its counters were taken would have
    the benchmark report its traffic as null)."""
    import glob
    import hashlib
    import os
    import re
    blocks = []
    for path in sorted(glob.glob(os.path.join(bench.ROOT, "profiles", "*.md"))):
        for b in re.findall(r"<!-- figures.*?-->", open(path).read(), re.S):
            blocks.append((os.path.basename(path), dict(re.findall(r"^(\w+): (.+)$", b, re.M))))
    assert blocks
    for name, kv in blocks:
        h = hashlib.sha256()
        for f in kv["sources"].split():
            with open(os.path.join(bench.ROOT, "paper_1805_00923_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        assert h.hexdigest() == kv["source_sha256"], (name, kv.get("kernel"), kv.get("plan"))
        assert int(kv["traffic_bytes_per_launch"]) > 0, name
