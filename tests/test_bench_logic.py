"""Host logic of the benchmark (CPU): the committed counter summaries are
well formed, a changed kernel source (not a changed comment) voids a
summary's traffic, the
memo-free search's algorithmic bytes follow their per-unit figures, and a
request for more than one GPU is refused before anything runs."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_counter_summaries_are_well_formed():
    # each summary holds one record: kernel, workload, fetch + write bytes and
    # the hash of the sources it was taken from (bench.py reports its traffic
    # only while that hash matches)
    for path, kernel, workload, key in ((bench.TRAFFIC_FILE, "k_celf_persistent", "c4", "bytes_per_launch"),
                                        (bench.BFS_TRAFFIC_FILE, "k_bfs_level", "d1", "bytes_per_step"),
                                        (bench.CC_TRAFFIC_FILE, "components", "c4", "bytes_components")):
        if path == bench.CC_TRAFFIC_FILE and not os.path.exists(path):
            continue  # taken after the labelling kernels' latest change
        lines = [l for l in open(path) if l.startswith("TRAFFIC_JSON ")]
        assert len(lines) == 1, path
        rec = json.loads(lines[0][len("TRAFFIC_JSON "):])
        assert rec["kernel"] == kernel and rec["workload"] == workload
        assert rec[key] == rec["fetch_bytes"] + rec["write_bytes"] > 0
        assert len(rec["source_hash"]) == 16 and int(rec["source_hash"], 16) >= 0
        assert rec["algorithmic_bytes"] > 0
        if "per_kernel_bytes" in rec:  # the components phase: its kernels' traffic adds up
            assert set(rec["per_kernel_bytes"]) == set(bench.CC_KERNELS)
            assert sum(rec["per_kernel_bytes"].values()) == rec[key]


def test_changed_source_voids_the_traffic_record(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel one\n")
    rec = {"kernel": "k", "workload": "w", "bytes_per_step": 3, "fetch_bytes": 2, "write_bytes": 1,
           "source_hash": bench.roof_source_hash([str(src)])}
    summary = tmp_path / "k_traffic.txt"
    summary.write_text("# header\nTRAFFIC_JSON " + json.dumps(rec) + "\n")
    assert bench.read_traffic(str(summary), [str(src)]) == rec
    # an edited comment or re-indented line is not a change of the kernel
    src.write_text("// a comment\nkernel   one /* an\n other */\n")
    assert bench.read_traffic(str(summary), [str(src)]) == rec
    src.write_text("kernel two\n")
    assert bench.read_traffic(str(summary), [str(src)]) is None
    assert bench.read_traffic(str(tmp_path / "missing.txt"), [str(src)]) is None


def test_search_algorithmic_bytes():
    work = dict(levels=3, items=10, arcs=100, live_pairs=7)
    assert bench.bfs_algorithmic_bytes(work, True) == 72 * 10 + 12 * 100 + 96 * 7
    assert bench.bfs_algorithmic_bytes(work, False) == 72 * 10 + 8 * 100 + 96 * 7


def test_celf_algorithmic_bytes():
    # mask words per evaluation and commit, 1 KiB per listed tile, 8 B per gathered column
    assert bench.celf_algorithmic_bytes(evals=10, K=2, mwords=1, listed_tiles=5, gathers=100) == \
        4 * 12 + 1024 * 5 + 8 * 100


def test_cc_algorithmic_bytes():
    work = dict(live_pairs=50, union_attempts=7, flatten_rewrites=3, count_atomics=11, row_tiles=4, hub_tiles=2,
                gain_gathers=13, hub_link_waves=1)
    b = bench.cc_algorithmic_bytes(work, n=100, mwords=1, light_slots=300, hub_slots=90, listed=6, link_tiles=2)
    assert b["hook"] == 8 * 300 + 1024 * 4 + 8 * 100
    assert b["hook_hubs"] == 8 * 90 + 1024 * 2
    assert b["lists"] == 8 * 100 + 4 * (6 + 2) + 8 * 100
    assert b["link+link_hubs"] == 1024 * 2 + 12 * 7
    assert b["flatten"] == 1024 * 6 + 4 * 3
    assert b["count"] == 1024 * 6 + 8 * 11
    assert b["gain0"] == 1024 * 6 + 4 * 13 + 8 * 100


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout.strip()
