"""Host-side checks of bench.py's contract that need no GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profiled_traffic_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    # a committed summary that matches the tree gives its bytes per launch;
    # another workload, or a summary of other kernel sources, gives None
    wl = "rti3d_128x128x512"
    t = bench.profiled_traffic("fp32", wl, "k_collide_nphi")
    assert t is None or 3.0e9 < t < 5.0e9
    assert bench.profiled_traffic("fp32", "rti3d_128x128x256", "k_collide_nphi") is None
    assert bench.profiled_traffic("fp32", wl, "kb_step") is None
    monkeypatch.setattr(bench, "PROFILES_DIR", str(tmp_path))
    fake = tmp_path / ("k_collide_nphi_k_phi_merge_%s_fp32_hbm_bytes.md" % wl)
    fake.write_text("x\n```json\n" + json.dumps({"kernel": "k_collide_nphi", "sources_sha256": "0" * 64,
                                                   "traffic_bytes_per_launch": 1}) + "\n```\n")
    assert bench.profiled_traffic("fp32", wl, "k_collide_nphi") is None


def test_algorithmic_bytes_follow_the_storage_sizes():
    # read and write every population once (+ phi for the two-kernel form)
    assert bench.ALG_BYTES[("fp32", 3)]["collide"] == 27 * 4 * 4 + 4
    assert bench.ALG_BYTES[("fp32", 3)]["method"] == 27 * 4 * 4 + 8
    assert bench.ALG_BYTES[("fp64", 3)]["collide"] == 2 * bench.ALG_BYTES[("fp32", 3)]["collide"]
    assert bench.ALG_BYTES[("fp32", 2)]["method"] == 9 * 4 * 4 + 8


def test_phi_summing_update_bytes():
    # the update's 436 B plus its partial sums: three per cell and three more
    # per cell of a tile's two edge rows; the merge reads them and writes phi
    assert bench.nphi_bytes("fp32", 4) == (436 + 4 * 4.5, 4 * 4.5 + 4)
    assert bench.nphi_bytes("fp32", 1) == (436 + 4 * 9, 4 * 9 + 4)
    up, merge = bench.nphi_bytes("fp64", 2)
    assert up == 872 + 8 * 6 and merge == 8 * 6 + 8
    # a step moves more than the method's minimum, less than with the phi pass
    ab = bench.ALG_BYTES[("fp32", 3)]
    assert ab["method"] < sum(bench.nphi_bytes("fp32", 4)) < ab["collide"] + ab["phi"]
