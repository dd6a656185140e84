"""Host-side parts of bench.py: the one-GPU guard, the algorithmic byte model
behind the roofline figure, and that the committed counter profile was taken on
the current fused-pass sources (bench.py reports measured traffic only then)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_fine_pass_bytes_at_400x128x512():
    """128 real planes of 398 x 510 interior unknowns; level 1 has 199 x 255.
    Up pass: read u and f, write u (24 B per unknown) and read the coarse
    correction (8 B per level-1 unknown)."""
    b = bench.alg_bytes({"level_shapes": [(400, 512), (201, 257)]}, 128)
    assert b["n0"] == 25_981_440
    assert b["up"] == 675_517_440
    assert b["down"] == b["up"]
    assert b["down_first"] == b["down"] - 8 * 25_981_440


def test_counter_profile_matches_the_fused_pass_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert rec["source_hash"] == bench.source_hash(), (
        "profiles/traffic.json was taken on other fused-pass sources: retake the FETCH_SIZE and "
        "WRITE_SIZE profiles and ingest them with bench.py --ingest-counters")
    assert {"fine_up", "fine_down"} <= set(rec["bytes_per_launch"])
    for k in ("fine_up", "fine_down"):
        assert 0.9 < rec["bytes_per_launch"][k] / bench.alg_bytes(
            {"level_shapes": [(400, 512), (201, 257)]}, 128)["up"] < 1.25
