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
    # merged pass: read u and f, write u; read the coarse correction and write
    # the coarse right-hand side (8 B each per level-1 unknown)
    assert b["merged"] == 24 * 25_981_440 + 16 * 128 * 199 * 255


def test_counter_profile_matches_the_fused_pass_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert rec["source_hash"] == bench.source_hash(), (
        "profiles/traffic.json was taken on other fused-pass sources: retake the FETCH_SIZE and "
        "WRITE_SIZE profiles and ingest them with bench.py --ingest-counters")
    assert {"fine_up", "fine_down", "fine_merged"} <= set(rec["bytes_per_launch"])
    alg = bench.alg_bytes({"level_shapes": [(400, 512), (201, 257)]}, 128)
    for k, model in (("fine_up", "up"), ("fine_down", "down"), ("fine_merged", "merged")):
        assert 0.9 < rec["bytes_per_launch"][k] / alg[model] < 1.25


def test_accuracy_measures_on_a_planted_error():
    """One interior node off by d: rel-L_inf is d / max|ref|, rel-L2 is
    d / ||ref||, and the charge-driven part divides by ||ref - 300 z / L||."""
    import numpy as np

    import workloads as W

    p = W.SMALL
    ref = W.manufactured_potential(p, 12345)
    phi = ref.copy()
    d = 1e-9
    phi[3, 7, 11] += d
    a = bench.accuracy(phi, ref, p, "x")
    inner = ref[:, 1:-1, 1:-1]
    _, z, r = W.node_coordinates(p)
    blobs = inner - (300.0 * z / p.length)[None, 1:-1, None]
    assert np.isclose(a["rel_linf_vs_x"], d / np.abs(inner).max(), rtol=1e-12)
    assert np.isclose(a["rel_l2_vs_x"], d / np.linalg.norm(inner), rtol=1e-12)
    assert np.isclose(a["rel_l2_charge_part_vs_x"], d / np.linalg.norm(blobs), rtol=1e-12)
    w = np.broadcast_to(r[None, None, 1:-1], inner.shape)
    assert np.isclose(a["eps2_vs_x"], d * np.sqrt(r[11] / np.sum(w * inner * inner)), rtol=1e-12)
    # the error on boundary nodes is not counted
    phi[0, 0, 0] += 1.0
    assert bench.accuracy(phi, ref, p, "x") == a


def test_full_multigrid_byte_model():
    """A V-cycle: 52 B per unknown of each level on passes (weighted 4^-l) down
    to the exactly solved level (32 B per unknown of it), 69.3 B with every
    level on passes.  Start: read f, write the level-1 right-hand side, one
    V-cycle from level 1 (the cycle's bytes below the finest level); the first
    down pass reads the level-1 answer (2 B) instead of the iterate (8 B)."""
    assert abs(bench.cycle_bytes(-1) - 52 * 4 / 3) < 1e-12
    assert abs(bench.cycle_bytes(2) - (52 + 13 + 2)) < 1e-12  # 400 x 128 x 512: level 2 exact
    assert abs(bench.fmg_bytes(-1) - (8 + 2 + 69.3333333333333 / 4 + 2 - 8)) < 1e-9
    assert abs(bench.fmg_bytes(2) - (8 + 2 + 15 + 2 - 8)) < 1e-12
