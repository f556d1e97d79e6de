"""Host logic of bench.py: the roofline accounting of the dominant kernel
(algorithmic bytes per launch over the measured launch time), the
memory-side bytes taken from the committed counter summaries only while the
kernel sources and the tile match, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

HEADLINE_TILE = {"fused": 1, "two_step": 1, "two_step_tx": 128, "two_step_rows": 1,
                 "two_step_zc": 512, "two_step_prefetch": 1, "two_step_threads": 1024,
                 "two_step_ty": 16}


def test_words_per_launch_and_per_cell_step_agree():
    """A launch of kind k covers STEPS_PER_LAUNCH[k] steps and moves
    WORDS[k] words per cell (read R, I, V and write R, I once per pass; a
    half-step reads its stencil array, the updated array and V and writes
    the updated array)."""
    for k in bench.WORDS:
        assert bench.WORDS[k] / bench.STEPS_PER_LAUNCH[k] == bench.WORDS_PER_CELL_STEP[k]
    assert bench.WORDS_PER_CELL_STEP["two_step"] * 4 == 10.0   # 10 B per FP32 cell-step
    assert bench.WORDS_PER_CELL_STEP["fused"] * 8 == 40.0      # 40 B per FP64 cell-step


def test_roofline_of_the_dominant_kind():
    cells = 512 * 512 * 1024
    # 100 two-step launches of 1.2 ms, 4 recording ones, one odd one-pass step
    kt = {"half_i": (0.0, 0), "half_r": (0.0, 0), "fused": (1.05, 1), "two_step": (120.0, 100),
          "half_i_rec": (0.0, 0), "half_r_rec": (0.0, 0), "fused_rec": (0.0, 0),
          "two_step_rec": (5.0, 4)}
    r = bench.roofline_of(kt, cells, "f32", "no-such-workload", HEADLINE_TILE)
    assert r["kernel"] == bench.KERNEL_NAMES["two_step"]
    assert r["avg_launch_ms"] == pytest.approx(1.2)
    assert r["alg_bytes_per_launch"] == 5 * 4 * cells
    assert r["achieved"] == pytest.approx(20 * cells / 1.2e-3 / 1e9, abs=0.1)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["record_launch_avg_ms"] == pytest.approx(1.25)
    assert r["traffic"] is None   # no committed counters for this workload
    r64 = bench.roofline_of(kt, cells, "f64", "no-such-workload", HEADLINE_TILE)
    assert r64["alg_bytes_per_launch"] == 2 * r["alg_bytes_per_launch"]


def test_traffic_only_for_the_kernel_and_tile_the_counters_were_taken_with():
    path = os.path.join(ROOT, "profiles", "two_step_surface-512x512x1024_f32_traffic.json")
    with open(path) as f:
        t = json.load(f)
    tile = t["tile"]   # the tile the counters were taken with
    got = bench.traffic_from_profiles("surface-512x512x1024", "f32", "two_step", tile)
    if t["kernel_src_sha"] == bench.kernel_src_sha():
        assert got == pytest.approx(t["hbm_bytes_per_launch"])
        # the summary's own arithmetic: scaled counters over the algorithmic bytes
        fb = t["fetch_kib_per_launch_raw"] * 1024 * t["scale_fetch"]
        wb = t["write_kib_per_launch_raw"] * 1024 * t["scale_write"]
        assert fb + wb == pytest.approx(t["hbm_bytes_per_launch"])
        assert (fb + wb) / t["alg_bytes_per_launch"] == pytest.approx(t["traffic_over_alg"])
    else:
        assert got is None
    other = dict(tile, two_step_zc=tile["two_step_zc"] + 8)
    assert bench.traffic_from_profiles("surface-512x512x1024", "f32", "two_step", other) is None
    assert bench.traffic_from_profiles("surface-512x512x1024", "f32", "fused", tile) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
