"""Host logic of bench.py that needs no GPU: the one-GPU guard, the algorithmic
flop count of a K_hat V product, and the roofline record built from a launch time
and the stored counter readings (reported only while they describe the current
kernel sources and grid, weighted by the launch mix of one evaluation)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_tile_flops_count_the_distance_the_product_and_the_map():
    # 2 n^2 (d + t) + n^2 at the bench shape (n = 100,000, d = 16, t = 65)
    assert bench.tile_flops(100000, 16, 65) == pytest.approx(1.63e12, rel=1e-12)
    assert bench.tile_flops(10, 1, 1) == 2 * 100 * 2 + 100


def test_launch_mix_follows_the_three_piece_iterations():
    assert bench.tile_launch_mix("bf16x3", 32) == {"v3": 16, "v2": 16}
    assert bench.tile_launch_mix("bf16x3", 10) == {"v3": 10, "v2": 0}
    assert bench.tile_launch_mix("fp16x3", 32) == {"v2": 32}


def _run(ms, reps=32, grid=(391, 5)):
    return {"tile_ms": ms, "tile_grid": list(grid), "tile_launches_timed": reps}


def test_roofline_fraction_and_mix_weighted_counters():
    tc = bench.TILE_COUNTERS["bf16x3"]
    roof = bench.tile_roofline(100000, 16, 65, _run(5.0), "bf16x3")
    assert roof["bound"] == "mfma" and roof["peak"] == 2500.0
    assert roof["achieved"] == pytest.approx(1.63e12 / 5e-3 / 1e12)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 2500.0)
    if bench.bf16_tile_source_hash() != tc["kernel_source_sha256_16"]:
        assert roof["traffic"] is None
        return
    def bytes_of(r):
        return 1024.0 * (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"])
    assert roof["traffic"] == pytest.approx(0.5 * bytes_of(tc["v3"]) + 0.5 * bytes_of(tc["v2"]))
    issued = 0.5 * (tc["v3"]["mfma_insts"] + tc["v2"]["mfma_insts"]) * 16384.0
    assert roof["issued_mfma_flops_per_launch"] == pytest.approx(issued)


def test_stale_counters_are_not_reported():
    # another grid, another size, or a mix that needs an instance without readings
    assert bench.tile_roofline(100000, 16, 65, _run(5.0, grid=(391, 6)), "bf16x3")["traffic"] is None
    assert bench.tile_roofline(50000, 16, 65, _run(5.0), "bf16x3")["traffic"] is None
    assert bench.tile_roofline(100000, 16, 65, _run(5.0, reps=0), "bf16x3")["traffic"] is None
    saved = dict(bench.TILE_COUNTERS["bf16x3"])
    try:
        bench.TILE_COUNTERS["bf16x3"].pop("v3")
        assert bench.tile_roofline(100000, 16, 65, _run(5.0), "bf16x3")["traffic"] is None
        bench.TILE_COUNTERS["bf16x3"]["v3"] = saved["v3"]
        bench.TILE_COUNTERS["bf16x3"]["kernel_source_sha256_16"] = "0" * 16
        assert bench.tile_roofline(100000, 16, 65, _run(5.0), "bf16x3")["traffic"] is None
    finally:
        bench.TILE_COUNTERS["bf16x3"].clear()
        bench.TILE_COUNTERS["bf16x3"].update(saved)


def test_tile_source_hash_covers_the_tile_kernels_but_not_the_staging_section():
    khat = open(os.path.join(ROOT, "paper_2107_00243_amd", "csrc", "k_khat.hip")).read()
    kept = bench.tile_source_text(khat)
    # the part-0 sections (staging, split-K reduction) are gone, the tile kernels stay
    assert "#if GPMLL_KHAT_PART == 0" in khat and "#if GPMLL_KHAT_PART == 0" not in kept
    assert "k_khat_reduce(" in khat and "k_khat_reduce(" not in kept
    assert "void k_khat_bf16(" in kept and "void k_khat_fp(" in kept
    # an edit inside a part-0 section leaves the text unchanged, one in the tile kernel does not
    i = khat.index("#if GPMLL_KHAT_PART == 0\n") + len("#if GPMLL_KHAT_PART == 0\n")
    assert bench.tile_source_text(khat[:i] + "// edit\n" + khat[i:]) == kept
    j = khat.index("void k_khat_bf16(")
    assert bench.tile_source_text(khat[:j] + "// edit\n" + khat[j:]) != kept
