"""Host-side parts of the benchmark's contract, on the CPU: more than one GPU
is refused before any GPU is touched, the kernel-source hash that ties the
stored HBM-traffic figures to the code ignores comments and white space but
not code, and stored traffic is reported only for the matching hash."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KERNELS = os.path.join("paper_2411_01919_amd", "csrc", "pp_kernels.hip")


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def _tree(tmp_path, text):
    d = tmp_path / os.path.dirname(KERNELS)
    d.mkdir(parents=True, exist_ok=True)
    (tmp_path / KERNELS).write_text(text, encoding="utf-8")
    return str(tmp_path)


def test_source_hash_ignores_comments_and_white_space_only(tmp_path, monkeypatch):
    src = open(os.path.join(ROOT, KERNELS), encoding="utf-8").read()
    base = bench.source_hash()
    monkeypatch.setattr(bench, "ROOT", _tree(tmp_path / "a", "// a new comment\n" + src.replace("\n", "\n\n  ")
                                             + "\n/* block\n comment */\n"))
    assert bench.source_hash() == base
    monkeypatch.setattr(bench, "ROOT", _tree(tmp_path / "b", src.replace("kFinalBlocks = 2048", "kFinalBlocks = 1024")))
    assert bench.source_hash() != base


def test_stored_traffic_only_for_its_own_kernel_source(tmp_path, monkeypatch):
    stored = json.load(open(os.path.join(ROOT, "profiles", "score_traffic.json")))
    h = stored["kernel_source_hash"]
    assert bench.load_traffic(h) == stored["bytes_per_launch"] > 0
    assert bench.load_traffic("0" * 16) is None
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))  # no profiles at all
    assert bench.load_traffic(h) is None
    (tmp_path / "profiles").mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", "score_traffic.json"), tmp_path / "profiles")
    assert bench.load_traffic(h) == stored["bytes_per_launch"]


def test_hbm_fractions_by_algorithmic_and_counted_bytes():
    """The per-stage HBM rates of the bench line: bytes per pixel times pixels
    over the stage time, against 8 TB/s, with the 60 % flags per stage."""
    n_px = 1_000_000
    stage = {"diffusion": 0.02, "normals": 0.01}  # ms
    counted = {"diffusion_bytes_per_px": 80.0, "normals_and_valid_list_bytes_per_px": 50.0}
    out = bench.hbm_fractions(stage, n_px, 20, 4, 0.9, counted)
    d, n = out["diffusion"], out["normals_and_valid_list"]
    # 80 B x 1e6 px in 20 us = 4 TB/s (50 %); 50 B x 1e6 px in 10 us = 5 TB/s (62.5 %)
    assert d["counter_gb_per_s"] == 4000.0 and d["counter_frac_of_8tbs"] == 0.5
    assert n["counter_gb_per_s"] == 5000.0 and n["counter_frac_of_8tbs"] == 0.625
    assert out["counter_target_met_by_stage"] == {"diffusion": False, "normals_and_valid_list": True}
    assert out["counter_target_met"] is False
    assert abs(d["gb_per_s"] - d["bytes_per_px"] * n_px / 0.02e-3 / 1e9) < 0.1
    plain = bench.hbm_fractions(stage, n_px, 20, 4, 0.9)
    assert plain["counter_target_met"] is None and plain["counter_target_met_by_stage"] is None
    assert "counter_frac_of_8tbs" not in plain["diffusion"]
