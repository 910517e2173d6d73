"""Autotuner of the batched path's launch shapes.

For a batch layout (the multiset of frame sizes, iterations, hypotheses and
scoring form) it times, on the device, every diffusion tile shape x temporal
depth (iterations fused per pass) and every scoring block shape
(hypotheses per block x points per block), using the library's per-stage
event timing of eager batch runs, and keeps the fastest of each.  Every
tuning computes bitwise-identical results, so the choice only moves time.
Results are cached in a JSON file keyed by device and layout
(PP_AUTOTUNE_CACHE, default ~/.cache/pp_autotune.json).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Sequence

TILES = (1, 2, 3, 4, 5, 6)           # LDS 64x16, 128x16, 64x32, 128x32; register columns of 8, 16 rows
DEPTHS = (1, 2, 3, 4, 5, 8, 10)      # iterations per diffusion pass
HB = (1, 2, 3, 4, 5, 6)              # 8, 16, 32 hypotheses per VALU scoring block; 64, 128, 256 with tile culling
CHUNKS = (1, 2, 3, 4)                # 1024 ... 8192 points per scoring block


def cache_path() -> str:
    return os.environ.get("PP_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                               "pp_autotune.json")


def layout_key(frames, device_name: str) -> str:
    sizes = sorted((int(f.depth.shape[1]), int(f.depth.shape[0])) for f in frames)
    hist: Dict[tuple, int] = {}
    for s in sizes:
        hist[s] = hist.get(s, 0) + 1
    f0 = frames[0]
    parts = [f"{w}x{h}*{n}" for (w, h), n in sorted(hist.items())]
    return (f"{device_name}|{'+'.join(parts)}|it{f0.diffuse.iters}|h{f0.ransac.hyps}|"
            f"r{f0.ransac.max_planes}|p{f0.ransac.precision}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_stage(pp, frames, ctx, stage: str, reps: int) -> float:
    import torch
    best = float("inf")
    for i in range(reps + 1):
        pp.batch_run(frames, graph=False, ctx=ctx)
        torch.cuda.current_stream().synchronize()
        if i:  # the first run warms caches and the staging ring
            best = min(best, ctx.stage_breakdown()[stage])
    return best


def tune(frames: Sequence, ctx=None, reps: int = 2, path: Optional[str] = None, force: bool = False,
         log=None) -> dict:
    """Pick and set the fastest tuning for this batch layout on ctx; returns it
    (with the measured stage times)."""
    import torch

    import paper_2411_01919_amd as pp
    ctx = ctx or pp.default_context(frames[0].depth.device.index)
    path = path or cache_path()
    key = layout_key(frames, torch.cuda.get_device_name(frames[0].depth.device))
    db = _load(path)
    if key in db and not force:
        t = db[key]
        ctx.set_tuning(t["diffuse_tile"], t["diffuse_t"], t["score_hb"], t["score_chunk"])
        return dict(t, cached=True)
    ctx.set_stage_timing(True)
    ctx.reset_tuning()
    base = ctx.get_tuning()
    diff = {}
    for tile in TILES:
        for T in DEPTHS:
            ctx.set_tuning(diffuse_tile=tile, diffuse_t=T)
            diff[(tile, T)] = _time_stage(pp, frames, ctx, "diffusion", reps)
    tile, T = min(diff, key=diff.get)
    score = {}
    hbs = HB if frames[0].ransac.precision == pp.PP_SCORE_FP32 else (4, 5, 6)
    for hb in hbs:
        for ch in CHUNKS:
            ctx.set_tuning(diffuse_tile=tile, diffuse_t=T, score_hb=hb, score_chunk=ch)
            score[(hb, ch)] = _time_stage(pp, frames, ctx, "scoring", reps)
    hb, ch = min(score, key=score.get)
    ctx.set_tuning(tile, T, hb, ch)
    ctx.set_stage_timing(False)
    t = dict(diffuse_tile=tile, diffuse_t=T, score_hb=hb, score_chunk=ch,
             diffusion_ms=round(diff[(tile, T)], 4), scoring_ms=round(score[(hb, ch)], 4),
             diffusion_default_ms=round(diff.get((base["diffuse_tile"], base["diffuse_t"]), float("nan")), 4),
             scoring_default_ms=round(score.get((base["score_hb"], base["score_chunk"]), float("nan")), 4))
    if log:
        log(f"autotune {key}: {t}")
    db[key] = t
    try:
        _save(path, db)
    except OSError:
        pass
    return dict(t, cached=False)
