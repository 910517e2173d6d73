"""Writes the stored oracle record for the 160x120 two-step workload.

Calls only ``oracle`` and the seeded scene generator; run from the repository
root with ``python tests/golden/make_golden.py``.  The record pins the oracle
against unintended changes of its arithmetic: a change to the oracle that
moves these numbers must name the passage of the paper that justifies it.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import scenes  # noqa: E402


def record():
    cfg = scenes.CONFIGS[1]
    f = scenes.make_frame(1, 0)
    W, H = cfg.sizes[0]
    prm = oracle.RansacParams(hyps=cfg.hyps, max_planes=cfg.max_planes, min_inliers=cfg.min_inliers(W, H),
                              thresh=cfg.thresh_m, seed=cfg.ransac_seed, frame=0)
    res = oracle.pipeline(f.depth, f.K, cfg.diffuse_iters, cfg.lam, cfg.kappa_mm, prm)
    rr = res.ransac
    return {
        "workload": "160x120 two-step stair, frame 0, 10 iterations, 256 hypotheses, t = 10 mm",
        "depth_sum_mm": float(res.depth.sum()),
        "depth_checksum": float((res.depth * np.arange(res.depth.size).reshape(res.depth.shape) % 977).sum()),
        "n_normal_valid": int(res.nvalid.sum()),
        "n_planes": rr.n_planes,
        "planes": rr.planes.tolist(),
        "inliers": rr.inliers.tolist(),
        "jstar": rr.jstar.tolist(),
        "label_counts": np.bincount(rr.labels.reshape(-1).astype(int) + 1).tolist(),
        "residuals": rr.residuals,
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "c1_oracle_record.json")
    with open(out, "w") as fh:
        json.dump(record(), fh, indent=1)
    print("wrote", out)
