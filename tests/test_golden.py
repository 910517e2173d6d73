"""The oracle still reproduces its stored record of the 160x120 workload
(written by tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_its_stored_record(orc):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    got = mg.record()
    want = json.load(open(os.path.join(HERE, "golden", "c1_oracle_record.json")))
    assert got["n_planes"] == want["n_planes"]
    assert got["inliers"] == want["inliers"] and got["jstar"] == want["jstar"]
    assert got["label_counts"] == want["label_counts"]
    assert got["n_normal_valid"] == want["n_normal_valid"]
    assert np.allclose(got["planes"], want["planes"], rtol=0, atol=1e-12)
    assert abs(got["depth_sum_mm"] - want["depth_sum_mm"]) <= 1e-9 * want["depth_sum_mm"]
    assert abs(got["depth_checksum"] - want["depth_checksum"]) <= 1e-6 * abs(want["depth_checksum"])
    assert got["residuals"] == want["residuals"]
