"""The oracle still reproduces its stored trajectory summary (regression guard)."""
import json
import os

import numpy as np

from tests.golden.make_golden import trajectory_summary

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_matches_stored_64x64_k16_trajectory():
    with open(os.path.join(HERE, "ocsc_64x64_k16_f64_first5.json")) as fh:
        want = json.load(fh)
    got = trajectory_summary(want["workload"], len(want["steps"]))
    assert got["order"] == want["order"]
    for g, w in zip(got["steps"], want["steps"]):
        assert g["codes_nnz"] == w["codes_nnz"]
        for key in ("objective", "codes_l1", "dict_fro", "dict_sum"):
            assert np.isclose(g[key], w[key], rtol=1e-11, atol=1e-12), key
