"""The oracle still produces the stored fixture (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

import oracle
from paper_2601_14414_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "plain_fp64_k200.json")


def test_oracle_matches_stored_fixture():
    d = json.load(open(GOLD))
    for case in d["cases"]:
        r = oracle.solve(W.plain_fp64_problem(case["seed"]))
        np.testing.assert_allclose(r["u0"], case["u0"], rtol=0, atol=1e-13)
        np.testing.assert_allclose(r["state"][1][0], case["z1"], rtol=0, atol=1e-13)
        c, rp, rd, _ = r["hist"][-1]
        assert abs(c - case["c"]) <= 1e-12 * max(1, abs(case["c"]))
        assert abs(rp - case["r_prim"]) <= 1e-13 and abs(rd - case["r_dual"]) <= 1e-13
