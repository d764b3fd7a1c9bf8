"""Write the oracle regression fixtures in this folder.

Calls only the CPU oracle and the seeded generators:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2601_14414_amd import workloads as W  # noqa: E402


def main():
    out = {"description": "CPU FP64 oracle, 4-mass chain (nx=8, nu=3), N=20, rho=1, "
                          "200 plain ADMM iterations from a cold start; u0 = du_0 of the "
                          "last step 1 (Algorithm 1 output), residuals of the last iteration.",
           "cases": []}
    for seed in range(3):
        p = W.plain_fp64_problem(seed)
        r = oracle.solve(p)
        c, rp, rd, _ = r["hist"][-1]
        out["cases"].append(dict(seed=seed, u0=r["u0"].tolist(), c=c, r_prim=rp, r_dual=rd,
                                 z1=r["state"][1][0].tolist()))
    with open(os.path.join(HERE, "plain_fp64_k200.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
