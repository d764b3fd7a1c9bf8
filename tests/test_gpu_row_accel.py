"""Restart acceleration (Algorithm 1 steps 6-7) on the row family (long
horizons: a reducer wave per workgroup gathers c^{i+1} of the whole horizon
every iteration and takes the same decision in every workgroup).

Fixed-K parity: the decision c^{i+1} <= eta c^i is a comparison of two
residual levels, which FP32 and FP64 agree on only when the ratio c^{i+1}/c^i
is not within rounding of eta.  Each fixed-K case therefore uses an eta for
which every ratio of the oracle's run stays at least 0.5 % away from eta
(checked here on the oracle's history); then both sides take the same
decisions, and every iterate, du, xbar, the iteration count and the restart
count must match to the FP32 tolerance.  Converged mode compares solutions,
as for the lane family."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

from test_gpu_lane import TOL32, compare, scaled_err, tiny_problem

pytestmark = pytest.mark.gpu


def decision_margin(hist, eta):
    """Smallest relative distance of c^{i+1}/c_prev from eta over the run
    (c_prev = 1 before the first decision, c^i after)."""
    c = hist[:, 0]
    ratio = np.concatenate([[c[0]], c[1:] / c[:-1]])
    return float(np.min(np.abs(ratio - eta)) / eta)


# (problem, eta, K); K keeps c^{K} >= 1e-6, where FP32 still resolves the
# iterate differences c is made of (the packed case converges fast)
CASES = {
    "chain24_N300": (lambda: W.long_horizon_problem(seed=5, N=300, K=150), 0.8, 150),
    "chain24_N1024": (lambda: W.long_horizon_problem(seed=0, N=1024, K=150), 0.8, 150),
    "packed3x2_N700": (lambda: tiny_problem(11, 3, 2, 700, 0), 0.8, 45),
    "tv4x1_N600": (lambda: tiny_problem(16, 4, 1, 600, 1), 0.9, 150),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_row_accel_fixed_k_parity(name):
    make, eta, K = CASES[name]
    p = make()
    ref = oracle.solve(p, K=K, accel=True, eta=eta)
    assert decision_margin(ref["hist"], eta) >= 5e-3
    assert ref["hist"][-1][0] >= 1e-6
    restarts = int(ref["hist"][:, 3].sum())
    assert 3 <= restarts <= K - 3  # both branches of step 6 are taken
    s = P.Solver([p], rho=p.rho, max_iter=K, precision=P.PIMPC_FP32, accel=True, eta=eta,
                 family=P.PIMPC_FAMILY_ROW)
    u0, info = s.solve()
    assert info["status"][0] == 0 and info["iters"][0] == K
    assert info["restarts"][0] == restarts
    compare(s, [p], [ref], TOL32)
    assert scaled_err(u0, ref["u0"]) <= TOL32
    c, rp, rd, _ = ref["hist"][-1]
    assert abs(info["c"][0] - c) <= 1e-4 * max(1.0, c)
    assert abs(info["r_prim"][0] - rp) <= 1e-4 and abs(info["r_dual"][0] - rd) <= 1e-4
    s.close()


def test_row_accel_eps_stop():
    """Step 5 is tested on every iteration before steps 6-7: the stop
    iteration, the restarts up to it and the final iterate match."""
    p = tiny_problem(11, 3, 2, 700, 0)
    eta, eps = 0.8, 1e-5
    ref = oracle.solve(p, K=5000, eps=eps, accel=True, eta=eta)
    assert ref["iters"] < 5000
    assert decision_margin(ref["hist"], eta) >= 5e-3
    c = ref["hist"][:, 0]
    assert abs(c[-1] - eps) / eps > 0.05 and abs(c[-2] - eps) / eps > 0.05  # the stop is not a near tie
    s = P.Solver([p], rho=p.rho, max_iter=5000, eps=eps, precision=P.PIMPC_FP32, accel=True, eta=eta,
                 family=P.PIMPC_FAMILY_ROW)
    u0, info = s.solve()
    assert info["iters"][0] == ref["iters"]
    assert info["restarts"][0] == int(ref["hist"][:, 3].sum())
    assert info["c"][0] <= eps
    compare(s, [p], [ref], TOL32)
    s.close()


def test_row_accel_fp32_converged():
    """Default eta = 0.999, run to c <= 1e-9: u0 and z within 1.5e-3 of the
    oracle's accelerated solution at c <= 1e-13 (the tolerance of the lane
    family's converged test, for the same reason: a flipped decision changes
    the trajectory, not the limit)."""
    p = tiny_problem(9, 3, 2, 700, 0)
    s = P.Solver([p], rho=p.rho, max_iter=40000, eps=1e-9, precision=P.PIMPC_FP32, accel=True,
                 family=P.PIMPC_FAMILY_ROW)
    u0, info = s.solve()
    ref = oracle.solve(p, K=40000, eps=1e-13, accel=True)
    assert ref["hist"][-1][0] <= 1e-13
    assert info["status"][0] == 0 and info["c"][0] <= 1e-9
    assert info["r_prim"][0] <= 1e-4 and info["r_dual"][0] <= 1e-4
    assert scaled_err(u0, ref["u0"]) <= 1.5e-3
    assert scaled_err(s.iterate(P.IT_Z)[0], ref["state"][1]) <= 1.5e-3
    s.close()


def test_row_accel_in_a_batch_with_lane_instances():
    """A long horizon (row family, accelerated) beside lane-family instances
    (accelerated per bin) in one batched solve: each against the oracle."""
    problems = [W.long_horizon_problem(seed=5, N=700, K=100)]
    problems += [W.random_batch_instance(seed=2100 + i, K=100) for i in range(5)]
    eta = 0.8
    refs = [oracle.solve(p, K=100, accel=True, eta=eta) for p in problems]
    assert decision_margin(refs[0]["hist"], eta) >= 5e-3
    s = P.Solver(problems, max_iter=100, precision=P.PIMPC_FP32, accel=True, eta=eta)
    u0, info = s.solve()
    assert np.all(info["status"] == 0)
    assert info["restarts"][0] == int(refs[0]["hist"][:, 3].sum())
    compare(s, problems[:1], refs[:1], TOL32)
    s.close()
