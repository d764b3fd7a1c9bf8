"""Non-box constraint sets on the row family (a stage's entries spread over
the lanes of its group, so each projection reduces across those lanes):
FP32 parity against the oracle, tolerances as in test_gpu_lane.py, on the
packed narrow classes (8 and 4 stages per wave), the wide class (one stage
per wave), time-varying data and with restart acceleration."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

from test_gpu_lane import TOL32, check_info, compare, scaled_err, tiny_problem
from test_gpu_row_accel import decision_margin

pytestmark = pytest.mark.gpu

SETS = {
    "u_l1": lambda n, m: (None, ("l1ball", 0.3 * m)),
    "u_soc": lambda n, m: (None, ("soc",)),
    "u_half": lambda n, m: (None, ("halfspace", np.linspace(1.0, -0.5, m), 0.1)),
    "x_half": lambda n, m: (("halfspace", np.linspace(-1.0, 1.0, n) + 0.2, -0.3), None),
    "x_hyper_u_l1": lambda n, m: (("hyperplane", np.r_[1.0, 1.0, np.zeros(n - 2)], 0.05), ("l1ball", 0.5)),
    "x_soc": lambda n, m: (("soc",), None),
    "x_l1": lambda n, m: (("l1ball", 1.0), None),
}
# (nx, nu, N): padded 4+4 (8 stages per wave), 8+8 (4 per wave), 24+12 (one per wave)
SHAPES = [(3, 2, 700), (5, 3, 600), (20, 6, 530)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}_N{s[2]}")
@pytest.mark.parametrize("kind", sorted(SETS))
def test_row_sets_fp32(kind, shape):
    n, m, N = shape
    xset, uset = SETS[kind](n, m)
    p = tiny_problem(7 * n + m + len(kind), n, m, N, 0).copy(xset=xset, uset=uset)
    K = 60
    s = P.Solver([p], rho=p.rho, max_iter=K, precision=P.PIMPC_FP32, family=P.PIMPC_FAMILY_ROW)
    u0, info = s.solve()
    ref = oracle.solve(p, K=K)
    compare(s, [p], [ref], TOL32)
    assert scaled_err(u0, ref["u0"]) <= TOL32
    check_info(info, [ref], 1e-4)
    # the set is active: the box-only run differs
    r0 = oracle.solve(p.copy(xset=None, uset=None), K=K)
    assert np.max(np.abs(r0["state"][1] - ref["state"][1])) > 1e-3
    s.close()


def test_row_sets_time_varying_fp32():
    p = tiny_problem(31, 4, 2, 640, 1).copy(uset=("soc",), xset=("l1ball", 0.9))
    s = P.Solver([p], rho=p.rho, max_iter=60, precision=P.PIMPC_FP32, family=P.PIMPC_FAMILY_ROW)
    u0, info = s.solve()
    ref = oracle.solve(p, K=60)
    compare(s, [p], [ref], TOL32)
    check_info(info, [ref], 1e-4)
    s.close()


def test_row_sets_with_restart_acceleration_fp32():
    """Acceleration and a non-box set together on a long wide horizon, with
    an eta whose decisions FP32 and FP64 agree on (see test_gpu_row_accel.py)."""
    p = W.long_horizon_problem(seed=5, N=300, K=120).copy(uset=("l1ball", 2.0))
    eta, K = 0.8, 120
    ref = oracle.solve(p, K=K, accel=True, eta=eta)
    assert decision_margin(ref["hist"], eta) >= 5e-3 and ref["hist"][-1][0] >= 1e-6
    s = P.Solver([p], max_iter=K, precision=P.PIMPC_FP32, accel=True, eta=eta, family=P.PIMPC_FAMILY_ROW)
    u0, info = s.solve()
    assert info["restarts"][0] == int(ref["hist"][:, 3].sum())
    compare(s, [p], [ref], TOL32)
    s.close()
