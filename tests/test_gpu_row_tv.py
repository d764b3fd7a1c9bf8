"""Row family with time-varying stage data (long horizons of re-linearised
models): each wave (or group of lanes) holds its own stage's fused matrices
and rows, read once per solve from the stage-minor layout.  FP32 against the
FP64 oracle, tolerance 1e-4 of max(1, |oracle|_inf) (derivation in
test_gpu_lane.py); the residual levels (whose dual part uses the stage's own
Bbar and the next stage's Abar) to 1e-4 absolute."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P

from test_gpu_lane import TOL32, check_info, compare, scaled_err, tiny_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,N,K", [(3, 2, 700, 60), (2, 1, 1029, 50), (6, 3, 600, 60), (20, 6, 520, 40)])
def test_row_time_varying_parity(n, m, N, K):
    """Narrow (4+4, 8+8: stages packed per wave) and wide (24+12) classes,
    affine time-varying stage data, linear term, dense Q and R, u_prev != 0.
    (The 32+16 class has no time-varying variant: its second column set
    would exceed the workgroup's LDS; pimpc_setup reports that.)"""
    p = tiny_problem(7 * N + n, n, m, N, 1)
    s = P.Solver([p], rho=p.rho, max_iter=K, precision=P.PIMPC_FP32)
    u0, info = s.solve()
    ref = oracle.solve(p, K=K)
    compare(s, [p], [ref], TOL32)
    assert scaled_err(u0, ref["u0"]) <= TOL32
    check_info(info, [ref], 1e-4)
    s.close()


def test_row_time_varying_linearize_and_warm_start():
    """pimpc_linearize replaces the stage data of a long time-varying horizon
    (the fused blocks are rebuilt per stage); the warm-started solve after it
    equals the oracle continuing from the same iterate with the new data."""
    p = tiny_problem(11, 3, 1, 800, 1)
    q = tiny_problem(12, 3, 1, 800, 1)
    q = q.copy(Q=p.Q, R=p.R, qbar=p.qbar, x0=p.x0, u_prev=p.u_prev)
    s = P.Solver([p], rho=p.rho, max_iter=30, precision=P.PIMPC_FP32, warm_start=True)
    s.solve()
    st = oracle.solve(p, K=30)["state"]
    s.linearize(q.A.ravel(), q.B.ravel(), q.e.ravel())
    u0, info = s.solve()
    ref = oracle.solve(q, K=30, state=st)
    compare(s, [q], [ref], TOL32)
    s.close()
