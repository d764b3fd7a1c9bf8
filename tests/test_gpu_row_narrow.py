"""Row family with narrow stages packed side by side in a wave (padded
classes 4+4: eight stages per wave, and 8+8: four stages per wave); the
cases from (30, 14) on are the wide classes: 32+16 (one stage per wave),
24+12 with two stages per wave (N = 1500 does not fit one stage per wave), and
24+12 with one stage per wave, where the last stage's wave holds the rows of
a non-diagonal H_{N-1} (dense Q and R) in registers, and 24+12 with four
stages per wave up to the longest horizon whose grid is co-resident on a
256-CU part (N = 4096).  Horizons
beyond one lane-family workgroup (N > 512) with small stages land here.

FP32 iteration vs the FP64 oracle, tolerance 1e-4 of max(1, |oracle|_inf)
(derivation in test_gpu_lane.py).  The horizons are chosen so that the last
wave holds a partial set of stage groups and the last workgroup a partial set
of waves."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P

from test_gpu_lane import TOL32, check_info, compare, scaled_err, tiny_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,N,K", [(3, 2, 513, 60), (4, 4, 700, 80), (2, 1, 1029, 60),
                                     (6, 3, 600, 60), (8, 8, 2053, 40), (5, 1, 777, 50),
                                     (30, 14, 600, 30), (20, 10, 1500, 30),
                                     (12, 8, 600, 40), (24, 11, 530, 30),
                                     (24, 11, 3000, 12), (24, 11, 4096, 8)])
def test_narrow_row_parity(n, m, N, K):
    """Affine stage data, linear term, dense Q and R, u_prev != 0."""
    p = tiny_problem(N + n, n, m, N, 0)
    s = P.Solver([p], rho=p.rho, max_iter=K, precision=P.PIMPC_FP32)
    u0, info = s.solve()
    ref = oracle.solve(p, K=K)
    compare(s, [p], [ref], TOL32)
    assert scaled_err(u0, ref["u0"]) <= TOL32
    check_info(info, [ref], 1e-4)
    s.close()


@pytest.mark.parametrize("n,m,N", [(3, 1, 900), (7, 2, 1100)])
def test_narrow_row_eps_stop_and_warm_start(n, m, N):
    """Residuals on every iteration (the dual residual takes dd of the next
    stage from the next group of lanes, the next wave or the next workgroup),
    the eps stop, and a warm-started continuation."""
    p = tiny_problem(N, n, m, N, 0, dense_q=False)
    eps = 1e-6
    s = P.Solver([p], rho=p.rho, max_iter=3000, eps=eps, check_every=1, precision=P.PIMPC_FP32)
    _, info = s.solve()
    ref = oracle.solve(p, K=3000, eps=eps)
    assert ref["iters"] < 3000
    assert abs(int(info["iters"][0]) - ref["iters"]) <= max(3, ref["iters"] // 50)
    s.close()
    K1 = 40
    r40 = oracle.solve(p, K=K1)
    s1 = P.Solver([p], rho=p.rho, max_iter=K1, precision=P.PIMPC_FP32)
    _, info1 = s1.solve()
    c, rp, rd, _ = r40["hist"][-1]
    assert abs(info1["r_prim"][0] - rp) <= 1e-4 and abs(info1["r_dual"][0] - rd) <= 1e-4
    assert abs(info1["c"][0] - c) <= 1e-4 * max(1.0, c)
    s1.close()
    s2 = P.Solver([p], rho=p.rho, max_iter=20, precision=P.PIMPC_FP32, warm_start=True)
    s2.solve()
    s2.solve()
    compare(s2, [p], [oracle.solve(p, K=40)], TOL32)
    s2.close()


def test_horizon_beyond_one_resident_grid_is_unsupported():
    """A horizon that no co-resident row grid holds is refused at setup with
    PIMPC_E_UNSUPPORTED (no kernel runs)."""
    p = tiny_problem(7, 24, 11, 20000, 0)
    with pytest.raises(P.PimpcError) as ei:
        P.Solver([p], rho=p.rho, max_iter=5, precision=P.PIMPC_FP32)
    assert ei.value.code == P.PIMPC_E_UNSUPPORTED
