"""GPU parity of the row-per-lane (long horizon) path against the oracle.

FP32 iteration vs FP64 oracle, tolerance 1e-4 of max(1, |oracle|_inf)
(see test_gpu_lane.py for the derivation)."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

from test_gpu_lane import TOL32, check_info, compare, scaled_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,K", [(1, 30), (7, 40), (64, 60), (257, 80)])
def test_row_small_horizons(N, K):
    """12-mass chain (nx=24, nu=11) on short horizons, incl. a partial last
    block and a single stage."""
    p = W.long_horizon_problem(seed=N, N=N, K=K)
    s = P.Solver([p], max_iter=K, precision=P.PIMPC_FP32)
    u0, info = s.solve()
    ref = oracle.solve(p, K=K)
    compare(s, [p], [ref], TOL32)
    assert scaled_err(u0, ref["u0"]) <= TOL32
    check_info(info, [ref], 1e-4)


def test_row_long_horizon_full():
    """The full long-horizon workload: N=1024, 500 iterations, x0 ~ U[-2,2]."""
    p = W.long_horizon_problem(seed=0)
    s = P.Solver([p], max_iter=p.K, precision=P.PIMPC_FP32)
    u0, info = s.solve()
    ref = oracle.solve(p)
    compare(s, [p], [ref], TOL32)
    check_info(info, [ref], 1e-4)
    # some input bounds are active at this point of the iteration
    z = s.state(0)[1]
    assert np.sum(np.isclose(np.abs(z[:, 24:]), 0.5)) > 10


def test_row_eps_stop_and_warm_start():
    p = W.long_horizon_problem(seed=3, N=96, K=2000)
    s = P.Solver([p], max_iter=2000, eps=1e-5, check_every=1, precision=P.PIMPC_FP32)
    _, info = s.solve()
    ref = oracle.solve(p, K=2000, eps=1e-5)
    assert abs(int(info["iters"][0]) - ref["iters"]) <= 2  # FP32 c vs FP64 c near the threshold
    s2 = P.Solver([p], max_iter=50, precision=P.PIMPC_FP32, warm_start=True)
    s2.solve()
    s2.solve()
    compare(s2, [p], [oracle.solve(p, K=100)], TOL32)


def test_several_row_instances_with_lane_instances():
    """A batch holding two full-size long horizons (the row family, each grid
    filling the GPU, run one after the other) and lane-family instances on
    the other streams: every instance against the oracle."""
    problems = [W.long_horizon_problem(seed=1, N=1024, K=40), W.long_horizon_problem(seed=2, N=900, K=40)]
    problems += [W.random_batch_instance(seed=2000 + i, K=40) for i in range(6)]
    # schedule 1: counter-claimed bins on four streams (a batch this small
    # would otherwise be tuned onto one stream)
    s = P.Solver(problems, max_iter=40, precision=P.PIMPC_FP32, schedule=1)
    u0, info = s.solve()
    refs = [oracle.solve(p, K=40) for p in problems]
    compare(s, problems, refs, TOL32)
    check_info(info, refs, 1e-4)
    s.close()
