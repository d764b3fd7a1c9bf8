"""The output form of eqn. (1) (output matrix C, output weight and
reference, output bounds, input reference) through the C ABI, on the
AFTI-16 aircraft of Section V-A with its input-rate weight W_du: an open-loop
unstable, ill-conditioned case (W_y = 100 against W_du = 0.1) -- against the
oracle fed the same Problem."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

import _refs
from test_gpu_lane import TOL32, TOL64, check_info, compare, scaled_err

pytestmark = pytest.mark.gpu


def _mixed(seed, N):
    rng = np.random.default_rng(seed)
    A, B = W.mass_spring(2)
    C = rng.standard_normal((3, 4))
    return W.Problem(nx=4, nu=1, N=N, A=A, B=B, Q=0.05 * np.eye(4), R=0.1 * np.eye(1),
                     xmin=np.full(4, -3.0), xmax=np.full(4, 3.0), umin=np.full(1, -0.3), umax=np.full(1, 0.3),
                     x0=rng.uniform(-1, 1, 4), u_prev=np.zeros(1), rho=1.0, K=200, C=C,
                     Wy=np.diag(rng.uniform(0.5, 2.0, 3)), ry=rng.uniform(-0.5, 0.5, 3), ru=np.array([0.1]))


@pytest.mark.parametrize("N", [5, 40])
def test_afti16_fp64_parity(N):
    """Fixed K, FP64 lane family: every iterate to rounding order."""
    p = W.afti16_problem(N=N, K=400, rho=10.0)
    s = P.Solver([p], rho=p.rho, max_iter=p.K, precision=P.PIMPC_FP64)
    u0, info = s.solve()
    ref = oracle.solve(p)
    compare(s, [p], [ref], TOL64)
    assert scaled_err(u0, ref["u0"]) <= TOL64
    check_info(info, [ref], 1e-9)
    s.close()


@pytest.mark.parametrize("N,family", [(40, P.PIMPC_FAMILY_LANE), (600, P.PIMPC_FAMILY_ROW)])
def test_afti16_fp32_parity(N, family):
    """Fixed K in FP32 (lane family, and the row family on a long horizon):
    every iterate within the FP32 tolerance of the FP64 oracle."""
    p = W.afti16_problem(N=N, K=400, rho=10.0)
    s = P.Solver([p], rho=p.rho, max_iter=p.K, precision=P.PIMPC_FP32, family=family)
    u0, info = s.solve()
    ref = oracle.solve(p)
    its = {w: s.iterate(w)[0] for w in range(7)}
    refs = [ref["state"][w] for w in range(5)] + [ref["du"], ref["xs"]]
    errs = [scaled_err(its[w], refs[w]) for w in range(7)]
    print(f"AFTI-16 N={N} FP32 scaled iterate errors: {['%.1e' % e for e in errs]}")
    assert max(errs) <= TOL32
    assert scaled_err(u0, ref["u0"]) <= TOL32
    s.close()


def test_general_output_matrix_fp64():
    """Outputs mixing states (no bounds on them), output and input references:
    FP64 parity on a batch of two horizons."""
    problems = [_mixed(0, 8), _mixed(1, 70)]
    s = P.Solver(problems, rho=1.0, max_iter=200, precision=P.PIMPC_FP64)
    u0, info = s.solve()
    refs = [oracle.solve(p) for p in problems]
    compare(s, problems, refs, TOL64)
    s.close()


def test_afti16_converged_fp32_limit_and_fp64():
    """Converged mode on the ill-conditioned case (N = 30, rho = 100; the FP64
    oracle needs about 135 000 iterations to c <= 1e-20).  FP32 iteration
    stops improving at c of a few 1e-6 here (W_y = 100 against W_du = 0.1
    puts the dual residual's scale far above the primal one): it reaches
    c <= 1e-5 and r_prim <= 1e-4, but r_dual stays near 2e-2 and the input
    trajectory within 2e-2 (scaled by the 25-degree input range) of the
    optimum.  FP64 iteration on the same case (lane family) meets the
    residual target and matches the interior-point optimum to 1e-6."""
    p = W.afti16_problem(N=30, K=0, rho=100.0)
    ip = _refs.ipm_qp(p)
    assert ip["ok"]
    s = P.Solver([p], rho=p.rho, max_iter=1000000, eps=1e-5, check_every=10, precision=P.PIMPC_FP32)
    _, info = s.solve()
    u = s.iterate(P.IT_XBAR)[0][:, p.nx:]
    err32 = float(np.max(np.abs(u - ip["us"]))) / 25.0
    print(f"AFTI-16 N=30 FP32: {info['iters'][0]} iterations, c = {info['c'][0]:.2e}, "
          f"r_prim = {info['r_prim'][0]:.2e}, r_dual = {info['r_dual'][0]:.2e}, input error / 25 = {err32:.2e}")
    assert info["status"][0] == 0 and info["c"][0] <= 1e-5 and info["r_prim"][0] <= 1e-4
    assert info["r_dual"][0] <= 5e-2 and err32 <= 2e-2
    s.close()
    s = P.Solver([p], rho=p.rho, max_iter=1000000, eps=1e-16, check_every=10, precision=P.PIMPC_FP64)
    _, info = s.solve()
    u = s.iterate(P.IT_XBAR)[0][:, p.nx:]
    err64 = float(np.max(np.abs(u - ip["us"]))) / 25.0
    print(f"AFTI-16 N=30 FP64: {info['iters'][0]} iterations, c = {info['c'][0]:.2e}, "
          f"r_prim = {info['r_prim'][0]:.2e}, r_dual = {info['r_dual'][0]:.2e}, input error / 25 = {err64:.2e}")
    assert info["status"][0] == 0 and info["c"][0] <= 1e-16
    assert info["r_prim"][0] <= 1e-4 and info["r_dual"][0] <= 1e-4 and err64 <= 1e-6
    s.close()
