"""Input-rate weight W_du (the cost term 1/2 ||u_k - u_{k-1}||^2_W of the
paper's experiments, Section V): GPU parity against the oracle.

W_du changes only the du cache of Algorithm 1, J_k = (W/rho + Bbar'Bbar)^-1
Bbar' (the oracle forms (W + rho Bbar'Bbar)^-1 rho Bbar' and is pinned to the
dense sub-problem, the KKT optimum and finite differences in
test_oracle_pins.py).  Tolerances as in test_gpu_lane.py (FP64 1e-11, FP32
1e-4 of max(1, |oracle|_inf)) and test_gpu_adjoint.py (2e-3)."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

from test_gpu_lane import TOL32, TOL64, check_info, compare, run_both, scaled_err, tiny_problem

pytestmark = pytest.mark.gpu


def rate_weight(seed, m, scale=0.3):
    rng = np.random.default_rng(70 + seed)
    Wh = rng.standard_normal((m, m))
    return scale * (Wh @ Wh.T / m + 0.1 * np.eye(m))


@pytest.mark.parametrize("seed", [0, 1])
def test_rate_weight_plain_fp64(seed):
    """4-mass chain with W_du and u_prev != 0, FP64 both sides, 200 iterations."""
    p = W.plain_fp64_problem(seed)
    p = p.copy(Wdu=rate_weight(seed, 3), u_prev=np.array([0.2, -0.1, 0.05]), rho=0.7)
    s, u0, info, refs = run_both([p], P.PIMPC_FP64)
    compare(s, [p], refs, TOL64)
    assert scaled_err(u0, refs[0]["u0"]) <= TOL64
    check_info(info, refs, 1e-10)
    # the weight changes the iterates (so the test sees it)
    r0 = oracle.solve(p.copy(Wdu=None))
    assert scaled_err(r0["u0"], refs[0]["u0"]) > 1e-3


@pytest.mark.parametrize("n,m,tv", [(3, 2, 1), (5, 3, 0), (2, 1, 1)])
def test_rate_weight_padded_time_varying_fp64(n, m, tv):
    """Padded classes, time-varying stage data (J_k per stage), mixed with an
    instance without W_du in the same batch."""
    problems = [tiny_problem(10 * n + m, n, m, N, tv) for N in (5, 70)]
    problems[0] = problems[0].copy(Wdu=rate_weight(n, m))
    s, u0, info, refs = run_both(problems, P.PIMPC_FP64)
    compare(s, problems, refs, TOL64)
    check_info(info, refs, 1e-10)


def test_rate_weight_uneven_batch_fp32():
    """24 instances of the uneven random batch, every other one with W_du, FP32."""
    problems = W.random_batch(24, base_seed=2000, K=300)
    problems = [p.copy(Wdu=rate_weight(i, p.nu)) if i % 2 == 0 else p for i, p in enumerate(problems)]
    s, u0, info, refs = run_both(problems, P.PIMPC_FP32)
    compare(s, problems, refs, TOL32)
    check_info(info, refs, 1e-4)


def test_rate_weight_row_family_fp32():
    """Long wide horizon (row family, fused stage data include B J): W_du = 0.1 I."""
    p = W.long_horizon_problem(seed=5, N=600, K=150)
    p = p.copy(Wdu=0.1 * np.eye(p.nu), u_prev=np.full(p.nu, 0.05))
    s = P.Solver([p], max_iter=p.K, precision=P.PIMPC_FP32)
    u0, info = s.solve()
    ref = oracle.solve(p)
    compare(s, [p], [ref], TOL32)
    assert scaled_err(u0, ref["u0"]) <= TOL32
    check_info(info, [ref], 1e-4)


def test_rate_weight_adjoint():
    """Differentiable layer with a fixed W_du: gradients against the oracle's
    reverse mode (which includes W_du in the chain through J)."""
    torch = pytest.importorskip("torch")
    from paper_2601_14414_amd.autograd import PiMPCLayer
    db = W.diff_batch(count=6, seed=4, N=24, K=30)
    Wd = rate_weight(1, 3)
    dev = torch.device("cuda")
    layer = PiMPCLayer(6, 8, 3, db.N, iters=db.K, ckpt_every=7, Wdu=Wd)
    f = lambda a: torch.tensor(np.ascontiguousarray(a[:6]), dtype=torch.float32, device=dev,
                               requires_grad=True)
    x0, Qd, Rd, A, B = f(db.x0), f(db.Qdiag), f(db.Rdiag), f(db.A), f(db.Bm)
    u0 = layer(x0, Qd, Rd, A, B)
    target = torch.tensor(db.u_target[:6], dtype=torch.float32, device=dev)
    ((u0 - target) ** 2).sum().backward()
    torch.cuda.synchronize()
    got = {k: t.grad.detach().cpu().numpy().astype(np.float64) for k, t in
           dict(dx0=x0, dQd=Qd, dRd=Rd, dA=A, dB=B).items()}
    u0n = u0.detach().cpu().numpy().astype(np.float64)
    layer.solver.close()
    for i in range(6):
        p = db.instance(i).copy(Wdu=Wd)
        r = oracle.solve(p)
        assert scaled_err(u0n[i], r["u0"]) <= 1e-4
        g = oracle.grad(8, 3, db.N, p.A, p.B, db.Qdiag[i], db.Rdiag[i], p.lb(), p.ub(), p.x0, p.rho,
                        db.K, 2 * (r["u0"] - db.u_target[i]), Wdu=Wd)
        for key in ("dx0", "dQd", "dRd", "dA", "dB"):
            e = float(np.max(np.abs(got[key][i] - g[key])) / max(1e-6, float(np.max(np.abs(g[key])))))
            assert e <= 2e-3, (i, key, e)
