"""Real-time iteration (time-varying stage data re-linearised every step,
warm start across steps): per-step parity of the GPU solver against the
oracle running the same RTI loop, and the closed-loop driver."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import rti
from paper_2601_14414_amd import workloads as W

from test_gpu_lane import TOL32, compare, scaled_err

pytestmark = pytest.mark.gpu


def oracle_rti(steps, N, iters):
    """The RTI loop run entirely by the oracle (inputs for the GPU side)."""
    p0 = W.cartpole_problem(N=N, K=iters)
    x, up, st, pred = p0.x0.copy(), np.zeros(1), None, None
    log = []
    for t in range(steps):
        if pred is None:
            xs, us = np.broadcast_to(x, (N, 4)).copy(), np.zeros((N, 1))
        else:
            xs, us = W.rti_shift(x, pred)
        A, B, e = W.cartpole_linearize(xs, us)
        p = p0.copy(A=A, B=B, e=e, x0=x.copy(), u_prev=up.copy())
        r = oracle.solve(p, K=iters, state=st)
        log.append((p, r))
        st, pred = r["state"], r["xs"]
        x = W.cartpole_rk4(x, r["u0"])
        up = r["u0"]
    return p0, log


@pytest.mark.parametrize("precision,tol,family", [(P.PIMPC_FP64, 1e-10, P.PIMPC_FAMILY_AUTO),
                                                  (P.PIMPC_FP32, TOL32, P.PIMPC_FAMILY_AUTO),
                                                  (P.PIMPC_FP32, TOL32, P.PIMPC_FAMILY_LANE)])
def test_rti_per_step_parity(precision, tol, family):
    """20 RTI steps x 100 iterations, N=256: at every step the GPU (fed the
    same linearisations, x(t) and u(t-1)) matches the oracle iterates."""
    p0, log = oracle_rti(steps=20, N=256, iters=100)
    s = P.Solver([p0], max_iter=100, precision=precision, warm_start=True, family=family)
    worst = 0.0
    for t, (p, r) in enumerate(log):
        s.linearize(p.A.ravel(), p.B.ravel(), p.e.ravel())
        u0, info = s.solve(x0=p.x0, u_prev=p.u_prev)
        assert scaled_err(u0, r["u0"]) <= tol, t
        worst = max(worst, compare(s, [p], [r], tol))
    print(f"largest scaled iterate error over 20 RTI steps: {worst:.2e}")
    s.close()


def test_rti_closed_loop_driver():
    """The closed-loop driver runs (GPU decides the inputs) and keeps the
    inputs inside |u| <= 10; the first step saturates the input."""
    log = rti.run_cartpole_rti(steps=20, N=256, iters=100)
    assert len(log) == 20
    u = np.array([st.u0[0] for st in log])
    # u0 is the xbar iterate of a finite iteration count, not yet exactly feasible
    assert np.all(np.isfinite(u)) and np.all(np.abs(u) <= 10.0 + 0.05)
    assert abs(u[0]) > 5.0
    assert all(st.info["status"][0] == 0 for st in log)
