"""Real-time-iteration (RTI) NMPC driver over the C ABI.

Per sampling step (Sections I-II: online-linearised / RTI NMPC with a
construction-free solver):
  1. linearise the plant along the previous predicted trajectory, shifted by
     one stage (caller-side model code, here the cart-pole of workloads.py);
  2. pimpc_linearize: replace the stage data and refactor on the device
     (no QP construction);
  3. pimpc_solve with a warm start from the previous iterate and u(t-1);
  4. apply u0 to the plant, read the predicted trajectory for the next step.

The solver's iterate is kept across steps unshifted (Algorithm 1 output used
as the next warm start).  Every solver step runs in the HIP library.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np

from . import pimpc as P
from . import workloads as W


@dataclasses.dataclass
class RTIStep:
    t: int
    x: np.ndarray          # plant state before applying u0
    u0: np.ndarray
    A: np.ndarray          # stage data used at this step
    B: np.ndarray
    e: np.ndarray
    u_prev: np.ndarray
    info: np.ndarray
    xbar: np.ndarray       # predicted xbar_{k+1}, (N, nb)


def run_cartpole_rti(steps: int = 20, N: int = 256, iters: int = 100, precision: int = P.PIMPC_FP32,
                     plant: Optional[Callable] = None, stream: Optional[int] = None) -> List[RTIStep]:
    """Swing-up of the cart-pole from the hanging position with RTI."""
    plant = plant or W.cartpole_rk4
    p = W.cartpole_problem(N=N, K=iters)
    solver = P.Solver([p], max_iter=iters, precision=precision, warm_start=True, stream=stream)
    x = p.x0.copy()
    u_prev = np.zeros(1)
    xbar_pred = None
    log: List[RTIStep] = []
    try:
        for t in range(steps):
            if xbar_pred is None:
                xs = np.broadcast_to(x, (N, 4)).copy()
                us = np.zeros((N, 1))
            else:
                xs, us = W.rti_shift(x, xbar_pred)
            A, B, e = W.cartpole_linearize(xs, us)
            solver.linearize(A.ravel(), B.ravel(), e.ravel())
            u0, info = solver.solve(x0=x, u_prev=u_prev)
            xbar_pred = solver.iterate(P.IT_XBAR)[0]
            log.append(RTIStep(t=t, x=x.copy(), u0=u0.copy(), A=A, B=B, e=e, u_prev=u_prev.copy(),
                               info=info.copy(), xbar=xbar_pred.copy()))
            x = plant(x, u0)
            u_prev = u0
    finally:
        solver.close()
    return log
