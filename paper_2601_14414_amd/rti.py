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
    jac_s: float = 0.0     # wall time of the host Jacobians along the shifted trajectory
    lib_s: float = 0.0     # wall time of pimpc_linearize + pimpc_solve
    step_s: float = 0.0    # whole RTI step: shift, Jacobians, library calls, predicted trajectory read-back


def run_cartpole_rti(steps: int = 20, N: int = 256, iters: int = 100, precision: int = P.PIMPC_FP32,
                     plant: Optional[Callable] = None, stream: Optional[int] = None,
                     family: int = P.PIMPC_FAMILY_AUTO) -> List[RTIStep]:
    """Swing-up of the cart-pole from the hanging position with RTI."""
    import time
    plant = plant or W.cartpole_rk4
    p = W.cartpole_problem(N=N, K=iters)
    solver = P.Solver([p], max_iter=iters, precision=precision, warm_start=True, stream=stream, family=family)
    x = p.x0.copy()
    u_prev = np.zeros(1)
    xbar_pred = None
    log: List[RTIStep] = []
    try:
        for t in range(steps):
            t0 = time.perf_counter()
            if xbar_pred is None:
                xs = np.broadcast_to(x, (N, 4)).copy()
                us = np.zeros((N, 1))
            else:
                xs, us = W.rti_shift(x, xbar_pred)
            A, B, e = W.cartpole_linearize(xs, us)
            t1 = time.perf_counter()
            solver.linearize(A.ravel(), B.ravel(), e.ravel())
            u0, info = solver.solve(x0=x, u_prev=u_prev)
            t2 = time.perf_counter()
            xbar_pred = solver.iterate(P.IT_XBAR)[0]
            t3 = time.perf_counter()
            log.append(RTIStep(t=t, x=x.copy(), u0=u0.copy(), A=A, B=B, e=e, u_prev=u_prev.copy(),
                               info=info.copy(), xbar=xbar_pred.copy(), jac_s=t1 - t0, lib_s=t2 - t1,
                               step_s=t3 - t0))
            x = plant(x, u0)
            u_prev = u0
    finally:
        solver.close()
    return log


@dataclasses.dataclass
class CSTRStep:
    t: int
    x: np.ndarray          # plant state before applying u0
    u0: np.ndarray
    u_prev: np.ndarray
    info: np.ndarray
    solve_s: float         # wall time of pimpc_linearize + pimpc_solve


def run_cstr_nmpc(steps: int = 20, N: int = 5000, iters: int = 1000, rho: float = 0.1,
                  precision: int = P.PIMPC_FP32, stream: Optional[int] = None) -> List[CSTRStep]:
    """Online-linearised NMPC of the reactor of Section V: at every sample the
    Euler model is linearised at the current state and input (the same stage
    data for the whole horizon), the device refactors (pimpc_linearize) and
    runs `iters` warm-started iterations, and the first input drives the RK4
    plant under the inlet-temperature disturbance."""
    import time
    p = W.cstr_problem(N=N, K=iters, rho=rho)
    solver = P.Solver([p], rho=rho, max_iter=iters, precision=precision, warm_start=True, stream=stream)
    x = p.x0.copy()
    u_prev = p.u_prev.copy()
    log: List[CSTRStep] = []
    try:
        for t in range(steps):
            tm = t * W.CSTR_TS
            t0 = time.perf_counter()
            A, B, e = W.cstr_linearize(x, u_prev, W.cstr_ti(tm))
            solver.linearize(A.ravel(), B.ravel(), e.ravel())
            u0, info = solver.solve(x0=x, u_prev=u_prev)
            dt = time.perf_counter() - t0
            log.append(CSTRStep(t=t, x=x.copy(), u0=u0.copy(), u_prev=u_prev.copy(), info=info.copy(),
                                solve_s=dt))
            x = W.cstr_plant(x, u0, tm)
            u_prev = u0
    finally:
        solver.close()
    return log
