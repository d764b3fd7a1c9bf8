"""CPU FP64 oracle of the piMPC ADMM iteration -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP implementation; the two
meet only in the seeded input generators.

Thin ctypes binding over oracle/pimpc_oracle.c (plain C99, double precision).
The C file states which passage of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_factor.restype = ctypes.c_int
    lib.orc_factor.argtypes = [ctypes.c_int] * 3 + [_dp] * 5 + [ctypes.c_double, _dp, _dp]
    lib.orc_solve.restype = ctypes.c_int
    lib.orc_solve.argtypes = ([ctypes.c_int] * 3 + [_dp] * 9 + [ctypes.c_int, _dp, ctypes.c_int, _dp]
                              + [_dp] + [ctypes.c_double, ctypes.c_int,
                              ctypes.c_double, ctypes.c_int, ctypes.c_double] + [_dp] * 4 + [_ip])
    lib.orc_project.restype = None
    lib.orc_project.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
    lib.orc_grad.restype = ctypes.c_int
    lib.orc_grad.argtypes = ([ctypes.c_int] * 3 + [_dp] * 8 + [ctypes.c_double, ctypes.c_int]
                             + [_dp] * 7)
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _wdu(p):
    """Input-rate weight W_du of problem `p` as (m, m) float64, or None (= 0)."""
    W = getattr(p, "Wdu", None)
    return None if W is None else _c(W)


SET_KINDS = {"box": 0, "halfspace": 1, "hyperplane": 2, "soc": 3, "l1ball": 4}


def _set_spec(spec, n):
    """(kind, par[n+1]) of a factor set: None / ("box",) / ("halfspace", a, b) /
    ("hyperplane", a, b) / ("soc",) / ("l1ball", r)."""
    if spec is None or spec[0] == "box":
        return 0, None
    kind = SET_KINDS[spec[0]]
    par = np.zeros(n + 1)
    if spec[0] in ("halfspace", "hyperplane"):
        par[:n] = np.asarray(spec[1], np.float64)
        par[n] = float(spec[2])
    elif spec[0] == "l1ball":
        par[n] = float(spec[1])
    return kind, par


def project(spec, w, lo=None, hi=None):
    """Projection of w onto one factor set, by the oracle's own routine (test use)."""
    lib = _load()
    w = _c(w).copy()
    n = w.size
    kind, par = _set_spec(spec, n)
    lo = _c(np.full(n, -np.inf) if lo is None else lo)
    hi = _c(np.full(n, np.inf) if hi is None else hi)
    lib.orc_project(kind, n, _ptr(par), _ptr(lo), _ptr(hi), _ptr(w))
    return w


def effective(p):
    """Problem `p` with the output form of eqn. (1) written into the velocity-
    form weights: cost 1/2||C x - ry||^2_Wy + 1/2||u - ru||^2_R, expanded with
    its constant dropped, adds C'Wy C to Q, C'Wy ry to the x part and R ru to
    the u part of the linear term qbar (the cost is -qbar' xbar); an output
    bound on a row of C with one nonzero c_ij bounds x_j by [ymin, ymax]/c_ij.
    Problems without the output form are returned unchanged."""
    C = getattr(p, "C", None)
    ru = getattr(p, "ru", None)
    if C is None and ru is None:
        return p
    Q = np.array(p.Q, np.float64)
    qbar = np.zeros(p.nx + p.nu) if p.qbar is None else np.array(p.qbar, np.float64)
    xmin = np.array(p.xmin, np.float64)
    xmax = np.array(p.xmax, np.float64)
    if C is not None:
        C = np.asarray(C, np.float64)
        Wy = np.asarray(p.Wy, np.float64)
        Q = Q + C.T @ Wy @ C
        if getattr(p, "ry", None) is not None:
            qbar[:p.nx] += C.T @ (Wy @ np.asarray(p.ry, np.float64))
        ny = C.shape[0]
        lo = np.full(ny, -np.inf) if getattr(p, "ymin", None) is None else np.asarray(p.ymin, np.float64)
        hi = np.full(ny, np.inf) if getattr(p, "ymax", None) is None else np.asarray(p.ymax, np.float64)
        for i in range(ny):
            if lo[i] == -np.inf and hi[i] == np.inf:
                continue
            nz = np.flatnonzero(C[i])
            if nz.size != 1:
                raise OracleError("a bounded output must select one state")
            j = int(nz[0])
            a, b = lo[i] / C[i, j], hi[i] / C[i, j]
            if C[i, j] < 0:
                a, b = b, a
            xmin[j] = max(xmin[j], a)
            xmax[j] = min(xmax[j], b)
    if ru is not None:
        qbar[p.nx:] += np.asarray(p.R, np.float64) @ np.asarray(ru, np.float64)
    return p.copy(Q=Q, qbar=qbar, xmin=xmin, xmax=xmax, C=None, Wy=None, ry=None, ymin=None,
                  ymax=None, ru=None)


def factor(p):
    """Stage caches (H_k, J_k) of Algorithm 1 for problem `p` (FP64)."""
    lib = _load()
    p = effective(p)
    nb = p.nx + p.nu
    H = np.zeros((p.N, nb, nb))
    J = np.zeros((p.N, p.nu, nb))
    rc = lib.orc_factor(p.nx, p.nu, p.N, _ptr(_c(p.stage_A())), _ptr(_c(p.stage_B())),
                        _ptr(_c(p.Q)), _ptr(_c(p.R)), _ptr(_wdu(p)), float(p.rho), _ptr(H), _ptr(J))
    if rc != 0:
        raise OracleError("stage matrix not positive definite")
    return H, J


def zero_state(p) -> np.ndarray:
    return np.zeros((5, p.N, p.nx + p.nu))


def solve(p, K: Optional[int] = None, eps: float = 0.0, accel: bool = False, eta: float = 0.999,
          state: Optional[np.ndarray] = None, xbar0: Optional[np.ndarray] = None) -> dict:
    """Run Algorithm 1 on problem `p` from `state` (default: cold start).

    Returns dict(state=(5,N,nb) final iterate (v, z, theta, beta, lambda),
    du=(N,m), xs=(N,nb) step-1 results of the last iteration,
    hist=(iters,4) [c, r_prim, r_dual, restart], iters, u0 = u_prev + du_0).
    """
    lib = _load()
    p = effective(p)
    K = p.K if K is None else K
    nb = p.nx + p.nu
    st = zero_state(p) if state is None else _c(state).copy()
    assert st.shape == (5, p.N, nb)
    du = np.zeros((p.N, p.nu))
    xs = np.zeros((p.N, nb))
    hist = np.zeros((max(K, 1), 4))
    it = ctypes.c_int(0)
    e = None if p.e is None else _c(p.stage_e())
    qbar = None if p.qbar is None else _c(p.qbar)
    xb0 = _c(p.xbar0() if xbar0 is None else xbar0)
    xkind, xpar = _set_spec(getattr(p, "xset", None), p.nx)
    ukind, upar = _set_spec(getattr(p, "uset", None), p.nu)
    rc = lib.orc_solve(p.nx, p.nu, p.N, _ptr(_c(p.stage_A())), _ptr(_c(p.stage_B())), _ptr(e),
                       _ptr(_c(p.Q)), _ptr(_c(p.R)), _ptr(_wdu(p)), _ptr(qbar), _ptr(_c(p.lb())),
                       _ptr(_c(p.ub())), xkind, _ptr(xpar), ukind, _ptr(upar),
                       _ptr(xb0), float(p.rho), int(K), float(eps), int(bool(accel)), float(eta),
                       _ptr(st), _ptr(du), _ptr(xs), _ptr(hist), ctypes.byref(it))
    if rc != 0:
        raise OracleError(f"orc_solve failed ({rc})")
    n_it = it.value
    return dict(state=st, du=du, xs=xs, hist=hist[:n_it].copy(), iters=n_it,
                u0=np.asarray(p.u_prev, np.float64) + du[0])


def grad(nx, nu, N, A, B, Qd, Rd, lb, ub, x0, rho, K, ubar, Wdu=None) -> dict:
    """Vector-Jacobian product of u_0 (output of the K-th step 1, cold start,
    u_prev = 0, e = 0) with respect to (x0, diag Q, diag R, A, B); Wdu is a
    fixed input-rate weight (None = 0)."""
    lib = _load()
    out = dict(u0=np.zeros(nu), dA=np.zeros((nx, nx)), dB=np.zeros((nx, nu)),
               dQd=np.zeros(nx), dRd=np.zeros(nu), dx0=np.zeros(nx))
    W = None if Wdu is None else _c(Wdu)
    rc = lib.orc_grad(nx, nu, N, _ptr(_c(A)), _ptr(_c(B)), _ptr(_c(Qd)), _ptr(_c(Rd)), _ptr(W),
                      _ptr(_c(lb)), _ptr(_c(ub)), _ptr(_c(x0)), float(rho), int(K), _ptr(_c(ubar)),
                      _ptr(out["u0"]), _ptr(out["dA"]), _ptr(out["dB"]), _ptr(out["dQd"]),
                      _ptr(out["dRd"]), _ptr(out["dx0"]))
    if rc != 0:
        raise OracleError(f"orc_grad failed ({rc})")
    return out
