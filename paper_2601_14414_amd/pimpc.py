"""ctypes binding of libpimpc.so (include/pimpc.h).

Argument marshalling only: every step of the solver runs in the HIP library.
If the library is missing this module raises on first use; there is no
Python or CPU fallback.

Functions carry the C names (pimpc_setup, pimpc_solve, ...); `Solver` wraps
a context for convenience.  Device buffers for pimpc_solve_batch /
pimpc_set_params_dev / pimpc_backward are torch tensors (PyTorch provides
device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpimpc.so")

PIMPC_OK = 0
PIMPC_E_ARG = -1
PIMPC_E_DIM = -2
PIMPC_E_NOT_PSD = -3
PIMPC_E_NONFINITE = -4
PIMPC_E_HIP = -5
PIMPC_E_NOMEM = -6
PIMPC_E_STATE = -7
PIMPC_E_UNSUPPORTED = -8
PIMPC_FP64 = 0
PIMPC_FP32 = 1
PIMPC_MEM_HOST = 0
PIMPC_MEM_DEVICE = 1
PIMPC_FAMILY_AUTO, PIMPC_FAMILY_LANE, PIMPC_FAMILY_ROW = 0, 1, 2
PIMPC_SET_BOX, PIMPC_SET_HALFSPACE, PIMPC_SET_HYPERPLANE, PIMPC_SET_SOC, PIMPC_SET_L1BALL = 0, 1, 2, 3, 4
IT_V, IT_Z, IT_THETA, IT_BETA, IT_LAMBDA, IT_DU, IT_XBAR = range(7)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class pimpc_problem(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("nx", _ip), ("nu", _ip), ("N", _ip),
                ("time_varying", ctypes.c_int32), ("A", _dp), ("B", _dp), ("e", _dp),
                ("Q", _dp), ("R", _dp), ("qbar", _dp), ("xmin", _dp), ("xmax", _dp),
                ("umin", _dp), ("umax", _dp), ("Wdu", _dp), ("xset", _ip), ("uset", _ip),
                ("xset_par", _dp), ("uset_par", _dp), ("ny", _ip), ("C", _dp), ("Wy", _dp),
                ("ry", _dp), ("ymin", _dp), ("ymax", _dp), ("ru", _dp)]


class pimpc_options(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("max_iter", ctypes.c_int32), ("eps", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("accel", ctypes.c_int32), ("eta", ctypes.c_double), ("warm_start", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("schedule", ctypes.c_int32), ("family", ctypes.c_int32)]


class pimpc_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("c", ctypes.c_double),
                ("r_prim", ctypes.c_double), ("r_dual", ctypes.c_double),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


INFO_DTYPE = np.dtype([("iters", np.int32), ("restarts", np.int32), ("c", np.float64),
                       ("r_prim", np.float64), ("r_dual", np.float64), ("status", np.int32),
                       ("pad", np.int32)])
assert INFO_DTYPE.itemsize == ctypes.sizeof(pimpc_info) == 40

EXPORTS = ["pimpc_default_options", "pimpc_setup", "pimpc_linearize", "pimpc_solve",
           "pimpc_solve_batch", "pimpc_set_params_dev", "pimpc_backward", "pimpc_get_iterates",
           "pimpc_set_iterates", "pimpc_destroy", "pimpc_last_error", "pimpc_version", "pimpc_tape_id",
           "pimpc_solve_batch_noalloc"]

_lib = None


class PimpcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pimpc error {code}: {msg}")
        self.code = code
        self.msg = msg


def lib():
    """Load libpimpc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2601_14414_amd.build` (no CPU fallback exists)")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
    # soname).  Loading it first lets libpimpc bind to that copy, so device
    # pointers and streams from torch tensors are valid here; loading libpimpc
    # first would pull in a second HIP / HSA runtime next to torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.pimpc_default_options.argtypes = [ctypes.POINTER(pimpc_options)]
    L.pimpc_default_options.restype = None
    L.pimpc_setup.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(pimpc_problem),
                              ctypes.POINTER(pimpc_options), vp]
    L.pimpc_linearize.argtypes = [vp, vp, vp, vp, ctypes.c_int32]
    L.pimpc_solve.argtypes = [vp, _dp, _dp, _dp, ctypes.POINTER(pimpc_info)]
    L.pimpc_solve_batch.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pimpc_solve_batch_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pimpc_set_params_dev.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pimpc_backward.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, vp, vp, vp, vp]
    L.pimpc_tape_id.argtypes = [vp]
    L.pimpc_tape_id.restype = ctypes.c_uint64
    L.pimpc_get_iterates.argtypes = [vp, ctypes.c_int32, _dp]
    L.pimpc_set_iterates.argtypes = [vp, ctypes.c_int32, _dp]
    L.pimpc_destroy.argtypes = [vp]
    L.pimpc_destroy.restype = None
    L.pimpc_last_error.argtypes = [vp]
    L.pimpc_last_error.restype = ctypes.c_char_p
    L.pimpc_version.argtypes = []
    for f in ["pimpc_setup", "pimpc_linearize", "pimpc_solve", "pimpc_solve_batch", "pimpc_solve_batch_noalloc",
              "pimpc_set_params_dev", "pimpc_backward", "pimpc_get_iterates", "pimpc_set_iterates",
              "pimpc_version"]:
        getattr(L, f).restype = ctypes.c_int32
    _lib = L
    return L


def _check(rc: int, ctx) -> None:
    if rc != PIMPC_OK:
        msg = lib().pimpc_last_error(ctx)
        raise PimpcError(rc, msg.decode() if msg else "")


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


def _tptr(t) -> Optional[int]:
    """Raw device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device tensors must be contiguous")
    return t.data_ptr()


# --- the C entry points, same names ------------------------------------------

def pimpc_default_options() -> pimpc_options:
    o = pimpc_options()
    lib().pimpc_default_options(ctypes.byref(o))
    return o


SET_KINDS = {"box": PIMPC_SET_BOX, "halfspace": PIMPC_SET_HALFSPACE, "hyperplane": PIMPC_SET_HYPERPLANE,
             "soc": PIMPC_SET_SOC, "l1ball": PIMPC_SET_L1BALL}


def _set_arrays(specs, sizes):
    """Packed kinds (int32 per instance) and parameters ((n + 1) per instance)
    of the x or u factor sets; (None, None) when every factor is a box.  A
    spec is None / ("box",) / ("halfspace", a, b) / ("hyperplane", a, b) /
    ("soc",) / ("l1ball", r)."""
    if all(sp is None or sp[0] == "box" for sp in specs):
        return None, None
    kinds = np.zeros(len(specs), np.int32)
    pars = []
    for i, (sp, n) in enumerate(zip(specs, sizes)):
        par = np.zeros(n + 1)
        if sp is not None:
            kinds[i] = SET_KINDS[sp[0]]
            if sp[0] in ("halfspace", "hyperplane"):
                par[:n] = np.asarray(sp[1], np.float64)
                par[n] = float(sp[2])
            elif sp[0] == "l1ball":
                par[n] = float(sp[1])
        pars.append(par)
    return kinds, _f64(np.concatenate(pars))


def pimpc_setup(problems: Sequence, opts: pimpc_options, stream: Optional[int] = None):
    """Create a context for a list of workloads.Problem (all time-invariant or
    all time-varying).  Returns (ctx, keepalive)."""
    tv = int(any(p.time_varying for p in problems))
    keep = {}
    nx = np.array([p.nx for p in problems], np.int32)
    nu = np.array([p.nu for p in problems], np.int32)
    N = np.array([p.N for p in problems], np.int32)
    if tv:
        A = _f64(np.concatenate([p.stage_A().ravel() for p in problems]))
        B = _f64(np.concatenate([p.stage_B().ravel() for p in problems]))
        e = _f64(np.concatenate([p.stage_e().ravel() for p in problems]))
    else:
        A = _f64(np.concatenate([np.asarray(p.A).ravel() for p in problems]))
        B = _f64(np.concatenate([np.asarray(p.B).ravel() for p in problems]))
        e = None
        if any(p.e is not None for p in problems):
            e = _f64(np.concatenate([(np.zeros(p.nx) if p.e is None else np.asarray(p.e)).ravel()
                                     for p in problems]))
    Q = _f64(np.concatenate([np.asarray(p.Q).ravel() for p in problems]))
    R = _f64(np.concatenate([np.asarray(p.R).ravel() for p in problems]))
    qbar = None
    if any(p.qbar is not None for p in problems):
        qbar = _f64(np.concatenate([(np.zeros(p.nb) if p.qbar is None else np.asarray(p.qbar))
                                    for p in problems]))
    xmin = _f64(np.concatenate([p.xmin for p in problems]))
    xmax = _f64(np.concatenate([p.xmax for p in problems]))
    umin = _f64(np.concatenate([p.umin for p in problems]))
    umax = _f64(np.concatenate([p.umax for p in problems]))
    Wdu = None
    if any(getattr(p, "Wdu", None) is not None for p in problems):
        Wdu = _f64(np.concatenate([(np.zeros((p.nu, p.nu)) if getattr(p, "Wdu", None) is None
                                    else np.asarray(p.Wdu)).ravel() for p in problems]))
    xk, xpar = _set_arrays([getattr(p, "xset", None) for p in problems], [p.nx for p in problems])
    uk, upar = _set_arrays([getattr(p, "uset", None) for p in problems], [p.nu for p in problems])
    # output form of eqn. (1): y = C x with weight Wy, reference ry, bounds
    ny = C = Wy = ry = ymin = ymax = ru = None
    if any(getattr(p, "C", None) is not None for p in problems):
        nys = [0 if getattr(p, "C", None) is None else int(np.asarray(p.C).shape[0]) for p in problems]
        ny = np.array(nys, np.int32)
        part = lambda p, name, n, fill: (np.full(n, fill) if getattr(p, name, None) is None
                                         else np.asarray(getattr(p, name), np.float64).ravel())
        C = _f64(np.concatenate([part(p, "C", n * p.nx, 0.0) for p, n in zip(problems, nys)]))
        Wy = _f64(np.concatenate([part(p, "Wy", n * n, 0.0) for p, n in zip(problems, nys)]))
        ry = _f64(np.concatenate([part(p, "ry", n, 0.0) for p, n in zip(problems, nys)]))
        ymin = _f64(np.concatenate([part(p, "ymin", n, -np.inf) for p, n in zip(problems, nys)]))
        ymax = _f64(np.concatenate([part(p, "ymax", n, np.inf) for p, n in zip(problems, nys)]))
    if any(getattr(p, "ru", None) is not None for p in problems):
        ru = _f64(np.concatenate([np.zeros(p.nu) if getattr(p, "ru", None) is None else np.asarray(p.ru)
                                  for p in problems]))
    keep.update(nx=nx, nu=nu, N=N, A=A, B=B, e=e, Q=Q, R=R, qbar=qbar, xmin=xmin, xmax=xmax,
                umin=umin, umax=umax, Wdu=Wdu, xk=xk, xpar=xpar, uk=uk, upar=upar, ny=ny, C=C, Wy=Wy,
                ry=ry, ymin=ymin, ymax=ymax, ru=ru)
    prob = pimpc_problem(count=len(problems), nx=nx.ctypes.data_as(_ip), nu=nu.ctypes.data_as(_ip),
                         N=N.ctypes.data_as(_ip), time_varying=tv, A=_p(A), B=_p(B), e=_p(e),
                         Q=_p(Q), R=_p(R), qbar=_p(qbar), xmin=_p(xmin), xmax=_p(xmax),
                         umin=_p(umin), umax=_p(umax), Wdu=_p(Wdu),
                         xset=None if xk is None else xk.ctypes.data_as(_ip),
                         uset=None if uk is None else uk.ctypes.data_as(_ip), xset_par=_p(xpar),
                         uset_par=_p(upar), ny=None if ny is None else ny.ctypes.data_as(_ip),
                         C=_p(C), Wy=_p(Wy), ry=_p(ry), ymin=_p(ymin), ymax=_p(ymax), ru=_p(ru))
    ctx = ctypes.c_void_p()
    rc = lib().pimpc_setup(ctypes.byref(ctx), ctypes.byref(prob), ctypes.byref(opts), stream)
    _check(rc, None)
    return ctx, keep


def pimpc_linearize(ctx, A, B, e=None, mem_kind=PIMPC_MEM_HOST):
    if mem_kind == PIMPC_MEM_HOST:
        A, B = _f64(A), _f64(B)
        e = None if e is None else _f64(e)
        rc = lib().pimpc_linearize(ctx, A.ctypes.data, B.ctypes.data,
                                   None if e is None else e.ctypes.data, mem_kind)
    else:
        rc = lib().pimpc_linearize(ctx, _tptr(A), _tptr(B), _tptr(e), mem_kind)
    _check(rc, ctx)


def pimpc_solve(ctx, x0, u_prev, sum_nu: int, count: int):
    x0 = _f64(x0)
    up = None if u_prev is None else _f64(u_prev)
    u0 = np.zeros(sum_nu)
    info = (pimpc_info * count)()
    rc = lib().pimpc_solve(ctx, _p(x0), _p(up), _p(u0), info)
    infos = np.frombuffer(bytes(info), dtype=INFO_DTYPE).copy()
    _check(rc, ctx)
    return u0, infos


def pimpc_solve_batch(ctx, x0_dev, uprev_dev, u0_dev, info_dev=None, stream: Optional[int] = None):
    rc = lib().pimpc_solve_batch(ctx, _tptr(x0_dev), _tptr(uprev_dev), _tptr(u0_dev),
                                 _tptr(info_dev), stream)
    _check(rc, ctx)


def pimpc_solve_batch_noalloc(ctx, x0_dev, uprev_dev, u0_dev, info_dev=None, stream: Optional[int] = None):
    rc = lib().pimpc_solve_batch_noalloc(ctx, _tptr(x0_dev), _tptr(uprev_dev), _tptr(u0_dev),
                                         _tptr(info_dev), stream)
    _check(rc, ctx)


def pimpc_set_params_dev(ctx, A, B, Qdiag, Rdiag, stream: Optional[int] = None):
    rc = lib().pimpc_set_params_dev(ctx, _tptr(A), _tptr(B), _tptr(Qdiag), _tptr(Rdiag), stream)
    _check(rc, ctx)


def pimpc_tape_id(ctx) -> int:
    return int(lib().pimpc_tape_id(ctx))


def pimpc_backward(ctx, tape_id: int, dL_du0, dx0=None, dQdiag=None, dRdiag=None, dA=None, dB=None,
                   stream: Optional[int] = None):
    rc = lib().pimpc_backward(ctx, tape_id, _tptr(dL_du0), _tptr(dx0), _tptr(dQdiag), _tptr(dRdiag),
                              _tptr(dA), _tptr(dB), stream)
    _check(rc, ctx)


def pimpc_get_iterates(ctx, which: int, n: int) -> np.ndarray:
    out = np.zeros(n)
    _check(lib().pimpc_get_iterates(ctx, which, _p(out)), ctx)
    return out


def pimpc_set_iterates(ctx, which: int, values) -> None:
    v = _f64(values)
    _check(lib().pimpc_set_iterates(ctx, which, _p(v)), ctx)


def pimpc_destroy(ctx) -> None:
    if ctx is not None:
        lib().pimpc_destroy(ctx)


def pimpc_version() -> int:
    return int(lib().pimpc_version())


# --- convenience wrapper -------------------------------------------------------

class Solver:
    """A context over a list of workloads.Problem."""

    def __init__(self, problems: Sequence, rho: float = 1.0, max_iter: int = 200, eps: float = 0.0,
                 check_every: int = 1, precision: int = PIMPC_FP32, warm_start: bool = False,
                 ckpt_every: int = 0, schedule: int = 0, stream: Optional[int] = None,
                 accel: bool = False, eta: float = 0.999, family: int = PIMPC_FAMILY_AUTO):
        self.problems = list(problems)
        o = pimpc_default_options()
        o.rho, o.max_iter, o.eps, o.check_every = rho, max_iter, eps, check_every
        o.precision, o.warm_start, o.ckpt_every, o.schedule = precision, int(warm_start), ckpt_every, schedule
        o.accel, o.eta, o.family = int(bool(accel)), eta, family
        self.opts = o
        self.ctx, self._keep = pimpc_setup(self.problems, o, stream)
        self.count = len(self.problems)
        self.sum_nx = sum(p.nx for p in self.problems)
        self.sum_nu = sum(p.nu for p in self.problems)
        self.nx = self.problems[0].nx
        self.nu = self.problems[0].nu

    def solve(self, x0=None, u_prev=None):
        """x0/u_prev: packed arrays (default: each problem's own); returns
        (u0 packed, info structured array)."""
        if x0 is None:
            x0 = np.concatenate([p.x0 for p in self.problems])
        if u_prev is None and any(np.any(p.u_prev != 0) for p in self.problems):
            u_prev = np.concatenate([p.u_prev for p in self.problems])
        return pimpc_solve(self.ctx, x0, u_prev, self.sum_nu, self.count)

    def iterate(self, which: int):
        """Iterate `which` split per instance: (N, nb) arrays ((N, nu) for IT_DU)."""
        sizes = [p.N * (p.nu if which == IT_DU else p.nb) for p in self.problems]
        flat = pimpc_get_iterates(self.ctx, which, sum(sizes))
        out, pos = [], 0
        for p, s in zip(self.problems, sizes):
            out.append(flat[pos:pos + s].reshape(p.N, -1))
            pos += s
        return out

    def state(self, i: int = 0) -> np.ndarray:
        """(5, N, nb) iterate (v, z, theta, beta, lambda) of instance i."""
        return np.stack([self.iterate(w)[i] for w in range(5)])

    def set_state(self, states: Sequence[np.ndarray]) -> None:
        for w in range(5):
            pimpc_set_iterates(self.ctx, w, np.concatenate([s[w].ravel() for s in states]))

    def linearize(self, A, B, e=None):
        pimpc_linearize(self.ctx, A, B, e, PIMPC_MEM_HOST)

    def close(self):
        if self.ctx is not None:
            pimpc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
