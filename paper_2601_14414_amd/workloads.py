"""Seeded synthetic MPC problem generators.

This module builds the *inputs* of the piMPC solver: stage matrices, weights,
bounds, initial states, batches and the cart-pole plant used for real-time
iteration (RTI).  It holds none of the solver's arithmetic (no factorisation,
no ADMM step, no residual), so both the CPU oracle's tests and the HIP path
draw their inputs from here and nothing else is shared between them.

Problem statement being instantiated: the linear time-varying MPC problem of
Section II (eqn. (1)): dynamics x_{k+1} = A_k x_k + B_k u_k + e_k, quadratic
weights, box sets X and U, horizon N and the current state x(t).  With C = I,
W_y = Q, W_u = R and zero references, the velocity-form data of Theorem 2 is
Qbar = blkdiag(Q, R), qbar = 0, Xbar = X x U.

Every generator is deterministic given its seed (numpy default_rng).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg


@dataclasses.dataclass
class Problem:
    """One MPC instance in the form of eqn. (1) (Section II).

    A: (n, n) time-invariant or (N, n, n) time-varying; B likewise (n, m) or
    (N, n, m); e: None or (n,) / (N, n).  Q (n, n), R (m, m) symmetric PSD.
    qbar: None or (n+m,) linear term of the velocity-form cost (Theorem 2).
    Wdu: None or (m, m) symmetric PSD input-rate weight, cost term
    1/2 ||u_k - u_{k-1}||^2_{Wdu} (used by the paper's experiments, Section V).
    xset / uset: None (the box xmin..xmax / umin..umax) or another closed
    convex set for every x_k / u_k (the sets the proof of Theorem 1 lists):
    ("halfspace", a, b) = {a'w <= b}, ("hyperplane", a, b) = {a'w = b},
    ("soc",) = {||w[:-1]||_2 <= w[-1]}, ("l1ball", r) = {||w||_1 <= r}.
    Bounds are per-component boxes; +-inf allowed.  x0 = x(t), u_prev = u(t-1).
    Output form of eqn. (1), optional: C (ny, nx) with y = C x, Wy (ny, ny),
    ry (ny,), output bounds ymin / ymax (ny,), input reference ru (nu,) with
    W_u = R; the cost then has 1/2 ||C x - ry||^2_Wy + 1/2 ||u - ru||^2_R on
    top of 1/2 x'Q x (Q may be zero).
    """

    nx: int
    nu: int
    N: int
    A: np.ndarray
    B: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    xmin: np.ndarray
    xmax: np.ndarray
    umin: np.ndarray
    umax: np.ndarray
    x0: np.ndarray
    u_prev: np.ndarray
    rho: float = 1.0
    K: int = 200
    e: Optional[np.ndarray] = None
    qbar: Optional[np.ndarray] = None
    Wdu: Optional[np.ndarray] = None
    xset: Optional[tuple] = None
    uset: Optional[tuple] = None
    C: Optional[np.ndarray] = None
    Wy: Optional[np.ndarray] = None
    ry: Optional[np.ndarray] = None
    ymin: Optional[np.ndarray] = None
    ymax: Optional[np.ndarray] = None
    ru: Optional[np.ndarray] = None

    @property
    def nb(self) -> int:
        return self.nx + self.nu

    @property
    def time_varying(self) -> bool:
        return self.A.ndim == 3

    def stage_A(self) -> np.ndarray:
        """A as (N, n, n) float64."""
        return _per_stage(self.A, self.N)

    def stage_B(self) -> np.ndarray:
        return _per_stage(self.B, self.N)

    def stage_e(self) -> np.ndarray:
        if self.e is None:
            return np.zeros((self.N, self.nx))
        e = np.asarray(self.e, dtype=np.float64)
        if e.ndim == 2:
            assert e.shape == (self.N, self.nx)
            return e
        return np.broadcast_to(e, (self.N, self.nx)).copy()

    def lb(self) -> np.ndarray:
        return np.concatenate([self.xmin, self.umin]).astype(np.float64)

    def ub(self) -> np.ndarray:
        return np.concatenate([self.xmax, self.umax]).astype(np.float64)

    def xbar0(self) -> np.ndarray:
        """Initial augmented state col(x(t), u(t-1)) (Theorem 2)."""
        return np.concatenate([self.x0, self.u_prev]).astype(np.float64)

    def copy(self, **changes) -> "Problem":
        d = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}
        for k, v in d.items():
            if isinstance(v, np.ndarray):
                d[k] = v.copy()
        d.update(changes)
        return Problem(**d)


def _per_stage(M: np.ndarray, N: int) -> np.ndarray:
    M = np.asarray(M, dtype=np.float64)
    if M.ndim == 3:
        assert M.shape[0] == N
        return M
    return np.broadcast_to(M, (N,) + M.shape).copy()


# ---------------------------------------------------------------------------
# Mass-spring chain (zero-order hold)
# ---------------------------------------------------------------------------

def mass_spring_continuous(p: int, k: float = 1.0, c: float = 0.1, mass: float = 1.0):
    """Chain of p unit masses, springs k between neighbours and to walls at both
    ends, dampers c parallel to every spring, p-1 tension inputs between
    neighbouring masses (+u_j on mass j, -u_j on mass j+1).

    State = (positions, velocities): nx = 2p, nu = p-1.
    Returns the continuous-time (A_c, B_c).
    """
    T = 2.0 * np.eye(p) - np.eye(p, k=1) - np.eye(p, k=-1)
    F = np.zeros((p, p - 1))
    for j in range(p - 1):
        F[j, j] = 1.0
        F[j + 1, j] = -1.0
    Ac = np.block([[np.zeros((p, p)), np.eye(p)], [-(k / mass) * T, -(c / mass) * T]])
    Bc = np.vstack([np.zeros((p, p - 1)), F / mass])
    return Ac, Bc


def zoh(Ac: np.ndarray, Bc: np.ndarray, dt: float):
    """Zero-order-hold discretisation via the exponential of the augmented
    matrix [[Ac, Bc], [0, 0]] * dt."""
    n, m = Bc.shape
    M = np.zeros((n + m, n + m))
    M[:n, :n] = Ac
    M[:n, n:] = Bc
    E = scipy.linalg.expm(M * dt)
    return E[:n, :n].copy(), E[:n, n:].copy()


def mass_spring(p: int, dt: float = 0.1, k: float = 1.0, c: float = 0.1, mass: float = 1.0):
    Ac, Bc = mass_spring_continuous(p, k, c, mass)
    return zoh(Ac, Bc, dt)


def mass_spring_problem(p: int, N: int, seed: int, x0_scale: float, K: int,
                        rho: float = 1.0, xbound: float = 4.0, ubound: float = 0.5,
                        r_weight: float = 0.1) -> Problem:
    A, B = mass_spring(p)
    nx, nu = 2 * p, p - 1
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-x0_scale, x0_scale, size=nx)
    return Problem(
        nx=nx, nu=nu, N=N, A=A, B=B, Q=np.eye(nx), R=r_weight * np.eye(nu),
        xmin=-xbound * np.ones(nx), xmax=xbound * np.ones(nx),
        umin=-ubound * np.ones(nu), umax=ubound * np.ones(nu),
        x0=x0, u_prev=np.zeros(nu), rho=rho, K=K)


def plain_fp64_problem(seed: int = 0) -> Problem:
    """Plain linear MPC: 4-mass chain (nx=8, nu=3), N=20, Q=I, R=0.1 I,
    |u|<=0.5, |x|<=4, rho=1, 200 iterations, x0 ~ U[-1,1]."""
    return mass_spring_problem(4, 20, seed, 1.0, 200)


def long_horizon_problem(seed: int = 0, N: int = 1024, K: int = 500) -> Problem:
    """Long horizon: 12-mass chain (nx=24, nu=11), N=1024, 500 iterations,
    x0 ~ U[-2,2]."""
    return mass_spring_problem(12, N, seed, 2.0, K)


# ---------------------------------------------------------------------------
# Random linear systems (uneven batch)
# ---------------------------------------------------------------------------

def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    G = rng.standard_normal((n, n))
    Qm, Rm = np.linalg.qr(G)
    return Qm * np.sign(np.diag(Rm))[None, :]


def random_batch_instance(seed: int, K: int = 300) -> Problem:
    """One instance of the uneven batch: nx in {4,8,12,16}, nu in {1,2,3,4},
    N uniform in [32, 512]; A = orthogonal x diag(d), d_j ~ U[0.95, 1.05];
    B ~ N(0,1)/sqrt(nx); Q = I, R = 0.1 I, |u|<=1, |x|<=5, x0 ~ U[-1,1]."""
    rng = np.random.default_rng(seed)
    nx = int(rng.choice([4, 8, 12, 16]))
    nu = int(rng.choice([1, 2, 3, 4]))
    N = int(rng.integers(32, 513))
    O = haar_orthogonal(nx, rng)
    d = rng.uniform(0.95, 1.05, size=nx)
    A = O * d[None, :]
    B = rng.standard_normal((nx, nu)) / math.sqrt(nx)
    x0 = rng.uniform(-1.0, 1.0, size=nx)
    return Problem(nx=nx, nu=nu, N=N, A=A, B=B, Q=np.eye(nx), R=0.1 * np.eye(nu),
                   xmin=-5.0 * np.ones(nx), xmax=5.0 * np.ones(nx),
                   umin=-np.ones(nu), umax=np.ones(nu), x0=x0, u_prev=np.zeros(nu),
                   rho=1.0, K=K)


def random_batch(count: int = 4096, base_seed: int = 1000, K: int = 300) -> List[Problem]:
    return [random_batch_instance(base_seed + i, K) for i in range(count)]


def paper_random_system(n: int, m: int, N: int, seed: int, K: int = 200) -> Problem:
    """Random-system recipe of the scalability study (Section V-B): A, B with
    N(0,1) entries, A scaled to unit spectral radius, |x|<=5, |u|<=0.1,
    W_y = I, W_u = I."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A / np.max(np.abs(np.linalg.eigvals(A)))
    B = rng.standard_normal((n, m))
    x0 = rng.uniform(-1.0, 1.0, size=n)
    return Problem(nx=n, nu=m, N=N, A=A, B=B, Q=np.eye(n), R=np.eye(m),
                   xmin=-5.0 * np.ones(n), xmax=5.0 * np.ones(n),
                   umin=-0.1 * np.ones(m), umax=0.1 * np.ones(m), x0=x0,
                   u_prev=np.zeros(m), rho=1.0, K=K)


# ---------------------------------------------------------------------------
# Differentiable batch (copies of the 4-mass chain)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DiffBatch:
    """Batch of B copies of the 4-mass chain with N=128 and per-instance
    differentiable parameters."""

    x0: np.ndarray        # (B, 8)
    Qdiag: np.ndarray     # (B, 8)
    Rdiag: np.ndarray     # (B, 3)
    A: np.ndarray         # (B, 8, 8)
    Bm: np.ndarray        # (B, 8, 3)
    u_target: np.ndarray  # (B, 3)
    N: int
    K: int
    rho: float
    xbound: float
    ubound: float

    def instance(self, i: int) -> Problem:
        nx, nu = self.A.shape[1], self.Bm.shape[2]
        return Problem(nx=nx, nu=nu, N=self.N, A=self.A[i].copy(), B=self.Bm[i].copy(),
                       Q=np.diag(self.Qdiag[i]), R=np.diag(self.Rdiag[i]),
                       xmin=-self.xbound * np.ones(nx), xmax=self.xbound * np.ones(nx),
                       umin=-self.ubound * np.ones(nu), umax=self.ubound * np.ones(nu),
                       x0=self.x0[i].copy(), u_prev=np.zeros(nu), rho=self.rho, K=self.K)


def diff_batch(count: int = 1024, seed: int = 7, N: int = 128, K: int = 200) -> DiffBatch:
    A, B = mass_spring(4)
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-1.0, 1.0, size=(count, 8))
    u_target = rng.normal(0.0, 0.1, size=(count, 3))
    return DiffBatch(x0=x0, Qdiag=np.ones((count, 8)), Rdiag=0.1 * np.ones((count, 3)),
                     A=np.broadcast_to(A, (count, 8, 8)).copy(),
                     Bm=np.broadcast_to(B, (count, 8, 3)).copy(),
                     u_target=u_target, N=N, K=K, rho=1.0, xbound=4.0, ubound=0.5)


# ---------------------------------------------------------------------------
# Cart-pole plant for real-time iteration
# ---------------------------------------------------------------------------

CARTPOLE = dict(M=1.0, m=0.1, l=0.5, g=9.81, dt=0.02)


def cartpole_f(x, u, M=1.0, m=0.1, l=0.5, g=9.81):
    """Frictionless cart-pole, state (p, pdot, th, thdot), th = 0 upright.
    The pole is a uniform rod of half-length l (pivot inertia 4/3 m l^2).
    Works on complex inputs (used for complex-step Jacobians)."""
    p, pd, th, thd = x[0], x[1], x[2], x[3]
    F = u[0]
    s, c = np.sin(th), np.cos(th)
    tot = M + m
    tmp = (F + m * l * thd * thd * s) / tot
    thdd = (g * s - c * tmp) / (l * (4.0 / 3.0 - m * c * c / tot))
    pdd = tmp - m * l * thdd * c / tot
    return np.array([pd, pdd, thd, thdd], dtype=np.result_type(x, u, 1.0))


def cartpole_fd(x, u, dt=0.02):
    """Forward-Euler discretisation x + dt f(x, u)."""
    return x + dt * cartpole_f(x, u)


def cartpole_jacobians(x, u, dt=0.02, h=1e-30):
    """Complex-step Jacobians of the Euler map (exact to rounding)."""
    n, mu = 4, 1
    A = np.zeros((n, n))
    B = np.zeros((n, mu))
    for j in range(n):
        xc = x.astype(np.complex128)
        xc[j] += 1j * h
        A[:, j] = np.imag(cartpole_fd(xc, u.astype(np.complex128), dt)) / h
    for j in range(mu):
        uc = u.astype(np.complex128)
        uc[j] += 1j * h
        B[:, j] = np.imag(cartpole_fd(x.astype(np.complex128), uc, dt)) / h
    return A, B


def cartpole_linearize(xs: np.ndarray, us: np.ndarray, dt=0.02, h=1e-30):
    """Stage data (A_k, B_k, e_k) of the Euler map linearised at the points
    (xs[k], us[k]), k = 0..N-1, with e_k = f_d(x_k, u_k) - A_k x_k - B_k u_k.
    The complex-step Jacobians of cartpole_jacobians, evaluated for all
    stages at once (the model works elementwise on (4, N) arrays)."""
    X = xs.T.astype(np.complex128)
    U = us.T.astype(np.complex128)
    N = xs.shape[0]
    A = np.zeros((N, 4, 4))
    B = np.zeros((N, 4, 1))
    for j in range(4):
        Xc = X.copy()
        Xc[j] += 1j * h
        A[:, :, j] = (np.imag(cartpole_fd(Xc, U, dt)) / h).T
    Uc = U.copy()
    Uc[0] += 1j * h
    B[:, :, 0] = (np.imag(cartpole_fd(X, Uc, dt)) / h).T
    fd = cartpole_fd(np.asarray(xs, np.float64).T, np.asarray(us, np.float64).T, dt).T
    e = fd - np.einsum("nij,nj->ni", A, xs) - np.einsum("nij,nj->ni", B, us)
    return A, B, e


def cartpole_rk4(x, u, dt=0.02, substeps=4):
    """Plant: fixed-step RK4 integration of the continuous cart-pole."""
    h = dt / substeps
    for _ in range(substeps):
        k1 = cartpole_f(x, u)
        k2 = cartpole_f(x + 0.5 * h * k1, u)
        k3 = cartpole_f(x + 0.5 * h * k2, u)
        k4 = cartpole_f(x + h * k3, u)
        x = x + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return x


def cartpole_problem(N: int = 256, K: int = 100) -> Problem:
    """Swing-up MPC data: x(0) = (0,0,pi,0), target 0, Q = diag(10,1,10,1),
    R = 0.01, |u| <= 10, unbounded states.  The stage matrices are the
    linearisation at x(0) repeated with u = 0 (first RTI step)."""
    x0 = np.array([0.0, 0.0, math.pi, 0.0])
    xs = np.broadcast_to(x0, (N, 4)).copy()
    us = np.zeros((N, 1))
    A, B, e = cartpole_linearize(xs, us)
    inf = np.inf
    return Problem(nx=4, nu=1, N=N, A=A, B=B, e=e, Q=np.diag([10.0, 1.0, 10.0, 1.0]),
                   R=np.array([[0.01]]), xmin=-inf * np.ones(4), xmax=inf * np.ones(4),
                   umin=np.array([-10.0]), umax=np.array([10.0]), x0=x0,
                   u_prev=np.zeros(1), rho=1.0, K=K)


def rti_shift(x_now: np.ndarray, xbar_pred: np.ndarray):
    """Linearisation points for the next RTI step from the previous predicted
    augmented trajectory xbar_pred[k] = col(x_{k+1}, u_k), k = 0..N-1:
    x_hat_0 = x(t), x_hat_k = x_{k+1}^{prev}, u_hat_k = u_{k+1}^{prev}
    (shift by one stage, last entry repeated)."""
    N = xbar_pred.shape[0]
    nx = x_now.shape[0]
    xs = np.empty((N, nx))
    us = np.empty((N, xbar_pred.shape[1] - nx))
    xs[0] = x_now
    for k in range(1, N):
        xs[k] = xbar_pred[k][:nx]
    for k in range(N):
        us[k] = xbar_pred[min(k + 1, N - 1)][nx:]
    return xs, us


# ---------------------------------------------------------------------------
# AFTI-16 (Section V-A), printed continuous-time model, ZOH at 0.05 s
# ---------------------------------------------------------------------------

def afti16(dt: float = 0.05):
    Ac = np.array([[-0.0151, -60.5651, 0.0, -32.174],
                   [-0.0001, -1.3411, 0.9929, 0.0],
                   [0.00018, 43.2541, -0.86939, 0.0],
                   [0.0, 0.0, 1.0, 0.0]])
    Bc = np.array([[-2.516, -13.136],
                   [-0.1689, -0.2514],
                   [-17.251, -1.5766],
                   [0.0, 0.0]])
    return zoh(Ac, Bc, dt)


def afti16_problem(N: int = 5, K: int = 500, rho: float = 10.0, pitch_ref: float = 10.0,
                   x0: Optional[np.ndarray] = None) -> Problem:
    """AFTI-16 tracking problem of Section V-A in the output form of eqn. (1):
    y = C x with C selecting the angle of attack (y_1) and the pitch angle
    (y_2), W_y = diag(100, 100), W_u = 0, W_du = diag(0.1, 0.1), |u_i| <= 25,
    -0.5 <= y_1 <= 0.5, -100 <= y_2 <= 100, reference y_2 -> pitch_ref.
    Not printed, so chosen here: the reference value, the initial state (0)
    and rho."""
    A, B = afti16()
    C = np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    return Problem(nx=4, nu=2, N=N, A=A, B=B, Q=np.zeros((4, 4)), R=np.zeros((2, 2)),
                   xmin=np.full(4, -np.inf), xmax=np.full(4, np.inf), umin=np.full(2, -25.0),
                   umax=np.full(2, 25.0), x0=np.zeros(4) if x0 is None else np.asarray(x0, np.float64),
                   u_prev=np.zeros(2), rho=rho, K=K, Wdu=np.diag([0.1, 0.1]), C=C,
                   Wy=np.diag([100.0, 100.0]), ry=np.array([0.0, pitch_ref]),
                   ymin=np.array([-0.5, -100.0]), ymax=np.array([0.5, 100.0]))


# ---------------------------------------------------------------------------
# Batch packing (flat arrays with per-instance offsets)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PackedBatch:
    """Instances packed back to back.  Per instance i: matrices at
    A[a_off[i]:], ..., one copy for time-invariant data (N copies otherwise).
    All arrays float64, row-major."""

    count: int
    nx: np.ndarray
    nu: np.ndarray
    N: np.ndarray
    time_varying: int
    A: np.ndarray
    B: np.ndarray
    e: Optional[np.ndarray]
    Q: np.ndarray
    R: np.ndarray
    xmin: np.ndarray
    xmax: np.ndarray
    umin: np.ndarray
    umax: np.ndarray
    x0: np.ndarray
    u_prev: np.ndarray


def pack(problems: Sequence[Problem]) -> PackedBatch:
    tv = int(any(p.time_varying or (p.e is not None and np.ndim(p.e) == 2) for p in problems))
    A, B, e, Q, R = [], [], [], [], []
    have_e = any(p.e is not None for p in problems)
    for p in problems:
        if tv:
            A.append(p.stage_A().ravel())
            B.append(p.stage_B().ravel())
            if have_e:
                e.append(p.stage_e().ravel())
        else:
            A.append(np.asarray(p.A, np.float64).ravel())
            B.append(np.asarray(p.B, np.float64).ravel())
            if have_e:
                e.append((np.zeros(p.nx) if p.e is None else np.asarray(p.e, np.float64)).ravel())
        Q.append(np.asarray(p.Q, np.float64).ravel())
        R.append(np.asarray(p.R, np.float64).ravel())
    cat = lambda xs: np.ascontiguousarray(np.concatenate(xs), dtype=np.float64)
    return PackedBatch(
        count=len(problems),
        nx=np.array([p.nx for p in problems], np.int32),
        nu=np.array([p.nu for p in problems], np.int32),
        N=np.array([p.N for p in problems], np.int32),
        time_varying=tv, A=cat(A), B=cat(B), e=cat(e) if have_e else None,
        Q=cat(Q), R=cat(R),
        xmin=cat([p.xmin for p in problems]), xmax=cat([p.xmax for p in problems]),
        umin=cat([p.umin for p in problems]), umax=cat([p.umax for p in problems]),
        x0=cat([p.x0 for p in problems]), u_prev=cat([p.u_prev for p in problems]))


# --------------------------------------------------------------------- CSTR
# Continuous stirred-tank reactor of Section V (online-linearised NMPC):
# state (C_A [kgmol/m^3], T [K]), input the coolant temperature T_c [K],
# output y = C_A.  Constants as printed; inlet temperature disturbance
# T_i(t) = 298.15 + 5 sin(0.05 t), t in minutes.
CSTR_CAI = 10.0
CSTR_K0 = 34930800.0
CSTR_EAR = 5963.6
CSTR_TS = 0.5


def cstr_ti(t_min: float) -> float:
    return 298.15 + 5.0 * math.sin(0.05 * t_min)


def cstr_f(x, u, Ti):
    """Right-hand side of the CSTR model (works on complex inputs)."""
    ca, T = x[0], x[1]
    kappa = CSTR_K0 * np.exp(-CSTR_EAR / T)
    return np.array([CSTR_CAI - ca - kappa * ca,
                     Ti + 0.3 * u[0] - 1.3 * T + 11.92 * kappa * ca], dtype=np.result_type(x, u, 1.0))


def cstr_linearize(x, u, Ti, dt=CSTR_TS, h=1e-30):
    """Forward-Euler map x + dt f(x, u) linearised at (x, u) by complex step:
    returns (A, B, e) with e = f_d(x, u) - A x - B u."""
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    fd = lambda xx, uu: xx + dt * cstr_f(xx, uu, Ti)
    A = np.zeros((2, 2))
    B = np.zeros((2, 1))
    for j in range(2):
        xc = x.astype(np.complex128)
        xc[j] += 1j * h
        A[:, j] = np.imag(fd(xc, u.astype(np.complex128))) / h
    uc = u.astype(np.complex128)
    uc[0] += 1j * h
    B[:, 0] = np.imag(fd(x.astype(np.complex128), uc)) / h
    e = fd(x, u) - A @ x - B @ u
    return A, B, e


def cstr_plant(x, u, t_min, dt=CSTR_TS, substeps=20):
    """Plant: RK4 integration of the continuous model over one sample, with
    the inlet disturbance evaluated along the way."""
    h = dt / substeps
    t = t_min
    for _ in range(substeps):
        k1 = cstr_f(x, u, cstr_ti(t))
        k2 = cstr_f(x + 0.5 * h * k1, u, cstr_ti(t + 0.5 * h))
        k3 = cstr_f(x + 0.5 * h * k2, u, cstr_ti(t + 0.5 * h))
        k4 = cstr_f(x + h * k3, u, cstr_ti(t + h))
        x = x + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        t += h
    return x


CSTR_X0 = np.array([8.57, 311.0])
CSTR_REF = 2.0


def cstr_steady_input(x) -> float:
    """Coolant temperature that holds dT/dt = 0 at state x (T_i nominal)."""
    ca, T = x
    kappa = CSTR_K0 * math.exp(-CSTR_EAR / T)
    return (1.3 * T - 298.15 - 11.92 * kappa * ca) / 0.3


def cstr_problem(N: int = 5000, K: int = 1000, rho: float = 1.0, t_min: float = 0.0,
                 x=None, u_prev=None) -> Problem:
    """CSTR tracking MPC in the form of eqn. (1): W_y = 1 on y = C_A (so
    Q = diag(1, 0) and qbar = (W_y r_y, 0, 0) with r_y = 2), W_u = 0,
    W_du = 0.1, horizon N.  The stage data are the Euler linearisation at
    (x, u_prev) (same for every stage).  Bounds (not printed in the paper):
    0 <= C_A <= 10, T unbounded, 280 K <= T_c <= 330 K."""
    x = CSTR_X0.copy() if x is None else np.asarray(x, np.float64)
    u_prev = np.array([cstr_steady_input(CSTR_X0)]) if u_prev is None else np.asarray(u_prev, np.float64)
    A, B, e = cstr_linearize(x, u_prev, cstr_ti(t_min))
    inf = np.inf
    return Problem(nx=2, nu=1, N=N, A=A, B=B, e=e, Q=np.diag([1.0, 0.0]), R=np.zeros((1, 1)),
                   qbar=np.array([CSTR_REF, 0.0, 0.0]), Wdu=np.array([[0.1]]),
                   xmin=np.array([0.0, -inf]), xmax=np.array([10.0, inf]),
                   umin=np.array([280.0]), umax=np.array([330.0]), x0=x, u_prev=u_prev, rho=rho, K=K)
