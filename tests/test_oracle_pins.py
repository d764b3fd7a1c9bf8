"""Pins of the CPU oracle against what the paper and the mathematics fix.

The paper prints no iterates, so every pin is a definition written out in a
different form (dense F, G, h of the splitting), a textbook special case
(LQR, equality-constrained KKT), an independent algorithm with the same
optimum (the general-QP ADMM of eqn. (3)) or an invariant (the monotone c of
Section IV-B's second lemma).  Each test says which passage it pins.
"""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import workloads as W

import _refs


def tiny_tv_problem(seed, n=3, m=2, N=5, bounded=True, affine=True):
    """Small time-varying affine instance (random A_k, B_k, e_k)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, n, n)) * 0.5
    B = rng.standard_normal((N, n, m))
    e = rng.standard_normal((N, n)) * 0.3 if affine else None
    Qh = rng.standard_normal((n, n))
    Rh = rng.standard_normal((m, m))
    Q = Qh @ Qh.T / n + 0.5 * np.eye(n)
    R = Rh @ Rh.T / m + 0.2 * np.eye(m)
    xb = 0.6 if bounded else np.inf
    ubd = 0.3 if bounded else np.inf
    qbar = rng.standard_normal(n + m) * 0.2
    return W.Problem(nx=n, nu=m, N=N, A=A, B=B, e=e, Q=Q, R=R, qbar=qbar,
                     xmin=-xb * np.ones(n), xmax=xb * np.ones(n),
                     umin=-ubd * np.ones(m), umax=ubd * np.ones(m),
                     x0=rng.uniform(-1, 1, n), u_prev=rng.uniform(-0.2, 0.2, m), rho=1.3, K=50)


def random_state(p, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((5, p.N, p.nx + p.nu)) * 0.5


# --- one iteration vs the three ADMM blocks written densely (eqn. (9) form) ---

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p_update_equals_dense_subproblem(seed):
    """Step 1 (eqn. (8), first block): the stage closed forms (du_k, xbar_{k+1})
    equal the dense minimiser of f(p) + rho/2||Fp + Gq - h + s||^2 over the
    whole horizon -- the decoupling claim of Section IV."""
    p = tiny_tv_problem(seed)
    st0 = random_state(p, 100 + seed)
    r = oracle.solve(p, K=1, state=st0)
    D = _refs.velocity_dense(p)
    q, s = _refs.state_to_qs(st0)
    pv = _refs.p_subproblem(D, p.rho, q, s)
    N, m, nb = p.N, p.nu, p.nb
    np.testing.assert_allclose(r["du"].ravel(), pv[: N * m], rtol=0, atol=1e-11)
    np.testing.assert_allclose(r["xs"].ravel(), pv[N * m:], rtol=0, atol=1e-11)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_q_update_equals_bounded_least_squares(seed):
    """Step 2 (Theorem 1): (v, z) equals the bounded least-squares minimiser of
    I_box(z) + rho/2||F p^{i+1} + G q - h + s^i||^2 -- the constrained
    sub-problem itself, solved by scipy's BVLS, not by the closed form."""
    p = tiny_tv_problem(seed)
    st0 = random_state(p, 200 + seed) * 2.0
    r = oracle.solve(p, K=1, state=st0)
    D = _refs.velocity_dense(p)
    q0, s0 = _refs.state_to_qs(st0)
    pv = np.concatenate([r["du"].ravel(), r["xs"].ravel()])
    qv = _refs.q_subproblem(D, p.rho, pv, s0)
    q1, _ = _refs.state_to_qs(r["state"])
    # some z components must be at a bound for the test to exercise the projection
    z = r["state"][1]
    assert np.any(np.isclose(z, p.lb()[None, :])) or np.any(np.isclose(z, p.ub()[None, :]))
    np.testing.assert_allclose(q1, qv, rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_dual_update_and_residual_definitions(seed):
    """Step 3 and the residuals of Section IV-B: s^{i+1} = s^i + F p + G q - h;
    r_prim = ||F p + G q - h||_inf; r_dual = rho ||F'G(q^{i+1} - q^i)||_inf;
    c^{i+1} = rho ||s^{i+1}-s^i||^2 + rho ||G(q^{i+1}-q^i)||^2."""
    p = tiny_tv_problem(seed)
    st0 = random_state(p, 300 + seed)
    r = oracle.solve(p, K=1, state=st0)
    D = _refs.velocity_dense(p)
    F, G, h = D["F"], D["G"], D["h"]
    q0, s0 = _refs.state_to_qs(st0)
    q1, s1 = _refs.state_to_qs(r["state"])
    pv = np.concatenate([r["du"].ravel(), r["xs"].ravel()])
    prim = F @ pv + G @ q1 - h
    np.testing.assert_allclose(s1, s0 + prim, rtol=0, atol=1e-12)
    c, rp, rd, _ = r["hist"][0]
    dq = q1 - q0
    assert rp == pytest.approx(np.max(np.abs(prim)), rel=1e-12, abs=1e-14)
    assert rd == pytest.approx(p.rho * np.max(np.abs(F.T @ G @ dq)), rel=1e-12, abs=1e-14)
    c_dense = p.rho * np.sum((s1 - s0) ** 2) + p.rho * np.sum((G @ dq) ** 2)
    assert c == pytest.approx(c_dense, rel=1e-12)


def _rate_weight(seed, m):
    rng = np.random.default_rng(50 + seed)
    Wh = rng.standard_normal((m, m))
    return Wh @ Wh.T / m + 0.1 * np.eye(m)


@pytest.mark.parametrize("seed", [0, 1])
def test_p_update_with_rate_weight_equals_dense_subproblem(seed):
    """With the input-rate weight of Section V the du block of the first ADMM
    sub-problem gains 1/2 du'W du; the oracle's stage closed forms must still
    equal the dense minimiser over the whole horizon."""
    p = tiny_tv_problem(seed)
    p = p.copy(Wdu=_rate_weight(seed, p.nu))
    st0 = random_state(p, 150 + seed)
    r = oracle.solve(p, K=1, state=st0)
    D = _refs.velocity_dense(p)
    q, s = _refs.state_to_qs(st0)
    pv = _refs.p_subproblem(D, p.rho, q, s)
    N, m = p.N, p.nu
    np.testing.assert_allclose(r["du"].ravel(), pv[: N * m], rtol=0, atol=1e-11)
    np.testing.assert_allclose(r["xs"].ravel(), pv[N * m:], rtol=0, atol=1e-11)


@pytest.mark.parametrize("seed", [0, 1])
def test_rate_weight_fixed_point_is_kkt(seed):
    """Time-varying affine data, no active bounds, input-rate weight and
    u(t-1) != 0: the fixed point equals the KKT solution of problem (1) with
    the rate term sum_k 1/2 (u_k - u_{k-1})'W(u_k - u_{k-1}) added."""
    p = tiny_tv_problem(seed, bounded=False)
    p = p.copy(qbar=None, Wdu=_rate_weight(seed, p.nu))
    r = oracle.solve(p, K=80000, eps=1e-28)
    xs_k, us_k = _refs.eq_qp_original(p)
    np.testing.assert_allclose(r["xs"][:, :p.nx], xs_k, rtol=0, atol=1e-8)
    np.testing.assert_allclose(r["xs"][:, p.nx:], us_k, rtol=0, atol=1e-8)
    # the rate weight changes the optimum (so the test sees it)
    xs_0, us_0 = _refs.eq_qp_original(p.copy(Wdu=None))
    assert np.max(np.abs(us_0 - us_k)) > 1e-3


# --- fixed points ------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_unconstrained_fixed_point_is_lqr(seed):
    """With no active constraints the MPC problem is a finite-horizon LQR
    (Section III-B); the converged oracle must reproduce the Riccati solution."""
    p = W.plain_fp64_problem(seed)
    p = p.copy(N=8, xmin=-np.inf * np.ones(8), xmax=np.inf * np.ones(8),
               umin=-np.inf * np.ones(3), umax=np.inf * np.ones(3))
    r = oracle.solve(p, K=40000, eps=1e-26)
    xs_l, us_l = _refs.lqr(p.A, p.B, p.Q, p.R, p.x0, p.N)
    xbar = r["xs"]
    np.testing.assert_allclose(xbar[:, :p.nx], xs_l, rtol=0, atol=1e-9)
    np.testing.assert_allclose(xbar[:, p.nx:], us_l, rtol=0, atol=1e-9)
    np.testing.assert_allclose(r["u0"], us_l[0], rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_time_varying_affine_fixed_point_is_kkt(seed):
    """Time-varying A_k, B_k and affine e_k, no active bounds: the fixed point
    must equal the KKT solution of the equality-constrained QP (1).  This pins
    reading R1 (h_k uses Abar_{k+1}, ebar_{k+1}); the index-k reading printed
    in Algorithm 1 converges to a different point on such data."""
    p = tiny_tv_problem(seed, bounded=False)
    p = p.copy(qbar=None)
    r = oracle.solve(p, K=60000, eps=1e-28)
    xs_k, us_k = _refs.eq_qp_original(p)
    np.testing.assert_allclose(r["xs"][:, :p.nx], xs_k, rtol=0, atol=1e-8)
    np.testing.assert_allclose(r["xs"][:, p.nx:], us_k, rtol=0, atol=1e-8)


def _u_bound_case(seed):
    """4-state spring pair, input bound active (|u| <= 0.15)."""
    A, B = W.mass_spring(2)
    rng = np.random.default_rng(seed)
    return W.Problem(nx=4, nu=1, N=6, A=A, B=B, Q=np.eye(4), R=0.1 * np.eye(1),
                     xmin=-1.5 * np.ones(4), xmax=1.5 * np.ones(4), umin=-0.15 * np.ones(1),
                     umax=0.15 * np.ones(1), x0=rng.uniform(-0.9, 0.9, 4), u_prev=np.zeros(1),
                     rho=1.0, K=0)


def _x_bound_case(seed):
    """Fully actuated 2-state system; state bound set at 85% of the
    unconstrained (LQR) excursion so that state bounds are active."""
    rng = np.random.default_rng(seed)
    A = np.array([[1.05, 0.2], [0.0, 1.05]]) + 0.05 * rng.standard_normal((2, 2))
    B = np.eye(2) + 0.1 * rng.standard_normal((2, 2))
    x0 = np.array([0.9, 0.8]) + 0.05 * rng.standard_normal(2)
    Q, R = 0.05 * np.eye(2), np.eye(2)
    xl, _ = _refs.lqr(A, B, Q, R, x0, 6)
    xmax = 0.85 * np.max(np.abs(xl), axis=0)
    return W.Problem(nx=2, nu=2, N=6, A=A, B=B, Q=Q, R=R, xmin=-xmax, xmax=xmax,
                     umin=-2.0 * np.ones(2), umax=2.0 * np.ones(2), x0=x0, u_prev=np.zeros(2),
                     rho=1.0, K=0)


def _u_bound_rate_case(seed):
    """The input-bound case with an input-rate weight and u(t-1) != 0, so the
    rate term couples u_0 to u(t-1) and the bound is still active."""
    p = _u_bound_case(seed)
    return p.copy(Wdu=0.5 * np.eye(1), u_prev=np.array([0.1]))


@pytest.mark.parametrize("case,seed", [("u", 0), ("u", 1), ("x", 0), ("x", 1), ("uw", 0), ("uw", 1)])
def test_constrained_fixed_point_matches_qp_admm(case, seed):
    """Active bounds: the converged oracle equals the optimum found by the
    general-QP ADMM of eqn. (3) (an independent algorithm on the sparse QP
    (2)), whose own convergence, feasibility and KKT conditions are checked.
    Case "uw" adds the input-rate weight of Section V."""
    p = {"u": _u_bound_case, "x": _x_bound_case, "uw": _u_bound_rate_case}[case](seed)
    ref = _refs.qp_admm(p, rho=1.0, iters=100000, tol=1e-13)
    assert ref["iters"] < 100000
    E, y, w = ref["E"], ref["y"], ref["w"]
    assert np.max(np.abs(E @ y - w)) < 1e-11
    mu = ref["rho"] * ref["lam"]
    assert np.max(np.abs(ref["H"] @ y + ref["f"] + E.T @ mu)) < 1e-9
    at_lo = np.isclose(w, ref["Ylo"], atol=1e-10)
    at_hi = np.isclose(w, ref["Yhi"], atol=1e-10)
    free = ~(at_lo | at_hi)
    assert np.all(np.abs(mu[free]) < 1e-8)
    assert np.all(mu[at_hi & ~at_lo] > -1e-8) and np.all(mu[at_lo & ~at_hi] < 1e-8)
    box = slice(p.N * p.nx, None)
    nact = np.sum((at_hi | at_lo)[box])
    assert nact >= 2, "this case must have active bounds"
    r = oracle.solve(p, K=100000, eps=1e-26)
    assert r["hist"][-1][0] <= 1e-26
    np.testing.assert_allclose(r["xs"][:, :p.nx], ref["xs"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(r["xs"][:, p.nx:], ref["us"], rtol=0, atol=1e-10)


@pytest.mark.parametrize("case,seed", [("u", 0), ("x", 1), ("uw", 0), ("tv", 2)])
def test_interior_point_reference_equals_qp_admm_and_oracle(case, seed):
    """The interior-point reference (`_refs.ipm_qp`, Mehrotra predictor-
    corrector on the sparse QP (2)), used for the converged-mode checks of
    long horizons, reaches the same optimum as the general-QP ADMM and as the
    converged oracle, with active bounds, the input-rate weight, and
    time-varying affine data with a linear cost term."""
    if case == "tv":
        p = tiny_tv_problem(seed, bounded=True)
    else:
        p = {"u": _u_bound_case, "x": _x_bound_case, "uw": _u_bound_rate_case}[case](seed)
    ip = _refs.ipm_qp(p)
    assert ip["ok"] and ip["kkt"] <= 1e-12
    r = oracle.solve(p, K=200000, eps=1e-26)
    assert r["hist"][-1][0] <= 1e-26
    np.testing.assert_allclose(ip["xs"], r["xs"][:, :p.nx], rtol=0, atol=1e-9)
    np.testing.assert_allclose(ip["us"], r["xs"][:, p.nx:], rtol=0, atol=1e-9)
    if case != "tv":
        ref = _refs.qp_admm(p, rho=1.0, iters=100000, tol=1e-13)
        np.testing.assert_allclose(ip["us"], ref["us"], rtol=0, atol=1e-9)


def test_optimum_invariant_to_rho_and_uprev():
    """The minimiser of (1) depends on neither the ADMM penalty rho nor on
    u(t-1) (no input-rate weight): every run converges to the same U."""
    base = W.plain_fp64_problem(3).copy(N=10)
    sols = []
    for rho, up in [(1.0, np.zeros(3)), (0.5, np.zeros(3)), (2.5, np.array([0.3, -0.2, 0.1]))]:
        p = base.copy(rho=rho, u_prev=up)
        r = oracle.solve(p, K=60000, eps=1e-24)
        sols.append(r["xs"][:, p.nx:].copy())
    np.testing.assert_allclose(sols[1], sols[0], atol=1e-7)
    np.testing.assert_allclose(sols[2], sols[0], atol=1e-7)


# --- invariants ---------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_c_monotone_plain_admm(seed):
    """Second lemma of Section IV-B: c^{i+1} <= c^i for plain (scaled) ADMM."""
    p = W.plain_fp64_problem(seed)
    r = oracle.solve(p, K=400)
    c = r["hist"][:, 0]
    assert np.all(c[1:] <= c[:-1] * (1 + 1e-9) + 1e-300)


def test_stop_rule_and_accel_restart():
    """Steps 5-7 of Algorithm 1: eps stop ends at the first c <= eps; the
    restart-accelerated run reaches the same c level in fewer iterations and
    reaches the same optimum."""
    p = W.plain_fp64_problem(0)
    eps = 1e-8
    r_plain = oracle.solve(p, K=20000, eps=eps)
    r_acc = oracle.solve(p, K=20000, eps=eps, accel=True)
    for r in (r_plain, r_acc):
        c = r["hist"][:, 0]
        assert c[-1] <= eps and np.all(c[:-1] > eps)
    assert r_acc["iters"] < r_plain["iters"]
    assert r_acc["hist"][:, 3].sum() >= 1  # at least one restart happened
    np.testing.assert_allclose(r_acc["xs"], r_plain["xs"], atol=1e-3)


@pytest.mark.parametrize("seed", [1, 4])
def test_accel_restart_iterates_equal_dense_algorithm(seed):
    """Steps 6-7 of Algorithm 1, iterate by iterate: the oracle's accelerated
    run equals Algorithm 1 carried out on the dense splitting (dense p
    sub-problem, BVLS q sub-problem, s update and c from F, G, h) for 300
    iterations on a time-varying affine instance with active bounds: the same
    restart decisions, the same c^{i+1} and the same iterate after every
    iteration.  Three plausible misreadings of the steps (momentum
    coefficient (alpha_{i+1} - 1) / alpha_{i+1}, a restart to the previous
    iterate as in the pseudo-code (11), c^i kept on a restart) are shown to
    leave this agreement, so the pin can tell them apart."""
    p = tiny_tv_problem(seed, n=2, m=1, N=3)
    K = 300
    ref = _refs.accel_admm_dense(p, K)
    run = oracle.solve(p, K=K, accel=True)
    assert run["iters"] == K
    flags = run["hist"][:, 3].astype(int)
    assert flags.sum() >= 3, "the instance must restart several times"
    assert np.any(flags[:50] == 0), "and extrapolate between restarts"
    np.testing.assert_array_equal(flags, ref["restart"])
    # every decision is taken with a margin far above rounding
    c_prev = np.concatenate([[1.0], ref["c"][:-1]])
    assert np.min(np.abs(ref["c"] - ref["eta"] * c_prev) / ref["c"]) > 1e-5
    np.testing.assert_allclose(run["hist"][:, 0], ref["c"], rtol=1e-6, atol=1e-20)
    for i in range(K):
        st = oracle.solve(p, K=i + 1, accel=True)["state"]
        q, s = _refs.state_to_qs(st)
        np.testing.assert_allclose(q, ref["q"][i], rtol=0, atol=1e-10, err_msg=f"q after {i + 1}")
        np.testing.assert_allclose(s, ref["s"][i], rtol=0, atol=1e-10, err_msg=f"s after {i + 1}")


@pytest.mark.parametrize("variant", ["coef_next", "restart_prev", "cprev_kept"])
def test_accel_pin_tells_misreadings_apart(variant):
    """Each misreading of steps 6-7 changes the restart decisions or the
    iterates of at least one instance of the pin above by far more than its
    tolerance, so that pin would fail on an oracle built that way."""
    K = 300
    gaps = []
    for seed in (1, 4):
        p = tiny_tv_problem(seed, n=2, m=1, N=3)
        ref = _refs.accel_admm_dense(p, K)
        bad = _refs.accel_admm_dense(p, K, variant=variant)
        gap = max(np.max(np.abs(bad["q"][i] - ref["q"][i])) for i in range(K))
        gaps.append(gap > 1e-4 or not np.array_equal(bad["restart"], ref["restart"]))
    assert any(gaps), variant


def test_residuals_at_fixed_iterations_plain_fp64_problem():
    """Reference levels at the fixed 200 iterations of the 4-mass problem: the
    iteration is not converged there (r_prim ~ 1e-2), which is why GPU parity
    is checked iterate-by-iterate and not against the optimum."""
    r = oracle.solve(W.plain_fp64_problem(0))
    c, rp, rd, _ = r["hist"][-1]
    assert 1e-3 < rp < 1e-1 and 1e-4 < rd < 1e-1


# --- adjoint vs central finite differences -------------------------------------

def _loss_and_grad_fd(nx, nu, N, A, B, Qd, Rd, lb, ub, x0, rho, K, ut, h=1e-6, Wdu=None):
    def loss(A_, B_, Qd_, Rd_, x0_):
        p = W.Problem(nx=nx, nu=nu, N=N, A=A_, B=B_, Q=np.diag(Qd_), R=np.diag(Rd_),
                      xmin=lb[:nx], xmax=ub[:nx], umin=lb[nx:], umax=ub[nx:], x0=x0_,
                      u_prev=np.zeros(nu), rho=rho, K=K, Wdu=Wdu)
        u0 = oracle.solve(p)["u0"]
        return float(np.sum((u0 - ut) ** 2))

    params = dict(A=A, B=B, Qd=Qd, Rd=Rd, x0=x0)
    grads = {}
    for name, val in params.items():
        g = np.zeros_like(val)
        for idx in np.ndindex(val.shape):
            vp = val.copy(); vp[idx] += h
            vm = val.copy(); vm[idx] -= h
            args_p = {**params, name: vp}
            args_m = {**params, name: vm}
            g[idx] = (loss(args_p["A"], args_p["B"], args_p["Qd"], args_p["Rd"], args_p["x0"]) -
                      loss(args_m["A"], args_m["B"], args_m["Qd"], args_m["Rd"], args_m["x0"])) / (2 * h)
        grads[name] = g
    return grads


@pytest.mark.parametrize("seed,masses,rho,rate", [(0, 2, 1.0, False), (1, 2, 1.0, False),
                                                  (2, 3, 1.7, True)])
def test_oracle_adjoint_matches_finite_differences(seed, masses, rho, rate):
    """Reverse mode through the unrolled iteration (differentiable layer)
    equals central differences (h = 1e-6, FP64) of the oracle's own loss;
    the last case adds a fixed input-rate weight and rho != 1."""
    rng = np.random.default_rng(seed)
    A, B = W.mass_spring(masses)
    nx, nu, N, K = 2 * masses, masses - 1, 6, 25
    Wdu = _rate_weight(seed, nu) if rate else None
    Qd = rng.uniform(0.5, 1.5, nx)
    Rd = rng.uniform(0.05, 0.2, nu)
    x0 = rng.uniform(-1, 1, nx)
    lb = np.concatenate([-1.0 * np.ones(nx), -0.3 * np.ones(nu)])
    ub = -lb
    ut = rng.normal(0, 0.1, nu)
    p = W.Problem(nx=nx, nu=nu, N=N, A=A, B=B, Q=np.diag(Qd), R=np.diag(Rd), xmin=lb[:nx],
                  xmax=ub[:nx], umin=lb[nx:], umax=ub[nx:], x0=x0, u_prev=np.zeros(nu),
                  rho=rho, K=K, Wdu=Wdu)
    u0 = oracle.solve(p)["u0"]
    g = oracle.grad(nx, nu, N, A, B, Qd, Rd, lb, ub, x0, rho, K, 2 * (u0 - ut), Wdu=Wdu)
    np.testing.assert_allclose(g["u0"], u0, atol=1e-14)
    fd = _loss_and_grad_fd(nx, nu, N, A, B, Qd, Rd, lb, ub, x0, rho, K, ut, Wdu=Wdu)
    for name, key in [("A", "dA"), ("B", "dB"), ("Qd", "dQd"), ("Rd", "dRd"), ("x0", "dx0")]:
        np.testing.assert_allclose(g[key], fd[name], rtol=1e-5, atol=1e-7, err_msg=name)


def _mixed_output_problem(seed):
    """Outputs that mix states (general C, no bounds on them), an output and
    an input reference, a small state weight, active input bounds."""
    rng = np.random.default_rng(seed)
    A, B = W.mass_spring(2)
    C = rng.standard_normal((3, 4))
    Wy = np.diag(rng.uniform(0.5, 2.0, 3))
    return W.Problem(nx=4, nu=1, N=8, A=A, B=B, Q=0.05 * np.eye(4), R=0.1 * np.eye(1),
                     xmin=np.full(4, -3.0), xmax=np.full(4, 3.0), umin=np.full(1, -0.3), umax=np.full(1, 0.3),
                     x0=rng.uniform(-1, 1, 4), u_prev=np.zeros(1), rho=1.0, K=0, C=C, Wy=Wy,
                     ry=rng.uniform(-0.5, 0.5, 3), ru=np.array([0.1]))


@pytest.mark.parametrize("case", ["afti_N5", "afti_N30", "mixed0", "mixed1"])
def test_output_form_fixed_point_equals_interior_point(case):
    """Eqn. (1) with an output matrix C, output weight, references and output
    bounds: the oracle (which folds them into Q, qbar and the state box) at
    its fixed point equals the interior-point optimum of the QP written with
    the outputs as variables of their own (w_k = C x_{k+1}, bounds on w)."""
    if case.startswith("afti"):
        N = int(case[6:])
        p = W.afti16_problem(N=N, rho=10.0 if N == 5 else 100.0)
    else:
        p = _mixed_output_problem(int(case[-1]))
    ip = _refs.ipm_qp(p)
    assert ip["ok"] and ip["kkt"] <= 1e-12
    r = oracle.solve(p, K=300000, eps=1e-22)
    assert r["hist"][-1][0] <= 1e-22
    np.testing.assert_allclose(r["xs"][:, p.nx:], ip["us"], rtol=0, atol=1e-7)
    np.testing.assert_allclose(r["xs"][:, :p.nx], ip["xs"], rtol=0, atol=1e-7)
    if case.startswith("afti"):
        # the angle-of-attack bound y_1 <= 0.5 and the input bounds are active
        assert np.any(np.isclose(ip["xs"][:, 1], 0.5, atol=1e-8))
        assert np.any(np.isclose(np.abs(ip["us"]), 25.0, atol=1e-8))
