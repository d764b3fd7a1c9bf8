"""Pins of the oracle's non-box constraint sets (the closed convex sets the
proof of Theorem 1 lists besides the box: halfspace, affine hyperplane,
second-order cone, l1 ball), each checked against something independent of
the oracle's projection code:

  * the defining property of a Euclidean projection P onto a closed convex
    set C: P(y) is in C and (y - P(y))'(w - P(y)) <= 0 for every w in C
    (checked on many feasible w);
  * Moreau's decomposition for the self-dual second-order cone:
    y = P_K(y) - P_K(-y);
  * an independent bisection for the l1-ball threshold;
  * the ADMM q sub-problem and the fixed point of a small MPC problem with
    such sets, each solved by scipy's SLSQP on the problem itself.
"""
import numpy as np
import pytest
import scipy.optimize

import oracle
from paper_2601_14414_amd import workloads as W

import _refs


def in_set(spec, w, tol=1e-10):
    kind = spec[0]
    if kind == "halfspace":
        return np.dot(spec[1], w) <= spec[2] + tol
    if kind == "hyperplane":
        return abs(np.dot(spec[1], w) - spec[2]) <= tol
    if kind == "soc":
        return np.linalg.norm(w[:-1]) <= w[-1] + tol
    if kind == "l1ball":
        return np.sum(np.abs(w)) <= spec[1] + tol
    raise ValueError(kind)


def feasible_points(spec, n, rng, count=200):
    """Points of the set drawn independently of the projection code."""
    pts = []
    kind = spec[0]
    while len(pts) < count:
        w = rng.standard_normal(n) * 2.0
        if kind == "halfspace":
            a, b = np.asarray(spec[1]), spec[2]
            s = a @ w - b
            if s > 0:
                w = w - (s + rng.uniform(0, 1)) * a / (a @ a)
        elif kind == "hyperplane":
            a, b = np.asarray(spec[1]), spec[2]
            w = w - (a @ w - b) * a / (a @ a)
        elif kind == "soc":
            w[-1] = np.linalg.norm(w[:-1]) + abs(rng.standard_normal())
        elif kind == "l1ball":
            w = w / np.sum(np.abs(w)) * spec[1] * rng.uniform(0, 1)
        assert in_set(spec, w, 1e-9)
        pts.append(w)
    return pts


SPECS = [("halfspace", [1.0, -2.0, 0.5], 0.3), ("hyperplane", [0.5, 1.5, -1.0], -0.2), ("soc",),
         ("l1ball", 1.3)]


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: s[0])
def test_projection_variational_inequality(spec):
    rng = np.random.default_rng(5)
    feas = feasible_points(spec, 3, rng)
    inside = 0
    for _ in range(300):
        y = rng.standard_normal(3) * 3.0
        p = oracle.project(spec, y)
        assert in_set(spec, p), (y, p)
        g = y - p
        worst = max(float(g @ (w - p)) for w in feas)
        assert worst <= 1e-10 * max(1.0, np.linalg.norm(g)), (y, p, worst)
        inside += int(np.allclose(p, y))
    # both branches (already inside / projected) are exercised
    assert 0 < inside < 300 or spec[0] == "hyperplane"


def test_soc_moreau_decomposition():
    """The second-order cone is self-dual, so y = P_K(y) - P_K(-y) and the two
    parts are orthogonal."""
    rng = np.random.default_rng(6)
    for n in (2, 3, 5):
        for _ in range(200):
            y = rng.standard_normal(n) * 2.0
            p, q = oracle.project(("soc",), y), oracle.project(("soc",), -y)
            np.testing.assert_allclose(p - q, y, atol=1e-12)
            assert abs(p @ q) <= 1e-11


def test_l1_threshold_matches_bisection():
    """Outside the ball the projection is a soft threshold at theta with
    sum max(|y_i| - theta, 0) = r; theta found here by bisection."""
    rng = np.random.default_rng(7)
    for n in (1, 2, 4, 9):
        for _ in range(100):
            y = rng.standard_normal(n) * 2.0
            y[rng.integers(0, n)] = y[0]  # ties
            r = rng.uniform(0.1, 2.0)
            p = oracle.project(("l1ball", r), y)
            if np.sum(np.abs(y)) <= r:
                np.testing.assert_array_equal(p, y)
                continue
            lo, hi = 0.0, float(np.max(np.abs(y)))
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if np.sum(np.maximum(np.abs(y) - mid, 0.0)) > r:
                    lo = mid
                else:
                    hi = mid
            ref = np.sign(y) * np.maximum(np.abs(y) - 0.5 * (lo + hi), 0.0)
            np.testing.assert_allclose(p, ref, atol=1e-12)


def set_problem(seed, xset=None, uset=None, N=3):
    rng = np.random.default_rng(seed)
    n, m = 3, 3
    A = np.eye(n) + 0.2 * rng.standard_normal((n, n))
    B = rng.standard_normal((n, m)) * 0.7
    inf = np.inf
    return W.Problem(nx=n, nu=m, N=N, A=A, B=B, Q=np.eye(n), R=0.2 * np.eye(m),
                     xmin=-inf * np.ones(n), xmax=inf * np.ones(n), umin=-inf * np.ones(m),
                     umax=inf * np.ones(m), x0=np.array([1.5, -1.0, 0.8]), u_prev=np.zeros(m),
                     rho=1.1, K=1, xset=xset, uset=uset)


def slsqp_constraints(spec, sl):
    """scipy constraint dicts restricting vector slice `sl` to the set."""
    kind = spec[0]
    if kind == "halfspace":
        a, b = np.asarray(spec[1]), spec[2]
        return [{"type": "ineq", "fun": lambda v: b - a @ v[sl], "jac": None}]
    if kind == "hyperplane":
        a, b = np.asarray(spec[1]), spec[2]
        return [{"type": "eq", "fun": lambda v: a @ v[sl] - b}]
    if kind == "soc":
        return [{"type": "ineq", "fun": lambda v: v[sl][-1] - np.sqrt(np.sum(v[sl][:-1] ** 2) + 1e-300)}]
    if kind == "l1ball":
        return [{"type": "ineq", "fun": lambda v: spec[1] - np.sum(np.abs(v[sl]))}]
    raise ValueError(kind)


CASES = [(("halfspace", [1.0, 1.0, 1.0], 0.4), None), (None, ("soc",)), (None, ("l1ball", 0.5)),
         (("hyperplane", [1.0, -1.0, 0.5], 0.2), ("halfspace", [1.0, 0.0, 1.0], 0.1))]


@pytest.mark.parametrize("xset,uset", CASES)
def test_q_update_equals_constrained_least_squares(xset, uset):
    """Step 2 with a non-box set: (v, z) equals the minimiser of
    I_Xbar(z) + rho/2 ||F p + G q - h + s||^2 found by SLSQP on the
    sub-problem itself (z_k constrained to X x U for every stage)."""
    p = set_problem(3, xset, uset)
    rng = np.random.default_rng(11)
    st0 = rng.standard_normal((5, p.N, p.nb)) * 1.5
    r = oracle.solve(p, K=1, state=st0)
    D = _refs.velocity_dense(p)
    F, G, h = D["F"], D["G"], D["h"]
    q0, s0 = _refs.state_to_qs(st0)
    pv = np.concatenate([r["du"].ravel(), r["xs"].ravel()])
    target = h - F @ pv - s0
    N, nb, n = p.N, p.nb, p.nx
    cons = []
    for k in range(N):
        base = N * nb + k * nb  # z_{k+1} inside q
        if xset is not None:
            cons += slsqp_constraints(xset, slice(base, base + n))
        if uset is not None:
            cons += slsqp_constraints(uset, slice(base + n, base + nb))
    fun = lambda q: 0.5 * np.sum((G @ q - target) ** 2)
    jac = lambda q: G.T @ (G @ q - target)
    q1, _ = _refs.state_to_qs(r["state"])
    # optimality of the oracle's point: feasible, zero gradient in the free v
    # part, and the variational inequality grad'(w - q1) >= 0 over feasible z
    gr = jac(q1)
    np.testing.assert_allclose(gr[: N * nb], 0.0, atol=1e-10)
    z1 = q1[N * nb:].reshape(N, nb)
    feas = {}
    for k in range(N):
        if xset is not None:
            assert in_set(xset, z1[k, :n])
            feas.setdefault("x", feasible_points(xset, n, rng, 100))
        if uset is not None:
            assert in_set(uset, z1[k, n:])
            feas.setdefault("u", feasible_points(uset, nb - n, rng, 100))
    gz = gr[N * nb:].reshape(N, nb)
    for k in range(N):
        for key, sl in (("x", slice(0, n)), ("u", slice(n, nb))):
            if key in feas:
                worst = min(float(gz[k, sl] @ (w - z1[k, sl])) for w in feas[key])
                assert worst >= -1e-9 * max(1.0, np.linalg.norm(gz[k, sl])), (k, key, worst)
            else:
                np.testing.assert_allclose(gz[k, sl], 0.0, atol=1e-10)
    # and no better point is found by SLSQP on the same sub-problem
    res = scipy.optimize.minimize(fun, q1 + 0.01, jac=jac, constraints=cons, method="SLSQP",
                                  options={"ftol": 1e-15, "maxiter": 2000})
    assert fun(q1) <= res.fun + 1e-9
    if res.success:
        np.testing.assert_allclose(q1, res.x, atol=2e-5)


def side_project(spec, w):
    """Projection written on the test side (not the oracle's code): closed
    forms for the halfspace, hyperplane and cone, bisection for the l1 ball."""
    kind = spec[0]
    if kind in ("halfspace", "hyperplane"):
        a, b = np.asarray(spec[1], np.float64), spec[2]
        s = a @ w - b
        return w - (s / (a @ a)) * a if (kind == "hyperplane" or s > 0) else w.copy()
    if kind == "soc":
        x, t = w[:-1], w[-1]
        nx = np.linalg.norm(x)
        if nx <= t:
            return w.copy()
        if nx <= -t:
            return np.zeros_like(w)
        al = 0.5 * (nx + t)
        return np.concatenate([al * x / nx, [al]])
    r = spec[1]
    if np.sum(np.abs(w)) <= r:
        return w.copy()
    lo, hi = 0.0, float(np.max(np.abs(w)))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.sum(np.maximum(np.abs(w) - mid, 0.0)) > r:
            lo = mid
        else:
            hi = mid
    return np.sign(w) * np.maximum(np.abs(w) - 0.5 * (lo + hi), 0.0)


def qp_admm_sets(p, xset, uset, rho=1.0, iters=300000, tol=1e-13):
    """General-QP ADMM of eqn. (3) on the sparse QP (2) (an algorithm
    independent of the parallel-in-horizon one) with Y = {beq} x (the set of
    every x_k and u_k), projected block by block with side_project."""
    D = _refs.original_qp(p)
    H, Aeq, beq = D["H"], D["Aeq"], D["beq"]
    ny = H.shape[0]
    ne = Aeq.shape[0]
    E = np.vstack([Aeq, np.eye(ny)])
    Minv = np.linalg.inv(H + rho * E.T @ E)
    w = np.zeros(E.shape[0])
    lam = np.zeros(E.shape[0])
    y = np.zeros(ny)

    def proj(t):
        out = t.copy()
        out[:ne] = beq
        for k in range(p.N):
            for spec, sl in ((xset, D["xx"](k)), (uset, D["uu"](k))):
                blk = slice(ne + sl.start, ne + sl.stop)
                out[blk] = t[blk] if spec is None else side_project(spec, t[blk])
        return out

    for it in range(1, iters + 1):
        y = Minv @ (-D["f"] + rho * E.T @ (w - lam))
        Ey = E @ y
        w_new = proj(Ey + lam)
        lam = lam + Ey - w_new
        r_p = np.max(np.abs(Ey - w_new))
        r_d = rho * np.max(np.abs(E.T @ (w_new - w)))
        w = w_new
        if r_p < tol and r_d < tol:
            break
    us = np.array([y[D["uu"](k)] for k in range(p.N)])
    xs = np.array([y[D["xx"](k)] for k in range(p.N)])
    return xs, us, it


@pytest.mark.parametrize("xset,uset", CASES)
def test_set_constrained_fixed_point_matches_qp_admm(xset, uset):
    """The converged oracle solves problem (1) with the set constraints: it
    equals the optimum reached by the general-QP ADMM of eqn. (3) with the
    test-side projections."""
    p = set_problem(4, xset, uset, N=4)
    r = oracle.solve(p, K=200000, eps=1e-24)
    assert r["hist"][-1][0] <= 1e-24
    xs, us, it = qp_admm_sets(p, xset, uset)
    assert it < 300000
    np.testing.assert_allclose(r["xs"][:, :p.nx], xs, atol=1e-8)
    np.testing.assert_allclose(r["xs"][:, p.nx:], us, atol=1e-8)
    # the set constraint changes the optimum (so the test sees it)
    unc = oracle.solve(p.copy(xset=None, uset=None), K=200000, eps=1e-24)
    assert np.max(np.abs(unc["xs"] - r["xs"])) > 1e-3


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: s[0])
def test_test_side_projection_agrees(spec):
    """The test-side projection (used by the reference QP-ADMM above) agrees
    with the oracle's on random points."""
    rng = np.random.default_rng(8)
    for _ in range(200):
        y = rng.standard_normal(3) * 2.5
        np.testing.assert_allclose(oracle.project(spec, y), side_project(spec, y), atol=1e-12)
