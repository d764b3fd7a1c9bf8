"""GPU parity of the lane-per-stage path against the CPU FP64 oracle.

Each case runs the HIP path through the C ABI and the oracle on the same
seeded inputs and compares every iterate element by element.  Tolerances:
FP64 iteration: 1e-11 relative to max(1, |oracle|_inf) (rounding order only);
FP32 iteration: 1e-4 of the same scale -- the iteration map is nonexpansive,
so FP32 rounding (~6e-8 per operation) accumulates at most about linearly
over the K <= 500 iterations; residual levels are compared to 1e-4 absolute.
"""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-4


def scaled_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(1.0, float(np.max(np.abs(b)))))


def compare(solver, problems, refs, tol, which=range(len(P.EXPORTS))):
    """Compare every iterate of every instance with the oracle results;
    returns the largest scaled error."""
    its = {w: solver.iterate(w) for w in range(7)}
    worst = 0.0
    for i, (p, r) in enumerate(zip(problems, refs)):
        for w in range(5):
            e = scaled_err(its[w][i], r["state"][w])
            worst = max(worst, e)
            assert e <= tol, f"instance {i} iterate {w}: {e:.3e}"
        e = scaled_err(its[P.IT_DU][i], r["du"])
        worst = max(worst, e)
        assert e <= tol, f"instance {i} du"
        e = scaled_err(its[P.IT_XBAR][i], r["xs"])
        worst = max(worst, e)
        assert e <= tol, f"instance {i} xbar"
    return worst


def run_both(problems, precision, K=None, **kw):
    """Solve on the lane family (requested explicitly: a lone FP32 instance
    would otherwise run on the row family) and with the oracle."""
    K = K or problems[0].K
    kw.setdefault("family", P.PIMPC_FAMILY_LANE)
    s = P.Solver(problems, rho=problems[0].rho, max_iter=K, precision=precision, **kw)
    u0, info = s.solve()
    refs = [oracle.solve(p, K=K, eps=kw.get("eps", 0.0)) for p in problems]
    return s, u0, info, refs


def check_info(info, refs, tol_abs):
    for i, r in enumerate(refs):
        c, rp, rd, _ = r["hist"][-1]
        assert info["iters"][i] == r["iters"]
        assert info["status"][i] == 0
        assert abs(info["c"][i] - c) <= tol_abs * max(1.0, c)
        assert abs(info["r_prim"][i] - rp) <= tol_abs
        assert abs(info["r_dual"][i] - rd) <= tol_abs


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_fp64_parity(seed):
    """4-mass chain, N=20, 200 iterations, FP64 on both sides."""
    p = W.plain_fp64_problem(seed)
    s, u0, info, refs = run_both([p], P.PIMPC_FP64)
    compare(s, [p], refs, TOL64)
    assert scaled_err(u0, refs[0]["u0"]) <= TOL64
    check_info(info, refs, 1e-10)


def test_plain_fp32_parity():
    p = W.plain_fp64_problem(0)
    s, u0, info, refs = run_both([p], P.PIMPC_FP32)
    compare(s, [p], refs, TOL32)
    assert scaled_err(u0, refs[0]["u0"]) <= TOL32
    check_info(info, refs, 1e-4)


def tiny_problem(seed, n, m, N, tv, qbar=True, affine=True, dense_q=True):
    rng = np.random.default_rng(seed)
    shape_a = (N, n, n) if tv else (n, n)
    shape_b = (N, n, m) if tv else (n, m)
    A = rng.standard_normal(shape_a) * (0.9 / np.sqrt(n))
    B = rng.standard_normal(shape_b) / np.sqrt(n)
    e = (rng.standard_normal((N, n) if tv else (n,)) * 0.1) if affine else None
    if dense_q:
        Qh = rng.standard_normal((n, n))
        Q = Qh @ Qh.T / n + 0.5 * np.eye(n)
        Rh = rng.standard_normal((m, m))
        R = Rh @ Rh.T / m + 0.2 * np.eye(m)
    else:
        Q, R = np.eye(n), 0.1 * np.eye(m)
    return W.Problem(nx=n, nu=m, N=N, A=A, B=B, e=e, Q=Q, R=R,
                     qbar=rng.standard_normal(n + m) * 0.2 if qbar else None,
                     xmin=-0.8 * np.ones(n), xmax=0.8 * np.ones(n), umin=-0.4 * np.ones(m),
                     umax=0.4 * np.ones(m), x0=rng.uniform(-1, 1, n),
                     u_prev=rng.uniform(-0.2, 0.2, m), rho=1.3, K=60)


@pytest.mark.parametrize("n,m,tv", [(3, 2, 1), (2, 1, 1), (4, 1, 1), (5, 3, 0), (7, 1, 0), (3, 4, 0)])
def test_padding_time_varying_affine_fp64(n, m, tv):
    """Padded classes, time-varying stage data, affine e_k, linear term qbar,
    non-diagonal Q (full H_{N-1} path), nonzero u_prev: FP64 parity."""
    problems = [tiny_problem(10 * n + m, n, m, N, tv) for N in (5, 70)]
    s, u0, info, refs = run_both(problems, P.PIMPC_FP64)
    compare(s, problems, refs, TOL64)
    np.testing.assert_allclose(u0, np.concatenate([r["u0"] for r in refs]), atol=1e-11)
    check_info(info, refs, 1e-10)


@pytest.mark.parametrize("N", [1, 2, 63, 64, 65, 127, 200, 256, 257, 511, 512])
def test_wave_and_bin_boundaries_fp64(N):
    """Horizons at and around wave (64) and workgroup (512) boundaries; FP64
    classes whose horizons all fit four waves (N <= 256) run 256-thread
    workgroups, longer ones 512-thread workgroups."""
    p = tiny_problem(N, 4, 2, N, 0, dense_q=False)
    s, u0, info, refs = run_both([p], P.PIMPC_FP64, K=40)
    compare(s, [p], refs, TOL64)
    check_info(info, refs, 1e-10)

def test_fp64_class_mixing_short_and_long_horizons():
    """One FP64 class holding horizons on both sides of four waves: the whole
    class runs eight-wave bins; every instance matches the oracle."""
    problems = [tiny_problem(40 + i, 4, 2, N, 0, dense_q=False) for i, N in enumerate((30, 200, 300, 90))]
    s, u0, info, refs = run_both(problems, P.PIMPC_FP64, K=40)
    compare(s, problems, refs, TOL64)
    check_info(info, refs, 1e-10)



def test_eps_stop_matches_oracle_fp64():
    """Step 5: stop at the first iteration with c <= eps (checked every
    iteration), and at the first multiple of check_every otherwise."""
    p = W.plain_fp64_problem(1)
    eps = 1e-6
    s, u0, info, refs = run_both([p], P.PIMPC_FP64, K=5000, eps=eps)
    assert info["iters"][0] == refs[0]["iters"] < 5000
    compare(s, [p], refs, TOL64)
    s10 = P.Solver([p], max_iter=5000, eps=eps, check_every=10, precision=P.PIMPC_FP64)
    _, info10 = s10.solve()
    it10 = int(info10["iters"][0])
    assert it10 % 10 == 0 and refs[0]["iters"] <= it10 < refs[0]["iters"] + 10
    r10 = oracle.solve(p, K=it10)
    compare(s10, [p], [r10], TOL64)


def test_warm_start_continues_iteration_fp64():
    """Output iterates warm-start the next solve (Algorithm 1 output):
    100 + 100 warm iterations equal 200 cold ones; set_iterates injects a state."""
    p = W.plain_fp64_problem(2)
    s = P.Solver([p], max_iter=100, precision=P.PIMPC_FP64, warm_start=True)
    s.solve()
    u0, _ = s.solve()
    ref = oracle.solve(p, K=200)
    compare(s, [p], [ref], TOL64)
    st = oracle.solve(p, K=37)["state"]
    s.set_state([st])
    s.solve()
    compare(s, [p], [oracle.solve(p, K=100, state=st)], TOL64)


def test_uneven_batch_subset_fp32():
    """48 instances of the uneven random batch (mixed classes and horizons)
    in one solve, FP32, each against its own oracle run."""
    problems = W.random_batch(48, base_seed=1000, K=300)
    s, u0, info, refs = run_both(problems, P.PIMPC_FP32)
    compare(s, problems, refs, TOL32)
    check_info(info, refs, 1e-4)


@pytest.mark.parametrize("family", [P.PIMPC_FAMILY_LANE, P.PIMPC_FAMILY_ROW])
def test_nonfinite_iterate_reported(family):
    """Overflowing FP32 data is reported as PIMPC_E_NONFINITE by both families."""
    p = W.plain_fp64_problem(0)
    s = P.Solver([p], precision=P.PIMPC_FP32, family=family)
    with pytest.raises(P.PimpcError) as ei:
        s.solve(x0=np.full(8, 1e30))
    assert ei.value.code == P.PIMPC_E_NONFINITE


def test_linearize_equals_fresh_setup_fp64():
    """pimpc_linearize replaces the stage data and refactors: a solve after it
    equals a context set up with the new data (cart-pole linearisation)."""
    p0 = W.cartpole_problem(N=100, K=50)
    rng = np.random.default_rng(3)
    xs = rng.uniform(-1, 1, (100, 4)) + np.array([0, 0, np.pi, 0])
    us = rng.uniform(-2, 2, (100, 1))
    A, B, e = W.cartpole_linearize(xs, us)
    p1 = p0.copy(A=A, B=B, e=e)
    s = P.Solver([p0], max_iter=50, precision=P.PIMPC_FP64)
    s.linearize(A.ravel(), B.ravel(), e.ravel())
    s.solve()
    compare(s, [p1], [oracle.solve(p1, K=50)], TOL64)


@pytest.mark.parametrize("n,m,N,tv", [(7, 6, 150, 0), (14, 7, 90, 0), (6, 5, 70, 1)])
def test_wide_input_classes_fp32(n, m, N, tv):
    """Classes with up to eight inputs (padded 8+8 and 16+8), FP32 against
    the FP64 oracle; the time-varying case has no lane class that wide and
    runs on the row family's 8+8 class with a short horizon."""
    p = tiny_problem(100 + n + m, n, m, N, tv)
    fam = P.PIMPC_FAMILY_ROW if tv else P.PIMPC_FAMILY_LANE
    s, u0, info, refs = run_both([p], P.PIMPC_FP32, family=fam)
    compare(s, [p], refs, TOL32)
    check_info(info, refs, 1e-4)
