"""Batched persistent form: the 4096-instance uneven batch through
pimpc_solve_batch (device tensors, hipGraph capture/replay), its schedules,
and parameter updates from device tensors -- each against the oracle and
against the plain single-context path."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

from test_gpu_lane import TOL32, compare, scaled_err, tiny_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def side_stream():
    s = torch.cuda.Stream()
    yield s
    torch.cuda.synchronize()


def _solve_batch(solver, problems, stream, x0=None):
    dev = torch.device("cuda")
    with torch.cuda.stream(stream):
        if x0 is None:
            x0 = torch.tensor(np.concatenate([p.x0 for p in problems]), dtype=torch.float32, device=dev)
        u0 = torch.full((solver.sum_nu,), float("nan"), dtype=torch.float32, device=dev)
        info = torch.zeros((solver.count * 40,), dtype=torch.uint8, device=dev)
        P.pimpc_solve_batch(solver.ctx, x0, None, u0, info, stream.cuda_stream)
    stream.synchronize()
    inf = np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE)
    return u0.cpu().numpy().astype(np.float64), inf, x0


def stratified_sample(problems, extra=6, seed=0):
    """The shortest and the longest instance of every (nx, nu) class present,
    plus `extra` instances drawn at random."""
    by_cls = {}
    for i, p in enumerate(problems):
        by_cls.setdefault((p.nx, p.nu), []).append(i)
    pick = {j for ids in by_cls.values() for j in (min(ids, key=lambda i: (problems[i].N, i)),
                                                   max(ids, key=lambda i: (problems[i].N, -i)))}
    pick |= set(int(j) for j in np.random.default_rng(seed).choice(len(problems), extra, replace=False))
    return sorted(pick), len(by_cls)


def test_full_uneven_batch_sampled(side_stream):
    """All 4096 instances in one batched solve.  The shortest and longest
    instance of each of the 16 (nx, nu) classes, and 6 more, match their
    oracle runs to the FP32 tolerance on all five iterates, du, xbar, u0 and
    the residuals; the device path equals the host-pointer path bit for bit."""
    problems = W.random_batch(4096, base_seed=1000, K=300)
    s = P.Solver(problems, max_iter=300, precision=P.PIMPC_FP32, stream=side_stream.cuda_stream)
    u0_dev, info, _ = _solve_batch(s, problems, side_stream)
    assert np.all(np.isfinite(u0_dev)) and np.all(info["status"] == 0) and np.all(info["iters"] == 300)
    u0_host, info_host = s.solve()  # also writes du and xbar
    np.testing.assert_array_equal(u0_dev, u0_host)
    np.testing.assert_array_equal(info["c"], info_host["c"])
    pick, ncls = stratified_sample(problems)
    assert ncls == 16 and len(pick) >= 32
    offs = np.concatenate([[0], np.cumsum([p.nu for p in problems])])
    its = {w: s.iterate(w) for w in range(7)}
    worst = 0.0
    for i in pick:
        r = oracle.solve(problems[i])
        refs = [r["state"][w] for w in range(5)] + [r["du"], r["xs"]]
        for w in range(7):
            e = scaled_err(its[w][i], refs[w])
            worst = max(worst, e)
            assert e <= TOL32, (i, w, e)
        assert scaled_err(u0_dev[offs[i]:offs[i + 1]], r["u0"]) <= TOL32, i
        c, rp, rd, _ = r["hist"][-1]
        assert abs(info["r_prim"][i] - rp) <= 1e-4 and abs(info["r_dual"][i] - rd) <= 1e-4
    print(f"largest scaled error over {len(pick)} instances: {worst:.2e}")
    s.close()


def test_graph_replay_is_stable(side_stream):
    """Replays of the captured graph, with unrelated eager work and host
    synchronisation between them, give identical results; changing x0 in
    place (same pointer) changes the result like a fresh host-path solve."""
    problems = W.random_batch(96, base_seed=77, K=120)
    s = P.Solver(problems, max_iter=120, precision=P.PIMPC_FP32, stream=side_stream.cuda_stream)
    first, _, x0 = _solve_batch(s, problems, side_stream)
    for rep in range(3):
        a = torch.randn(512, 512, device="cuda")
        (a @ a).sum().item()
        again, _, _ = _solve_batch(s, problems, side_stream, x0=x0)
        np.testing.assert_array_equal(again, first)
    with torch.cuda.stream(side_stream):
        x0.mul_(0.5)
    side_stream.synchronize()
    half, _, _ = _solve_batch(s, problems, side_stream, x0=x0)
    u_host, _ = s.solve(x0=0.5 * np.concatenate([p.x0 for p in problems]).astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(half, u_host, atol=1e-6)
    assert np.max(np.abs(half - first)) > 1e-3
    s.close()


@pytest.mark.parametrize("schedule", list(range(1, 15)))
def test_every_schedule_gives_the_same_iterates(schedule):
    """The autotuner's candidates only change which workgroup runs which bin,
    so every fixed schedule yields bit-identical results."""
    problems = W.random_batch(64, base_seed=5, K=80)
    ref = P.Solver(problems, max_iter=80, precision=P.PIMPC_FP32, schedule=1)
    u_ref, _ = ref.solve()
    s = P.Solver(problems, max_iter=80, precision=P.PIMPC_FP32, schedule=schedule)
    u, _ = s.solve()
    np.testing.assert_array_equal(u, u_ref)
    for w in (P.IT_Z, P.IT_THETA):
        for a, b in zip(s.iterate(w), ref.iterate(w)):
            np.testing.assert_array_equal(a, b)


def test_set_params_from_device_tensors(side_stream):
    """pimpc_set_params_dev (differentiable path) re-factors from device
    tensors: the solve equals a context set up with the same parameters."""
    db = W.diff_batch(count=32, N=128, K=60)
    rng = np.random.default_rng(1)
    Qd = db.Qdiag * rng.uniform(0.5, 2.0, db.Qdiag.shape)
    Rd = db.Rdiag * rng.uniform(0.5, 2.0, db.Rdiag.shape)
    A = db.A + 0.01 * rng.standard_normal(db.A.shape)
    B = db.Bm + 0.01 * rng.standard_normal(db.Bm.shape)
    base = [db.instance(i) for i in range(32)]
    s = P.Solver(base, max_iter=60, precision=P.PIMPC_FP32, stream=side_stream.cuda_stream)
    f32 = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    tA, tB, tQ, tR = f32(A), f32(B), f32(Qd), f32(Rd)
    side_stream.synchronize()
    torch.cuda.synchronize()
    P.pimpc_set_params_dev(s.ctx, tA, tB, tQ, tR, side_stream.cuda_stream)
    side_stream.synchronize()
    u_dev, _ = s.solve()
    new = [db.instance(i).copy(A=A[i].astype(np.float32).astype(np.float64),
                               B=B[i].astype(np.float32).astype(np.float64),
                               Q=np.diag(Qd[i].astype(np.float32).astype(np.float64)),
                               R=np.diag(Rd[i].astype(np.float32).astype(np.float64))) for i in range(32)]
    fresh = P.Solver(new, max_iter=60, precision=P.PIMPC_FP32)
    u_fresh, _ = fresh.solve()
    np.testing.assert_allclose(u_dev, u_fresh, atol=1e-6)
    for i in (0, 17):
        r = oracle.solve(new[i], K=60)
        assert scaled_err(u_dev[3 * i:3 * i + 3], r["u0"]) <= TOL32
    s.close()
    fresh.close()


def test_graph_replay_with_row_family_instances(side_stream):
    """A captured batch holding two long horizons (row family, run first)
    and lane-family instances on four streams: replays equal the host-path
    solve of the same context, and every instance matches the oracle."""
    problems = [W.long_horizon_problem(seed=3, N=1024, K=30), W.long_horizon_problem(seed=4, N=700, K=30)]
    problems += [W.random_batch_instance(seed=3000 + i, K=30) for i in range(10)]
    s = P.Solver(problems, max_iter=30, precision=P.PIMPC_FP32, schedule=1, stream=side_stream.cuda_stream)
    first, _, x0 = _solve_batch(s, problems, side_stream)
    for rep in range(3):
        a = torch.randn(256, 256, device="cuda")
        (a @ a).sum().item()
        again, _, _ = _solve_batch(s, problems, side_stream, x0=x0)
        np.testing.assert_array_equal(again, first)
    u_host, _ = s.solve(x0=np.concatenate([p.x0 for p in problems]).astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(first, u_host, atol=1e-6)
    refs = [oracle.solve(p, K=30) for p in problems]
    compare(s, problems, refs, TOL32)
    s.close()


@pytest.mark.parametrize("accel", [False, True])
def test_graph_replay_row_family_reducer_kernel(side_stream, accel):
    """Graph replays of a batch whose row-family instance runs the reducer
    kernel (eps stop, or restart acceleration) beside lane-family instances:
    every replay equals the first and the host-path solve."""
    problems = [tiny_problem(11, 3, 2, 700, 0)]  # row family; meets eps within 45 iterations
    problems += [W.random_batch_instance(seed=3100 + i, K=300) for i in range(6)]
    s = P.Solver(problems, max_iter=300, eps=1e-3, check_every=5, precision=P.PIMPC_FP32, accel=accel,
                 schedule=1, stream=side_stream.cuda_stream)
    first, info, x0 = _solve_batch(s, problems, side_stream)
    assert np.all(info["status"] == 0) and info["iters"][0] < 300
    for rep in range(3):
        a = torch.randn(256, 256, device="cuda")
        (a @ a).sum().item()
        again, info2, _ = _solve_batch(s, problems, side_stream, x0=x0)
        np.testing.assert_array_equal(again, first)
        np.testing.assert_array_equal(info2["iters"], info["iters"])
    # the device calls pass no u_prev: the host path gets zeros too (the
    # problems' own u_prev enter the initial augmented state)
    u_host, info_h = s.solve(x0=np.concatenate([p.x0 for p in problems]).astype(np.float32).astype(np.float64),
                             u_prev=np.zeros(s.sum_nu))
    np.testing.assert_array_equal(u_host, first)
    np.testing.assert_array_equal(info_h["iters"], info["iters"])
    s.close()
