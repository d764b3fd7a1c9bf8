"""Robustness of the C ABI on the device: a tape that was replaced cannot be
differentiated, a stage matrix that is not SPD after a device-side parameter
update is reported through the solve's status, the device-pointer
construction-free update (pimpc_linearize with device memory) reads the
caller's arrays on the context's stream and gives the same solve as the host
path, and the per-context cache of launch argument sets stays bounded."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

from test_gpu_lane import TOL32, scaled_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _layer_inputs(count, seed=3):
    db = W.diff_batch(count=count, seed=seed, N=24, K=30)
    dev = torch.device("cuda")
    f = lambda a: torch.tensor(np.ascontiguousarray(a[:count]), dtype=torch.float32, device=dev,
                               requires_grad=True)
    return db, [f(db.x0), f(db.Qdiag), f(db.Rdiag), f(db.A), f(db.Bm)]


def test_backward_of_a_replaced_tape_is_an_error():
    """Two forwards of the layer before a backward: the first output's
    backward must fail (its tape was overwritten); the second's succeeds."""
    from paper_2601_14414_amd.autograd import PiMPCLayer
    db, args = _layer_inputs(4)
    layer = PiMPCLayer(4, 8, 3, db.N, iters=db.K, ckpt_every=10)
    u_a = layer(*args)
    u_b = layer(*[a * 1.0 for a in args])
    with pytest.raises(P.PimpcError) as ei:
        u_a.sum().backward()
    assert ei.value.code == P.PIMPC_E_STATE
    u_b.sum().backward()
    torch.cuda.synchronize()
    assert all(torch.isfinite(a.grad).all() for a in args)
    layer.solver.close()


def test_backward_after_a_parameter_update_is_an_error():
    """pimpc_set_params_dev after the taped forward invalidates its tape."""
    from paper_2601_14414_amd.autograd import PiMPCLayer
    db, args = _layer_inputs(4)
    layer = PiMPCLayer(4, 8, 3, db.N, iters=db.K, ckpt_every=10)
    u = layer(*args)
    tid = P.pimpc_tape_id(layer.solver.ctx)
    assert tid > 0
    x0, Qd, Rd, A, B = (a.detach().contiguous() for a in args)
    P.pimpc_set_params_dev(layer.solver.ctx, A, B, Qd, Rd, torch.cuda.current_stream().cuda_stream)
    assert P.pimpc_tape_id(layer.solver.ctx) == 0
    with pytest.raises(P.PimpcError) as ei:
        u.sum().backward()
    assert ei.value.code == P.PIMPC_E_STATE
    layer.solver.close()


def test_not_spd_parameters_raise_in_the_layer():
    """A negative diagonal weight makes Qbar + rho I indefinite for one
    instance: the layer raises PIMPC_E_NOT_PSD instead of returning NaN, and
    the info records flag exactly that instance."""
    from paper_2601_14414_amd.autograd import PiMPCLayer
    db, args = _layer_inputs(4)
    layer = PiMPCLayer(4, 8, 3, db.N, iters=db.K, ckpt_every=10)
    Qd = args[1].detach().clone()
    Qd[2, 1] = -5.0
    args[1] = Qd.requires_grad_(True)
    with pytest.raises(P.PimpcError) as ei:
        layer(*args)
    assert ei.value.code == P.PIMPC_E_NOT_PSD and "instance 2" in ei.value.msg
    # with valid weights again the same context solves normally
    Qd2 = Qd.detach().clone()
    Qd2[2, 1] = 1.0
    args[1] = Qd2.requires_grad_(True)
    u = layer(*args)
    assert torch.isfinite(u).all()
    layer.solver.close()


def test_not_spd_status_in_batch_info():
    """set_params_dev with an indefinite stage matrix, then pimpc_solve_batch
    with an info buffer: that instance reports PIMPC_E_NOT_PSD, the others 0."""
    db, args = _layer_inputs(3)
    p = db.instance(0)
    s = P.Solver([p] * 3, max_iter=db.K, precision=P.PIMPC_FP32)
    x0, Qd, Rd, A, B = (a.detach().contiguous().clone() for a in args)
    Rd[1, 0] = -3.0
    st = torch.cuda.current_stream().cuda_stream
    P.pimpc_set_params_dev(s.ctx, A, B, Qd, Rd, st)
    u0 = torch.empty(3 * 3, dtype=torch.float32, device="cuda")
    info = torch.zeros(3 * 10, dtype=torch.int32, device="cuda")
    P.pimpc_solve_batch(s.ctx, x0, None, u0, info, st)
    torch.cuda.synchronize()
    status = info.view(3, 10)[:, 8].cpu().numpy()
    assert list(status) == [0, P.PIMPC_E_NOT_PSD, 0]
    s.close()


def _tv_rate_problem(seed):
    """Cart-pole-like time-varying instance (lane family) for the
    construction-free update."""
    p = W.cartpole_problem(N=96, K=60)
    x = np.array([0.1, 0.0, 3.0, 0.2])
    xs = np.broadcast_to(x, (p.N, 4)).copy() + 0.01 * np.random.default_rng(seed).standard_normal((p.N, 4))
    A, B, e = W.cartpole_linearize(xs, np.zeros((p.N, 1)))
    return p.copy(A=A, B=B, e=e, x0=x)


@pytest.mark.parametrize("family", [P.PIMPC_FAMILY_LANE, P.PIMPC_FAMILY_ROW])
def test_linearize_from_device_memory_matches_host_path(family):
    """The Jacobians are formed by torch kernels on the context's own (side)
    stream; pimpc_linearize(PIMPC_MEM_DEVICE) must read them after those
    kernels and give the same solve, bit for bit, as the host-pointer path;
    both agree with the oracle."""
    p0 = _tv_rate_problem(0)
    p1 = _tv_rate_problem(1)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        sh = P.Solver([p0], max_iter=60, precision=P.PIMPC_FP32, warm_start=False, family=family,
                      stream=side.cuda_stream)
        sd = P.Solver([p0], max_iter=60, precision=P.PIMPC_FP32, warm_start=False, family=family,
                      stream=side.cuda_stream)
        sh.linearize(p1.A.ravel(), p1.B.ravel(), p1.e.ravel())
        u_h, _ = sh.solve(x0=p1.x0)
        # produce the device copies by kernels on the side stream (scaled by 2,
        # then halved again, so that the data only exist after those kernels)
        dA = torch.tensor(p1.A.ravel(), dtype=torch.float64, device="cuda") * 2.0
        dB = torch.tensor(p1.B.ravel(), dtype=torch.float64, device="cuda") * 2.0
        de = torch.tensor(p1.e.ravel(), dtype=torch.float64, device="cuda") * 2.0
        dA, dB, de = dA * 0.5, dB * 0.5, de * 0.5
        P.pimpc_linearize(sd.ctx, dA, dB, de, P.PIMPC_MEM_DEVICE)
        u_d, _ = sd.solve(x0=p1.x0)
    np.testing.assert_array_equal(u_d, u_h)
    for w in range(5):
        np.testing.assert_array_equal(sd.state(0)[w], sh.state(0)[w])
    r = oracle.solve(p1, K=60)
    assert scaled_err(u_d, r["u0"]) <= TOL32
    # non-finite device data is rejected
    dA[3] = float("nan")
    with pytest.raises(P.PimpcError) as ei:
        P.pimpc_linearize(sd.ctx, dA, dB, de, P.PIMPC_MEM_DEVICE)
    assert ei.value.code == P.PIMPC_E_NONFINITE
    sh.close()
    sd.close()


def test_launch_set_cache_is_bounded_and_stays_correct():
    """Twelve distinct argument sets (more than the context keeps) solved
    twice each through pimpc_solve_batch: every result equals the first
    solve of the same x0, so evicted sets are rebuilt correctly."""
    probs = W.random_batch(count=6, base_seed=77, K=40)
    s = P.Solver(probs, max_iter=40, precision=P.PIMPC_FP32,
                 stream=torch.cuda.current_stream().cuda_stream)
    st = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(5)
    x0s = [torch.tensor(rng.uniform(-1, 1, s.sum_nx), dtype=torch.float32, device="cuda") for _ in range(12)]
    outs = [torch.zeros(s.sum_nu, dtype=torch.float32, device="cuda") for _ in range(12)]
    first = []
    for x, o in zip(x0s, outs):
        P.pimpc_solve_batch(s.ctx, x, None, o, None, st)
        first.append(o.clone())
    for rep in range(2):
        for x, o, f in zip(x0s, outs, first):
            o.zero_()
            P.pimpc_solve_batch(s.ctx, x, None, o, None, st)
            torch.cuda.synchronize()
            assert torch.equal(o, f)
    # one of them against the oracle
    x = x0s[7].cpu().numpy().astype(np.float64)
    xo = uo = 0
    for p in probs:
        r = oracle.solve(p.copy(x0=x[xo:xo + p.nx]), K=40)
        u = first[7].cpu().numpy()[uo:uo + p.nu]
        assert scaled_err(u, r["u0"]) <= TOL32
        xo += p.nx
        uo += p.nu
    s.close()
