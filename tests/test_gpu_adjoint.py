"""Differentiable form: the hand-written adjoint through the unrolled,
checkpointed iterations against the oracle's reverse mode (itself pinned to
central finite differences in test_oracle_pins.py).

Tolerance: FP32 forward and adjoint over K iterations vs FP64; gradients are
compared relative to the largest oracle gradient entry of the same parameter,
at 1e-3 (the adjoint map is the transpose of a nonexpansive one, so rounding
accumulates at most about linearly in K; the largest error measured on the
differentiable batch is about 4e-5)."""
import numpy as np
import pytest

import oracle
from paper_2601_14414_amd import pimpc as P
from paper_2601_14414_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOLG = 1e-3


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-6, float(np.max(np.abs(b)))))


def run_gpu(db, count, ckpt, ut):
    from paper_2601_14414_amd.autograd import PiMPCLayer
    dev = torch.device("cuda")
    layer = PiMPCLayer(count, 8, 3, db.N, iters=db.K, ckpt_every=ckpt)
    f = lambda a: torch.tensor(np.ascontiguousarray(a[:count]), dtype=torch.float32, device=dev,
                               requires_grad=True)
    x0, Qd, Rd, A, B = f(db.x0), f(db.Qdiag), f(db.Rdiag), f(db.A), f(db.Bm)
    u0 = layer(x0, Qd, Rd, A, B)
    target = torch.tensor(ut[:count], dtype=torch.float32, device=dev)
    loss = ((u0 - target) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    out = {k: t.grad.detach().cpu().numpy().astype(np.float64) for k, t in
           dict(dx0=x0, dQd=Qd, dRd=Rd, dA=A, dB=B).items()}
    out["u0"] = u0.detach().cpu().numpy().astype(np.float64)
    layer.solver.close()
    return out


def oracle_grad(db, i, ut, u0=None):
    p = db.instance(i)
    r = oracle.solve(p)
    g = oracle.grad(8, 3, db.N, p.A, p.B, db.Qdiag[i], db.Rdiag[i], p.lb(), p.ub(), p.x0, p.rho, db.K,
                    2 * (r["u0"] - ut[i]))
    return r, g


@pytest.mark.parametrize("ckpt", [1, 5, 7, 30])
def test_adjoint_matches_oracle_small(ckpt):
    """8 perturbed instances, N=24, 30 iterations, several checkpoint spacings
    (incl. one not dividing K and one larger than K), and the full tape the
    forward records itself (ckpt_every = 1)."""
    db = W.diff_batch(count=8, seed=3, N=24, K=30)
    rng = np.random.default_rng(9)
    db.Qdiag *= rng.uniform(0.5, 2.0, db.Qdiag.shape)
    db.Rdiag *= rng.uniform(0.5, 2.0, db.Rdiag.shape)
    db.A += 0.02 * rng.standard_normal(db.A.shape)
    db.Bm += 0.02 * rng.standard_normal(db.Bm.shape)
    g = run_gpu(db, 8, ckpt, db.u_target)
    for i in range(8):
        r, go = oracle_grad(db, i, db.u_target)
        assert rel(g["u0"][i], r["u0"]) <= 1e-4
        for key in ("dx0", "dQd", "dRd", "dA", "dB"):
            assert rel(g[key][i], go[key]) <= TOLG, (i, key, rel(g[key][i], go[key]))


def test_adjoint_differentiable_batch_sampled():
    """The differentiable batch: 1024 chains (nx=8, nu=3, N=128), 200
    iterations, checkpoints every 20; 32 instances (every 32nd, the last
    one included) vs the oracle's reverse mode."""
    db = W.diff_batch(count=1024, seed=7, N=128, K=200)
    g = run_gpu(db, 1024, 20, db.u_target)
    worst = {}
    for i in list(range(0, 1024, 33)) + [1023]:
        r, go = oracle_grad(db, i, db.u_target)
        assert rel(g["u0"][i], r["u0"]) <= 1e-4
        for key in ("dx0", "dQd", "dRd", "dA", "dB"):
            e = rel(g[key][i], go[key])
            worst[key] = max(worst.get(key, 0.0), e)
            assert e <= TOLG, (i, key, e)
    print("largest relative gradient errors:", {k: f"{v:.2e}" for k, v in worst.items()})


def test_checkpoint_spacing_does_not_change_gradients():
    """Re-running segments from checkpoints reproduces the forward iterates
    exactly, and the records the forward writes itself (ckpt_every = 1) are
    the ones a re-run writes, so the gradient depends on neither the spacing
    nor the kind of tape."""
    db = W.diff_batch(count=16, seed=4, N=64, K=40)
    ga = run_gpu(db, 16, 40, db.u_target)
    gb = run_gpu(db, 16, 8, db.u_target)
    gc = run_gpu(db, 16, 1, db.u_target)
    for key in ("u0", "dx0", "dQd", "dRd", "dA", "dB"):
        np.testing.assert_array_equal(ga[key], gb[key])
        np.testing.assert_array_equal(ga[key], gc[key])


def test_backward_without_tape_is_an_error():
    p = W.plain_fp64_problem(0)
    s = P.Solver([p], precision=P.PIMPC_FP32)
    g = torch.zeros(3, device="cuda")
    with pytest.raises(P.PimpcError) as ei:
        P.pimpc_backward(s.ctx, P.pimpc_tape_id(s.ctx), g)
    assert ei.value.code == P.PIMPC_E_STATE


@pytest.mark.parametrize("nx,nu,N,K,ck", [(4, 2, 40, 20, 6), (12, 4, 70, 16, 5), (6, 1, 130, 12, 4),
                                         (4, 2, 40, 20, 1), (12, 4, 70, 16, 1), (6, 1, 130, 12, 1),
                                         (2, 2, 200, 10, 1), (8, 8, 90, 12, 4), (7, 5, 256, 10, 1)])
def test_adjoint_other_classes(nx, nu, N, K, ck):
    """Backward kernels of other (nx, nu) classes (padded 4+2, 12+4, 8+1, 2+2
    and 8+8, the widest, whose matrices stream through SGPRs) and horizons
    over one, two and four waves (N = 256 fills four), against the oracle's
    reverse mode, from checkpoints and from the full tape (ck = 1)."""
    from paper_2601_14414_amd.autograd import PiMPCLayer
    rng = np.random.default_rng(nx * 100 + nu)
    count = 5
    A = np.stack([np.eye(nx) * 0.95 + 0.05 * rng.standard_normal((nx, nx)) for _ in range(count)])
    B = rng.standard_normal((count, nx, nu)) / np.sqrt(nx)
    Qd = rng.uniform(0.5, 1.5, (count, nx))
    Rd = rng.uniform(0.05, 0.2, (count, nu))
    x0 = rng.uniform(-1, 1, (count, nx))
    ut = rng.normal(0, 0.1, (count, nu))
    dev = torch.device("cuda")
    layer = PiMPCLayer(count, nx, nu, N, iters=K, ckpt_every=ck, xbound=1.5, ubound=0.4)
    f = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev, requires_grad=True)
    tx0, tQ, tR, tA, tB = f(x0), f(Qd), f(Rd), f(A), f(B)
    u0 = layer(tx0, tQ, tR, tA, tB)
    ((u0 - torch.tensor(ut, dtype=torch.float32, device=dev)) ** 2).sum().backward()
    torch.cuda.synchronize()
    got = {k: t.grad.detach().cpu().numpy().astype(np.float64) for k, t in
           dict(dx0=tx0, dQd=tQ, dRd=tR, dA=tA, dB=tB).items()}
    u0n = u0.detach().cpu().numpy().astype(np.float64).reshape(count, nu)
    layer.solver.close()
    lb = np.concatenate([-1.5 * np.ones(nx), -0.4 * np.ones(nu)])
    ub = -lb
    for i in range(count):
        p = W.Problem(nx=nx, nu=nu, N=N, A=A[i], B=B[i], Q=np.diag(Qd[i]), R=np.diag(Rd[i]), xmin=lb[:nx],
                      xmax=ub[:nx], umin=lb[nx:], umax=ub[nx:], x0=x0[i], u_prev=np.zeros(nu), rho=1.0, K=K)
        r = oracle.solve(p)
        assert rel(u0n[i], r["u0"]) <= 1e-4
        g = oracle.grad(nx, nu, N, A[i], B[i], Qd[i], Rd[i], lb, ub, x0[i], 1.0, K, 2 * (r["u0"] - ut[i]))
        for key in ("dx0", "dQd", "dRd", "dA", "dB"):
            assert rel(got[key][i], g[key]) <= TOLG, (i, key, rel(got[key][i], g[key]))


def _mixed_problems(K):
    """Six instances of three shapes in one context, interleaved: 4 states +
    2 inputs with N = 40, 8 + 3 with N = 100 and 12 + 4 with N = 70 (three
    lane classes; the last one keeps J_bar and B_bar in separate tiles)."""
    rng = np.random.default_rng(21)
    ps = []
    for i in range(6):
        nx, nu, N = [(4, 2, 40), (8, 3, 100), (12, 4, 70)][i % 3]
        A = np.eye(nx) * 0.95 + 0.05 * rng.standard_normal((nx, nx))
        B = rng.standard_normal((nx, nu)) / np.sqrt(nx)
        ps.append(W.Problem(nx=nx, nu=nu, N=N, A=A, B=B, Q=np.diag(rng.uniform(0.5, 1.5, nx)),
                            R=np.diag(rng.uniform(0.05, 0.2, nu)), xmin=-1.5 * np.ones(nx), xmax=1.5 * np.ones(nx),
                            umin=-0.4 * np.ones(nu), umax=0.4 * np.ones(nu), x0=rng.uniform(-1, 1, nx),
                            u_prev=np.zeros(nu), rho=1.0, K=K))
    return ps


def _mixed_grads(ps, K, ck, ut):
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    s = P.Solver(ps, max_iter=K, precision=P.PIMPC_FP32, ckpt_every=ck, stream=stream)
    f = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    x0 = f(np.concatenate([p.x0 for p in ps]))
    u0 = torch.empty(s.sum_nu, dtype=torch.float32, device=dev)
    P.pimpc_solve_batch(s.ctx, x0, None, u0, None, stream)
    g = 2 * (u0 - f(ut))
    sx, su = sum(p.nx for p in ps), sum(p.nu for p in ps)
    out = dict(dx0=torch.full((sx,), np.nan, device=dev), dQd=torch.full((sx,), np.nan, device=dev),
               dRd=torch.full((su,), np.nan, device=dev),
               dA=torch.full((sum(p.nx * p.nx for p in ps),), np.nan, device=dev),
               dB=torch.full((sum(p.nx * p.nu for p in ps),), np.nan, device=dev))
    P.pimpc_backward(s.ctx, P.pimpc_tape_id(s.ctx), g, out["dx0"], out["dQd"], out["dRd"], out["dA"], out["dB"],
                     stream)
    torch.cuda.synchronize()
    s.close()
    res = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    res["u0"] = u0.cpu().numpy().astype(np.float64)
    return res


def test_backward_mixed_shapes_packs_per_instance():
    """One taped context holding three classes: the gradients come packed per
    instance in instance order (dx0 and diag Q like x0, diag R like u0, the
    dA and dB blocks one after another), every entry written, each instance's
    block equal to the oracle's reverse mode; the full tape (ckpt_every = 1)
    and checkpoints give the same gradients bit for bit."""
    K = 16
    ps = _mixed_problems(K)
    ut = np.random.default_rng(5).normal(0, 0.1, sum(p.nu for p in ps))
    ga = _mixed_grads(ps, K, 1, ut)
    gb = _mixed_grads(ps, K, 5, ut)
    for key in ga:
        assert np.all(np.isfinite(ga[key])), key
        np.testing.assert_array_equal(ga[key], gb[key])
    ox = ou = oa = ob = 0
    for i, p in enumerate(ps):
        nx, nu = p.nx, p.nu
        r = oracle.solve(p)
        assert rel(ga["u0"][ou:ou + nu], r["u0"]) <= 1e-4
        go = oracle.grad(nx, nu, p.N, p.A, p.B, np.diag(p.Q), np.diag(p.R), p.lb(), p.ub(), p.x0, p.rho, K,
                         2 * (r["u0"] - ut[ou:ou + nu]))
        got = dict(dx0=ga["dx0"][ox:ox + nx], dQd=ga["dQd"][ox:ox + nx], dRd=ga["dRd"][ou:ou + nu],
                   dA=ga["dA"][oa:oa + nx * nx].reshape(nx, nx), dB=ga["dB"][ob:ob + nx * nu].reshape(nx, nu))
        for key, v in got.items():
            assert rel(v, np.asarray(go[key]).reshape(v.shape)) <= TOLG, (i, key, rel(v, go[key]))
        ox, ou, oa, ob = ox + nx, ou + nu, oa + nx * nx, ob + nx * nu


@pytest.mark.parametrize("ck", [1, 8])
def test_host_path_taped_forward_feeds_the_backward(ck):
    """pimpc_solve (host pointers) records the same tape as the device-pointer
    path: u0 and the backward after it equal those of pimpc_solve_batch bit
    for bit, with the full tape and with checkpoints."""
    db = W.diff_batch(count=16, seed=4, N=64, K=40)
    ps = [db.instance(i) for i in range(16)]
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    x32 = np.ascontiguousarray(db.x0[:16]).ravel().astype(np.float32)
    ut = torch.tensor(db.u_target[:16].ravel(), dtype=torch.float32, device=dev)
    outs = []
    for path in ("host", "device"):
        s = P.Solver(ps, max_iter=40, precision=P.PIMPC_FP32, ckpt_every=ck, stream=stream)
        if path == "host":
            u0h, info = s.solve(x0=x32.astype(np.float64))
            assert np.all(info["status"] == 0)
            u0 = torch.tensor(u0h, dtype=torch.float32, device=dev)
        else:
            x0 = torch.tensor(x32, device=dev)
            u0 = torch.empty(s.sum_nu, dtype=torch.float32, device=dev)
            P.pimpc_solve_batch(s.ctx, x0, None, u0, None, stream)
        grads = [torch.full((n,), float("nan"), device=dev) for n in (16 * 8, 16 * 8, 16 * 3, 16 * 64, 16 * 24)]
        P.pimpc_backward(s.ctx, P.pimpc_tape_id(s.ctx), 2 * (u0 - ut), *grads, stream=stream)
        torch.cuda.synchronize()
        outs.append([u0.cpu().numpy()] + [t.cpu().numpy() for t in grads])
        s.close()
    for a, b in zip(*outs):
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)
