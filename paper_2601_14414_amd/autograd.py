"""Differentiable piMPC layer: torch.autograd.Function over the C ABI.

forward(x0, Qdiag, Rdiag, A, B) -> u0 for a batch of instances with equal
(nx, nu): re-factors the stage caches from the device tensors
(pimpc_set_params_dev), runs the taped batched solve (pimpc_solve_batch with
checkpoints every `ckpt_every` iterations, or every step recorded when it is
1) and returns u0 = du_0 of the last
step 1 (cold start, u(t-1) = 0).  backward(dL/du0) runs the adjoint kernels
(pimpc_backward) and returns dL/dx0, dL/dQdiag, dL/dRdiag, dL/dA, dL/dB.
PyTorch only provides memory and the stream; all arithmetic is in libpimpc.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import pimpc as P
from . import workloads as W


class PiMPCFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, Qdiag, Rdiag, A, B, solver):
        stream = torch.cuda.current_stream().cuda_stream
        x0c, Qc, Rc, Ac, Bc = (t.detach().contiguous().float() for t in (x0, Qdiag, Rdiag, A, B))
        P.pimpc_set_params_dev(solver.ctx, Ac, Bc, Qc, Rc, stream)
        u0 = torch.empty(solver.count * solver.nu, dtype=torch.float32, device=x0.device)
        info = torch.empty(solver.count * (P.INFO_DTYPE.itemsize // 4), dtype=torch.int32, device=x0.device)
        P.pimpc_solve_batch(solver.ctx, x0c, None, u0, info, stream)
        ctx.tape_id = P.pimpc_tape_id(solver.ctx)
        # a stage matrix that is not SPD (e.g. a negative weight) is reported
        # through the per-instance status of the info records
        status = info.view(solver.count, -1)[:, P.INFO_DTYPE.fields["status"][1] // 4]
        if bool((status != 0).any()):  # one reduction and one read-back; the index only on failure
            i = int(torch.nonzero(status).flatten()[0])
            raise P.PimpcError(int(status[i]), f"instance {i} of the differentiable batch failed "
                                               f"({'stage matrix not SPD' if int(status[i]) == P.PIMPC_E_NOT_PSD else 'non-finite iterate'})")
        ctx.solver = solver
        ctx.save_for_backward(x0c, Qc, Rc, Ac, Bc)  # keep the forward's inputs alive
        return u0.view(solver.count, solver.nu)

    @staticmethod
    def backward(ctx, gu0):
        solver = ctx.solver
        x0c, Qc, Rc, Ac, Bc = ctx.saved_tensors
        stream = torch.cuda.current_stream().cuda_stream
        g = gu0.detach().contiguous().float()
        dx0 = torch.empty_like(x0c)
        dQ = torch.empty_like(Qc)
        dR = torch.empty_like(Rc)
        dA = torch.empty_like(Ac)
        dB = torch.empty_like(Bc)
        P.pimpc_backward(solver.ctx, ctx.tape_id, g, dx0, dQ, dR, dA, dB, stream)
        return dx0, dQ, dR, dA, dB, None


class PiMPCLayer(torch.nn.Module):
    """Batch of `count` MPC instances of one shape (nx, nu, N) with box bounds,
    solved with `iters` plain ADMM iterations and differentiated through them.
    ckpt_every = k >= 2 keeps the iterate every k iterations and the backward
    re-runs each segment; ckpt_every = 1 records every step in the forward
    (2 nb + nx + 1 floats a stage and iteration) and the backward re-runs
    nothing."""

    def __init__(self, count: int, nx: int, nu: int, N: int, iters: int = 200, ckpt_every: int = 20,
                 rho: float = 1.0, xbound: float = 4.0, ubound: float = 0.5, Wdu=None):
        super().__init__()
        # Wdu: optional fixed (nu, nu) input-rate weight shared by the instances
        proto = W.Problem(nx=nx, nu=nu, N=N, A=np.eye(nx) * 0.9, B=np.ones((nx, nu)) / nx, Q=np.eye(nx),
                          R=0.1 * np.eye(nu), xmin=-xbound * np.ones(nx), xmax=xbound * np.ones(nx),
                          umin=-ubound * np.ones(nu), umax=ubound * np.ones(nu), x0=np.zeros(nx),
                          u_prev=np.zeros(nu), rho=rho, K=iters, Wdu=Wdu)
        self.solver = P.Solver([proto] * count, rho=rho, max_iter=iters, precision=P.PIMPC_FP32,
                               ckpt_every=ckpt_every,
                               stream=torch.cuda.current_stream().cuda_stream)
        self.solver.nu = nu

    def forward(self, x0, Qdiag, Rdiag, A, B):
        return PiMPCFunction.apply(x0, Qdiag, Rdiag, A, B, self.solver)
