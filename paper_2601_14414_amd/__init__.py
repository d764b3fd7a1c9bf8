"""piMPC on MI355X: parallel-in-horizon, construction-free ADMM for MPC.

Submodules:
  workloads  seeded problem generators (no solver arithmetic)
  pimpc      ctypes binding of the C-ABI library libpimpc.so (HIP, gfx950)
  autograd   torch.autograd.Function over the batched solve + adjoint
  rti        real-time-iteration driver (re-linearise, solve, apply u0)

Importing the package loads nothing native; `pimpc` loads the HIP library
on first use and raises if it is missing.
"""
__all__ = ["workloads"]
