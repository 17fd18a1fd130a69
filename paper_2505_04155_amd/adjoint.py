"""Differentiable solve x = A(theta)^{-1} b for the finite-volume diffusion
operator with cell coefficients exp(theta), behind torch.autograd.

Forward: assemble A(theta) on the device (amp_fv_csr), refresh the matrix
and Jacobi handles, AMP-PCG solve.  Backward: the adjoint lambda = A^{-1} g
is one more AMP-PCG solve with the same (symmetric) matrix; dL/db = lambda;
dL/dtheta comes from the per-cell face gather amp_fv_grad_theta.  Every
numerical step runs in libamppcg.so.
"""

from __future__ import annotations

import ctypes

import torch

from . import binding as B
from .solver import Matrix, Preconditioner, _ptr, _stream, solve


class FVSystem:
    """A(theta) on a fixed dim-dimensional grid; shape = (nz, ny, nx) or (ny, nx)."""

    def __init__(self, shape, device="cuda", preset="amp64", tol=1e-10, maxit=20000, **opts):
        shape = tuple(int(s) for s in shape)
        if len(shape) not in (2, 3):
            raise ValueError("shape must be (ny, nx) or (nz, ny, nx)")
        self.shape = shape
        self.dim = len(shape)
        self.nx, self.ny = shape[-1], shape[-2]
        self.nz = shape[0] if self.dim == 3 else 1
        self.n = self.nx * self.ny * self.nz
        L = B.load()
        nnz = ctypes.c_int64()
        B.check(L.amp_fv_nnz(self.dim, self.nx, self.ny, self.nz, ctypes.byref(nnz)), "amp_fv_nnz")
        self.device = torch.device(device)
        self.row_ptr = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        self.col_idx = torch.empty(nnz.value, dtype=torch.int32, device=self.device)
        self.val = torch.empty(nnz.value, dtype=torch.float64, device=self.device)
        self.A = None
        self.M = None
        self.theta_version = None
        self.preset, self.tol, self.maxit, self.opts = preset, tol, maxit, opts
        self.last_info = {}

    def assemble(self, theta: torch.Tensor):
        theta = theta.detach().to(self.device, torch.float32).contiguous().reshape(-1)
        if theta.numel() != self.n:
            raise ValueError(f"theta must have {self.n} entries")
        L = B.load()
        B.check(L.amp_fv_csr(self.dim, self.nx, self.ny, self.nz, _ptr(theta), _ptr(self.row_ptr),
                             _ptr(self.col_idx), _ptr(self.val), _stream()), "amp_fv_csr")
        if self.A is None:
            self.A = Matrix(self.row_ptr, self.col_idx, self.val)
            self.M = Preconditioner(self.A, "jacobi")
        else:
            csr = B.Csr(self.n, self.col_idx.numel(), self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                        self.val.data_ptr())
            B.check(L.amp_matrix_update_values(self.A.handle, ctypes.byref(csr), _stream()),
                    "amp_matrix_update_values")
            B.check(L.amp_precond_update(self.M.handle, _stream()), "amp_precond_update")
        self.theta = theta

    def solve(self, rhs: torch.Tensor):
        x, info = solve(self.A, self.M, rhs.detach().to(self.device, torch.float64).contiguous().reshape(-1),
                        tol=self.tol, maxit=self.maxit, preset=self.preset, raise_on_error=True, **self.opts)
        self.last_info = info
        return x

    def grad_theta(self, x: torch.Tensor, lam: torch.Tensor):
        out = torch.empty(self.n, dtype=torch.float32, device=self.device)
        B.check(B.load().amp_fv_grad_theta(self.dim, self.nx, self.ny, self.nz, _ptr(self.theta), _ptr(x),
                                           _ptr(lam), _ptr(out), _stream()), "amp_fv_grad_theta")
        return out


class DiffSolve(torch.autograd.Function):
    """x = A(theta)^{-1} b; gradients for theta (float32, grid-shaped) and b."""

    @staticmethod
    def forward(ctx, theta, b, system: FVSystem):
        system.assemble(theta)
        x = system.solve(b)
        ctx.system = system
        ctx.theta_shape = theta.shape
        ctx.save_for_backward(theta.detach().clone(), x)
        return x

    @staticmethod
    def backward(ctx, gx):
        theta, x = ctx.saved_tensors
        system = ctx.system
        if not torch.equal(system.theta, theta.to(system.device, torch.float32).reshape(-1)):
            system.assemble(theta)
        lam = system.solve(gx.contiguous())
        dtheta = system.grad_theta(x, lam).reshape(ctx.theta_shape)
        return dtheta, lam, None


def diff_solve(theta: torch.Tensor, b: torch.Tensor, system: FVSystem) -> torch.Tensor:
    return DiffSolve.apply(theta, b, system)
