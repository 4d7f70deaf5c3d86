"""Differentiable simulation through the PSF library, for fitting disk models.

``simulate`` is S = A Z as a ``torch.autograd.Function`` whose backward is the
adjoint A^T g (``psflib_apply_adjoint``); ``render_disk`` renders the
parametric disk with its parameter gradient (``psflib_render_disk`` and
``psflib_render_disk_grad``).  Chaining them gives d(loss)/d(theta) for any
loss written in torch on the simulated image, e.g. the chi-square of
``chi2``.  Both run the HIP kernels of libpsflib; torch only holds tensors and
the autograd tape.  This is the gradient analogue of the parameter retrieval
the paper's conclusions plan (Sec. 5).
"""
from __future__ import annotations

import math

import torch

from . import psflib


def _stream(dev):
    return torch.cuda.current_stream(dev).cuda_stream


class _Simulate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Z, lib):
        ctx.lib = lib
        return lib.apply(Z.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.lib.apply_adjoint(g.contiguous().to(torch.float32)), None


def simulate(lib: "psflib.Library", Z: torch.Tensor) -> torch.Tensor:
    """S = A Z, differentiable in Z (backward: A^T g)."""
    return _Simulate.apply(Z, lib)


class _RenderDisk(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, N, S, rmax):
        theta = theta.detach().to(torch.float64).contiguous()
        Z = torch.empty(N * N, dtype=torch.float32, device=theta.device)
        psflib.render_disk(N, S, rmax, theta.data_ptr(), Z.data_ptr(), _stream(theta.device))
        ctx.save_for_backward(theta)
        ctx.geom = (N, S, rmax)
        return Z

    @staticmethod
    def backward(ctx, dZ):
        (theta,) = ctx.saved_tensors
        N, S, rmax = ctx.geom
        dZ = dZ.contiguous().to(torch.float32)
        dth = torch.empty(5, dtype=torch.float64, device=theta.device)
        psflib.render_disk_grad(N, S, rmax, theta.data_ptr(), dZ.data_ptr(), dth.data_ptr(),
                                _stream(theta.device))
        return dth, None, None, None


def render_disk(theta: torch.Tensor, N: int, S: float, rmax: float) -> torch.Tensor:
    """Disk scene for theta = (incl [rad], r0, width, gamma, flux) (float64 CUDA [5])."""
    return _RenderDisk.apply(theta, N, S, rmax)


def chi2(model: torch.Tensor, counts: torch.Tensor, var: torch.Tensor, K: float) -> torch.Tensor:
    """sum_i (K S_i - D_i)^2 / var_i, accumulated in float64."""
    r = K * model.to(torch.float64) - counts
    return (r * r / var).sum()


def loss_and_grad(lib, theta, counts, var, K, rmax):
    """Chi-square of the simulated disk image and its gradient in theta."""
    th = theta.detach().clone().requires_grad_(True)
    L = chi2(simulate(lib, render_disk(th, lib.N, lib.S, rmax)), counts, var, K)
    L.backward()
    return L.detach(), th.grad.detach()


def fit_disk(lib, counts, var, K, theta0, rmax, steps: int = 64, lr: float = 0.05):
    """Adam on the chi-square, in coordinates where every parameter moves on a
    comparable scale: theta = (incl, r0 e^u1, w e^u2, gamma, F e^u4) with u = 0
    at theta0.  Returns (theta, losses)."""
    dev = counts.device
    t0 = torch.as_tensor(theta0, dtype=torch.float64, device=dev)
    u = torch.zeros(5, dtype=torch.float64, device=dev, requires_grad=True)
    opt = torch.optim.Adam([u], lr=lr)
    logm = torch.tensor([0.0, 1.0, 1.0, 0.0, 1.0], dtype=torch.float64, device=dev)

    def theta_of(u):
        return torch.where(logm > 0, t0 * torch.exp(u), t0 + u)

    losses = []
    for _ in range(steps):
        opt.zero_grad()
        L = chi2(simulate(lib, render_disk(theta_of(u), lib.N, lib.S, rmax)), counts, var, K)
        L.backward()
        opt.step()
        losses.append(float(L.detach()))
    return theta_of(u).detach(), losses
