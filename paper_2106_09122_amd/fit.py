"""Differentiable simulation through the PSF library, for fitting disk models.

``simulate`` is S = A Z as a ``torch.autograd.Function`` whose backward is the
adjoint A^T g (``psflib_apply_adjoint``); ``render_disk`` renders the
parametric disk with its parameter gradient (``psflib_render_disk`` and
``psflib_render_disk_grad``); ``chi2`` is the chi-square misfit with its
gradient in the image (``psflib_chi2``).  Chaining them gives d(loss)/d(theta);
``loss_and_grad`` runs the chain directly, without the autograd tape.  Both run the HIP kernels of libpsflib; torch only holds tensors and
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


def _float64_vec(x, name, M, dev):
    if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.device == dev
            and x.numel() == M):
        raise ValueError(f"{name} must be a float64 tensor of {M} elements on {dev}")
    return x.contiguous()


class _Chi2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, counts, var, K):
        S = model.detach().contiguous()
        if S.dtype != torch.float32:
            raise ValueError("model must be a float32 image")
        M = S.numel()
        D = _float64_vec(counts, "counts", M, S.device)
        V = _float64_vec(var, "var", M, S.device)
        loss = torch.empty((), dtype=torch.float64, device=S.device)
        grad = torch.empty_like(S)
        psflib.chi2(M, float(K), S.data_ptr(), D.data_ptr(), V.data_ptr(), loss.data_ptr(),
                    grad.data_ptr(), _stream(S.device))
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, gL):
        (grad,) = ctx.saved_tensors
        return grad * gL.to(grad.dtype), None, None, None


def chi2(model: torch.Tensor, counts: torch.Tensor, var: torch.Tensor, K: float) -> torch.Tensor:
    """sum_i (K S_i - D_i)^2 / var_i (``psflib_chi2``: float64, fixed-order sum),
    differentiable in the float32 image S (backward: 2 K (K S_i - D_i) / var_i
    from the same kernel)."""
    return _Chi2.apply(model, counts, var, K)


def loss_and_grad(lib, theta, counts, var, K, rmax):
    """Chi-square of the simulated disk image and its gradient in theta, every
    step in the library's kernels: render Z(theta), S = A Z, the chi-square and
    dL/dS, A^T (dL/dS), and dL/dtheta through the renderer's gradient.  Not to
    be captured in a graph (psflib_chi2 and psflib_render_disk_grad refuse a
    capturing stream)."""
    dev = counts.device
    th = theta.detach().to(device=dev, dtype=torch.float64).contiguous()
    st = _stream(dev)
    N = lib.N
    Z = torch.empty(N * N, dtype=torch.float32, device=dev)
    psflib.render_disk(N, lib.S, rmax, th.data_ptr(), Z.data_ptr(), st)
    S = lib.apply(Z)
    M = S.numel()
    D = _float64_vec(counts, "counts", M, dev)
    V = _float64_vec(var, "var", M, dev)
    L = torch.empty((), dtype=torch.float64, device=dev)
    gS = torch.empty_like(S)
    psflib.chi2(M, float(K), S.data_ptr(), D.data_ptr(), V.data_ptr(), L.data_ptr(), gS.data_ptr(), st)
    gZ = lib.apply_adjoint(gS)
    dth = torch.empty(5, dtype=torch.float64, device=dev)
    psflib.render_disk_grad(N, lib.S, rmax, th.data_ptr(), gZ.data_ptr(), dth.data_ptr(), st)
    return L, dth


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
