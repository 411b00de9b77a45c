"""torch.autograd.Function for the misfit J(v) of section 2 / eq. (2).

``J = fwi_misfit(v, problem)`` runs the forward sweep of every shot in the
HIP library (``fwi_misfit_forward``): it records the traces, keeps each
shot's sqrt(nt) FP32 snapshots and per-step boundary strips in the problem's
workspace, and returns J (float64 scalar on the device).  ``J.backward()``
calls ``fwi_misfit_backward``: the hand-written adjoint kernel reconstructs
the source wavefield backwards from those checkpoints, propagates the
adjoint wavefield and accumulates dJ/dv, scaled by the incoming gradient.
The eq. (1) illumination H1 and the offset-Hessian diagonal D come out of the
same backward sweep as side outputs (``problem.illum``, ``problem.offset``).

The gradient is taken on the model cells with the sponge padding held fixed
(the padding replicates the model's edge cells), so directional derivatives
agree with it for directions that vanish on the model's outermost cells.
"""
from __future__ import annotations

import torch

from . import binding as B


class FWIProblem:
    """Everything J(v) depends on besides v, resident on the device."""

    def __init__(self, grid, geom, wavelet, d_obs, misfit="int", exec_=None, illum=True, hmax=None,
                 rcv_model="pm", device="cuda"):
        self.grid = grid
        self.geom = B.GeometryC(geom)
        self.ntrace = geom.ntrace
        self.exec = exec_
        self.misfit = misfit
        self.wavelet, self.wstride = B._wavelet(wavelet, grid.nt_max, device)
        self.d_obs = B._dev(d_obs, torch.float32, device)
        self.hmax = hmax
        self.rcv_model = rcv_model
        self.want_illum = illum
        self.device = device
        self.ws = B.workspace(grid, self.geom, B.WS_AUTOGRAD, exec_, hmax or 0, device=device)
        self.illum = None
        self.offset = None


class FWIMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, problem: FWIProblem):
        pr = problem
        vd = v.detach()
        if vd.dtype != torch.float32 or not vd.is_contiguous():
            raise ValueError("v must be a contiguous float32 device tensor")
        J = torch.empty((), dtype=torch.float64, device=v.device)
        B.fwi_misfit_forward(pr.grid, pr.geom, pr.exec, vd, pr.wavelet, pr.wstride, pr.d_obs, pr.misfit, J,
                             pr.ws, pr.ws.numel())
        ctx.problem = pr
        ctx.save_for_backward(vd)
        return J

    @staticmethod
    def backward(ctx, gJ):
        pr = ctx.problem
        (vd,) = ctx.saved_tensors
        grad = torch.empty_like(vd)
        scale = gJ.detach().to(torch.float64).contiguous()
        g = pr.grid
        pr.illum = torch.empty((g.nz, g.nx), dtype=torch.float32, device=vd.device) if pr.want_illum else None
        pr.offset = None
        if pr.hmax is not None:
            pr.offset = torch.empty((2 * pr.hmax + 1, g.nz, g.nx), dtype=torch.float32, device=vd.device)
        B.fwi_misfit_backward(pr.grid, pr.geom, pr.exec, vd, pr.wavelet, pr.wstride, scale, grad, pr.illum,
                              pr.hmax or 0, pr.rcv_model, pr.offset, pr.ws, pr.ws.numel())
        return grad, None


def fwi_misfit(v, problem: FWIProblem):
    """J(v) as a differentiable float64 scalar."""
    return FWIMisfit.apply(v, problem)
