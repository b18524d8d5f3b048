"""torch.autograd wrapper: forward modelling with the adjoint gradient.

``FictitiousForward.apply(log_rho, plan)`` returns E at the receivers
(complex128 [ns][nr][ncomp][nf]) for the resistivity exp(log_rho) (shape
[nz][ny][nx]; or [2][nz][ny][nx] = (ln rho_h, ln rho_v) for a VTI model,
whose gradient then has the same two parts, Section 3.1); its
backward returns d loss / d log_rho (Section 3.5 chain rule) by one of two
adjoints:
  method="basis" (default)  one adjoint simulation driven by the
      basis-function adjoint sources (Section 3.3); the forward keeps the
      volume transform of E, the frequency-domain checkpoint that is all the
      gradient needs (``snapshot_every`` is not used);
  method="time"  the time-domain adjoint of the Appendix on the stepped
      system (exact, also inside the CPML): the backward reruns the forward
      with checkpoints every ``snapshot_every`` steps (200 if 0) and steps the
      transposed system backward.

PyTorch hands the backward the conjugate Wirtinger gradient
gE = dL/dRe E + i dL/dIm E; for the data misfit L = 1/2 ||W (d - E)||^2
this is -W^2 (d - E), so the library's weighted residual is -gE.

One plan may serve several forwards before their backwards (a loss summed
over models): a backward whose model is no longer the plan's (the plan's
model serial moved on) sets it again, and rebuilds the basis if the time
step changed, before the adjoint.
"""
from __future__ import annotations

import numpy as np
import torch

from .fwdem import Plan


class FictitiousForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_rho: torch.Tensor, plan: Plan, snapshot_every: int = 0,
                gamma_rel: float = 1e-12, method: str = "basis"):
        rho = torch.exp(log_rho.detach().to(torch.float64)).cpu().numpy()
        _set_model(plan, rho)
        ctx.serial = plan.model_serial
        ctx.rho = rho
        ctx.gamma_rel = gamma_rel
        ctx.plan = plan
        ctx.method = method
        ctx.snapshot_every = snapshot_every
        ctx.in_dtype = log_rho.dtype
        ctx.in_device = log_rho.device
        if method == "time":
            ctx.vol = None
            return plan.forward()
        if method != "basis":
            raise ValueError(f"unknown adjoint method {method!r}")
        if not plan.info.have_basis:
            plan.basis_build(gamma_rel=gamma_rel)
        E, vol = plan.forward(vol=plan.volume_buffer(), want_volume=True)
        ctx.vol = vol
        return E

    @staticmethod
    def backward(ctx, gE):
        plan: Plan = ctx.plan
        if plan.model_serial != ctx.serial:
            # the plan's model changed since this forward: restore ours
            _set_model(plan, ctx.rho)
            if ctx.method == "basis" and not plan.info.have_basis:
                plan.basis_build(gamma_rel=ctx.gamma_rel)
            ctx.serial = plan.model_serial
        resid = (-gE).to(torch.complex128).contiguous()
        if ctx.method == "time":
            grad = plan.adjoint_td(resid, segment=ctx.snapshot_every or 200)
        else:
            grad = plan.adjoint(ctx.vol, resid)
        return grad.to(dtype=ctx.in_dtype, device=ctx.in_device), None, None, None, None


def _set_model(plan: Plan, rho: np.ndarray) -> None:
    """rho [nz][ny][nx], or [2][nz][ny][nx] = (rho_h, rho_v) for VTI, whose
    gradient is then split (FWD_OPT_VTI_GRADIENT)."""
    from .fwdem import FWD_OPT_VTI_GRADIENT
    vti = rho.ndim == 4
    if vti:
        plan.set_model(rho[0], rho[1])
    else:
        plan.set_model(rho)
    plan.set_option(FWD_OPT_VTI_GRADIENT, 1 if vti else 0)


def misfit(E: torch.Tensor, d: torch.Tensor, W=1.0) -> torch.Tensor:
    """phi_d = 1/2 sum |W (d - E)|^2 (eq. phid, electric data)."""
    r = (d - E) * W
    return 0.5 * (r.real ** 2 + r.imag ** 2).sum()
