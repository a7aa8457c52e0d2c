"""torch.autograd wrapper of the checkpointed RK4 flow and its discrete adjoint.

``rk4_flow(x0, sys, dt, nsteps, K, pparams=None, pp_slot=(), gparams=None,
kahan=False)`` returns x(T) = Phi^nsteps(x0) computed by
``ff_integrate_checkpointed``; its backward calls ``ff_adjoint`` and returns
dL/dx0, dL/d(per-particle parameters) and, if ``gparams`` (a float64 tensor of
the system's global parameter values) is given, dL/d(global parameters)
summed over particles in FP64.  All arithmetic happens in the HIP kernels.
"""
from __future__ import annotations

import torch

from . import api as A


class RK4Flow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, pparams, gparams, sys, dt, nsteps, K, pp_slot, kahan):
        if gparams is not None:
            sys.set_params([float(v) for v in gparams.detach().cpu().tolist()])
        # the values this pass runs with: the system may be given others
        # before backward (another flow on it, or the caller)
        ctx.params = sys.get_params()
        x = x0.detach().clone().contiguous()
        pp = None if pparams is None else pparams.detach().contiguous()
        comp = torch.zeros_like(x) if kahan else None
        nbytes = A.adjoint_workspace_size(sys, x, nsteps, K, pparams=pp, pp_slot=pp_slot, comp=comp)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=x.device)
        A.integrate_checkpointed(sys, x, dt, nsteps, K, ws, pparams=pp, pp_slot=pp_slot, comp=comp)
        ctx.sys, ctx.dt, ctx.nsteps, ctx.K, ctx.pp_slot, ctx.kahan = sys, dt, nsteps, K, tuple(pp_slot), kahan
        ctx.ws, ctx.pp, ctx.has_g = ws, pp, gparams is not None
        ctx.gdtype = None if gparams is None else gparams.dtype
        ctx.shape_x = x.shape
        return x

    @staticmethod
    def backward(ctx, grad_xT):
        lam = grad_xT.detach().contiguous().clone()
        pp = ctx.pp
        mu = None if pp is None else torch.empty_like(pp)
        mu_g = torch.empty(ctx.sys.n_params, dtype=torch.float64, device=lam.device) if ctx.has_g else None
        # the reverse sweep runs with the forward pass's parameters; the
        # launch takes them by value, so the caller's are restored right after
        current = ctx.sys.get_params()
        if current != ctx.params:
            ctx.sys.set_params(ctx.params)
        try:
            # the batch only describes the particles here; its state is not read
            A.adjoint(ctx.sys, lam, ctx.dt, ctx.nsteps, ctx.K, ctx.ws, lam, mu=mu, mu_global=mu_g,
                      pparams=pp, pp_slot=ctx.pp_slot, prec="fp32_kahan" if ctx.kahan else None)
        finally:
            if current != ctx.params:
                ctx.sys.set_params(current)
        g_global = None if mu_g is None else mu_g.to(ctx.gdtype)
        return lam, mu, g_global, None, None, None, None, None, None


def rk4_flow(x0, sys, dt, nsteps, K, pparams=None, pp_slot=(), gparams=None, kahan=False):
    return RK4Flow.apply(x0, pparams, gparams, sys, dt, nsteps, K, tuple(pp_slot), kahan)
