"""Differentiable Vegas estimate of a Gaussian integral.

VegasIntegral.apply(mu, a, vegas, n_events) returns the estimate of
integral_[0,1]^d (a sqrt(pi))^-d exp(-sum_i (x_i - mu_i)^2 / a^2) dx from one
iteration of n_events events on the context's current grid (the grid is
frozen: nothing is refined, and the iteration is not recorded, so any number
of forward passes fit one context).  Its backward pass regenerates the same
points (counter-based Philox, same iteration index) and runs the library's
adjoint kernel, which returns (1/M) sum_e w_e df/dtheta(x_e) for
theta = (mu, a), times the incoming gradient.  Nothing per event is stored
between the passes.

The backward pass needs the grid and parameters its forward pass used.  If
the context's parameters changed in between (another forward pass on the same
context, say), they are set back for the adjoint and restored afterwards; if
its grid changed (a refinement, new edges or a loaded state), backward raises.
"""
from __future__ import annotations

import torch

from .integrator import Vegas


class VegasIntegral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu: torch.Tensor, a: torch.Tensor, vegas: Vegas, n_events: int):
        if vegas.desc.integrand != 0:
            raise ValueError("VegasIntegral needs a Gaussian-integrand context")
        d = vegas.dim
        if mu.numel() != d or a.numel() != 1:
            raise ValueError(f"mu must have {d} elements and a one")
        # parameter layout of the Gaussian integrand: a, mu[0..d-1]; FP32
        # parameters go to the library as they are (it widens them, exactly)
        pt = torch.float32 if mu.dtype == torch.float32 and a.dtype == torch.float32 else torch.float64
        params = torch.cat([a.detach().reshape(1).to(pt), mu.detach().reshape(-1).to(pt)])
        vegas.set_params_device(params)
        t = vegas.iteration_index
        # frozen grid: no histograms (the sums are bitwise those of the
        # histogram variant) and no record slot
        vegas.iterate(n_events, refine=False, combine=False, hist=False, record=False)
        out = torch.empty(2, dtype=torch.float64, device=mu.device)
        vegas.last_iteration_device(out)
        ctx.vegas, ctx.t, ctx.n = vegas, t, n_events
        ctx.params = params  # a tensor of its own: nothing else writes it
        ctx.versions = vegas.versions()
        ctx.mu_meta = (mu.dtype, mu.shape)
        ctx.a_meta = (a.dtype, a.shape)
        return out[0]

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        v: Vegas = ctx.vegas
        d = v.dim
        grid_v, params_v = v.versions()
        if grid_v != ctx.versions[0]:
            raise RuntimeError("VegasIntegral.backward: the context's grid changed after the forward pass "
                               "(refinement, set_edges or set_state); the adjoint needs the forward grid")
        restore = None
        if params_v != ctx.versions[1]:
            restore = v.get_params_device()
            v.set_params_device(ctx.params)
        g = gout.detach().to(torch.float64).reshape(1).contiguous()
        mu_dtype, mu_shape = ctx.mu_meta
        a_dtype, a_shape = ctx.a_meta
        if mu_dtype == a_dtype and mu_dtype in (torch.float32, torch.float64):
            # the adjoint writes the parameters' dtype itself
            grad = torch.empty(d + 1, dtype=mu_dtype, device=g.device)
            v.adjoint(ctx.t, ctx.n, g, grad)
            gmu, ga = grad[:d].reshape(mu_shape), grad[d].reshape(a_shape)
        else:
            grad = torch.empty(d + 1, dtype=torch.float64, device=g.device)
            v.adjoint(ctx.t, ctx.n, g, grad)
            gmu, ga = grad[:d].to(mu_dtype).reshape(mu_shape), grad[d].to(a_dtype).reshape(a_shape)
        if restore is not None:
            v.set_params_device(restore)
        return gmu, ga, None, None


def vegas_integral(mu: torch.Tensor, a: torch.Tensor, vegas: Vegas, n_events: int) -> torch.Tensor:
    return VegasIntegral.apply(mu, a, vegas, n_events)
