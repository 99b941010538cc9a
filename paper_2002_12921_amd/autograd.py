"""Differentiable Vegas estimate of a Gaussian integral.

VegasIntegral.apply(mu, a, vegas, n_events) returns the estimate of
integral_[0,1]^d (a sqrt(pi))^-d exp(-sum_i (x_i - mu_i)^2 / a^2) dx from one
iteration of n_events events on the context's current grid (the grid is
frozen: nothing is refined).  Its backward pass regenerates the same points
(counter-based Philox, same iteration index) and runs the library's adjoint
kernel, which returns (1/M) sum_e w_e df/dtheta(x_e) for theta = (mu, a), times
the incoming gradient.  Nothing per event is stored between the passes.
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
        params = torch.cat([a.detach().reshape(1).to(pt), mu.detach().reshape(-1).to(pt)]).contiguous()
        vegas.set_params_device(params)
        t = vegas.iteration_index
        # frozen grid: no histograms (the sums are bitwise those of the
        # histogram variant)
        vegas.iterate(n_events, refine=False, combine=False, hist=False)
        out = torch.empty(2, dtype=torch.float64, device=mu.device)
        vegas.last_iteration_device(out)
        ctx.vegas, ctx.t, ctx.n = vegas, t, n_events
        ctx.mu_meta = (mu.dtype, mu.shape)
        ctx.a_meta = (a.dtype, a.shape)
        return out[0]

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        v: Vegas = ctx.vegas
        d = v.dim
        g = gout.detach().to(torch.float64).reshape(1).contiguous()
        grad = torch.empty(d + 1, dtype=torch.float64, device=g.device)
        v.adjoint(ctx.t, ctx.n, g, grad)
        mu_dtype, mu_shape = ctx.mu_meta
        a_dtype, a_shape = ctx.a_meta
        return grad[:d].to(mu_dtype).reshape(mu_shape), grad[d].to(a_dtype).reshape(a_shape), None, None


def vegas_integral(mu: torch.Tensor, a: torch.Tensor, vegas: Vegas, n_events: int) -> torch.Tensor:
    return VegasIntegral.apply(mu, a, vegas, n_events)
