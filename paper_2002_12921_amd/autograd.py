"""Differentiable Vegas estimate of a Gaussian integral.

VegasIntegral.apply(mu, a, vegas, n_events, fused) returns the estimate of
integral_[0,1]^d (a sqrt(pi))^-d exp(-sum_i (x_i - mu_i)^2 / a^2) dx from one
iteration of n_events events on the context's current grid (the grid is
frozen: nothing is refined, and the iteration is not recorded, so any number
of forward passes fit one context).  Its gradient with respect to (mu, a) is
(1/M) sum_e w_e df/dtheta(x_e) over the same events, at fixed samples and
grid, times the incoming gradient.

fused=True (the default): the forward launch itself also sums the gradient
terms (vegas_iterate_grad: the same events and the same estimate, bit for
bit), so backward only scales d + 1 numbers.  fused=False: the backward pass
regenerates the same points (counter-based Philox, same iteration index) in
the library's adjoint kernel (vegas_adjoint); nothing per event is stored
between the passes, but it needs the forward's grid and parameters: if the
context's parameters changed in between (another forward pass on the same
context, say), they are set back for the adjoint and restored afterwards; if
its grid changed (a refinement, new edges or a loaded state), backward raises.
"""
from __future__ import annotations

import torch

from .integrator import Vegas


class VegasIntegral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu: torch.Tensor, a: torch.Tensor, vegas: Vegas, n_events: int, fused: bool = True):
        if vegas.desc.integrand != 0:
            raise ValueError("VegasIntegral needs a Gaussian-integrand context")
        d = vegas.dim
        if mu.numel() != d or a.numel() != 1:
            raise ValueError(f"mu must have {d} elements and a one")
        if not (mu.is_cuda and a.is_cuda):
            raise ValueError("mu and a must be GPU tensors")
        # parameter layout of the Gaussian integrand: a, mu[0..d-1]; FP32
        # parameters go to the library as they are (it widens them, exactly)
        pt = torch.float32 if mu.dtype == torch.float32 and a.dtype == torch.float32 else torch.float64
        ctx.G = None
        if fused:
            # one library call: the parameters, then the frozen-grid iteration
            # (no histograms, no record slot) whose launch also sums the
            # gradient terms, its (I_t, sigma_t) written to out; a and mu go
            # as two arrays when they already have the type (no concatenation)
            buf = torch.empty(d + 3, dtype=torch.float64, device=mu.device)
            G, out = buf[:d + 1], buf[d + 1:]
            if a.dtype == pt and mu.dtype == pt and mu.is_contiguous():
                vegas._forward_grad(a.detach(), n_events, G, out, mu.detach())
            else:
                params = torch.cat([a.detach().reshape(1).to(pt), mu.detach().reshape(-1).to(pt)])
                vegas._forward_grad(params, n_events, G, out)
            ctx.G = G
        else:
            params = torch.cat([a.detach().reshape(1).to(pt), mu.detach().reshape(-1).to(pt)])
            out = torch.empty(2, dtype=torch.float64, device=mu.device)
            vegas.set_params_device(params)
            ctx.t = vegas.iteration_index
            # frozen grid: no histograms (the sums are bitwise those of the
            # histogram variant) and no record slot
            vegas.iterate(n_events, refine=False, combine=False, hist=False, record=False)
            vegas.last_iteration_device(out)
            ctx.params = params  # a tensor of its own: nothing else writes it
            ctx.versions = vegas.versions()
        ctx.vegas, ctx.n = vegas, n_events
        ctx.mu_meta = (mu.dtype, mu.shape)
        ctx.a_meta = (a.dtype, a.shape)
        return out[0]

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        v: Vegas = ctx.vegas
        d = v.dim
        g = gout.detach().to(torch.float64).reshape(1).contiguous()
        mu_dtype, mu_shape = ctx.mu_meta
        a_dtype, a_shape = ctx.a_meta
        same = mu_dtype == a_dtype and mu_dtype in (torch.float32, torch.float64)
        # the library writes the parameters' dtype itself (one rounding)
        grad = torch.empty(d + 1, dtype=mu_dtype if same else torch.float64, device=g.device)
        if ctx.G is not None:
            v._grad_scale(ctx.G, g, grad)
        else:
            grid_v, params_v = v.versions()
            if grid_v != ctx.versions[0]:
                raise RuntimeError("VegasIntegral.backward: the context's grid changed after the forward pass "
                                   "(refinement, set_edges or set_state); the adjoint needs the forward grid")
            restore = None
            if params_v != ctx.versions[1]:
                restore = v.get_params_device()
                v.set_params_device(ctx.params)
            v.adjoint(ctx.t, ctx.n, g, grad)
            if restore is not None:
                v.set_params_device(restore)
        if same:
            return grad[:d].reshape(mu_shape), grad[d].reshape(a_shape), None, None, None
        return grad[:d].to(mu_dtype).reshape(mu_shape), grad[d].to(a_dtype).reshape(a_shape), None, None, None


def vegas_integral(mu: torch.Tensor, a: torch.Tensor, vegas: Vegas, n_events: int, fused: bool = True) -> torch.Tensor:
    return VegasIntegral.apply(mu, a, vegas, n_events, fused)
