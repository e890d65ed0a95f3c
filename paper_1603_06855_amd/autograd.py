"""Band frequencies as a differentiable function of the design field (PyTorch).

``BandFrequencies.apply(rho, problem)`` returns omega (nk, nbands) on the
device; its backward is the adjoint of Eq. (15) (Methods, "Topology
optimization formulation") evaluated in field-energy form by the HIP
library (``phx_adjoint_dev``): d omega / d rho_e is reduced on the device into
one weighted gradient.  Nothing is kept between forward and backward: the
eigenvectors of the k-points that the backward needs are recomputed, which
at large M costs less memory than storing 3N x nbands vectors per k.  Two
ways to pick what the backward recomputes:

* ``Problem.backward_bands`` given (the KS objective, whose weights touch every
  k): those bands at every k-point, the incoming gradient's columns passed as
  device weights with no copy to the host;
* otherwise only the (k, band) entries with a non-zero incoming gradient,
  found on the host (one small device-to-host copy): the hard min/max of
  Eq. (10) touches two k-points.

``normalized_gap`` is Eq. (10) on frequencies (every gap the paper reports is
a frequency ratio); ``ks_gap`` replaces its min/max over k by
Kreisselmeier-Steinhauser aggregates, so every k contributes to the gradient.
Both are plain torch expressions on omega, so torch supplies their partial
derivatives and the library supplies d omega / d rho.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np
import torch

from . import phx


@dataclass
class Problem:
    """What a band-structure evaluation needs besides the design."""
    ctx: "phx.Context"
    cell: object            # synth.Cell-like (lattice, a, nv, M, phase0, phase1, simp_p)
    q: np.ndarray           # (nk, 3) reciprocal coordinates
    nbands: int
    precision: str = "fp64"
    backward_bands: Optional[Tuple[int, ...]] = None  # 1-based; see the module docstring


class BandFrequencies(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho: torch.Tensor, prob: Problem) -> torch.Tensor:
        if not rho.is_cuda:
            raise ValueError("rho must be a device tensor")
        om = prob.ctx.bands_dev(prob.cell, rho.reshape(-1), prob.q, prob.nbands, prob.precision)
        ctx.save_for_backward(rho)
        ctx.prob = prob
        return om

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (rho,) = ctx.saved_tensors
        prob: Problem = ctx.prob
        if prob.backward_bands is not None:
            cols = torch.tensor([b - 1 for b in prob.backward_bands], device=g.device)
            w = g.detach().to(torch.float64).index_select(1, cols).contiguous()
            grad = prob.ctx.adjoint_dev(prob.cell, rho.reshape(-1), prob.q, prob.nbands, prob.backward_bands, w,
                                        prob.precision)
            return grad.reshape(rho.shape).to(rho.dtype), None
        gh = g.detach().to("cpu", torch.float64).numpy()
        ks = np.nonzero(np.any(gh != 0, axis=1))[0]
        bs = np.nonzero(np.any(gh != 0, axis=0))[0]
        if len(ks) == 0:
            return torch.zeros_like(rho), None
        w = torch.from_numpy(np.ascontiguousarray(gh[np.ix_(ks, bs)])).to(rho.device)
        q = np.ascontiguousarray(np.asarray(prob.q, dtype=np.float64).reshape(-1, 3)[ks])
        grad = prob.ctx.adjoint_dev(prob.cell, rho.reshape(-1), q, prob.nbands, [int(b) + 1 for b in bs], w,
                                    prob.precision)
        return grad.reshape(rho.shape).to(rho.dtype), None


class DesignProjection(torch.autograd.Function):
    """rho = the Heaviside projection of the design variables x (``phx_project_dev``); the
    backward is ``phx_project_adjoint_dev``."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, lib_ctx: "phx.Context", p: "phx.Projection") -> torch.Tensor:
        if not x.is_cuda:
            raise ValueError("x must be a device tensor")
        ctx.save_for_backward(x)
        ctx.lib_ctx, ctx.p = lib_ctx, p
        return lib_ctx.project_dev(p, x)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (x,) = ctx.saved_tensors
        return ctx.lib_ctx.project_adjoint_dev(ctx.p, x, g).to(x.dtype), None, None


def project(x: torch.Tensor, lib_ctx: "phx.Context", p: "phx.Projection") -> torch.Tensor:
    return DesignProjection.apply(x, lib_ctx, p)


def band_frequencies(rho: torch.Tensor, prob: Problem) -> torch.Tensor:
    return BandFrequencies.apply(rho, prob)


def normalized_gap(omega: torch.Tensor, t: int) -> torch.Tensor:
    """Eq. (10) between bands t and t+1 (1-based): 2 (a - b) / (a + b), a = min_k omega_{t+1},
    b = max_k omega_t."""
    a = omega[:, t].min()
    b = omega[:, t - 1].max()
    return 2.0 * (a - b) / (a + b)


def ks_max(x: torch.Tensor, beta: float) -> torch.Tensor:
    m = x.max().detach()
    return m + torch.log(torch.exp(beta * (x - m)).sum()) / beta


def ks_gap(omega: torch.Tensor, t: int, beta: float, scale: Optional[float] = None) -> torch.Tensor:
    """Eq. (10) with the min/max over k replaced by KS aggregates of omega / scale."""
    if scale is None:
        scale = float(omega[:, t].detach().mean())
    a = -ks_max(-omega[:, t] / scale, beta) * scale
    b = ks_max(omega[:, t - 1] / scale, beta) * scale
    return 2.0 * (a - b) / (a + b)
