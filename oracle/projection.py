"""Design parameterisation of the topology optimisation: Heaviside projection of a
reduced, optionally mirrored-octant design field.  Test infrastructure (oracle).

Paper: Methods, "Topology optimization formulation" (the Heaviside projection method with
design variables spaced at twice the element size, continuation on the Heaviside
parameter from 1, a projection radius) and "Study of cubic unit cells" (the SC design
optimised on one eighth of the cell, mirrored about the orthogonal mid-planes).  The paper
gives no formulas for these; this restates the projection method as published by Guest,
Prevost and Belytschko (2004) in the reading fixed for this build:

* elements e: the nv^3 voxels, centroids at i + 1/2 (element widths, per primitive axis);
* design nodes every `spacing` elements, node j at spacing j + spacing/2 (the centre of
  its block of elements); with the octant, nodes j < nn/2 carry the variables and node
  j >= nn/2 the value of node nn - 1 - j;
* w_en = max(0, r - |x_e - x_n|) with the periodic minimum-image distance;
* mu_e = sum_n w_en x_n / sum_n w_en;   rho_e = 1 - exp(-beta mu_e) + mu_e exp(-beta).

Written as dense matrices: rho = H(W E x / (W E 1)), with E the mirror expansion.
"""
from __future__ import annotations

import numpy as np


def node_count(nv: int, spacing: int, octant: bool) -> int:
    nn = nv // spacing
    return nn // 2 if octant else nn


def expansion(nv: int, spacing: int, octant: bool) -> np.ndarray:
    """E: full node grid (nn^3) from the design variables (node_count^3)."""
    nn = nv // spacing
    nd = node_count(nv, spacing, octant)
    mirror = np.array([j if (not octant or j < nn // 2) else nn - 1 - j for j in range(nn)])
    E = np.zeros((nn ** 3, nd ** 3))
    for j1 in range(nn):
        for j2 in range(nn):
            for j3 in range(nn):
                k = (mirror[j1] * nd + mirror[j2]) * nd + mirror[j3]
                E[(j1 * nn + j2) * nn + j3, k] = 1.0
    return E


def weights(nv: int, spacing: int, radius: float) -> np.ndarray:
    """W (nv^3 x nn^3): w_en = max(0, r - |x_e - x_n|), periodic minimum image."""
    nn = nv // spacing
    xe = np.arange(nv) + 0.5
    xn = spacing * np.arange(nn) + 0.5 * spacing
    d = xe[:, None] - xn[None, :]
    d = d - nv * np.round(d / nv)  # minimum image along the axis
    d2 = d ** 2
    dist = np.sqrt(d2[:, None, None, :, None, None] + d2[None, :, None, None, :, None]
                   + d2[None, None, :, None, None, :])
    return np.maximum(0.0, radius - dist).reshape(nv ** 3, nn ** 3)


def heaviside(mu: np.ndarray, beta: float) -> np.ndarray:
    return 1.0 - np.exp(-beta * mu) + mu * np.exp(-beta)


def heaviside_slope(mu: np.ndarray, beta: float) -> np.ndarray:
    return beta * np.exp(-beta * mu) + np.exp(-beta)


def filtered(x: np.ndarray, nv: int, spacing: int, radius: float, octant: bool) -> np.ndarray:
    """mu (nv^3) from the design variables."""
    W = weights(nv, spacing, radius)
    full = expansion(nv, spacing, octant) @ np.asarray(x, dtype=float).reshape(-1)
    return (W @ full) / W.sum(axis=1)


def project(x: np.ndarray, nv: int, spacing: int, radius: float, beta: float, octant: bool) -> np.ndarray:
    return heaviside(filtered(x, nv, spacing, radius, octant), beta).reshape(nv, nv, nv)


def project_adjoint(x: np.ndarray, grad_rho: np.ndarray, nv: int, spacing: int, radius: float, beta: float,
                    octant: bool) -> np.ndarray:
    """(d rho / d x)^T grad_rho = E^T W^T (H'(mu) grad_rho / (W 1))."""
    W = weights(nv, spacing, radius)
    E = expansion(nv, spacing, octant)
    mu = (W @ (E @ np.asarray(x, dtype=float).reshape(-1))) / W.sum(axis=1)
    c = heaviside_slope(mu, beta) * np.asarray(grad_rho, dtype=float).reshape(-1) / W.sum(axis=1)
    return E.T @ (W.T @ c)
