"""Density filter of the optimisation loop, written out as a plain sum.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's optimiser works on a reduced design field through a projection
(Methods, "Topology optimization formulation"); the plain loop the library
drives by default (reading Q18 of the build's readings) filters design
variables x on the voxel grid itself:

    rho_e = sum_j w(d_ej) x_j / sum_j w(d_ej),   w(d) = max(0, r - d),

with d_ej the distance between voxel indices e and j taken with periodic
wrap (minimum image, in voxel widths).  Every voxel sees the same offsets,
so the denominator is one constant and the operator is symmetric; its
transpose (the backward) is the same sum.
"""
from __future__ import annotations

import numpy as np


def hat_filter(x: np.ndarray, radius: float) -> np.ndarray:
    """rho (nv, nv, nv) from x (nv, nv, nv): the normalised periodic hat average."""
    nv = x.shape[0]
    out = np.zeros_like(x, dtype=float)
    den = 0.0
    n = int(np.ceil(radius))
    for a in range(-n, n + 1):
        for b in range(-n, n + 1):
            for c in range(-n, n + 1):
                w = max(0.0, radius - np.sqrt(a * a + b * b + c * c))
                if w == 0.0:
                    continue
                # x shifted so that out[e] accumulates x[e + (a, b, c)] (indices mod nv)
                out += w * np.roll(x, (-a, -b, -c), axis=(0, 1, 2))
                den += w
    assert 2 * n + 1 <= nv, "the filter radius must stay below half the cell"
    return out / den


def hat_filter_adjoint(g: np.ndarray, radius: float) -> np.ndarray:
    """d (sum_e g_e rho_e) / d x: the transpose of hat_filter, the same symmetric sum."""
    return hat_filter(g, radius)
