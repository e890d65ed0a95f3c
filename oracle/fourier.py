"""Centroid-rule Fourier coefficients of voxel fields by direct sums.

Paper: Methods, "Vectorization and parallel computations", Eqs. (16)-(19):
every matrix entry is an integral over the primitive cell of a material
field times exp[i 2 pi (K_p - K_q) . x], evaluated by the centroid rule
sum_e f^(e) v^(e).  Because (K_p - K_q) . x_e = (n_p - n_q) . s_e, the
integrals of Eqs. (6)-(7) only need, for each scalar field g,

    ghat(m) = v * sum_e g_e exp(i 2 pi m . s_e),   m in [-2M, 2M]^3,

with v = V / N_v^3.  The sum is written out directly (one axis at a time,
which is the same sum), in FP64.
"""
from __future__ import annotations

import numpy as np


def axis_phases(nv: int, M2: int) -> np.ndarray:
    """E[m, i] = exp(i 2 pi m (i + 1/2) / nv) for m in [-M2, M2]; shape (2*M2+1, nv)."""
    m = np.arange(-M2, M2 + 1)[:, None]
    s = (np.arange(nv) + 0.5)[None, :] / nv
    return np.exp(2j * np.pi * m * s)


def coefficients(field: np.ndarray, V: float, M2: int) -> np.ndarray:
    """ghat[m1+M2, m2+M2, m3+M2] for a scalar voxel field of shape (nv, nv, nv)."""
    g = np.asarray(field, dtype=float)
    nv = g.shape[0]
    assert g.shape == (nv, nv, nv)
    E = axis_phases(nv, M2)
    v = V / nv ** 3
    inner = g @ E.T  # (nv, nv, 2*M2+1): sum over i3
    out = np.einsum("ai,bj,ijc->abc", E, E, inner)  # sums over i1 and i2
    return v * out


def coefficients_bruteforce(field: np.ndarray, V: float, m: np.ndarray) -> np.ndarray:
    """The same sum as a plain loop over voxels, for a list of integer vectors m (k, 3)."""
    g = np.asarray(field, dtype=float).reshape(-1)
    nv = round(g.size ** (1 / 3))
    s = (np.stack(np.meshgrid(*(np.arange(nv),) * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) / nv
    v = V / nv ** 3
    return np.array([v * np.sum(g * np.exp(2j * np.pi * (s @ mm))) for mm in np.atleast_2d(m)])
