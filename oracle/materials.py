"""Material interpolation for a two-phase voxel design.

Paper: Methods, "Topology optimization formulation", Eq. (9) interpolates
Young's modulus linearly in rho_e, while Eqs. (20)-(21) take the
derivatives of Omega and Phi as (rho^1 - rho^2) and (D^1 - D^2) times the
element integral, i.e. density and compliance linear in rho_e.  The two
are not the same.  Reading used here: density and compliance tensor are
affine in w_e = rho_e^p (SIMP exponent p, p = 1 reproduces Eqs. 20-21
exactly), rho_e = 0 is phase 0 (epoxy), rho_e = 1 is phase 1 (tungsten
carbide).

Compliance is written in Voigt form with engineering shear strain, so that
sigma : epsilon = sigma_V . epsilon_V and D_V maps sigma_V to epsilon_V.
"""
from __future__ import annotations

import numpy as np


def voigt_compliance(E: float, nu: float) -> np.ndarray:
    """Isotropic Voigt compliance (engineering shear strain)."""
    D = np.zeros((6, 6))
    D[:3, :3] = -nu / E
    np.fill_diagonal(D[:3, :3], 1.0 / E)
    G = E / (2.0 * (1.0 + nu))
    D[3, 3] = D[4, 4] = D[5, 5] = 1.0 / G
    return D


def voigt_stiffness(E: float, nu: float) -> np.ndarray:
    return np.linalg.inv(voigt_compliance(E, nu))


def simp_weight(rho: np.ndarray, p: float) -> np.ndarray:
    return np.asarray(rho, float) ** p


def simp_weight_derivative(rho: np.ndarray, p: float) -> np.ndarray:
    rho = np.asarray(rho, float)
    if p == 1.0:
        return np.ones_like(rho)
    return p * rho ** (p - 1.0)


def voxel_fields(rho: np.ndarray, p: float, phase0, phase1):
    """Per-voxel density (nv^3,) and Voigt compliance (nv^3, 6, 6), C order."""
    w = simp_weight(np.asarray(rho, float).reshape(-1), p)
    dens = phase0.density + w * (phase1.density - phase0.density)
    D0 = voigt_compliance(phase0.youngs, phase0.poisson)
    D1 = voigt_compliance(phase1.youngs, phase1.poisson)
    D = D0[None, :, :] + w[:, None, None] * (D1 - D0)[None, :, :]
    return dens, D


def phase_contrasts(phase0, phase1):
    """(Delta density, Delta D_V) = phase1 - phase0."""
    dD = voigt_compliance(phase1.youngs, phase1.poisson) - voigt_compliance(phase0.youngs, phase0.poisson)
    return phase1.density - phase0.density, dD


def wave_speeds(mat):
    """Longitudinal and transverse speeds of an isotropic phase (m/s)."""
    E, nu, r = mat.youngs, mat.poisson, mat.density
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return np.sqrt((lam + 2 * mu) / r), np.sqrt(mu / r)
