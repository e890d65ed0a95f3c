"""Design sensitivities of the eigenvalues.

Paper: Methods, "Topology optimization formulation", Eqs. (12)-(15), and
"Vectorization and parallel computations", Eqs. (20)-(21).

For the Hermitian pencil (reading Q5) the left eigenvector of Eq. (12) is
psi = Omega theta with theta^H Omega theta = 1, and Eq. (15) becomes

    d lambda / d rho_e = - lambda theta^H Omega'_e theta - S^H Phi'_e S,
    S = Phi^{-1} H^* theta   (the stress coefficients).

Eqs. (20)-(21) make Omega'_e and Phi'_e single-element outer products
f^(e) f^(e)H v^(e) times the phase contrasts (times w'(rho_e) for the SIMP
weight), so both quadratic forms are field energies at the element
centroid:

    theta^H Omega'_e theta = v w'_e Drho |u_e|^2,
    S^H Phi'_e S          = v w'_e sigma_e^H DD_V sigma_e,

with u_e = sum_q theta_q exp(-i 2 pi n_q . s_e) and
sigma_e = sum_p S_p exp(-i 2 pi n_p . s_e) (the Bloch factor cancels in
the moduli).  ``dlambda_fields`` evaluates this form; ``dlambda_materialised``
in ``brute`` evaluates Eq. (15) with the matrices of Eqs. (20)-(21) built
explicitly, for tiny inputs.  d omega / d rho = (d lambda / d rho) / (2 omega),
taken as 0 where omega = 0 (the acoustic bands at Gamma).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import materials


def _synthesise(coef: np.ndarray, M: int, nv: int) -> np.ndarray:
    """g_e = sum_p coef_p exp(-i 2 pi n_p . s_e) for coef on the (2M+1)^3 wave grid; (nv^3,)."""
    m = np.arange(-M, M + 1)[None, :]
    s = (np.arange(nv) + 0.5)[:, None] / nv
    E = np.exp(-2j * np.pi * s * m)  # (nv, 2M+1)
    c = coef.reshape(2 * M + 1, 2 * M + 1, 2 * M + 1)
    g = np.einsum("ia,jb,kc,abc->ijk", E, E, E, c)
    return g.reshape(-1)


def fields(ops, theta: np.ndarray, S: np.ndarray):
    """Displacement (nv^3, 3) and Voigt stress (nv^3, 6) at the element centroids."""
    N, M, nv = ops.N, ops.M, ops.nv
    th = theta.reshape(N, 3)
    Sv = S.reshape(N, 6)
    u = np.stack([_synthesise(th[:, c], M, nv) for c in range(3)], axis=1)
    sig = np.stack([_synthesise(Sv[:, r], M, nv) for r in range(6)], axis=1)
    return u, sig


def stress_coefficients(ops, fac, Q, theta: np.ndarray) -> np.ndarray:
    H = ops.H(Q)
    return sla.cho_solve(fac.cf, H.conj().T @ theta, check_finite=False)


def dlambda_fields(ops, fac, Q, lam: float, theta: np.ndarray) -> np.ndarray:
    """d lambda / d rho_e for one Omega-normalised eigenvector; (nv^3,)."""
    S = stress_coefficients(ops, fac, Q, theta)
    u, sig = fields(ops, theta, S)
    drho, dD = materials.phase_contrasts(ops.phase0, ops.phase1)
    wp = materials.simp_weight_derivative(ops.rho.reshape(-1), ops.simp_p)
    v = ops.V / ops.nv ** 3
    kin = drho * np.sum(np.abs(u) ** 2, axis=1)
    pot = np.real(np.einsum("er,rc,ec->e", sig.conj(), dD, sig))
    return -v * wp * (lam * kin + pot)


def sum_rules(ops, fac, Q, lam: float, theta: np.ndarray):
    """(sum_e v rho_e |u_e|^2, sum_e v sigma_e^H D_e sigma_e); equal 1 and lambda exactly."""
    S = stress_coefficients(ops, fac, Q, theta)
    u, sig = fields(ops, theta, S)
    v = ops.V / ops.nv ** 3
    kin = np.sum(v * ops.dens * np.sum(np.abs(u) ** 2, axis=1))
    pot = np.real(np.sum(v * np.einsum("er,erc,ec->e", sig.conj(), ops.D, sig)))
    return kin, pot


def domega(lam: float, dlam: np.ndarray) -> np.ndarray:
    om = np.sqrt(max(lam, 0.0))
    if om == 0.0:
        return np.zeros_like(dlam)
    return dlam / (2.0 * om)


def sensitivities(cell, rho, Qs, nb, bands_1based):
    """omega (nk, nb) and d omega / d rho (nk, len(bands), nv^3)."""
    from .solve import bands as _bands
    om, lams, vecs, ops, fac = _bands(cell, rho, Qs, nb, return_vectors=True)
    out = np.zeros((len(Qs), len(bands_1based), ops.nv ** 3))
    for i, Q in enumerate(Qs):
        for j, b in enumerate(bands_1based):
            lam = lams[i, b - 1]
            dl = dlambda_fields(ops, fac, Q, lam, vecs[i][:, b - 1])
            out[i, j] = domega(lam, dl)
    return om, out
