"""Brute-force companions of the oracle, for tiny inputs and closed forms.

* ``homogeneous_lambda``  uniform medium: every plane wave p gives one
  longitudinal and two transverse modes, lambda = (2 pi |K_p| c_L)^2 and
  (2 pi |K_p| c_T)^2 (Christoffel; the basis exp[i 2 pi K.x] of "Phononic
  band structure calculation" carries K in cycles per length).
* ``saddle_lambda``        Eq. (3) made stationary in displacement *and*
  stress without eliminating the stress: the unreduced pencil
  [[0, H], [H^*, -Phi]] vs [[Omega, 0], [0, 0]], solved by a general
  eigensolver (QZ).
* ``dlambda_materialised`` Eq. (15) with psi = Omega theta and the element
  derivative matrices of Eqs. (20)-(21) built explicitly.
* ``pwe_lambda``           the displacement-only plane-wave (Rayleigh
  quotient) comparator named in "Phononic band structure calculation":
  K_PWE = H Chat H^* / V^2 with Chat the Fourier matrix of the stiffness.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import assembly, fourier, geometry, materials


def homogeneous_lambda(lattice, a, M, Q, mat, nb):
    A = geometry.primitive_vectors(lattice, a)
    T = geometry.reciprocal_vectors(A)
    K = geometry.wavevectors(Q, geometry.plane_wave_indices(M), T)
    cl, ct = materials.wave_speeds(mat)
    k2 = np.sum(K ** 2, axis=1)
    lam = np.concatenate([(2 * np.pi) ** 2 * k2 * cl ** 2,
                          (2 * np.pi) ** 2 * k2 * ct ** 2,
                          (2 * np.pi) ** 2 * k2 * ct ** 2])
    return np.sort(lam)[:nb]


def saddle_lambda(ops, Q, nb):
    """Finite eigenvalues of the unreduced saddle-point pencil, lowest nb."""
    H = ops.H(Q)
    N3, N6 = 3 * ops.N, 6 * ops.N
    # Scale the stress unknowns so that Phi is O(1) and Omega so that it is O(1).
    sphi = 1.0 / np.max(np.abs(np.diag(ops.Phi)))
    som = 1.0 / np.max(np.abs(np.diag(ops.Omega)))
    Hs = H * np.sqrt(sphi)
    A = np.zeros((N3 + N6, N3 + N6), dtype=complex)
    A[:N3, N3:] = Hs
    A[N3:, :N3] = Hs.conj().T
    A[N3:, N3:] = -ops.Phi * sphi
    B = np.zeros_like(A)
    B[:N3, :N3] = ops.Omega * som
    w = sla.eig(A, B, right=False, homogeneous_eigvals=True)
    alpha, beta = w
    finite = np.abs(beta) > 1e-8 * np.max(np.abs(beta))
    lam = (alpha[finite] / beta[finite]).real * som
    return np.sort(lam)[:nb]


def dlambda_materialised(ops, fac, Q, lam, theta):
    """Eq. (15) literally, with Omega^{-1}, Phi^{-1} and the element matrices built densely."""
    H = ops.H(Q)
    Kmat = H @ sla.cho_solve(fac.cf, H.conj().T)
    Oinv = np.linalg.inv(ops.Omega)
    Pinv = sla.cho_solve(fac.cf, np.eye(ops.Phi.shape[0]))
    psi = ops.Omega @ theta  # left eigenvector with psi^H theta = 1
    F = assembly.element_vectors(ops.M, ops.nv)  # (Ne, N)
    v = ops.V / ops.nv ** 3
    drho, dD = materials.phase_contrasts(ops.phase0, ops.phase1)
    wp = materials.simp_weight_derivative(ops.rho.reshape(-1), ops.simp_p)
    out = np.zeros(F.shape[0])
    for e in range(F.shape[0]):
        fe = np.outer(F[e], F[e].conj()) * v  # f^(e)_pq v^(e): exp(i2pi(n_p - n_q).s_e)
        dOm = wp[e] * drho * np.kron(fe, np.eye(3))
        dPhi = wp[e] * np.kron(fe, dD)
        term1 = -Oinv @ dOm @ Oinv @ Kmat
        term2 = -Oinv @ (H @ Pinv @ dPhi @ Pinv @ H.conj().T)
        out[e] = np.real(psi.conj() @ ((term1 + term2) @ theta))
    return out


def pwe_lambda(ops, Q, nb):
    """Lowest nb eigenvalues of the displacement-only plane-wave pencil."""
    nv, M, V = ops.nv, ops.M, ops.V
    C = np.linalg.inv(ops.D)  # per-voxel Voigt stiffness
    Ch = np.zeros((6, 6, 4 * M + 1, 4 * M + 1, 4 * M + 1), dtype=complex)
    for r in range(6):
        for c in range(6):
            Ch[r, c] = fourier.coefficients(C[:, r, c].reshape(nv, nv, nv), V, 2 * M)
    N = ops.N
    Cm = np.zeros((N, 6, N, 6), dtype=complex)
    for r in range(6):
        for c in range(6):
            Cm[:, r, :, c] = assembly.toeplitz_gather(Ch[r, c], M)
    Cm = Cm.reshape(6 * N, 6 * N)
    H = ops.H(Q)
    Kp = H @ Cm @ H.conj().T / V ** 2
    Kp = 0.5 * (Kp + Kp.conj().T)
    return sla.eigh(Kp, ops.Omega, eigvals_only=True, subset_by_index=[0, nb - 1])
