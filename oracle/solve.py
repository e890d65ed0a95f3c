"""Stress elimination and the generalized Hermitian eigenproblem.

Paper: Results, "Phononic band structure calculation".  Stationarity of
the mixed quotient, Eq. (3), in the stress coefficients gives
S = Phi^{-1} H^* U, and eliminating them gives Eq. (4),
H Phi^{-1} H^* U = lambda Omega U with lambda = omega^2.  The paper calls
the operation "*" the complex conjugate; the reading here is the
conjugate transpose (reading Q4), which makes K = H Phi^{-1} H^* Hermitian
positive semi-definite and Omega Hermitian positive definite, so the
eigenvalues are real and non-negative and LAPACK's generalized Hermitian
solver applies (the paper's remark that the problem is asymmetric, in
"Topology optimization formulation", does not hold for this pencil,
reading Q5).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assembly import Operators


class PhiFactor:
    """Cholesky factor of the k-independent compliance matrix Phi."""

    def __init__(self, ops: Operators):
        self.ops = ops
        self.cf = sla.cho_factor(ops.Phi, lower=True, check_finite=False)

    def schur(self, Q) -> np.ndarray:
        """K(Q) = H Phi^{-1} H^*, Eq. (4), symmetrised."""
        H = self.ops.H(Q)
        X = sla.cho_solve(self.cf, H.conj().T, check_finite=False)
        K = H @ X
        return 0.5 * (K + K.conj().T)


def lowest_eigs(K: np.ndarray, Omega: np.ndarray, nb: int):
    """Lowest nb eigenpairs of K theta = lambda Omega theta (theta^H Omega theta = 1)."""
    lam, th = sla.eigh(K, Omega, subset_by_index=[0, nb - 1], driver="gvx", check_finite=False)
    return lam, th


def omega_from_lambda(lam: np.ndarray) -> np.ndarray:
    return np.sqrt(np.maximum(lam, 0.0))


def bands(cell, rho, Qs, nb, return_vectors=False):
    """omega (rad/s), shape (nk, nb), for every Bloch vector in Qs."""
    ops = Operators(cell.lattice, cell.a, cell.nv, cell.M, rho, cell.phase0, cell.phase1, cell.simp_p)
    fac = PhiFactor(ops)
    om = np.zeros((len(Qs), nb))
    vecs = []
    lams = np.zeros((len(Qs), nb))
    for i, Q in enumerate(Qs):
        K = fac.schur(Q)
        lam, th = lowest_eigs(K, ops.Omega, nb)
        lams[i] = lam
        om[i] = omega_from_lambda(lam)
        if return_vectors:
            vecs.append(th)
    if return_vectors:
        return om, lams, vecs, ops, fac
    return om
