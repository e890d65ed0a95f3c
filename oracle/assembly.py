"""Literal assembly of the matrices of the mixed variational eigenproblem.

Paper: Results, "Phononic band structure calculation", Eqs. (5)-(7)
(H, Omega, Phi as integrals over the primitive cell), the unknown counts
of "Computation complexity and efficiency" (Omega 3N x 3N, Phi 6N x 6N,
H 3N x 6N with N = (2M+1)^3), and Methods, "Vectorization and parallel
computations", Eqs. (16)-(19) (centroid rule; the basic integral I_pq is
the outer product of the vector f with its own conjugate, summed over
elements).

Orientation (the paper's): entry (p, q) integrates against
exp[i 2 pi (K_p - K_q) . x].  Index of a displacement unknown: 3p + c
(c = x, y, z); of a stress unknown: 6p + r with r in Voigt order
(11, 22, 33, 23, 13, 12) and engineering shear strain ("tensorial
symmetries" of the paper, reading Q3).

H couples a displacement wave p to a stress wave q through the strain of
the displacement wave: H[(p,c), (q,r)] = i 2 pi I_pq B_V(K_p)[r, c] with
the 6x3 Voigt strain operator B_V.  With the centroid rule on an N_v^3
mesh with N_v > 2M, I_pq = V delta_pq exactly (tested), so which of the
two waves' K multiplies I in Eq. (5) makes no difference; meshes with
N_v <= 2M alias and are rejected.
"""
from __future__ import annotations

import numpy as np

from . import fourier, geometry, materials


def strain_operator(K: np.ndarray) -> np.ndarray:
    """6x3 Voigt operator: epsilon_V = i 2 pi B_V(K) U for u = U exp(i 2 pi K.x)."""
    k1, k2, k3 = K
    return np.array([[k1, 0, 0], [0, k2, 0], [0, 0, k3],
                     [0, k3, k2], [k3, 0, k1], [k2, k1, 0]], dtype=float)


def element_vectors(M: int, nv: int) -> np.ndarray:
    """f^(e)_p = exp(i 2 pi n_p . s_e) for every element (rows) and plane wave (cols), Eq. (18)."""
    n = geometry.plane_wave_indices(M)
    s = geometry.voxel_fractions(nv)
    return np.exp(2j * np.pi * (s @ n.T))


def basic_integral_outer(M: int, nv: int, V: float) -> np.ndarray:
    """I_pq = sum_e f^(e)_p conj(f^(e)_q) v^(e), Eq. (19), as the literal outer-product sum."""
    F = element_vectors(M, nv)
    v = V / nv ** 3
    return v * (F.T @ F.conj())


def basic_integral(M: int, nv: int, V: float) -> np.ndarray:
    """I_pq by the same centroid sum, evaluated through the coefficient table of g = 1."""
    ones = np.ones((nv, nv, nv))
    tab = fourier.coefficients(ones, V, 2 * M)
    return toeplitz_gather(tab, M)


def toeplitz_gather(tab: np.ndarray, M: int) -> np.ndarray:
    """G[p, q] = ghat(n_p - n_q) from a coefficient table indexed by m + 2M."""
    n = geometry.plane_wave_indices(M)
    d = n[:, None, :] - n[None, :, :] + 2 * M
    return tab[d[..., 0], d[..., 1], d[..., 2]]


class Operators:
    """k-independent matrices of one design: Omega (3N), Phi (6N), I (N)."""

    def __init__(self, lattice, a, nv, M, rho, phase0, phase1, simp_p):
        if nv < 2 * M + 1:
            raise ValueError("N_v must be at least 2M+1 (centroid rule aliases otherwise)")
        self.lattice, self.a, self.nv, self.M = lattice, a, nv, M
        self.A = geometry.primitive_vectors(lattice, a)
        self.T = geometry.reciprocal_vectors(self.A)
        self.V = geometry.cell_volume(self.A)
        self.n = geometry.plane_wave_indices(M)
        self.N = self.n.shape[0]
        rho = np.asarray(rho, float).reshape(nv, nv, nv)
        self.rho = rho
        self.simp_p = simp_p
        self.phase0, self.phase1 = phase0, phase1
        dens, D = materials.voxel_fields(rho, simp_p, phase0, phase1)
        self.dens, self.D = dens, D
        M2 = 2 * M
        dtab = fourier.coefficients(dens.reshape(nv, nv, nv), self.V, M2)
        Ds = np.zeros((6, 6) + dtab.shape, dtype=complex)
        for r in range(6):
            for c in range(r, 6):
                Ds[r, c] = fourier.coefficients(D[:, r, c].reshape(nv, nv, nv), self.V, M2)
                Ds[c, r] = Ds[r, c]
        self.dens_hat, self.D_hat = dtab, Ds
        N = self.N
        Os = toeplitz_gather(dtab, M)                      # N x N
        self.Omega = np.kron(Os, np.eye(3))               # (p, c) ordering
        Phi = np.zeros((N, 6, N, 6), dtype=complex)
        for r in range(6):
            for c in range(6):
                Phi[:, r, :, c] = toeplitz_gather(Ds[r, c], M)
        self.Phi = Phi.reshape(6 * N, 6 * N)
        self.I = basic_integral(M, nv, self.V)

    def H(self, Q) -> np.ndarray:
        """Coupling matrix of Eq. (5) at Bloch vector Q (reciprocal coordinates), 3N x 6N."""
        K = geometry.wavevectors(Q, self.n, self.T)
        N = self.N
        Hm = np.zeros((N, 3, N, 6), dtype=complex)
        for p in range(N):
            Bt = strain_operator(K[p]).T  # 3 x 6
            Hm[p, :, :, :] = (2j * np.pi) * self.I[p][None, :, None] * Bt[:, None, :]
        return Hm.reshape(3 * N, 6 * N)

    def wavevectors(self, Q) -> np.ndarray:
        return geometry.wavevectors(Q, self.n, self.T)
