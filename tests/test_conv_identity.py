"""CPU: the identity the Omega_s convolution kernel rests on, checked in NumPy.

Omega_s[p][q] is the density's Fourier coefficient at n_p - n_q (Eqs. (6)-(7)), a
Toeplitz matrix over the wave grid [-M, M]^3, so Omega_s x is the linear convolution of
the table (differences [-2M, 2M]^3) with x.  On a cyclic grid of L2 = 4M + 1 points per
axis no difference wraps: DFTs of length L2 along n3 and n2, a Toeplitz product along n1
with the table transformed along n2 and n3 (with the inverse transforms' 1/L2^2), and the
inverse DFTs reproduce the dense product up to rounding, also in the basis that pairs each
wave with its opposite (where the operator of a real field is real symmetric).  One point
fewer per axis (4M) wraps, and the result is wrong.  This pins the reasoning, not the
kernel: the GPU tests compare the kernel with the dense product and the solves with the
oracle.
"""
import numpy as np
import pytest


def dense_omega(T, M):
    """Omega_s[p][q] = T[n_p - n_q], waves lexicographic in n (n1 slowest)."""
    L = 2 * M + 1
    n = np.array([(a1, a2, a3) for a1 in range(L) for a2 in range(L) for a3 in range(L)]) - M
    d = n[:, None, :] - n[None, :, :] + 2 * M
    return T[d[..., 0], d[..., 1], d[..., 2]]


def pairing(N):
    """U: columns u_p = (e_p + e_pb)/sqrt2, u_pb = i (e_p - e_pb)/sqrt2, u_c = e_c."""
    c = (N - 1) // 2
    U = np.zeros((N, N), complex)
    r = np.sqrt(0.5)
    for p in range(c):
        pb = N - 1 - p
        U[p, p] = U[pb, p] = r
        U[p, pb], U[pb, pb] = 1j * r, -1j * r
    U[c, c] = 1
    return U


def convolve(T, x, M, L2):
    """The kernel's stages on plane-wave coefficients x (length (2M+1)^3), cyclic length L2."""
    L = 2 * M + 1
    m = np.arange(L) - M
    g = np.arange(L2)
    F = np.exp(-2j * np.pi * np.outer(g, m) / L2)        # forward, L2 x L
    G = np.exp(+2j * np.pi * np.outer(m, g) / L2)        # inverse (unnormalised), L x L2
    dd = np.arange(4 * M + 1) - 2 * M
    E = np.exp(-2j * np.pi * np.outer(g, dd) / L2)       # table transform, L2 x (4M+1)
    Ch = np.einsum("adf,bd,cf->abc", T, E, E) / L2 ** 2  # [d1][g2][g3]
    X = x.reshape(L, L, L)
    X = np.einsum("ga,xya->xyg", F, X)                   # along n3
    X = np.einsum("gb,xbz->xgz", F, X)                   # along n2
    i = np.arange(L)
    Y = np.einsum("ijyz,jyz->iyz", Ch[i[:, None] - i[None, :] + 2 * M], X)  # Toeplitz along n1
    Y = np.einsum("bg,xgz->xbz", G, Y)                   # back along n2
    Y = np.einsum("ag,xyg->xya", G, Y)                   # back along n3
    return Y.reshape(-1)


def hermitian_table(M, seed):
    """The Fourier table of a real field: T[-d] = conj(T[d])."""
    rng = np.random.default_rng(seed)
    L2 = 4 * M + 1
    idx = (np.arange(L2) - 2 * M) % L2
    return np.fft.fftn(rng.standard_normal((L2, L2, L2)))[np.ix_(idx, idx, idx)]


@pytest.mark.parametrize("M", [1, 2, 3])
def test_convolution_equals_the_dense_product(M):
    T = hermitian_table(M, 7 + M)
    N = (2 * M + 1) ** 3
    Om = dense_omega(T, M)
    rng = np.random.default_rng(M)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = Om @ x
    got = convolve(T, x, M, 4 * M + 1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("M", [1, 2, 3])
def test_paired_basis_operator_is_real_and_matches(M):
    T = hermitian_table(M, 11 + M)
    N = (2 * M + 1) ** 3
    U = pairing(N)
    Or = U.conj().T @ dense_omega(T, M) @ U
    assert np.abs(Or.imag).max() <= 1e-12 * np.abs(Or).max()
    assert np.allclose(Or.real, Or.real.T, rtol=0, atol=1e-12 * np.abs(Or).max())
    rng = np.random.default_rng(100 + M)
    y = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = Or.real @ y
    got = U.conj().T @ convolve(T, U @ y, M, 4 * M + 1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("M", [1, 2, 3])
def test_one_point_fewer_wraps(M):
    T = hermitian_table(M, 23 + M)
    N = (2 * M + 1) ** 3
    rng = np.random.default_rng(200 + M)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = dense_omega(T, M) @ x
    # with 4M points the extreme differences +-2M alias onto each other
    got = convolve(T[:, :, :], x, M, 4 * M)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()
