"""Oracle pins of the design projection (Heaviside projection of a reduced, optionally
mirrored-octant design field; Methods, "Topology optimization formulation" and "Study of
cubic unit cells"): exact special cases, brute-force weights on tiny grids, the mirror
symmetry, and the adjoint against central finite differences."""
import itertools
import math

import numpy as np
import pytest

from oracle import projection as P


def _brute_weights(nv, sp, r):
    nn = nv // sp
    W = np.zeros((nv ** 3, nn ** 3))
    for e in itertools.product(range(nv), repeat=3):
        for n in itertools.product(range(nn), repeat=3):
            best = np.inf
            for img in itertools.product((-1, 0, 1), repeat=3):
                d = [e[a] + 0.5 - (sp * n[a] + 0.5 * sp) - nv * img[a] for a in range(3)]
                best = min(best, math.sqrt(sum(x * x for x in d)))
            W[(e[0] * nv + e[1]) * nv + e[2], (n[0] * nn + n[1]) * nn + n[2]] = max(0.0, r - best)
    return W


@pytest.mark.parametrize("nv,sp,r", [(6, 2, 1.5), (6, 1, 1.2), (8, 2, 2.8)])
def test_weights_match_brute_force(nv, sp, r):
    assert np.array_equal(P.weights(nv, sp, r), _brute_weights(nv, sp, r))


@pytest.mark.parametrize("sp,octant", [(1, False), (2, False), (2, True)])
def test_constant_design_passes_through_and_heaviside_fixes_0_and_1(sp, octant):
    nv = 8
    n = P.node_count(nv, sp, octant) ** 3
    for c in (0.0, 0.3, 1.0):
        mu = P.filtered(np.full(n, c), nv, sp, 2.8, octant)
        assert np.allclose(mu, c, rtol=0, atol=1e-15)
    for beta in (0.0, 1.0, 37.0):
        assert P.heaviside(np.array([0.0]), beta)[0] == 0.0
        assert P.heaviside(np.array([1.0]), beta)[0] == pytest.approx(1.0, abs=1e-15)


def test_beta_zero_is_the_linear_filter_and_large_beta_a_step():
    rng = np.random.default_rng(7)
    nv, sp = 8, 2
    x = rng.random(P.node_count(nv, sp, False) ** 3)
    mu = P.filtered(x, nv, sp, 2.8, False).reshape(nv, nv, nv)
    assert np.allclose(P.project(x, nv, sp, 2.8, 0.0, False), mu, rtol=0, atol=1e-15)
    hard = P.project(x, nv, sp, 2.8, 500.0, False)
    assert np.all(np.abs(hard[mu > 0.05] - 1.0) < 1e-10)


def test_single_node_response():
    """One unit design variable: mu_e = w_en / sum_m w_em, and with spacing 1 every element
    has the same weight sum, the lattice sum of max(0, r - |offset|) over integer offsets."""
    nv, sp, r = 8, 1, 1.8
    nn = nv
    x = np.zeros(nn ** 3)
    x[0] = 1.0
    mu = P.filtered(x, nv, sp, r, False)
    W = sum(max(0.0, r - math.sqrt(a * a + b * b + c * c)) for a, b, c in itertools.product(range(-2, 3), repeat=3))
    assert mu[0] == pytest.approx(r / W, rel=1e-14)
    assert mu[1] == pytest.approx((r - 1.0) / W, rel=1e-14)                   # face neighbour
    assert mu[nv * nv + nv + 1] == pytest.approx((r - math.sqrt(3)) / W, rel=1e-14)  # corner neighbour
    assert mu[2] == 0.0


def test_octant_design_is_mirror_symmetric():
    rng = np.random.default_rng(3)
    nv, sp = 16, 2
    x = rng.random(P.node_count(nv, sp, True) ** 3)
    rho = P.project(x, nv, sp, 2.8, 4.0, True)
    assert np.allclose(rho, rho[::-1, :, :], rtol=0, atol=1e-15)
    assert np.allclose(rho, rho[:, ::-1, :], rtol=0, atol=1e-15)
    assert np.allclose(rho, rho[:, :, ::-1], rtol=0, atol=1e-15)


@pytest.mark.parametrize("sp,octant,beta", [(1, False, 1.0), (2, False, 8.0), (2, True, 3.0)])
def test_adjoint_matches_central_differences(sp, octant, beta):
    rng = np.random.default_rng(11)
    nv, r = 8, 2.2
    n = P.node_count(nv, sp, octant) ** 3
    x = rng.random(n)
    g = rng.standard_normal(nv ** 3)
    adj = P.project_adjoint(x, g, nv, sp, r, beta, octant)
    h = 1e-6
    for i in rng.choice(n, 6, replace=False):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (g @ P.project(xp, nv, sp, r, beta, octant).reshape(-1)
              - g @ P.project(xm, nv, sp, r, beta, octant).reshape(-1)) / (2 * h)
        assert adj[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


# ----------------------------------------------------------------------------- density filter

@pytest.mark.parametrize("r", [0.7, 1.5, 2.2])
def test_oracle_hat_filter_pins(r):
    """The oracle's voxel filter: a constant field is unchanged, the mean is preserved, the
    operator (built column by column on a 5^3 grid) is symmetric with unit row sums, a
    radius below one voxel leaves the field as it is, and a single voxel spreads to weights
    that fall linearly with distance and vanish at the radius."""
    from oracle import filter as filt
    rng = np.random.default_rng(5)
    x = rng.random((7, 7, 7))
    assert np.allclose(filt.hat_filter(np.full((7, 7, 7), 0.3), r), 0.3, atol=1e-15)
    assert abs(filt.hat_filter(x, r).sum() - x.sum()) < 1e-12
    n = 5
    Fm = np.zeros((n ** 3, n ** 3))
    for j in range(n ** 3):
        e = np.zeros(n ** 3)
        e[j] = 1
        Fm[:, j] = filt.hat_filter(e.reshape(n, n, n), min(r, 2.0)).reshape(-1)
    assert np.allclose(Fm, Fm.T, atol=1e-15) and np.allclose(Fm.sum(axis=1), 1, atol=1e-14)
    if r < 1:
        assert np.allclose(filt.hat_filter(x, r), x, atol=1e-15)
    d = np.zeros((7, 7, 7))
    d[3, 3, 3] = 1
    y = filt.hat_filter(d, r)
    # weights relative to the centre: (r - |offset|) / r along an axis, zero beyond r
    for k in range(0, 3):
        expect = max(0.0, r - k) / r
        assert abs(y[3 + k, 3, 3] / y[3, 3, 3] - expect) < 1e-14


def test_oracle_hat_filter_matches_the_library_kernel_on_the_cpu():
    """The product path's filter (a torch convolution) and the oracle's sum agree; both are
    CPU operations here, so this runs without a GPU."""
    import torch

    from oracle import filter as filt
    from paper_1603_06855_amd import optimize
    rng = np.random.default_rng(6)
    x = rng.random((9, 9, 9))
    for r in (1.5, 2.2):
        got = optimize.density_filter(torch.from_numpy(x), optimize.hat_kernel(r)).numpy()
        assert np.abs(got - filt.hat_filter(x, r)).max() < 1e-14
