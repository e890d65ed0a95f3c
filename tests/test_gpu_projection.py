"""GPU: the design projection (Heaviside projection of a reduced, optionally mirrored-octant
design field) through the C ABI against the oracle, forward and adjoint, host and device
entry points, and the rejection of invalid projections."""
import numpy as np
import pytest

from paper_1603_06855_amd import phx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = phx.Context(0)
    yield c
    c.close()


# the mirrored octant needs an even node count per axis (nv / sp), so (18, 2) runs without it
GEOMETRIES = [(16, 1, 1.5, False), (16, 2, 2.8, False), (18, 2, 1.2, False), (12, 1, 0.7, False),
              (16, 1, 1.5, True), (16, 2, 2.8, True), (12, 1, 0.7, True), (12, 2, 1.2, True)]


@pytest.mark.parametrize("nv,sp,r,octant", GEOMETRIES)
@pytest.mark.parametrize("beta", [0.0, 1.0, 8.0, 64.0])
def test_projection_matches_oracle(ctx, nv, sp, r, octant, beta):
    from oracle import projection as P
    assert not octant or (nv // sp) % 2 == 0
    p = phx.projection(nv, sp, r, beta, octant)
    n = phx.projection_size(p)
    rng = np.random.default_rng(nv * 100 + sp * 10 + int(beta))
    x = rng.random(n)
    g = rng.standard_normal(nv ** 3)
    rho = ctx.project(p, x)
    ref = P.project(x, nv, sp, r, beta, octant)
    assert np.abs(rho - ref).max() <= 1e-14
    adj = ctx.project_adjoint(p, x, g)
    aref = P.project_adjoint(x, g, nv, sp, r, beta, octant)
    assert np.abs(adj - aref).max() <= 1e-12 * np.abs(aref).max()


def test_device_entry_points_match_host(ctx):
    import torch
    p = phx.projection(32, 2, 2.8, 4.0, True)
    n = phx.projection_size(p)
    rng = np.random.default_rng(5)
    x = rng.random(n)
    g = rng.standard_normal(32 ** 3)
    rd = ctx.project_dev(p, torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    ad = ctx.project_adjoint_dev(p, torch.from_numpy(x).to("cuda:0"), torch.from_numpy(g).to("cuda:0")).cpu().numpy()
    assert np.array_equal(rd, ctx.project(p, x))
    assert np.array_equal(ad, ctx.project_adjoint(p, x, g))


@pytest.mark.parametrize("bad", [dict(nv=15, spacing=2), dict(radius=0.8), dict(radius=8.0), dict(beta=-1.0),
                                 dict(nv=18, spacing=2, octant=True)])
def test_invalid_projection_is_rejected(ctx, bad):
    kw = dict(nv=16, spacing=2, radius=2.8, beta=1.0, octant=False)
    kw.update(bad)
    p = phx.Projection(kw["nv"], kw["spacing"], kw["radius"], kw["beta"], 1 if kw["octant"] else 0)
    x = np.zeros(8 ** 3)
    rc = ctx.lib.phx_project(ctx.h, phx.byref(p), phx._dptr(x), phx._dptr(np.zeros(kw["nv"] ** 3)))
    assert rc == phx.EINVAL
