"""The band-gap optimisation driver: density filter properties on the CPU; a short
optimisation on the GPU (objective rises, a resumed run repeats the uninterrupted one)."""
import numpy as np
import pytest
import torch

from paper_1603_06855_amd import optimize


@pytest.mark.parametrize("r", [1.5, 2.2])
def test_hat_filter_is_normalised_symmetric_and_mean_preserving(r):
    w = optimize.hat_kernel(r)
    assert abs(float(w.sum()) - 1.0) < 1e-15
    assert torch.equal(w, w.flip(0)) and torch.equal(w, w.flip(1)) and torch.equal(w, w.flip(2))
    assert torch.equal(w, w.permute(1, 0, 2)) and torch.equal(w, w.permute(2, 1, 0))
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.random((9, 9, 9)))
    y = torch.from_numpy(rng.random((9, 9, 9)))
    fx = optimize.density_filter(x, w)
    assert abs(float(fx.sum() - x.sum())) < 1e-12
    # a symmetric kernel with periodic wrap is a self-adjoint operator
    assert abs(float((fx * y).sum() - (x * optimize.density_filter(y, w)).sum())) < 1e-12
    # a constant field is left unchanged, a single voxel spreads to exactly the kernel
    assert torch.allclose(optimize.density_filter(torch.ones(7, 7, 7, dtype=torch.float64), w),
                          torch.ones(7, 7, 7, dtype=torch.float64), atol=1e-15)
    d = torch.zeros(9, 9, 9, dtype=torch.float64)
    d[4, 4, 4] = 1
    n = w.shape[0] // 2
    assert torch.allclose(optimize.density_filter(d, w)[4 - n:5 + n, 4 - n:5 + n, 4 - n:5 + n], w)


@pytest.mark.gpu
def test_short_optimisation_rises_and_resumes(tmp_path):
    from paper_1603_06855_amd import phx, synth
    ctx = phx.Context(0)
    cell = synth.Cell("SC", 1.0, 10, 2)
    rho0 = synth.box_smoothed_uniform(10, 501)
    q = phx.kpath("SC", 10, "GXMGR")
    a = optimize.GapOptimizer(ctx, cell, q, 8, 6, rho0, "fp64", step=0.02)
    h = a.run(4)
    print("ks gap", h.ks_gap, "gap", h.gap, flush=True)
    assert h.ks_gap[-1] > h.ks_gap[0]
    b = optimize.GapOptimizer(ctx, cell, q, 8, 6, rho0, "fp64", step=0.02)
    path = str(tmp_path / "ck.npz")
    b.run(2, checkpoint=path, every=1)
    c = optimize.GapOptimizer(ctx, cell, q, 8, 6, rho0, "fp64", step=0.02)
    c.load(path)
    c.run(4)
    # same trajectory (the filter's convolution may accumulate in a different order)
    assert np.allclose(c.hist.ks_gap, h.ks_gap, rtol=1e-10, atol=0)
    assert float((c.x - a.x).abs().max()) <= 1e-9
    ctx.close()


@pytest.mark.gpu
def test_command_line_run_reports_the_final_higher_order_gap(capsys):
    """The driver's summary line carries the final design's gap re-evaluated one order up."""
    import json
    optimize.main(["--lattice", "SC", "--nv", "12", "--M", "2", "--nk", "12", "--iters", "2", "--precision", "fp64"])
    lines = [json.loads(l) for l in capsys.readouterr().out.splitlines() if l.startswith("{")]
    summary = lines[-1]
    assert summary["iters"] == 2 and summary["final_M"] == 3
    assert summary["gap_final_M"] is not None and abs(summary["gap_final_M"] - summary["gap_last"]) < 0.2


@pytest.mark.gpu
def test_projected_octant_optimisation_rises_and_stays_symmetric():
    """The paper's SC setting: design variables on every second element's node, one octant
    mirrored, Heaviside projection with beta doubling from 1; the KS gap rises and the
    physical design keeps the mirror symmetry."""
    from paper_1603_06855_amd import phx, synth
    ctx = phx.Context(0)
    cell = synth.Cell("SC", 1.0, 16, 2)
    rho0 = synth.sphere(16, "SC", 0.35) * 0.6 + 0.2
    q = phx.kpath("SC", 10, "GXMGR")
    hpm = optimize.HPM(spacing=2, radius=2.8, octant=True, beta0=1.0, beta_max=8.0, beta_every=2)
    a = optimize.GapOptimizer(ctx, cell, q, 8, 6, rho0, "fp64", step=0.05, hpm=hpm)
    assert tuple(a.x.shape) == (4, 4, 4)
    h = a.run(5)
    print("ks gap", h.ks_gap, "gap", h.gap, flush=True)
    assert h.ks_gap[-1] > h.ks_gap[0]
    rho = a.physical().cpu().numpy()
    assert np.allclose(rho, rho[::-1], atol=1e-14) and np.allclose(rho, rho[:, :, ::-1], atol=1e-14)
    assert hpm.beta(5) == 4.0
    ctx.close()


@pytest.mark.gpu
def test_projection_autograd_matches_the_oracle_adjoint():
    import torch

    from oracle import projection as P
    from paper_1603_06855_amd import autograd, phx
    ctx = phx.Context(0)
    p = phx.projection(16, 2, 2.8, 3.0, False)
    rng = np.random.default_rng(2)
    x = rng.random(phx.projection_size(p)).reshape(8, 8, 8)
    g = rng.standard_normal((16, 16, 16))
    xt = torch.from_numpy(x).to("cuda:0").requires_grad_(True)
    rho = autograd.project(xt, ctx, p)
    (rho * torch.from_numpy(g).to("cuda:0")).sum().backward()
    ref = P.project_adjoint(x, g, 16, 2, 2.8, 3.0, False)
    assert np.abs(xt.grad.cpu().numpy().reshape(-1) - ref).max() <= 1e-12 * np.abs(ref).max()
    ctx.close()
