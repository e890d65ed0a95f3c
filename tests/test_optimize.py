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
