"""Band-gap maximisation driver (the optimisation loop around the band solver).

Each iteration: density filter of the design variables, band frequencies and their
adjoint through ``autograd.BandFrequencies`` (the HIP library), the normalised gap of
Eq. (10) with its min/max over k replaced by Kreisselmeier-Steinhauser aggregates, and
a projected-gradient ascent step on the design variables (Methods, "Topology
optimization formulation": maximise Eq. (10) subject to 0 <= rho_e <= 1, Eq. (11)).

Settings not fixed by the paper: KS parameter beta on omega / omega_ref (omega_ref =
the mean of band t+1 at the first iteration), a linear "hat" density filter of radius r
voxels with periodic wrap, and the step rho <- clip(rho + eta g / max|g|, 0, 1).  The
filter and the step run as PyTorch operations on the device; the band structure and its
adjoint run in the library.  A run can be check-pointed to an ``.npz`` file (design,
iteration, history) and resumed from it.

With ``hpm`` the design variables instead live on nodes every `spacing` elements (the
paper's reduced design field) and the physical density is their Heaviside projection
(``phx_project_dev``, backward ``phx_project_adjoint_dev``), with continuation on the
Heaviside parameter from 1; ``octant`` optimises one eighth of the cell, mirrored about
its mid-planes, as the paper does for SC.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch
import torch.nn.functional as F

from . import autograd, phx


def hat_kernel(radius: float) -> torch.Tensor:
    """Normalised linear-decay weights w(d) = max(0, r - |d|) on the integer offsets |d| < r."""
    n = int(np.floor(radius - 1e-12))
    ax = torch.arange(-n, n + 1, dtype=torch.float64)
    d = torch.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2)
    w = torch.clamp(radius - d, min=0.0)
    return w / w.sum()


def density_filter(x: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """Periodic convolution of an nv^3 field with the (odd-sized, symmetric) kernel w."""
    p = w.shape[0] // 2
    xp = F.pad(x[None, None], (p, p, p, p, p, p), mode="circular")
    return F.conv3d(xp, w[None, None].to(x))[0, 0]


@dataclass
class History:
    ks_gap: List[float] = field(default_factory=list)
    gap: List[float] = field(default_factory=list)
    volume: List[float] = field(default_factory=list)
    seconds: List[float] = field(default_factory=list)


@dataclass
class HPM:
    """The paper's design parameterisation (Methods, "Topology optimization formulation"):
    Heaviside projection of design variables on nodes every `spacing` elements, projection
    radius in element widths, continuation on the Heaviside parameter (beta0, doubled every
    `beta_every` iterations up to beta_max); `octant` optimises one eighth of the cell,
    mirrored about its mid-planes (the paper's SC setting)."""
    spacing: int = 2
    radius: float = 2.8
    octant: bool = False
    beta0: float = 1.0
    beta_max: float = 64.0
    beta_every: int = 20

    def beta(self, it: int) -> float:
        return min(self.beta_max, self.beta0 * 2.0 ** (it // self.beta_every))


class GapOptimizer:
    def __init__(self, ctx: "phx.Context", cell, q: np.ndarray, nbands: int, t: int, rho0: np.ndarray,
                 precision: str = "mixed", beta: float = 100.0, radius: float = 1.5, step: float = 0.05,
                 device: str = "cuda:0", hpm: Optional[HPM] = None):
        # the KS aggregate weights bands t and t+1 at every k: the backward takes those two
        # bands at all k-points straight from the device gradient
        self.prob = autograd.Problem(ctx, cell, np.ascontiguousarray(q, dtype=np.float64), nbands, precision,
                                     backward_bands=(t, t + 1))
        self.t = t
        self.beta = beta
        self.step_size = step
        self.hpm = hpm
        self.ctx = ctx
        r0 = np.ascontiguousarray(rho0, dtype=np.float64)
        if hpm is None:
            self.w = hat_kernel(radius).to(device)
        else:
            # design variables: the start design averaged over each node's block of elements
            nv, sp = r0.shape[0], hpm.spacing
            nn = nv // sp
            r0 = r0.reshape(nn, sp, nn, sp, nn, sp).mean(axis=(1, 3, 5))
            if hpm.octant:
                r0 = np.ascontiguousarray(r0[: nn // 2, : nn // 2, : nn // 2])
        self.x = torch.from_numpy(np.ascontiguousarray(r0)).to(device)
        self.it = 0
        self.last_grad: Optional[torch.Tensor] = None  # d(KS gap)/dx of the last step
        self.omega_ref: Optional[float] = None
        self.hist = History()

    def projection(self):
        h = self.hpm
        return phx.projection(self.prob.cell.nv, h.spacing, h.radius, h.beta(self.it), h.octant)

    def design_map(self, x: torch.Tensor) -> torch.Tensor:
        if self.hpm is None:
            return density_filter(x, self.w)
        return autograd.project(x, self.ctx, self.projection())

    def physical(self) -> torch.Tensor:
        return self.design_map(self.x)

    def step(self) -> float:
        t0 = time.perf_counter()
        x = self.x.clone().requires_grad_(True)
        rho = self.design_map(x)
        om = autograd.band_frequencies(rho, self.prob)
        if self.omega_ref is None:
            self.omega_ref = float(om[:, self.t].detach().mean())
        f = autograd.ks_gap(om, self.t, self.beta, self.omega_ref)
        f.backward()
        g = x.grad.detach()
        self.last_grad = g
        gmax = float(g.abs().max())
        with torch.no_grad():
            if gmax > 0:
                self.x = torch.clamp(self.x + self.step_size * g / gmax, 0.0, 1.0)
        torch.cuda.synchronize()
        omd = om.detach()
        self.hist.ks_gap.append(float(f.detach()))
        self.hist.gap.append(float(autograd.normalized_gap(omd, self.t)))
        self.hist.volume.append(float(rho.detach().mean()))
        self.hist.seconds.append(time.perf_counter() - t0)
        self.it += 1
        return self.hist.ks_gap[-1]

    def run(self, iters: int, checkpoint: Optional[str] = None, every: int = 10) -> History:
        while self.it < iters:
            self.step()
            if checkpoint and (self.it % every == 0 or self.it == iters):
                self.save(checkpoint)
        return self.hist

    def save(self, path: str):
        tmp = path + ".tmp.npz"
        np.savez(tmp, x=self.x.cpu().numpy(), it=self.it, omega_ref=self.omega_ref,
                 hist=json.dumps(self.hist.__dict__))
        os.replace(tmp, path)

    def load(self, path: str):
        z = np.load(path, allow_pickle=False)
        self.x = torch.from_numpy(z["x"]).to(self.x.device)
        self.it = int(z["it"])
        self.omega_ref = float(z["omega_ref"])
        self.hist = History(**json.loads(str(z["hist"])))


def main(argv=None):
    """Band-gap maximisation on a seeded start: prints one JSON line per iteration and a summary."""
    import argparse

    from . import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--lattice", default="FCC", choices=["SC", "BCC", "FCC"])
    ap.add_argument("--nv", type=int, default=32)
    ap.add_argument("--M", type=int, default=5)
    ap.add_argument("--nk", type=int, default=40)
    ap.add_argument("--nbands", type=int, default=8)
    ap.add_argument("--t", type=int, default=6, help="gap between bands t and t+1")
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--seed", type=int, default=502)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--hpm", action="store_true", help="Heaviside projection of a reduced design field")
    ap.add_argument("--spacing", type=int, default=2, help="HPM: elements between design nodes")
    ap.add_argument("--proj-radius", type=float, default=2.8, help="HPM: projection radius (element widths)")
    ap.add_argument("--octant", action="store_true", help="HPM: design one octant, mirrored (SC)")
    ap.add_argument("--beta-every", type=int, default=20, help="HPM: iterations per doubling of beta")
    ap.add_argument("--beta-max", type=float, default=64.0)
    ap.add_argument("--final-M", type=int, default=None,
                    help="re-evaluate the final design at this plane-wave order (default M + 1)")
    ap.add_argument("--kstreams", type=int, default=1,
                    help="k-point ranges of each band solve on concurrent library streams (1..16)")
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--resume", action="store_true")
    a = ap.parse_args(argv)
    if a.kstreams > 1:
        # one hardware queue per stream (read when the HIP runtime starts: before any GPU use)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(32, max(4, a.kstreams + 1))))
    cell = synth.Cell(a.lattice, 1.0, a.nv, a.M)
    rho0 = synth.box_smoothed_uniform(a.nv, a.seed)
    ctx = phx.Context(0)
    ctx.set_option("kstreams", a.kstreams)
    q = phx.kpath(a.lattice, a.nk)
    hpm = HPM(a.spacing, a.proj_radius, a.octant, 1.0, a.beta_max, a.beta_every) if a.hpm else None
    opt = GapOptimizer(ctx, cell, q, a.nbands, a.t, rho0, a.precision, hpm=hpm)
    if a.resume and a.checkpoint and os.path.exists(a.checkpoint):
        opt.load(a.checkpoint)
    t0 = time.perf_counter()
    while opt.it < a.iters:
        opt.step()
        h = opt.hist
        rec = {"iter": opt.it, "ks_gap": h.ks_gap[-1], "gap": h.gap[-1], "volume": h.volume[-1],
               "seconds": h.seconds[-1]}
        if hpm is not None:
            rec["beta"] = hpm.beta(opt.it - 1)
        print(json.dumps(rec), flush=True)
        if a.checkpoint and (opt.it % 10 == 0 or opt.it == a.iters):
            opt.save(a.checkpoint)
    dt = time.perf_counter() - t0
    # The final band structure at a higher order than the optimisation used (Results,
    # "Topology optimized structures": optimised at M=3, final band structure at M=4).
    fm = a.final_M if a.final_M is not None else a.M + 1
    final = None
    if fm > 0 and a.nv >= 2 * fm + 1:
        fcell = synth.Cell(a.lattice, 1.0, a.nv, fm)
        om = ctx.bands_dev(fcell, opt.physical().reshape(-1), q, a.nbands, a.precision)
        final = float(autograd.normalized_gap(om, a.t))
    print(json.dumps({"lattice": a.lattice, "nv": a.nv, "M": a.M, "nk": a.nk, "iters": opt.it,
                      "gap_first": opt.hist.gap[0], "gap_last": opt.hist.gap[-1],
                      "final_M": fm, "gap_final_M": final,
                      "iters_per_s": len(opt.hist.seconds) / max(sum(opt.hist.seconds), 1e-9),
                      "wall_s": dt}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
