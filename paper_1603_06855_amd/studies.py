"""Sphere-inclusion and laminate studies (Results, "A note on normalized band gaps").

* ``sphere_sweep``: the normalised gap of Eq. (10) between bands t and t+1 of a single
  centred spherical inclusion of the stiff phase, as a function of its volume fraction, for
  the SC, BCC and FCC lattices.  Every band structure comes from the library (the HIP path);
  this module builds the designs and reads the band edges off the result.
* ``rytov_*``: the exact dispersion of a periodic two-layer laminate for waves travelling
  normal to the layers (the transfer matrix of one period, for the longitudinal or the
  shear polarisation), its first gap at the zone boundary and the normalised width of that
  gap as a function of the volume fraction: the 1-D reference the paper quotes beside its
  3-D results (155.5 % at a tungsten-carbide fraction of 0.737).  Host arithmetic.
* ``m_convergence``: one design's band structure at increasing plane-wave orders M (the paper
  computes its final band structures at a higher order than it optimised with).

``python -m paper_1603_06855_amd.studies`` runs all three and prints one JSON line per case.
"""
from __future__ import annotations

import json
import math
import time
from typing import Dict, List, Sequence

import numpy as np

from . import synth

VOLUME_FACTOR = {"SC": 1.0, "BCC": 0.5, "FCC": 0.25}  # primitive-cell volume / a^3


def sphere_radius(lattice: str, fraction: float, a: float = 1.0) -> float:
    """Radius of the ball that fills `fraction` of the primitive cell."""
    return (3.0 * fraction * VOLUME_FACTOR[lattice] * a ** 3 / (4.0 * math.pi)) ** (1.0 / 3.0)


def normalized_gap(omega: np.ndarray, t: int):
    """Eq. (10) between bands t and t+1 (1-based) over all k: (gap, lower edge, upper edge)."""
    lo = float(np.max(omega[:, t - 1]))
    hi = float(np.min(omega[:, t]))
    return 2.0 * (hi - lo) / (hi + lo), lo, hi


def sphere_sweep(ctx, lattice: str, fractions: Sequence[float], nv: int = 32, M: int = 3, nk: int = 40,
                 nbands: int = 8, t: int = 6, precision: str = "mixed",
                 phase0: synth.Material = synth.EPOXY_PAPER, phase1: synth.Material = synth.WC_PAPER) -> List[Dict]:
    """Gap of a centred ball of phase1 in phase0 for each target volume fraction (the
    voxelised fraction is reported beside it)."""
    cell = synth.Cell(lattice, 1.0, nv, M, phase0, phase1, 1.0)
    q = _kpath(lattice, nk)
    out = []
    for f in fractions:
        rho = synth.sphere(nv, lattice, sphere_radius(lattice, f))
        t0 = time.perf_counter()
        om = ctx.bands(cell, rho, q, nbands, precision)
        dt = time.perf_counter() - t0
        g, lo, hi = normalized_gap(om, t)
        out.append({"fraction": float(f), "voxel_fraction": float(rho.mean()), "gap": g, "lower": lo,
                    "upper": hi, "seconds": dt})
    return out


def _kpath(lattice: str, nk: int) -> np.ndarray:
    from . import phx
    return phx.kpath(lattice, nk)


# ---------------------------------------------------------------------------
# Two-layer laminate, waves normal to the layers
# ---------------------------------------------------------------------------


def layer_speed(mat: synth.Material, pol: str) -> float:
    """Longitudinal ("P") or shear ("S") speed of an isotropic phase."""
    E, nu, r = mat.youngs, mat.poisson, mat.density
    mu = E / (2.0 * (1.0 + nu))
    if pol == "S":
        return math.sqrt(mu / r)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return math.sqrt((lam + 2.0 * mu) / r)


def rytov_trace(omega, m1: synth.Material, m0: synth.Material, f: float, pol: str, a: float = 1.0):
    """Half the trace of the one-period transfer matrix at angular frequency omega: layer of
    phase m1 (thickness f a) and of phase m0 ((1 - f) a).  A Bloch wave of wavenumber k
    exists where it equals cos(k a); |value| > 1 is a gap."""
    c1, c0 = layer_speed(m1, pol), layer_speed(m0, pol)
    z1, z0 = m1.density * c1, m0.density * c0
    p1 = np.asarray(omega) * f * a / c1
    p0 = np.asarray(omega) * (1.0 - f) * a / c0
    return np.cos(p1) * np.cos(p0) - 0.5 * (z1 / z0 + z0 / z1) * np.sin(p1) * np.sin(p0)


def rytov_omega(k: float, m1: synth.Material, m0: synth.Material, f: float, pol: str, nbranch: int = 1,
                a: float = 1.0) -> np.ndarray:
    """The lowest nbranch angular frequencies with Bloch wavenumber k (rad per length)."""
    from scipy.optimize import brentq
    c_min = min(layer_speed(m1, pol), layer_speed(m0, pol))
    target = math.cos(k * a)
    res = lambda w: rytov_trace(w, m1, m0, f, pol, a) - target
    top = (nbranch + 1) * math.pi * c_min / a * 2.0
    grid = np.linspace(1e-9, top, 20000 * nbranch)
    r = res(grid)
    idx = np.nonzero(np.sign(r[:-1]) != np.sign(r[1:]))[0]
    roots = [brentq(res, grid[i], grid[i + 1], xtol=1e-13, rtol=1e-15) for i in idx[:nbranch]]
    return np.array(roots)


def rytov_first_gap(m1: synth.Material, m0: synth.Material, f: float, pol: str, a: float = 1.0):
    """Edges (omega_low, omega_high) of the first gap at the zone boundary (k a = pi), where
    the half trace first drops below -1, and its normalised width 2 (high - low)/(high + low)."""
    from scipy.optimize import brentq
    c_min = min(layer_speed(m1, pol), layer_speed(m0, pol))
    h = lambda w: rytov_trace(w, m1, m0, f, pol, a) + 1.0
    grid = np.linspace(1e-9, 4.0 * math.pi * c_min / a, 40000)
    v = h(grid)
    neg = np.nonzero(v < 0)[0]
    if len(neg) == 0:
        return float("nan"), float("nan"), 0.0
    i = neg[0]
    lo = brentq(h, grid[i - 1], grid[i], xtol=1e-13, rtol=1e-15)
    j = i + np.argmax(v[i:] >= 0)
    hi = brentq(h, grid[j - 1], grid[j], xtol=1e-13, rtol=1e-15)
    return lo, hi, 2.0 * (hi - lo) / (hi + lo)


def quarter_wave_fraction(m1: synth.Material, m0: synth.Material, pol: str) -> float:
    """Fraction of phase m1 at which both layers are a quarter wavelength thick at the
    first gap's centre (equal transit times)."""
    c1, c0 = layer_speed(m1, pol), layer_speed(m0, pol)
    return c1 / (c1 + c0)


def laminate_gap_sweep(m1: synth.Material, m0: synth.Material, fractions: Sequence[float], pol: str):
    return np.array([rytov_first_gap(m1, m0, f, pol)[2] for f in fractions])


def m_convergence(ctx, lattice: str, rho: np.ndarray, orders: Sequence[int], nk: int = 40, nbands: int = 8,
                  t: int = 6, precision: str = "fp64", phase0: synth.Material = synth.EPOXY,
                  phase1: synth.Material = synth.WC) -> List[Dict]:
    """Band structure of one design at increasing plane-wave orders M (the paper re-evaluates
    its optimised designs at a higher order than the one it optimised with): per order the
    gap of Eq. (10), and the largest and the root-mean-square relative change of the band
    frequencies from the previous order."""
    nv = rho.shape[0]
    q = _kpath(lattice, nk)
    out, prev = [], None
    for M in orders:
        if nv < 2 * M + 1:
            raise ValueError(f"order {M} needs at least {2 * M + 1} voxels per axis")
        cell = synth.Cell(lattice, 1.0, nv, M, phase0, phase1, 3.0)
        t0 = time.perf_counter()
        om = ctx.bands(cell, rho, q, nbands, precision)
        dt = time.perf_counter() - t0
        g, lo, hi = normalized_gap(om, t)
        change = rms = None
        if prev is not None:
            mask = prev > 1e-3 * prev.max()  # the acoustic bands near Gamma have no relative scale
            rel = np.abs(om[mask] - prev[mask]) / prev[mask]
            change, rms = float(rel.max()), float(np.sqrt(np.mean(rel ** 2)))
        out.append({"M": M, "gap": g, "lower": lo, "upper": hi, "max_rel_change": change,
                    "rms_rel_change": rms, "seconds": dt})
        prev = om
    return out


def main(argv=None):
    import argparse

    from . import phx
    ap = argparse.ArgumentParser()
    ap.add_argument("--nv", type=int, default=32)
    ap.add_argument("--M", type=int, default=3)
    ap.add_argument("--nk", type=int, default=40)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--fractions", default="0.20,0.25,0.30,0.35,0.40,0.45,0.50,0.55,0.60,0.65,0.70")
    ap.add_argument("--orders", default="2,3,4,5,6", help="plane-wave orders of the convergence study")
    a = ap.parse_args(argv)
    fr = [float(x) for x in a.fractions.split(",")]
    for pol in ("S", "P"):
        fs = np.linspace(0.5, 0.9, 401)
        g = laminate_gap_sweep(synth.WC_PAPER, synth.EPOXY_PAPER, fs, pol)
        i = int(np.argmax(g))
        print(json.dumps({"study": "laminate", "polarisation": pol, "max_gap": float(g[i]),
                          "at_fraction": float(fs[i]),
                          "quarter_wave_fraction": quarter_wave_fraction(synth.WC_PAPER, synth.EPOXY_PAPER, pol)}),
              flush=True)
    with phx.Context(0) as ctx:
        for lat in ("SC", "BCC", "FCC"):
            t0 = time.perf_counter()
            res = sphere_sweep(ctx, lat, fr, a.nv, a.M, a.nk, precision=a.precision)
            dt = time.perf_counter() - t0
            best = max(res, key=lambda r: r["gap"])
            print(json.dumps({"study": "sphere", "lattice": lat, "nv": a.nv, "M": a.M, "nk": a.nk,
                              "precision": a.precision, "best_gap": best["gap"],
                              "best_fraction": best["voxel_fraction"], "k_solves_per_s": len(fr) * a.nk / dt,
                              "sweep": [{k: round(v, 5) for k, v in r.items()} for r in res]}), flush=True)
        orders = [int(x) for x in a.orders.split(",")]
        for lat, seed in (("SC", 501), ("FCC", 502)):
            rho = synth.box_smoothed_uniform(a.nv, seed)
            res = m_convergence(ctx, lat, rho, orders, a.nk)
            print(json.dumps({"study": "orders", "lattice": lat, "nv": a.nv, "nk": a.nk, "seed": seed,
                              "precision": "fp64", "orders": res}), flush=True)


if __name__ == "__main__":
    main()
