"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module only *generates inputs*: design fields rho_e in [0, 1] on an
N_v^3 voxel grid, base-material tables and the five workload recipes.  It
holds none of the band-structure arithmetic, so both the HIP path and the
CPU oracle may import it without sharing any of the method.

Workload shapes follow the paper's design studies (Results, "Topology
optimized structures" and the SC/BCC/FCC subsections): homogeneous
mixtures, smoothed random starts and single centred inclusions on voxel
meshes laid along the primitive vectors (Methods, "Study of cubic unit
cells").  The paper uses no public dataset; every design here is drawn
from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import erfc, sqrt
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Base materials (SI).  phase0 is the compliant matrix (rho_e = 0), phase1 is
# the stiff, heavy inclusion (rho_e = 1).
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Material:
    density: float  # kg / m^3
    youngs: float   # Pa
    poisson: float  # -


# Workload materials: epoxy / tungsten carbide.
EPOXY = Material(1180.0, 4.35e9, 0.37)
WC = Material(15630.0, 550e9, 0.22)
# The values the paper quotes in "A note on normalized band gaps".
EPOXY_PAPER = Material(1180.0, 4.3438e9, 0.3679)
WC_PAPER = Material(13800.0, 387.5559e9, 0.3459)

LATTICES = ("SC", "BCC", "FCC")


@dataclass(frozen=True)
class Cell:
    lattice: str = "SC"          # "SC" | "BCC" | "FCC"
    a: float = 1.0               # conventional cube edge (m)
    nv: int = 8                  # voxels per primitive axis
    M: int = 2                   # plane-wave order, alpha,beta,gamma in [-M, M]
    phase0: Material = EPOXY     # rho_e = 0
    phase1: Material = WC        # rho_e = 1
    simp_p: float = 3.0          # w = rho^p


# ---------------------------------------------------------------------------
# Design generators
# ---------------------------------------------------------------------------


def box_smoothed_uniform(nv: int, seed: int) -> np.ndarray:
    """U[0,1] on nv^3 voxels, then a periodic 3x3x3 box mean.  C order [i1][i2][i3]."""
    rng = np.random.default_rng(seed)
    u = rng.random((nv, nv, nv))
    acc = np.zeros_like(u)
    for d1 in (-1, 0, 1):
        for d2 in (-1, 0, 1):
            for d3 in (-1, 0, 1):
                acc += np.roll(u, (d1, d2, d3), axis=(0, 1, 2))
    return acc / 27.0


def _primitive_rows(lattice: str, a: float) -> np.ndarray:
    if lattice == "SC":
        return a * np.eye(3)
    if lattice == "BCC":
        return 0.5 * a * np.array([[-1.0, 1.0, 1.0], [1.0, -1.0, 1.0], [1.0, 1.0, -1.0]])
    if lattice == "FCC":
        return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    raise ValueError(f"unknown lattice {lattice!r}")


def gaussian_blob(nv: int, lattice: str, seed: int, radius: float = 0.3,
                  blur: float = 0.05, noise: float = 0.1, a: float = 1.0) -> np.ndarray:
    """A blurred ball of the stiff phase at a random centre plus uniform noise.

    Centre c ~ U[0,1)^3 in primitive coordinates; d_e is the periodic
    minimum-image Cartesian distance over 5^3 lattice translations;
    rho_e = clip(erfc((d_e - r) / (sqrt(2) * blur)) / 2 + U[0, noise], 0, 1).
    """
    rng = np.random.default_rng(seed)
    A = _primitive_rows(lattice, a)
    c = rng.random(3)
    s = (np.arange(nv) + 0.5) / nv
    S = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)
    best = np.full(S.shape[0], np.inf)
    rng_t = range(-2, 3)
    for t1 in rng_t:
        for t2 in rng_t:
            for t3 in rng_t:
                ds = S - c + np.array([t1, t2, t3], dtype=float)
                d = np.linalg.norm(ds @ A, axis=1)
                best = np.minimum(best, d)
    ball = np.array([0.5 * erfc((d - radius * a) / (sqrt(2.0) * blur * a)) for d in best])
    rho = ball + noise * rng.random(S.shape[0])
    return np.clip(rho, 0.0, 1.0).reshape(nv, nv, nv)


def sphere(nv: int, lattice: str, radius: float, a: float = 1.0) -> np.ndarray:
    """Sharp ball of the stiff phase centred in the primitive cell (rho in {0, 1})."""
    A = _primitive_rows(lattice, a)
    s = (np.arange(nv) + 0.5) / nv
    S = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)
    best = np.full(S.shape[0], np.inf)
    for t1 in range(-2, 3):
        for t2 in range(-2, 3):
            for t3 in range(-2, 3):
                d = np.linalg.norm((S - 0.5 + np.array([t1, t2, t3], float)) @ A, axis=1)
                best = np.minimum(best, d)
    return (best <= radius * a).astype(float).reshape(nv, nv, nv)


def cubic_symmetric(nv: int, seed: int) -> np.ndarray:
    """A random SC design invariant under the 48 operations of the cube about its centre."""
    rng = np.random.default_rng(seed)
    u = rng.random((nv, nv, nv))
    acc = np.zeros_like(u)
    import itertools
    n = 0
    for perm in itertools.permutations(range(3)):
        v = np.transpose(u, perm)
        for f1 in (False, True):
            for f2 in (False, True):
                for f3 in (False, True):
                    w = v
                    if f1:
                        w = w[::-1, :, :]
                    if f2:
                        w = w[:, ::-1, :]
                    if f3:
                        w = w[:, :, ::-1]
                    acc += w
                    n += 1
    return acc / n


def random_voxels(nv: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.choice(nv ** 3, count, replace=False)


# ---------------------------------------------------------------------------
# Workload recipes (sizes and seeds).  k-point counts and paths are named by
# their high-symmetry letters; G = Gamma.
# ---------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    cells: List[Cell]
    designs: List[np.ndarray]
    nk: int
    path: str
    nbands: int
    sens_bands: Tuple[int, ...] = ()
    note: str = ""


def config1() -> Workload:
    cell = Cell("SC", 1.0, 8, 2)
    return Workload("SC 8^3 M=2, 10 k on G-X-M-G-R, 8 bands, FP64",
                    [cell], [box_smoothed_uniform(8, 101)], 10, "GXMGR", 8)


def config2() -> Workload:
    cell = Cell("SC", 1.0, 16, 3)
    return Workload("SC 16^3 M=3, 30 k on G-X-M-G-R-X|M-R, 10 bands, adjoint bands 3,4,6,7",
                    [cell], [box_smoothed_uniform(16, 202)], 30, "GXMGRX|MR", 10, (3, 4, 6, 7))


def config3() -> Workload:
    cell = Cell("BCC", 1.0, 24, 4)
    return Workload("BCC 24^3 M=4 blob, 48 k on G-H-N-G-P-H|P-N, 12 bands",
                    [cell], [gaussian_blob(24, "BCC", 303)], 48, "GHNGPH|PN", 12)


def config4(all_m5: bool = True, ndesign: int = 16) -> Workload:
    designs = [box_smoothed_uniform(32, 400 + i) for i in range(ndesign)]
    if all_m5:
        cells = [Cell("FCC", 1.0, 32, 5) for _ in range(ndesign)]
        name = f"FCC 32^3 M=5 x{ndesign} designs, 60 k, 12 bands, adjoint bands 6,7"
    else:
        cells = [Cell("FCC", 1.0, 32, (3, 4, 5)[i % 3]) for i in range(ndesign)]
        name = f"FCC 32^3 M in (3,4,5) x{ndesign} designs, 60 k, 12 bands, adjoint bands 6,7"
    return Workload(name, cells, designs, 60, "GXWKGLUWLK|UX", 12, (6, 7))


WORKLOADS = {1: config1, 2: config2, 3: config3, 4: config4}
