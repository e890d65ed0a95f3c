"""Lattice geometry, plane-wave index set and Brillouin-zone paths.

Paper: Results, "Phononic band structure calculation" (the basis
f = exp[i 2 pi K.x] with K = T_1(Q_1+alpha) + T_2(Q_2+beta) + T_3(Q_3+gamma),
alpha, beta, gamma in [-M, M]); Methods, "Study of cubic unit cells"
(SC/BCC/FCC primitive cells, meshes laid along the primitive vectors,
band structures along the edges of the irreducible Brillouin zone).

Conventions (the paper is silent on them):
* rows of ``A`` are the primitive vectors a_i; rows of ``T`` are the
  reciprocal vectors b_j with a_i . b_j = delta_ij (no 2 pi, since the basis
  carries the 2 pi itself);
* K_p = sum_j (Q_j + n_pj) b_j, in cycles per length;
* the voxel e = (i1, i2, i3) has centroid x_e = sum_j s_j a_j with
  s_j = (i_j + 1/2) / N_v;
* plane waves n_p = (alpha, beta, gamma) are ordered lexicographically with
  alpha slowest.
"""
from __future__ import annotations

import numpy as np


def primitive_vectors(lattice: str, a: float) -> np.ndarray:
    if lattice == "SC":
        return a * np.eye(3)
    if lattice == "BCC":
        return 0.5 * a * np.array([[-1.0, 1.0, 1.0], [1.0, -1.0, 1.0], [1.0, 1.0, -1.0]])
    if lattice == "FCC":
        return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    raise ValueError(lattice)


def reciprocal_vectors(A: np.ndarray) -> np.ndarray:
    """The paper's T: rows b_j with a_i . b_j = delta_ij."""
    return np.linalg.inv(A).T


def cell_volume(A: np.ndarray) -> float:
    return abs(float(np.linalg.det(A)))


def plane_wave_indices(M: int) -> np.ndarray:
    r = np.arange(-M, M + 1)
    n = np.array([(al, be, ga) for al in r for be in r for ga in r], dtype=np.int64)
    return n


def wavevectors(Q: np.ndarray, n: np.ndarray, T: np.ndarray) -> np.ndarray:
    """K_p = T^T (Q + n_p) for every plane wave p; shape (N, 3)."""
    return (np.asarray(Q, float)[None, :] + n) @ T


def voxel_fractions(nv: int) -> np.ndarray:
    """s_e = (i + 1/2) / N_v for every voxel in C order; shape (nv^3, 3)."""
    s = (np.arange(nv) + 0.5) / nv
    return np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)


def voxel_centroids(A: np.ndarray, nv: int) -> np.ndarray:
    return voxel_fractions(nv) @ A


# Standard high-symmetry points in Cartesian units of 1/a (cycles per length);
# the paper cites the standard set without printing coordinates.
SYMMETRY_POINTS = {
    "SC": {"G": (0, 0, 0), "X": (0, 0.5, 0), "M": (0.5, 0.5, 0), "R": (0.5, 0.5, 0.5)},
    "BCC": {"G": (0, 0, 0), "H": (0, 0, 1), "N": (0.5, 0.5, 0), "P": (0.5, 0.5, 0.5)},
    "FCC": {"G": (0, 0, 0), "X": (0, 1, 0), "W": (0.5, 1, 0), "K": (0.75, 0.75, 0),
            "L": (0.5, 0.5, 0.5), "U": (0.25, 1, 0.25)},
}
DEFAULT_PATHS = {"SC": "GXMGRX|MR", "BCC": "GHNGPH|PN", "FCC": "GXWKGLUWLK|UX"}


def kpath(lattice: str, nk: int, path: str | None = None) -> np.ndarray:
    """k-points along the IBZ boundary, as reciprocal coordinates Q (nk, 3).

    Every vertex is included; the remaining points are spread over the
    segments in proportion to their Cartesian length by the largest-remainder
    rule, evenly inside each segment; nothing is placed across a "|" break.
    """
    path = DEFAULT_PATHS[lattice] if path is None else path
    pts = SYMMETRY_POINTS[lattice]
    branches = [b for b in path.split("|") if b]
    nvert = sum(len(b) for b in branches)
    if nk < nvert:
        raise ValueError(f"need at least {nvert} k-points for path {path}")
    segs = []
    for b in branches:
        for u, v in zip(b[:-1], b[1:]):
            segs.append((np.array(pts[u], float), np.array(pts[v], float)))
    lengths = np.array([np.linalg.norm(v - u) for u, v in segs])
    extra = nk - nvert
    share = extra * lengths / lengths.sum() if lengths.sum() > 0 else np.zeros(len(segs))
    cnt = np.floor(share).astype(int)
    rem = extra - cnt.sum()
    order = np.argsort(-(share - cnt), kind="stable")
    cnt[order[:rem]] += 1
    out = []
    si = 0
    for b in branches:
        out.append(np.array(pts[b[0]], float))
        for _ in range(len(b) - 1):
            u, v = segs[si]
            c = cnt[si]
            for j in range(1, c + 1):
                out.append(u + (v - u) * j / (c + 1))
            out.append(v.copy())
            si += 1
    kc = np.array(out)
    A = primitive_vectors(lattice, 1.0)
    return kc @ A.T  # Q_j = a_j . k  (a = 1 here; Q is dimensionless)
