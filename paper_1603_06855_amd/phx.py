"""ctypes binding of libphx.so (argument marshalling only; every step runs in the HIP library).

The C ABI is declared in ``include/phx.h``.  Loading fails loudly when the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char, c_char_p, c_double, c_int, c_long, c_void_p
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphx.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENOTPD = 0, -1, -2, -3, -4, -5
WDEGEN = 1  # warning: a requested band lies in a degenerate cluster (its sensitivity is the cluster mean)
LATTICE = {"SC": 0, "BCC": 1, "FCC": 2}
PRECISION = {"fp64": 0, "mixed": 1}


class PhxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"phx error {code}: {msg}")
        self.code = code
        self.msg = msg


class Material(ctypes.Structure):
    _fields_ = [("density", c_double), ("youngs", c_double), ("poisson", c_double)]


class Cell(ctypes.Structure):
    _fields_ = [("lattice", c_int), ("a", c_double), ("nv", c_int), ("M", c_int),
                ("phase0", Material), ("phase1", Material), ("simp_p", c_double)]


_lib = None


def load():
    """Load libphx.so (raises if it is missing: no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or python -m "
                          "paper_1603_06855_amd.build")
    # PyTorch carries its own HIP runtime (same soname).  Loaded first, it is the one
    # libphx.so binds to, so tensors' device pointers and torch streams are objects of
    # the library's own runtime, and torch keeps seeing the device.  Without torch the
    # system ROCm runtime is used.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    D = POINTER(c_double)
    I = POINTER(c_int)
    P = c_void_p
    sig = {
        "phx_create": (c_int, [POINTER(c_void_p), c_int]),
        "phx_destroy": (c_int, [P]),
        "phx_last_error": (c_char_p, [P]),
        "phx_set_option": (c_int, [P, c_char_p, c_double]),
        "phx_get_stat": (c_int, [P, c_char_p, D]),
        "phx_kpath": (c_int, [c_int, c_char_p, c_int, D]),
        "phx_validate": (c_int, [POINTER(Cell), D, c_int, D, c_int, c_int, I, POINTER(c_char), c_int]),
        "phx_fourier": (c_int, [P, POINTER(Cell), D, D]),
        "phx_schur": (c_int, [P, POINTER(Cell), D, D, D]),
        "phx_bands": (c_int, [P, POINTER(Cell), D, c_int, D, c_int, c_int, D, D]),
        "phx_sens": (c_int, [P, POINTER(Cell), D, c_int, D, c_int, c_int, c_int, I, D, D]),
        "phx_adjoint": (c_int, [P, POINTER(Cell), D, c_int, D, c_int, c_int, c_int, I, D, D, D]),
        "phx_bands_batch": (c_int, [P, c_int, POINTER(Cell), POINTER(D), c_int, D, c_int, c_int, c_int, I,
                                    POINTER(D), POINTER(D)]),
        "phx_bands_dev": (c_int, [P, POINTER(Cell), c_void_p, c_int, D, c_int, c_int, c_void_p, c_void_p]),
        "phx_sens_dev": (c_int, [P, POINTER(Cell), c_void_p, c_int, D, c_int, c_int, c_int, I, c_void_p,
                                 c_void_p, c_void_p]),
        "phx_adjoint_dev": (c_int, [P, POINTER(Cell), c_void_p, c_int, D, c_int, c_int, c_int, I, c_void_p,
                                    c_void_p, c_void_p, c_void_p]),
        "phx_sens_batch_dev": (c_int, [P, c_int, POINTER(Cell), POINTER(c_void_p), c_int, D, c_int, c_int, c_int,
                                       I, POINTER(c_void_p), POINTER(c_void_p), c_void_p]),
        "phx_zgemm": (c_int, [P, c_int, c_char, c_char, c_int, c_int, c_int, D, D, c_long, c_long, D, c_long,
                              c_long, D, D, c_long, c_long, c_int]),
        "phx_zposv": (c_int, [P, c_int, c_int, c_int, c_int, D, D]),
        "phx_small_orth": (c_int, [P, c_int, c_int, D, c_double, D, I]),
        "phx_small_eig": (c_int, [P, c_int, c_int, c_int, D, I, D, D]),
        "phx_small_rr": (c_int, [P, c_int, c_int, c_int, D, c_double, D, D, D, I]),
        "phx_projection_size": (c_int, [POINTER(Projection), POINTER(c_long)]),
        "phx_project": (c_int, [P, POINTER(Projection), D, D]),
        "phx_project_adjoint": (c_int, [P, POINTER(Projection), D, D, D]),
        "phx_project_dev": (c_int, [P, POINTER(Projection), c_void_p, c_void_p, c_void_p]),
        "phx_project_adjoint_dev": (c_int, [P, POINTER(Projection), c_void_p, c_void_p, c_void_p, c_void_p]),
        "phx_project_adjoint_dev_noalloc": (c_int, [P, POINTER(Projection), c_void_p, c_void_p, c_void_p,
                                                    c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class Projection(ctypes.Structure):
    """phx_projection: the Heaviside projection of a reduced (optionally mirrored-octant)
    design field onto the nv^3 elements."""
    _fields_ = [("nv", c_int), ("spacing", c_int), ("radius", c_double), ("beta", c_double), ("octant", c_int)]


def projection(nv: int, spacing: int = 2, radius: float = 2.8, beta: float = 1.0, octant: bool = False) -> Projection:
    return Projection(nv, spacing, radius, beta, 1 if octant else 0)


def projection_size(p: Projection) -> int:
    lib = load()
    n = c_long(0)
    if lib.phx_projection_size(byref(p), byref(n)) != OK:
        raise PhxError(EINVAL, "invalid projection")
    return n.value


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_int))


def make_cell(cell) -> Cell:
    """Convert a ``synth.Cell``-like object (lattice name, a, nv, M, phase0/1, simp_p)."""
    lat = cell.lattice if isinstance(cell.lattice, int) else LATTICE[cell.lattice]
    m0, m1 = cell.phase0, cell.phase1
    return Cell(lat, float(cell.a), int(cell.nv), int(cell.M),
                Material(m0.density, m0.youngs, m0.poisson), Material(m1.density, m1.youngs, m1.poisson),
                float(cell.simp_p))


def kpath(lattice: str, nk: int, path: Optional[str] = None) -> np.ndarray:
    lib = load()
    q = np.zeros((nk, 3))
    rc = lib.phx_kpath(LATTICE[lattice], path.encode() if path else None, nk, _dptr(q))
    if rc != OK:
        raise PhxError(rc, "phx_kpath rejected its arguments")
    return q


def validate(cell, rho=None, q=None, nbands=0, band_no=()):
    lib = load()
    c = make_cell(cell)
    msg = ctypes.create_string_buffer(256)
    r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    qq = None if q is None else np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    nk = 0 if q is None else qq.size // 3
    b = np.ascontiguousarray(band_no, dtype=np.int32)
    rc = lib.phx_validate(byref(c), _dptr(r) if r is not None else None, nk, _dptr(qq) if qq is not None else None,
                          int(nbands), len(b), _iptr(b) if len(b) else None, msg, 256)
    return rc, msg.value.decode()


class Context:
    """One HIP device, one stream, grow-only device workspaces."""

    def __init__(self, device: int = 0, **options):
        self.lib = load()
        h = c_void_p()
        rc = self.lib.phx_create(byref(h), device)
        if rc != OK:
            raise PhxError(rc, "phx_create failed (no HIP device?)")
        self.h = h
        self.last_status = OK
        self.last_message = ""
        for k, v in options.items():
            self.set_option(k, v)

    def close(self):
        if getattr(self, "h", None):
            self.lib.phx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int, allow=()):
        """Raise on an error; warnings (PHX_WDEGEN) and the codes in `allow` are recorded in
        last_status / last_message instead."""
        self.last_status = rc
        self.last_message = self.lib.phx_last_error(self.h).decode() if rc != OK else ""
        if rc < 0 and rc not in allow:
            raise PhxError(rc, self.last_message)
        return rc

    def set_option(self, key: str, value: float):
        rc = self.lib.phx_set_option(self.h, key.encode(), float(value))
        if rc != OK:
            raise PhxError(rc, self.lib.phx_last_error(self.h).decode())

    def stat(self, key: str) -> float:
        """A statistic of the last solve (does not change last_status)."""
        v = c_double()
        if self.lib.phx_get_stat(self.h, key.encode(), byref(v)) != OK:
            raise PhxError(EINVAL, f"unknown statistic {key}")
        return v.value

    # -------------------------------------------------------------- stages
    def fourier(self, cell, rho) -> np.ndarray:
        c = make_cell(cell)
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        L2 = 4 * c.M + 1
        out = np.zeros(3 * L2 ** 3 * 2)
        self._check(self.lib.phx_fourier(self.h, byref(c), _dptr(r), _dptr(out)))
        return out.view(np.complex128).reshape(3, L2, L2, L2)

    def schur(self, cell, rho, q) -> np.ndarray:
        c = make_cell(cell)
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(3)
        n = 3 * (2 * c.M + 1) ** 3
        out = np.zeros(2 * n * n)
        self._check(self.lib.phx_schur(self.h, byref(c), _dptr(r), _dptr(qq), _dptr(out)))
        return out.view(np.complex128).reshape(n, n, order="F")

    # -------------------------------------------------------------- band structure
    def bands(self, cell, rho, q, nbands: int, precision: str = "fp64", bounds: bool = False,
              allow_noconv: bool = False):
        c = make_cell(cell)
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        om = np.zeros((nk, nbands))
        eb = np.zeros((nk, nbands))
        rc = self.lib.phx_bands(self.h, byref(c), _dptr(r), nk, _dptr(qq), nbands, PRECISION[precision],
                                _dptr(om), _dptr(eb))
        self._check(rc, (ENOCONV,) if allow_noconv else ())
        return (om, eb) if bounds else om

    def sens(self, cell, rho, q, nbands: int, band_no: Sequence[int], precision: str = "fp64",
             allow_noconv: bool = False):
        c = make_cell(cell)
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        b = np.ascontiguousarray(band_no, dtype=np.int32)
        om = np.zeros((nk, nbands))
        dw = np.zeros((nk, len(b), r.size))
        rc = self.lib.phx_sens(self.h, byref(c), _dptr(r), nk, _dptr(qq), nbands, PRECISION[precision], len(b),
                               _iptr(b), _dptr(om), _dptr(dw))
        self._check(rc, (ENOCONV,) if allow_noconv else ())
        return om, dw

    def adjoint(self, cell, rho, q, nbands: int, band_no: Sequence[int], weight, precision: str = "fp64"):
        c = make_cell(cell)
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        b = np.ascontiguousarray(band_no, dtype=np.int32)
        w = np.ascontiguousarray(weight, dtype=np.float64).reshape(nk, len(b))
        om = np.zeros((nk, nbands))
        g = np.zeros(r.size)
        self._check(self.lib.phx_adjoint(self.h, byref(c), _dptr(r), nk, _dptr(qq), nbands, PRECISION[precision],
                                         len(b), _iptr(b), _dptr(w), _dptr(om), _dptr(g)))
        return om, g

    def bands_batch(self, cells, rhos, q, nbands: int, precision: str = "fp64", band_no: Sequence[int] = ()):
        nd = len(cells)
        carr = (Cell * nd)(*[make_cell(c) for c in cells])
        rs = [np.ascontiguousarray(r, dtype=np.float64).reshape(-1) for r in rhos]
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        b = np.ascontiguousarray(band_no, dtype=np.int32)
        oms = [np.zeros((nk, nbands)) for _ in range(nd)]
        dws = [np.zeros((nk, len(b), r.size)) for r in rs] if len(b) else None
        DP = POINTER(c_double)
        rp = (DP * nd)(*[_dptr(r) for r in rs])
        op = (DP * nd)(*[_dptr(o) for o in oms])
        dp = (DP * nd)(*[_dptr(d) for d in dws]) if dws is not None else None
        self._check(self.lib.phx_bands_batch(self.h, nd, carr, rp, nk, _dptr(qq), nbands, PRECISION[precision],
                                             len(b), _iptr(b) if len(b) else None, op, dp))
        return (oms, dws) if dws is not None else oms

    def sens_dev(self, cell, rho_t, q, nbands: int, band_no: Sequence[int], precision: str = "fp64"):
        """torch CUDA tensors in and out: rho_t (nv^3 float64 on the device)."""
        import torch
        c = make_cell(cell)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        b = np.ascontiguousarray(band_no, dtype=np.int32)
        rho_t = rho_t.detach().contiguous().to(torch.float64)
        om = torch.empty((nk, nbands), dtype=torch.float64, device=rho_t.device)
        dw = torch.empty((nk, len(b), rho_t.numel()), dtype=torch.float64, device=rho_t.device)
        stream = torch.cuda.current_stream(rho_t.device).cuda_stream
        self._check(self.lib.phx_sens_dev(self.h, byref(c), c_void_p(rho_t.data_ptr()), nk, _dptr(qq), nbands,
                                          PRECISION[precision], len(b), _iptr(b), c_void_p(om.data_ptr()),
                                          c_void_p(dw.data_ptr()), c_void_p(stream)))
        return om, dw

    def bands_dev(self, cell, rho_t, q, nbands: int, precision: str = "fp64"):
        """torch CUDA tensors in and out: rho_t (nv^3 float64 on the device) -> omega (nk, nbands)."""
        import torch
        c = make_cell(cell)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        rho_t = rho_t.detach().contiguous().to(torch.float64)
        om = torch.empty((nk, nbands), dtype=torch.float64, device=rho_t.device)
        stream = torch.cuda.current_stream(rho_t.device).cuda_stream
        self._check(self.lib.phx_bands_dev(self.h, byref(c), c_void_p(rho_t.data_ptr()), nk, _dptr(qq), nbands,
                                           PRECISION[precision], c_void_p(om.data_ptr()), c_void_p(stream)))
        return om

    def adjoint_dev(self, cell, rho_t, q, nbands: int, band_no: Sequence[int], weight_t, precision: str = "fp64"):
        """grad (nv^3, device) = sum_{k,j} weight_t[k, j] d omega_{band_no[j]}(k) / d rho."""
        import torch
        c = make_cell(cell)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        b = np.ascontiguousarray(band_no, dtype=np.int32)
        rho_t = rho_t.detach().contiguous().to(torch.float64)
        w = weight_t.detach().to(device=rho_t.device, dtype=torch.float64).contiguous().reshape(nk, len(b))
        g = torch.empty(rho_t.numel(), dtype=torch.float64, device=rho_t.device)
        stream = torch.cuda.current_stream(rho_t.device).cuda_stream
        self._check(self.lib.phx_adjoint_dev(self.h, byref(c), c_void_p(rho_t.data_ptr()), nk, _dptr(qq), nbands,
                                             PRECISION[precision], len(b), _iptr(b), c_void_p(w.data_ptr()), None,
                                             c_void_p(g.data_ptr()), c_void_p(stream)))
        return g

    def sens_batch_dev(self, cells, rhos, q, nbands: int, band_no: Sequence[int] = (), precision: str = "fp64"):
        """Several designs (device float64 tensors, uneven M allowed) in one call; returns
        (omega list, domega list or None) as device tensors."""
        import torch
        nd = len(cells)
        carr = (Cell * nd)(*[make_cell(c) for c in cells])
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        nk = qq.shape[0]
        b = np.ascontiguousarray(band_no, dtype=np.int32)
        rs = [r.detach().contiguous().to(torch.float64).reshape(-1) for r in rhos]
        dev = rs[0].device
        oms = [torch.empty((nk, nbands), dtype=torch.float64, device=dev) for _ in range(nd)]
        dws = [torch.empty((nk, len(b), r.numel()), dtype=torch.float64, device=dev) for r in rs] if len(b) else None
        VP = c_void_p * nd
        rp = VP(*[r.data_ptr() for r in rs])
        op = VP(*[o.data_ptr() for o in oms])
        dp = VP(*[d.data_ptr() for d in dws]) if dws is not None else None
        stream = torch.cuda.current_stream(dev).cuda_stream
        self._check(self.lib.phx_sens_batch_dev(self.h, nd, carr, rp, nk, _dptr(qq), nbands, PRECISION[precision],
                                                len(b), _iptr(b) if len(b) else None, op, dp, c_void_p(stream)))
        return oms, dws

    # -------------------------------------------------------------- dense building blocks
    def zgemm(self, opa: str, opb: str, A, B, C=None, alpha=1.0, beta=0.0, precision: str = "fp64"):
        """Batched: A (batch, ., .) etc. complex arrays (column-major semantics via Fortran order)."""
        A = np.asarray(A, dtype=np.complex128)
        B = np.asarray(B, dtype=np.complex128)
        if A.ndim == 2:
            A, B = A[None], B[None]
            C = None if C is None else np.asarray(C)[None]
            squeeze = True
        else:
            squeeze = False
        batch = A.shape[0]
        m = A.shape[1] if opa == "N" else A.shape[2]
        k = A.shape[2] if opa == "N" else A.shape[1]
        n = B.shape[2] if opb == "N" else B.shape[1]
        Af = np.concatenate([np.asfortranarray(a).reshape(-1, order="F") for a in A])
        Bf = np.concatenate([np.asfortranarray(b).reshape(-1, order="F") for b in B])
        if C is None:
            C = np.zeros((batch, m, n), dtype=np.complex128)
        Cf = np.concatenate([np.asfortranarray(c).reshape(-1, order="F") for c in np.asarray(C, np.complex128)])
        Ad, Bd, Cd = Af.view(np.float64), Bf.view(np.float64), Cf.view(np.float64).copy()
        al = np.array([np.real(alpha), np.imag(alpha)], dtype=np.float64)
        be = np.array([np.real(beta), np.imag(beta)], dtype=np.float64)
        self._check(self.lib.phx_zgemm(self.h, PRECISION[precision], opa.encode(), opb.encode(), m, n, k, _dptr(al),
                                       _dptr(np.ascontiguousarray(Ad)), A.shape[1], A.shape[1] * A.shape[2],
                                       _dptr(np.ascontiguousarray(Bd)), B.shape[1], B.shape[1] * B.shape[2],
                                       _dptr(be), _dptr(Cd), m, m * n, batch))
        out = Cd.view(np.complex128).reshape(batch, n, m).transpose(0, 2, 1)
        return out[0] if squeeze else out

    def zposv(self, A, B, precision: str = "fp64"):
        A = np.asarray(A, dtype=np.complex128)
        B = np.asarray(B, dtype=np.complex128)
        batch, n, _ = A.shape
        nrhs = B.shape[2]
        Af = np.concatenate([np.asfortranarray(a).reshape(-1, order="F") for a in A]).view(np.float64)
        Bf = np.concatenate([np.asfortranarray(b).reshape(-1, order="F") for b in B]).view(np.float64).copy()
        self._check(self.lib.phx_zposv(self.h, PRECISION[precision], n, nrhs, batch, _dptr(np.ascontiguousarray(Af)),
                                       _dptr(Bf)))
        return Bf.view(np.complex128).reshape(batch, nrhs, n).transpose(0, 2, 1)

    def small_orth(self, G, drop: float = 1e-12):
        G = np.asarray(G, dtype=np.complex128)
        batch, m, _ = G.shape
        Gf = np.concatenate([np.asfortranarray(g).reshape(-1, order="F") for g in G]).view(np.float64)
        C0 = np.zeros(2 * m * m * batch)
        keep = np.zeros(m * batch, dtype=np.int32)
        self._check(self.lib.phx_small_orth(self.h, m, batch, _dptr(np.ascontiguousarray(Gf)), drop, _dptr(C0),
                                            _iptr(keep)))
        return C0.view(np.complex128).reshape(batch, m, m).transpose(0, 2, 1), keep.reshape(batch, m)

    def small_eig(self, G, keep, s: int):
        G = np.asarray(G, dtype=np.complex128)
        batch, m, _ = G.shape
        Gf = np.concatenate([np.asfortranarray(g).reshape(-1, order="F") for g in G]).view(np.float64)
        k = np.ascontiguousarray(keep, dtype=np.int32).reshape(-1)
        C = np.zeros(2 * m * s * batch)
        th = np.zeros(s * batch)
        self._check(self.lib.phx_small_eig(self.h, m, s, batch, _dptr(np.ascontiguousarray(Gf)), _iptr(k), _dptr(C),
                                           _dptr(th)))
        return C.view(np.complex128).reshape(batch, s, m).transpose(0, 2, 1), th.reshape(batch, s)

    def small_rr(self, G2, s: int, drop: float = 1e-12):
        """G2: (batch, m, 2m) = S^H [K S | Omega S]; returns Cx, Cp (batch, m, s), theta, keep."""
        G2 = np.asarray(G2, dtype=np.complex128)
        batch, m, _ = G2.shape
        Gf = np.concatenate([np.asfortranarray(g).reshape(-1, order="F") for g in G2]).view(np.float64)
        Cx = np.zeros(2 * m * s * batch)
        Cp = np.zeros(2 * m * s * batch)
        th = np.zeros(s * batch)
        keep = np.zeros(m * batch, dtype=np.int32)
        self._check(self.lib.phx_small_rr(self.h, m, s, batch, _dptr(np.ascontiguousarray(Gf)), drop, _dptr(Cx),
                                          _dptr(Cp), _dptr(th), _iptr(keep)))
        f = lambda a: a.view(np.complex128).reshape(batch, s, m).transpose(0, 2, 1)
        return f(Cx), f(Cp), th.reshape(batch, s), keep.reshape(batch, m)

    # ---------------------------------------------------------------- design projection
    def project(self, p: Projection, x) -> np.ndarray:
        xx = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        if xx.size != projection_size(p):
            raise ValueError("x has the wrong number of design variables")
        rho = np.zeros(p.nv ** 3)
        self._check(self.lib.phx_project(self.h, byref(p), _dptr(xx), _dptr(rho)))
        return rho.reshape(p.nv, p.nv, p.nv)

    def project_adjoint(self, p: Projection, x, grad_rho) -> np.ndarray:
        xx = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        g = np.ascontiguousarray(grad_rho, dtype=np.float64).reshape(-1)
        if xx.size != projection_size(p) or g.size != p.nv ** 3:
            raise ValueError("wrong array sizes")
        out = np.zeros(xx.size)
        self._check(self.lib.phx_project_adjoint(self.h, byref(p), _dptr(xx), _dptr(g), _dptr(out)))
        return out

    def project_dev(self, p: Projection, x_t):
        """torch CUDA tensors: design variables (projection_size(p) values) -> rho (nv, nv, nv)."""
        import torch
        x_t = x_t.detach().contiguous().to(torch.float64)
        if x_t.numel() != projection_size(p):
            raise ValueError("x has the wrong number of design variables")
        rho = torch.empty((p.nv, p.nv, p.nv), dtype=torch.float64, device=x_t.device)
        st = torch.cuda.current_stream(x_t.device).cuda_stream
        self._check(self.lib.phx_project_dev(self.h, byref(p), c_void_p(x_t.data_ptr()), c_void_p(rho.data_ptr()),
                                             c_void_p(st)))
        return rho

    def project_adjoint_dev(self, p: Projection, x_t, grad_rho_t):
        """torch CUDA tensors: the backward of project_dev (shaped like x_t)."""
        import torch
        x_t = x_t.detach().contiguous().to(torch.float64)
        g_t = grad_rho_t.detach().contiguous().to(torch.float64)
        if x_t.numel() != projection_size(p) or g_t.numel() != p.nv ** 3:
            raise ValueError("wrong tensor sizes")
        out = torch.empty(x_t.shape, dtype=torch.float64, device=x_t.device)
        st = torch.cuda.current_stream(x_t.device).cuda_stream
        self._check(self.lib.phx_project_adjoint_dev(self.h, byref(p), c_void_p(x_t.data_ptr()),
                                                     c_void_p(g_t.data_ptr()), c_void_p(out.data_ptr()),
                                                     c_void_p(st)))
        return out

    def project_adjoint_dev_noalloc(self, p: Projection, x_t, grad_rho_t, out_t):
        """The backward of project_dev into the caller's tensor out_t (shaped like x_t), through
        the library's fixed device scratch: neither the library nor this binding allocates.
        All tensors must be contiguous float64 device tensors; the work is queued on torch's
        current stream."""
        import torch
        for t in (x_t, grad_rho_t, out_t):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("contiguous float64 device tensors required")
        if x_t.numel() != projection_size(p) or out_t.numel() != x_t.numel() or grad_rho_t.numel() != p.nv ** 3:
            raise ValueError("wrong tensor sizes")
        st = torch.cuda.current_stream(x_t.device).cuda_stream
        self._check(self.lib.phx_project_adjoint_dev_noalloc(self.h, byref(p), c_void_p(x_t.data_ptr()),
                                                             c_void_p(grad_rho_t.data_ptr()),
                                                             c_void_p(out_t.data_ptr()), c_void_p(st)))
        return out_t
