"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and the host-only entry points (k-paths, argument validation) behave.
No compute call is made here (there may be no GPU)."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_1603_06855_amd import phx, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phx.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phx_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_solver_calls():
    syms = declared_symbols()
    for s in ("phx_create", "phx_destroy", "phx_last_error", "phx_kpath", "phx_fourier", "phx_schur",
              "phx_bands", "phx_sens", "phx_adjoint", "phx_bands_batch", "phx_sens_dev", "phx_validate"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(phx.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    out = subprocess.run(["nm", "-D", "--defined-only", phx.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (phx_\w+)", out))
    assert set(declared_symbols()) <= exported


def test_library_has_gfx950_code():
    out = subprocess.run(["/opt/rocm/llvm/bin/clang-offload-bundler", "--list", "--type=o",
                          "--input=" + phx.LIB_PATH], capture_output=True, text=True)
    blob = open(phx.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


@pytest.mark.parametrize("lat", ["SC", "BCC", "FCC"])
@pytest.mark.parametrize("nk", [None, 11, 40, 60])
def test_kpath_matches_oracle(lat, nk):
    from oracle import geometry
    nvert = len(geometry.DEFAULT_PATHS[lat].replace("|", ""))
    nk = nvert if nk is None else max(nk, nvert)
    assert np.allclose(phx.kpath(lat, nk), geometry.kpath(lat, nk), atol=1e-15)
    if lat == "SC":
        assert np.allclose(phx.kpath(lat, 10, "GXMGR"), geometry.kpath(lat, 10, "GXMGR"), atol=1e-15)


@pytest.mark.parametrize("lat", ["SC", "BCC", "FCC"])
def test_library_kpath_vertices_lie_on_the_brillouin_zone_boundary(lat):
    """The library's own vertex table and conversion to reciprocal coordinates, pinned like
    the oracle's: each non-Gamma vertex it emits is on the first Brillouin-zone boundary."""
    from oracle import geometry
    from tests.test_oracle import bz_boundary_defect
    path = geometry.DEFAULT_PATHS[lat]
    verts = path.replace("|", "")
    Q = phx.kpath(lat, len(verts))
    B = np.linalg.inv(geometry.primitive_vectors(lat, 1.0)).T
    for v, q in zip(verts, Q):
        if v == "G":
            continue
        on, inside = bz_boundary_defect(lat, q @ B)
        assert abs(on) < 1e-12 and inside > -1e-12, (lat, v)


def test_kpath_rejects_bad_arguments():
    lib = phx.load()
    q = np.zeros(300)
    ptr = q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.phx_kpath(0, b"GXZ", 20, ptr) == phx.EINVAL      # unknown point
    assert lib.phx_kpath(0, None, 3, ptr) == phx.EINVAL         # fewer points than vertices
    assert lib.phx_kpath(7, None, 20, ptr) == phx.EINVAL        # unknown lattice


def _cell(**kw):
    c = synth.Cell("SC", 1.0, 8, 2)
    d = c.__dict__.copy()
    d.update(kw)
    return synth.Cell(**d)


def test_validate_accepts_a_good_problem():
    rc, msg = phx.validate(_cell(), np.full(512, 0.5), np.zeros((4, 3)), 8, (6, 7))
    assert rc == phx.OK, msg


@pytest.mark.parametrize("kw,rho,q,nb,bands,frag", [
    (dict(nv=4), None, None, 0, (), "2M+1"),
    (dict(M=0, nv=4), None, None, 0, (), "M must"),
    (dict(a=-1.0), None, None, 0, (), "edge"),
    (dict(phase1=synth.Material(1000.0, 1e9, 0.5)), None, None, 0, (), "Poisson"),
    (dict(simp_p=0.5), None, None, 0, (), "simp_p"),
    ({}, np.full(512, np.nan), None, 0, (), "rho"),
    ({}, np.full(512, -0.1), None, 0, (), "rho"),
    ({}, None, np.full((2, 3), np.inf), 0, (), "finite"),
    ({}, None, np.zeros((0, 3)), 0, (), "nk must be positive"),
    ({}, None, None, 17, (), "nbands"),
    ({}, None, None, 8, (9,), "band_no"),
])
def test_validate_rejects(kw, rho, q, nb, bands, frag):
    rc, msg = phx.validate(_cell(**kw), rho, q, nb, bands)
    assert rc == phx.EINVAL and frag in msg


def test_create_without_device_reports_ehip():
    if os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"):
        pytest.skip("a GPU may be present")
    lib = phx.load()
    h = ctypes.c_void_p()
    assert lib.phx_create(ctypes.byref(h), 0) == phx.EHIP


def test_one_hip_runtime_per_process():
    """Loading the library and then using torch must leave a single HIP runtime in the
    process (two runtimes would not share devices, pointers or streams)."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1603_06855_amd import phx\n"
            "phx.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = sorted(set(l.split()[-1] for l in maps if 'libamdhip64' in l))\n"
            "print(len(libs), libs)\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("1 "), out.stdout


def test_projection_size_counts_design_variables():
    assert phx.projection_size(phx.projection(32, 2, 2.8, 1.0, False)) == 16 ** 3
    assert phx.projection_size(phx.projection(32, 2, 2.8, 1.0, True)) == 8 ** 3
    assert phx.projection_size(phx.projection(20, 1, 1.5, 1.0, False)) == 20 ** 3
    with pytest.raises(phx.PhxError):
        phx.projection_size(phx.projection(15, 2, 2.8, 1.0, False))
    with pytest.raises(phx.PhxError):
        phx.projection_size(phx.projection(18, 2, 2.8, 1.0, True))
