"""The library's host module (csrc/host.cpp: validation, Brillouin-zone path, chunk sizing,
factor-sharing groups, degenerate-cluster plan) built with the host compiler under the
address and undefined-behaviour sanitizers, driven by tests/host_check.cpp.

Any out-of-bounds access, use after free, leak, signed overflow or similar aborts the
driver (-fno-sanitize-recover=all), so every case below is also a sanitizer check.  The
results are compared with the oracle (the k-path) and with the definitions the module
implements (clusters of Ritz values, factor groups, validation rules).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LATTICES = {"SC": 0, "BCC": 1, "FCC": 2}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which(os.environ.get("CXX", "g++"))
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("host") / "host_check")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_check.cpp"),
           os.path.join(ROOT, "paper_1603_06855_amd", "csrc", "host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def run(mode, lines):
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        env.pop("LD_PRELOAD", None)
        p = subprocess.run([exe, mode], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env)
        assert p.returncode == 0, f"sanitizer or driver failure ({p.returncode}):\n{p.stderr[-4000:]}"
        out = p.stdout.strip().splitlines()
        assert len(out) == len(lines)
        return out

    return run


def fields(line):
    return [part.split() for part in line.split("|")]


# ---------------------------------------------------------------- k-path

KP_CASES = [(lat, nk, None) for lat in LATTICES for nk in (12, 13, 17, 40, 41, 97, 200)]
KP_CASES += [("SC", 12, "GXMGR"), ("SC", 5, "GXMGR"), ("SC", 1, "G"), ("SC", 3, "G|X|M"), ("SC", 9, "|GX||MR|"),
             ("BCC", 30, "GHNGPH|PN"), ("FCC", 33, "LGXWK"), ("FCC", 8, "GX|UW"), ("BCC", 4, "PP|PP")]


def test_kpath_matches_the_oracle_under_sanitizers(driver):
    lines = [f"{LATTICES[lat]} {nk} {path or '-'}" for lat, nk, path in KP_CASES]
    for (lat, nk, path), out in zip(KP_CASES, driver("kpath", lines)):
        v = out.split()
        assert int(v[0]) == 0, (lat, nk, path)
        q = np.array(v[1:], float).reshape(nk, 3)
        assert np.abs(q - geometry.kpath(lat, nk, path)).max() <= 1e-15, (lat, nk, path)


def test_kpath_rejects_bad_paths_under_sanitizers(driver):
    bad = [(0, 3, "-"),        # fewer points than vertices
           (0, 20, "GXZ"),     # no Z point on SC
           (1, 20, "GX"),      # X is not a BCC label
           (0, 10, "||"),      # no vertex at all
           (0, 10, "GG"),      # extra points but zero path length
           (0, 7, "G|X|M"),    # extra points but no segment to hold them
           (7, 10, "-"),       # unknown lattice
           (0, 0, "G"), (0, -4, "-")]
    out = driver("kpath", [f"{a} {b} {c}" for a, b, c in bad])
    assert [int(o.split()[0]) for o in out] == [-1] * len(bad)


# ---------------------------------------------------------------- degenerate-cluster plan

def clusters_by_definition(om, dtol):
    """Maximal runs of neighbours whose frequency gap is below dtol times the upper one."""
    runs, start = [], 0
    for i in range(1, len(om) + 1):
        if i == len(om) or not (om[i] - om[i - 1] < dtol * om[i]):
            runs.append((start, i - 1))
            start = i
    return runs


def random_plan_case(rng):
    nk, s = int(rng.integers(1, 5)), int(rng.integers(1, 22))
    dtol = float(rng.choice([0.0, 1e-8, 1e-3]))
    th = []
    for _ in range(nk):
        om = np.sort(rng.uniform(0.5, 3.0, s))
        for _ in range(int(rng.integers(0, 4))):   # planted clusters
            i = int(rng.integers(0, s))
            j = min(s, i + int(rng.integers(2, 4)))
            om[i:j] = om[i] * (1 + rng.uniform(-1, 1, j - i) * 1e-12)
        om = np.sort(om)
        if rng.random() < 0.2:
            om[0] = 0.0                                # a rigid-body zero at Gamma
        th.append(om ** 2)
    th = np.array(th)
    nsel = int(rng.integers(1, s + 1))
    sel = np.sort(rng.choice(s, nsel, replace=False))
    return nk, s, dtol, th, sel


def test_cluster_plan_follows_its_definition_under_sanitizers(driver):
    rng = np.random.default_rng(7)
    cases = [random_plan_case(rng) for _ in range(300)]
    lines = [f"{nk} {s} {len(sel)} {dtol!r} " + " ".join(repr(float(x)) for x in th.ravel()) + " "
             + " ".join(str(int(b)) for b in sel) for nk, s, dtol, th, sel in cases]
    for (nk, s, dtol, th, sel), out in zip(cases, driver("plan", lines)):
        nd, lo, hi, ext, coef = fields(out)
        lo, hi = np.array(lo, int).reshape(nk, len(sel)), np.array(hi, int).reshape(nk, len(sel))
        want_lo, want_hi = np.array(sel)[None].repeat(nk, 0), np.array(sel)[None].repeat(nk, 0)
        for k in range(nk):
            om = np.sqrt(np.maximum(th[k], 0.0))
            for a, b in clusters_by_definition(om, dtol) if dtol > 0 else []:
                for j, band in enumerate(sel):
                    if a <= band <= b and th[k, band] > 0:
                        want_lo[k, j], want_hi[k, j] = a, b
        assert np.array_equal(lo, want_lo) and np.array_equal(hi, want_hi)
        ndeg = int(np.count_nonzero(hi > lo))
        assert int(nd[0]) == ndeg
        ext = [int(x) for x in ext]
        if ndeg == 0:
            assert ext == [int(b) for b in sel] and coef == []
            continue
        members = set(int(b) for b in sel)
        for k in range(nk):
            for j in range(len(sel)):
                members.update(range(lo[k, j], hi[k, j] + 1))
        assert ext == sorted(members)
        C = np.array(coef, float).reshape(nk, len(sel), len(ext))
        assert np.allclose(C.sum(-1), 1.0, rtol=0, atol=1e-15)   # each result is a mean
        for k in range(nk):
            for j in range(len(sel)):
                on = [t for t, b in enumerate(ext) if lo[k, j] <= b <= hi[k, j]]
                assert np.all(C[k, j, on] == 1.0 / (hi[k, j] - lo[k, j] + 1))
                assert np.count_nonzero(C[k, j]) == len(on)


# ---------------------------------------------------------------- factor-sharing groups

def test_share_groups_invariants_under_sanitizers(driver):
    rng = np.random.default_rng(11)
    cases = []
    for lat in LATTICES:
        for nk in (1, 2, 12, 40):
            if nk < 12 and nk != 1:
                qr = rng.uniform(-0.5, 0.5, (nk, 3))
            elif nk == 1:
                qr = np.zeros((1, 3))
            else:
                qr = geometry.kpath(lat, nk)
            A = geometry.primitive_vectors(lat, 1.0)
            qc = qr @ np.linalg.inv(A).T                      # Cartesian, cycles per a
            for kmax, dist, rel, f0 in ((1, 0.15, 0.5, 0), (2, 0.15, 0.5, 3), (8, 1.0, 0.5, 0), (8, 1.0, 1.0, 5)):
                which = (rng.random(nk) < 0.7).astype(int)
                cases.append((qc, which, kmax, dist, rel, f0))
    lines = [f"{len(w)} {km} {d!r} {r!r} {f0} " + " ".join(repr(float(x)) for x in qc.ravel()) + " "
             + " ".join(str(x) for x in w) for qc, w, km, d, r, f0 in cases]
    for (qc, which, kmax, dist, rel, f0), out in zip(cases, driver("groups", lines)):
        ng, fmap, lead = fields(out)
        ng, fmap, lead = int(ng[0]), np.array(fmap, int), [int(x) for x in lead]
        act = np.flatnonzero(which)
        assert np.all(fmap[which == 0] == -1)
        assert ng == len(lead) and (len(act) == 0) == (ng == 0)
        if ng == 0:
            continue
        assert lead[0] == act[0] and sorted(lead) == lead
        assert np.array_equal(np.unique(fmap[act]), np.arange(f0, f0 + ng))
        assert np.all(np.diff(fmap[act]) >= 0)                 # groups are runs of the active k's
        for g, l in enumerate(lead):
            assert fmap[l] == f0 + g
            for k in act[fmap[act] == f0 + g]:
                d = np.linalg.norm(qc[k] - qc[l])
                assert k - l < kmax and d <= dist
                assert d <= rel * min(np.linalg.norm(qc[k]), np.linalg.norm(qc[l]))
            if g > 0:   # a new group starts only where the previous leader's bounds fail
                p = lead[g - 1]
                d = np.linalg.norm(qc[l] - qc[p])
                assert not (l - p < kmax and d <= dist and
                            d <= rel * min(np.linalg.norm(qc[l]), np.linalg.norm(qc[p])))
        for k in act:   # Gamma shares its factor with no other wave vector (rigid modes)
            if not qc[k].any():
                assert not any(qc[j].any() for j in act[fmap[act] == fmap[k]])


# ---------------------------------------------------------------- validation

GOOD = dict(lat=0, a=1.0, M=3, nv=16, r0=1.0, E0=1.0, n0=0.3, r1=10.0, E1=100.0, n1=0.25, simp=3.0, nb=8,
            block=0, nsens=2, band=(6, 7))


def cell_line(**kw):
    c = dict(GOOD, **kw)
    return (f"{c['lat']} {c['a']!r} {c['M']} {c['nv']} {c['r0']!r} {c['E0']!r} {c['n0']!r} {c['r1']!r} {c['E1']!r} "
            f"{c['n1']!r} {c['simp']!r} {c['nb']} {c['block']} {c['nsens']} " + " ".join(str(b) for b in c["band"]))


CELL_CASES = [
    ({}, "ok", "ok"),
    (dict(lat=3), "unknown lattice", None), (dict(lat=-1), "unknown lattice", None),
    (dict(a=0.0), "cube edge", None), (dict(a=float("nan")), "cube edge", None), (dict(a=float("inf")), "cube edge", None),
    (dict(M=0), "order M", None), (dict(M=9), "order M", None),
    (dict(M=3, nv=6), "nv must be at least", None), (dict(M=1, nv=257), "at most 256", None),
    (dict(r0=0.0), "material", None), (dict(E1=-1.0), "material", None), (dict(n0=0.5), "material", None),
    (dict(n1=-1.0), "material", None), (dict(r1=float("nan")), "material", None),
    (dict(simp=0.5), "simp_p", None), (dict(simp=float("inf")), "simp_p", None),
    (dict(nb=0), "ok", "nbands"), (dict(nb=17), "ok", "nbands"), (dict(M=1, nv=3, nb=16), "ok", "ok"),
    (dict(block=8), "ok", "option block"), (dict(block=9), "ok", "ok"), (dict(M=1, nv=3, nb=10, block=10), "ok", "option block"),
    (dict(nsens=-1, band=()), "ok", "nsens"), (dict(nsens=0, band=()), "ok", "ok"),
    (dict(band=(0, 7)), "ok", "band_no"), (dict(band=(6, 9)), "ok", "band_no"), (dict(nsens=3, band=(8, 8, 1)), "ok", "ok"),
]


def test_validation_rules_under_sanitizers(driver):
    out = driver("cell", [cell_line(**kw) for kw, _, _ in CELL_CASES])
    for (kw, want_cell, want_bands), o in zip(CELL_CASES, out):
        got_cell, got_bands = (x.strip() for x in o.split("|"))
        assert want_cell in got_cell, (kw, o)
        if want_bands is not None:
            assert want_bands in got_bands, (kw, o)


PROJ_CASES = [("32 2 2.8 1 0", 16 ** 3), ("32 2 2.8 1 1", 8 ** 3), ("32 1 1.5 0 0", 32 ** 3), ("30 2 2.8 64 1", -1),
              ("31 2 2.8 1 0", -1), ("32 3 2.8 1 0", -1), ("1 1 0.5 1 0", -1), ("32 2 0.8 1 0", -1),
              ("32 2 15 1 0", -1), ("32 2 2.8 -1 0", -1), ("32 2 2.8 1001 0", -1), ("32 2 nan 1 0", -1)]


def test_projection_checks_under_sanitizers(driver):
    out = driver("proj", [c for c, _ in PROJ_CASES])
    for (c, want), o in zip(PROJ_CASES, out):
        assert int(o.split("|")[0]) == want, (c, o)


# ---------------------------------------------------------------- chunk sizing

def test_block_and_chunk_sizing_under_sanitizers(driver):
    # order M = 5: N = 11^3 plane waves, n3 = 3N; the full-order pencil of the FCC design
    N, n3, Np = 1331, 3993, 1331 * 8
    cases = []
    for nb in (1, 8, 10, 16):
        for prec in (0, 1):
            for precond in (0, 1, 2):
                for mem in (1e-6, 0.5, 64.0, 1e6):
                    cases.append((40, mem, n3, Np, nb, N, prec, precond, 0))
    cases += [(7, 64.0, 3 * 27, 27 * 8, 8, 27, 0, 0, 0), (7, 64.0, 3 * 27, 27 * 8, 8, 27, 0, 0, 100),
              (3, 64.0, n3, Np, 8, N, 0, 0, 12)]
    out = driver("size", [" ".join(repr(x) if isinstance(x, float) else str(x) for x in c) for c in cases])
    res = {}
    for c, o in zip(cases, out):
        s, per, kc = (int(x) for x in o.split())
        nk, mem, n3_, Np_, nb, N_, prec, precond, block = c
        want_s = min(block if block > 0 else min(21, nb + max(8, nb)), 3 * N_)
        assert s == want_s and (s > nb or block > 0)
        assert per > 0 and 1 <= kc <= nk
        assert kc == max(1, min(nk, int(mem * 2 ** 30 // per)))
        res[c] = per
    for nb in (1, 8, 10, 16):
        for precond in (0, 1, 2):
            assert res[(40, 64.0, n3, Np, nb, N, 1, precond, 0)] <= res[(40, 64.0, n3, Np, nb, N, 0, precond, 0)]
        assert res[(40, 64.0, n3, Np, nb, N, 0, 1, 0)] < res[(40, 64.0, n3, Np, nb, N, 0, 0, 0)]
        # the FP64 pencil factor dominates: n3^2 complex doubles per k-point
        assert res[(40, 64.0, n3, Np, nb, N, 0, 0, 0)] >= 16 * n3 * n3
