"""GPU: Omega_s X applied as an exact convolution with the density's Fourier table (option
omega_conv = 1, the default for M <= 5) against the dense real operator in the paired basis
(omega_conv = 0), through whole solves: the two routes compute the same product up to
rounding, so the frequencies and the adjoint sensitivities agree far inside the solver
tolerance.  Cases: FCC 32^3 M = 5 (with the coarse start at M = 2 and at M = 3), BCC 24^3
M = 4 (with the coarse start at M = 2 and at M = 1), SC M = 1, 2 and 3; k-points off Gamma (no zero modes), FP64 and mixed precision.  The
solver-level parity tests against the oracle run with the default (the convolution).  At
M = 6, beyond the convolution kernel's orders, both settings take the dense product and give
identical results (with the coarse start off: its order-4 solve would take the
convolution).
"""
import sys

import numpy as np
import pytest

from paper_1603_06855_amd import phx, synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = phx.Context(0)
    yield c
    c.close()


CASES = {
    "FCC-M5-drop3": (synth.Cell("FCC", 1.0, 32, 5), lambda: synth.box_smoothed_uniform(32, 400), "FCC", 3),
    "FCC-M5-drop2": (synth.Cell("FCC", 1.0, 32, 5), lambda: synth.box_smoothed_uniform(32, 401), "FCC", 2),
    "BCC-M4": (synth.Cell("BCC", 1.0, 24, 4), lambda: synth.gaussian_blob(24, "BCC", 303), "BCC", 2),
    "SC-M3": (synth.Cell("SC", 1.0, 16, 3), lambda: synth.box_smoothed_uniform(16, 202), "SC", 2),
    "SC-M2": (synth.Cell("SC", 1.0, 8, 2), lambda: synth.box_smoothed_uniform(8, 101), "SC", 2),
    "SC-M1": (synth.Cell("SC", 1.0, 8, 1), lambda: synth.box_smoothed_uniform(8, 104), "SC", 2),
    "BCC-M4-drop3": (synth.Cell("BCC", 1.0, 24, 4), lambda: synth.gaussian_blob(24, "BCC", 304), "BCC", 3),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_convolution_equals_dense_operator(ctx, case, prec):
    cell, make_rho, lat, drop = CASES[case]
    rho = make_rho()
    q = phx.kpath(lat, 24)[[3, 9, 15, 21]]
    nb, bands = (12, (6, 7)) if cell.M >= 4 else (8, (3, 6))
    log("case", case, prec, "M", cell.M, "nk", len(q))
    ctx.set_option("tol_fp64", 1e-10)
    ctx.set_option("coarse_drop", drop)
    res = {}
    try:
        for conv in (0, 1):
            ctx.set_option("omega_conv", conv)
            om, dw = ctx.sens(cell, rho, q, nb, bands, prec)
            res[conv] = (om, dw)
            log("  omega_conv", conv, "status", ctx.last_status, "iters", ctx.stat("iters"))
    finally:
        ctx.set_option("omega_conv", 1)
        ctx.set_option("coarse_drop", 2)
        ctx.set_option("tol_fp64", 1e-8)
    (om0, dw0), (om1, dw1) = res[0], res[1]
    assert np.all(om0 > 0)
    om_rel = np.abs(om1 - om0) / om0
    # sensitivities: summed over each run of bands whose relative gaps are below 1e-4 (the
    # derivative of a cluster's sum is basis independent), within the computed bands
    sens_rel, n = 0.0, 0
    for k in range(len(q)):
        for j, b in enumerate(bands):
            lo, hi = b - 1, b - 1
            w = om0[k]
            while lo > 0 and w[lo] - w[lo - 1] < 1e-4 * w[lo]:
                lo -= 1
            while hi + 1 < nb and w[hi + 1] - w[hi] < 1e-4 * w[hi + 1]:
                hi += 1
            cl = [c + 1 for c in range(lo, hi + 1)]
            if not all(c in bands for c in cl) or hi == nb - 1:
                continue
            idx = [bands.index(c) for c in cl]
            a, r = dw1[k, idx].sum(axis=0), dw0[k, idx].sum(axis=0)
            sens_rel = max(sens_rel, float(np.abs(a - r).max() / np.abs(r).max()))
            n += 1
    log("  max rel omega diff", om_rel.max(), "max sens diff", sens_rel, "over", n, "clusters")
    assert n >= len(q)
    assert om_rel.max() <= (1e-9 if prec == "fp64" else 1e-8)
    assert sens_rel <= (1e-7 if prec == "fp64" else 1e-5)


def test_order_six_takes_the_dense_product(ctx):
    cell = synth.Cell("SC", 1.0, 16, 6)
    rho = synth.box_smoothed_uniform(16, 203)
    q = phx.kpath("SC", 24)[[3, 9]]
    log("case SC M=6 fp64 nk", len(q))
    res = {}
    ctx.set_option("coarse", 0)
    try:
        for conv in (0, 1):
            ctx.set_option("omega_conv", conv)
            res[conv] = ctx.sens(cell, rho, q, 8, (3, 6), "fp64")
            log("  omega_conv", conv, "status", ctx.last_status, "iters", ctx.stat("iters"))
    finally:
        ctx.set_option("omega_conv", 1)
        ctx.set_option("coarse", 1)
    assert np.all(res[0][0] > 0)
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
