"""The laminate and sphere-inclusion studies (Results, "A note on normalized band gaps"),
host parts: the transfer-matrix laminate analysis against the quarter-wave closed form,
the homogeneous limit and the paper's printed 1-D value; the sphere designs' volume."""
import json
import math
import os

import numpy as np
import pytest

from paper_1603_06855_amd import studies, synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "normalized_gap_studies.json")))


def _paper_materials():
    w, e = GOLDEN["materials"]["wc"], GOLDEN["materials"]["epoxy"]
    return synth.Material(*w), synth.Material(*e)


def test_paper_materials_match_synth():
    wc, ep = _paper_materials()
    assert wc == synth.WC_PAPER and ep == synth.EPOXY_PAPER


@pytest.mark.parametrize("pol", ["S", "P"])
def test_quarter_wave_stack_closed_form(pol):
    """Equal transit times through both layers: the first gap spans pi/2 +- arcsin(|Z1 - Z0| /
    (Z1 + Z0)) in phase per layer, so its normalised width is (4/pi) arcsin(|Z1 - Z0| / (Z1 + Z0))."""
    wc, ep = _paper_materials()
    f = studies.quarter_wave_fraction(wc, ep, pol)
    z1 = wc.density * studies.layer_speed(wc, pol)
    z0 = ep.density * studies.layer_speed(ep, pol)
    lo, hi, g = studies.rytov_first_gap(wc, ep, f, pol)
    assert g == pytest.approx(4.0 / math.pi * math.asin(abs(z1 - z0) / (z1 + z0)), rel=1e-10)
    # the gap centre is where each layer is a quarter wavelength thick
    c1 = studies.layer_speed(wc, pol)
    assert 0.5 * (lo + hi) == pytest.approx(math.pi / 2 * c1 / f, rel=0.05)


def test_homogeneous_laminate_has_no_gap_and_linear_branches():
    m = synth.Material(1000.0, 2e9, 0.3)
    assert studies.rytov_first_gap(m, m, 0.4, "S")[2] == 0.0
    c = studies.layer_speed(m, "S")
    for k in (0.3, 1.0, 2.5):
        w = studies.rytov_omega(k, m, m, 0.4, "S", 2)
        assert w[0] == pytest.approx(c * k, rel=1e-10)
        assert w[1] == pytest.approx(c * (2 * math.pi - k), rel=1e-10)


def test_laminate_reproduces_the_printed_1d_gap():
    """The paper's 1-D number: 155.5 % at a WC fraction of 0.737.  The shear branch's first
    gap peaks at 155.8 % at 0.736 (the quarter-wave fraction); the longitudinal one at
    154.5 % at 0.724."""
    wc, ep = _paper_materials()
    fs = np.linspace(0.6, 0.85, 251)
    g = studies.laminate_gap_sweep(wc, ep, fs, "S")
    i = int(np.argmax(g))
    ref = GOLDEN["laminate_1d"]
    assert abs(100 * g[i] - ref["max_gap_percent"]) < 0.5
    assert abs(fs[i] - ref["at_fraction"]) < 0.005


@pytest.mark.parametrize("lat", ["SC", "BCC", "FCC"])
def test_sphere_radius_and_voxel_fraction(lat):
    for f in (0.2, 0.45, 0.6):
        r = studies.sphere_radius(lat, f)
        assert 4.0 / 3.0 * math.pi * r ** 3 == pytest.approx(f * studies.VOLUME_FACTOR[lat], rel=1e-12)
        rho = synth.sphere(32, lat, r)
        assert abs(rho.mean() - f) < 0.02


def test_normalized_gap_edges():
    om = np.array([[1.0, 2.0, 5.0], [1.5, 3.0, 4.0]])
    g, lo, hi = studies.normalized_gap(om, 2)
    assert (lo, hi) == (3.0, 4.0) and g == pytest.approx(2.0 / 7.0)
