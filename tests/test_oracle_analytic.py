"""Pins against the analytic quadratic limb-darkening model (Mandel & Agol
2002), the model the paper measures its own accuracy against (Sect. 3.3):

* the analytic model and Oracle-B (adaptive quadrature of the plain
  definition, Eq. 1-2) agree to rounding for any (p, z, u1, u2);
* the uniform source and the out-of-transit region reduce to closed forms;
* Oracle-A's error against it shrinks with the grid resolution and is at the
  paper's level (a few ppm; the accuracy figure quotes ~5 ppm at its lowest
  resolution, `tests/golden/fig2_setup.json`) -- the resolutions of that figure
  are garbled in the text, so the grids here are our own sweep;
* the single-light-curve configuration (quadratic LD sampled at 100 mu) at
  the default grid is within 1 ppm of the analytic light curve."""

import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import analytic as an
from oracle import exact as ex
from oracle import orbit
from oracle import roadrunner as orr

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("u1,u2", [(0.4, 0.25), (0.1, 0.6), (0.8, -0.1)])
def test_analytic_matches_exact_definition(u1, u2):
    prof = lambda mu: 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2   # noqa: E731
    istar = ex.istar_exact(prof)
    for p in (0.01, 0.1, 0.25, 0.45):
        z = np.array([0.0, 0.03, p, 0.3, 0.6, 1.0 - p - 1e-3, 1.0 - p, 1.0 - p + 1e-3, 1.0,
                      1.0 + p - 1e-3, 1.0 + p + 1e-3])
        fa = an.quadratic_flux(z, p, u1, u2)
        fb = ex.flux_exact(z, p, prof, istar=istar)
        assert np.abs(fa - fb).max() <= 1e-12, (p, np.abs(fa - fb).max())


def test_analytic_special_cases():
    # uniform source: 1 - p^2 fully inside, lens area outside
    assert an.quadratic_flux([0.3], 0.1, 0.0, 0.0)[0] == pytest.approx(1.0 - 0.01, abs=1e-15)
    z = 1.02
    lens = an.lambda_e(0.1, z)
    assert an.quadratic_flux([z], 0.1, 0.0, 0.0)[0] == pytest.approx(1.0 - lens, abs=1e-15)
    # no overlap
    assert np.all(an.quadratic_flux([1.1, 1.5, 3.0], 0.1, 0.4, 0.25) == 1.0)
    # the inside and limb-crossing branches meet at z = 1 - p
    p = 0.1
    a, b = an.quadratic_flux([1.0 - p - 1e-9, 1.0 - p + 1e-9], p, 0.4, 0.25)
    assert abs(a - b) < 1e-7
    # symmetric in time for a circular orbit: depends on z only, and the
    # centre value is the deepest
    zz = np.linspace(0.0, 1.2, 121)
    f = an.quadratic_flux(zz, 0.1, 0.4, 0.25)
    assert np.all(np.diff(f) >= -1e-15)


def fig2_errors(zcut, nzin, nzlimb, ng, ks=(0.01, 0.05, 0.1), u1=0.4, u2=0.25):
    mu = np.linspace(0.0, 1.0, 1001)
    prof = 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2
    # k on nodes of the k grid (dk = 0.01): only the g-interpolation and the
    # annuli are approximations, as for the paper's figure
    tab = orr.Tables(mu, prof, zcut=zcut, nzin=nzin, nzlimb=nzlimb, ng=ng, nk=30,
                     k0=0.01, k1=0.30)
    g = np.linspace(0.0, 0.999, 400)
    return [np.abs(orr.flux_at_z(tab, 0, k, g * (1 + k)) -
                   an.quadratic_flux(g * (1 + k), k, u1, u2)).max() * 1e6 for k in ks]


def test_oracle_a_accuracy_against_analytic_converges():
    golden = json.load(open(os.path.join(HERE, "golden", "fig2_setup.json")))
    low = fig2_errors(0.7, 20, 40, 100)        # nz 60, ng 100
    mid = fig2_errors(0.7, 40, 80, 150)        # nz 120, ng 150
    high = fig2_errors(0.7, 60, 120, 200)      # nz 180, ng 200
    # the paper's class: a few ppm at low resolution
    assert max(low) <= 2.0 * golden["lowest_resolution_max_error_ppm"]
    assert max(mid) <= golden["lowest_resolution_max_error_ppm"]
    assert max(high) <= 3.0
    assert max(high) < max(mid) < max(low)


def test_single_light_curve_within_one_ppm_of_analytic():
    w = wl.single_light_curve()
    row = w["pv"][0]
    tab = orr.Tables(w["mu_s"], w["I_s"], **wl.DEFAULT_GRID)
    fa = orr.evaluate(tab, w["times"], w["pv"])[0]
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    fm = np.where(front, an.quadratic_flux(z, row[6], 0.4, 0.25), 1.0)
    assert np.abs(fa - fm).max() <= 1e-6
    assert np.count_nonzero(fm < 1.0) == 316          # the configuration's in-transit count
