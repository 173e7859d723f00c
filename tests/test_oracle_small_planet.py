"""Pins of the oracle's small-planet approximation (Sect. 3.4.2: below a
radius-ratio threshold, the LD-weighted mean over the planet's disk is
replaced by the LD value at the planet's centre):

* a uniform profile reproduces the uniform-source closed form exactly,
  at the limb as well (every LD value is 1);
* with linear LD, on g nodes fully inside the disk, the occulted fraction
  is the closed form I(mu_c) k^2 / (1 - u/3) with mu_c = sqrt(1 - z^2);
* with quadratic LD it is within 1e-9 of the analytic quadratic model at
  k = 0.004 for z <= 0.9, and its error there grows as k^4 (depth ~ k^2
  times the centre-value error ~ k^2 times the profile's Laplacian), which
  a wrong centre distance or a dropped normaliser would break;
* a k at or above the threshold follows the interpolated model exactly,
  and a k below the table's k0 but not below the threshold is a NaN row."""

import numpy as np
import pytest

import workloads as wl
from oracle import analytic as an
from oracle import orbit
from oracle import roadrunner as orr

# a g-resolved, k-coarse grid (nk = 2 keeps the 3-D weight table small)
SP_GRID = dict(zcut=0.7, nzin=10, nzlimb=10, ng=2048, nk=2, k0=0.01, k1=0.30)


@pytest.mark.parametrize("k", [0.002, 0.006])
def test_uniform_source_closed_form(k):
    w = wl.single_light_curve()
    mu = w["mu_s"]
    t = orr.Tables(mu, np.ones_like(mu), **wl.TEST_GRID)
    pv = w["pv"].copy()
    pv[0, 6] = k
    f = orr.evaluate_small_planet(t, w["times"], pv, 0.01)[0]
    row = pv[0]
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    ref = np.where(front, an.quadratic_flux(z, k, 0.0, 0.0), 1.0)
    assert np.count_nonzero(ref < 1.0) > 0
    assert np.abs(f - ref).max() <= 1e-13


def test_linear_ld_on_nodes_closed_form():
    u, k = 0.6, 0.005
    mu = np.linspace(0.0, 1.0, 11)           # linear profile: the interpolant is exact
    t = orr.Tables(mu, 1.0 - u * (1.0 - mu), **SP_GRID)
    ldw = orr.small_planet_ldw(t, 0, k)
    m = np.arange(0, 1500, 37)
    z = m / (t.ng - 1.0) * (1.0 + k)
    assert z.max() < 1.0 - k
    delta = orr.occulted_with(t, ldw, 0, k, z, np.ones(z.size, bool))
    ref = (1.0 - u * (1.0 - np.sqrt(1.0 - z * z))) * k * k / (1.0 - u / 3.0)
    assert np.abs(delta - ref).max() <= 1e-17


def _max_err_vs_analytic(t, k, z):
    ldw = orr.small_planet_ldw(t, 0, k)
    f = 1.0 - orr.occulted_with(t, ldw, 0, k, z, np.ones(z.size, bool))
    return np.abs(f - an.quadratic_flux(z, k, 0.4, 0.25)).max()


def test_quadratic_ld_against_analytic_and_fourth_order():
    mu = np.linspace(0.0, 1.0, 2001)
    t = orr.Tables(mu, wl.profile_quadratic(mu, 0.4, 0.25), **SP_GRID)
    z = np.linspace(0.0, 0.9, 500)
    e4 = _max_err_vs_analytic(t, 0.004, z)
    e8 = _max_err_vs_analytic(t, 0.008, z)
    assert e4 <= 1e-9, e4
    assert 12.0 <= e8 / e4 <= 20.0, e8 / e4


def test_threshold_split_and_invalid_rows():
    w = wl.single_light_curve()
    t = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    pv = np.repeat(w["pv"], 5, axis=0)
    pv[:, 6] = [0.05, 0.02, 0.004, 0.008, 0.0]   # threshold 0.009, k0 0.01
    pv[1, 6] = 0.02
    f = orr.evaluate_small_planet(t, w["times"], pv, 0.009)
    ref = orr.evaluate(t, w["times"], pv[:2])
    assert np.array_equal(f[:2], ref)
    assert np.isfinite(f[2]).all() and np.isfinite(f[3]).all()
    assert (f[2] < 1.0).any()
    assert np.isnan(f[4]).all()
    # at or above the threshold the table range applies
    pv2 = pv[3:4].copy()
    f2 = orr.evaluate_small_planet(t, w["times"], pv2, 0.008)
    assert np.isnan(f2).all()
