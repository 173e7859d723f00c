"""Pins of the oracle's direct model (weights built for each row's own k,
Sect. 3.1.1, with no k-grid, no k-interpolation and no k limits):

* its weights for a k on a table node equal that node's weights in the 3-D
  table, and every row of them sums to one;
* at a node k the direct model reproduces the interpolated model;
* a uniform profile gives the uniform-source closed form 1 - lambda_e at k
  inside and outside the interpolated model's range;
* with quadratic LD, at k = 0.005 and 0.5 (outside the table range) and
  0.1, it is within 5 ppm of the analytic quadratic model (the paper's
  accuracy figure covers the direct model up to k = 0.5, Sect. 3.3)."""

import numpy as np
import pytest

import workloads as wl
from oracle import analytic as an
from oracle import orbit
from oracle import roadrunner as orr


@pytest.fixture(scope="module")
def tab():
    w = wl.single_light_curve()
    return w, orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)


def test_weights_match_table_at_nodes(tab):
    w, t = tab
    for i in (0, 7, t.nk - 1):
        k = t.k0 + t.dk * i
        Wk = orr.weights_for_k(t.ze, k, t.ng)
        assert np.abs(Wk - t.W[i]).max() <= 1e-15
        assert np.allclose(Wk.sum(axis=1), 1.0, atol=1e-13)


def test_node_k_reproduces_interpolated_model(tab):
    w, t = tab
    pv = np.repeat(w["pv"], 3, axis=0)
    pv[:, 6] = [t.k0 + t.dk * 3, t.k0 + t.dk * 9, t.k0 + t.dk * 15]
    a = orr.evaluate_direct(t, w["times"], pv)
    b = orr.evaluate(t, w["times"], pv)
    assert np.abs(a - b).max() <= 1e-14


@pytest.mark.parametrize("k", [0.005, 0.1, 0.5])
def test_uniform_source_closed_form(k):
    w = wl.single_light_curve()
    mu = w["mu_s"]
    t = orr.Tables(mu, np.ones_like(mu), **wl.TEST_GRID)
    pv = w["pv"].copy()
    pv[0, 6] = k
    f = orr.evaluate_direct(t, w["times"], pv)[0]
    row = pv[0]
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    ref = np.where(front, an.quadratic_flux(z, k, 0.0, 0.0), 1.0)
    assert np.abs(f - ref).max() <= 1e-13


@pytest.mark.parametrize("k", [0.005, 0.1, 0.5])
def test_quadratic_within_five_ppm_of_analytic(k):
    w = wl.single_light_curve()
    mu = np.linspace(0.0, 1.0, 1001)
    prof = wl.profile_quadratic(mu, 0.4, 0.25)
    t = orr.Tables(mu, prof, **wl.DEFAULT_GRID)
    pv = w["pv"].copy()
    pv[0, 6] = k
    f = orr.evaluate_direct(t, w["times"], pv)[0]
    row = pv[0]
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    ref = np.where(front, an.quadratic_flux(z, k, 0.4, 0.25), 1.0)
    assert np.abs(f - ref).max() <= 5e-6, np.abs(f - ref).max()
    assert np.count_nonzero(ref < 1.0) > 0


def test_invalid_rows(tab):
    w, t = tab
    pv = np.repeat(w["pv"], 3, axis=0)
    pv[0, 6] = 0.0
    pv[1, 6] = 1.2
    f = orr.evaluate_direct(t, w["times"], pv)
    assert np.isnan(f[0]).all() and np.isnan(f[1]).all() and np.isfinite(f[2]).all()
