"""Pins of the oracle's analytic log-likelihood gradient: central finite
differences of the oracle's own forward model (parameters and LD profile
samples), consistency of its likelihood with Oracle-A's light curve, and the
treatment of invalid rows."""

import numpy as np
import pytest

import workloads as wl
from oracle import gradient as gr
from oracle import roadrunner as rr


@pytest.fixture(scope="module")
def setup():
    w = wl.loglik_walkers(npv=3, npt=3000, nss=3)
    w["times"] = np.linspace(0.0, 20.0, 3000)        # several transit epochs
    tab = rr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    obs = rr.evaluate(tab, w["times"], w["truth"][None, :], nss=w["nss"],
                      exptimes=w["exptimes"])[0] + w["noise"]
    return w, tab, obs


def test_loglik_matches_forward_model(setup):
    w, tab, obs = setup
    ll, _, _ = gr.loglik_grad(tab, w["times"], w["pv"], obs, w["sigma"], nss=w["nss"],
                              exptimes=w["exptimes"], want_profile=False)
    F = rr.evaluate(tab, w["times"], w["pv"], nss=w["nss"], exptimes=w["exptimes"])
    want = -0.5 * np.sum(((obs[None, :] - F) / w["sigma"]) ** 2, axis=1)
    np.testing.assert_allclose(ll, want, rtol=1e-12)


def test_parameter_gradient_matches_central_differences(setup):
    w, tab, obs = setup
    ll, g, _ = gr.loglik_grad(tab, w["times"], w["pv"], obs, w["sigma"], nss=w["nss"],
                              exptimes=w["exptimes"], want_profile=False)
    h = np.array([1e-6, 1e-7, 1e-6, 1e-6, 1e-6, 1e-6, 1e-7])

    for i, row in enumerate(w["pv"]):
        def L(r):
            return gr.loglik_grad(tab, w["times"], r[None, :], obs, w["sigma"], nss=w["nss"],
                                  exptimes=w["exptimes"], want_profile=False)[0][0]
        fd = gr.finite_difference(L, row, h)
        scale = np.abs(g[i]).max()
        np.testing.assert_allclose(g[i], fd, rtol=1e-4, atol=1e-6 * scale)


def test_profile_gradient_matches_central_differences(setup):
    w, tab, obs = setup
    _, _, gp = gr.loglik_grad(tab, w["times"], w["pv"], obs, w["sigma"], nss=w["nss"],
                              exptimes=w["exptimes"])
    assert gp.shape == w["I_s"].shape

    def L(I_s):
        t2 = rr.Tables(w["mu_s"], I_s, **wl.TEST_GRID)
        return gr.loglik_grad(t2, w["times"], w["pv"], obs, w["sigma"], nss=w["nss"],
                              exptimes=w["exptimes"], want_profile=False)[0].sum()

    hh = 1e-5
    for s in (10, 50, 120, 180, 199):
        Ip, Im = w["I_s"].copy(), w["I_s"].copy()
        Ip[0, s] += hh
        Im[0, s] -= hh
        fd = (L(Ip) - L(Im)) / (2 * hh)
        assert gp[0, s] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(gp).max())


def test_profile_gradient_sums_over_rows_and_passbands():
    """Two passbands, two light curves: the profile gradient of passband 1
    comes only from the light curve mapped to it; a uniform profile's
    gradient is orthogonal to the change that keeps the profile uniform."""
    w = wl.heterogeneous(npv=2, days=3.0)
    tab = rr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    obs = np.ones(w["times"].size)
    kw = dict(lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"], exptimes=w["exptimes"])
    ll, g, gp = gr.loglik_grad(tab, w["times"], w["pv"], obs, 2e-4, **kw)
    pv1 = w["pv"][:1]
    ll1, _, gp1 = gr.loglik_grad(tab, w["times"], pv1, obs, 2e-4, **kw)
    ll2, _, gp2 = gr.loglik_grad(tab, w["times"], w["pv"][1:], obs, 2e-4, **kw)
    np.testing.assert_allclose(gp, gp1 + gp2, rtol=1e-12, atol=1e-12 * np.abs(gp).max())
    # scaling every profile sample by the same factor leaves F unchanged
    # (Eq. 5 is homogeneous of degree 0 in the profile), so the gradient is
    # orthogonal to the profile itself
    for pb in range(4):
        assert abs(np.dot(gp[pb], w["I_s"][pb])) <= 1e-8 * np.abs(gp[pb]).sum() * np.abs(w["I_s"][pb]).max()


def test_invalid_rows(setup):
    w, tab, obs = setup
    pv = w["pv"].copy()
    pv[1, 4] = 1.2
    ll, g, _ = gr.loglik_grad(tab, w["times"], pv, obs, w["sigma"], nss=w["nss"],
                              exptimes=w["exptimes"])
    assert np.isnan(ll[1]) and np.isnan(g[1]).all()
    assert np.isfinite(ll[[0, 2]]).all() and np.isfinite(g[[0, 2]]).all()
