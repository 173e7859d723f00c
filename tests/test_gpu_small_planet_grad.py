"""GPU log-likelihood and parameter gradient of the small-planet
approximation (rr_loglik_grad_small_planet, Sect. 3.4.2) through the C ABI:
logL against the oracle's small-planet light curves, the gradient against
central differences of that oracle log-likelihood, and rows at or above the
threshold against rr_loglik_grad."""

import numpy as np
import pytest

import workloads as wl
from oracle import gradient as ogr
from oracle import roadrunner as orr

pytestmark = pytest.mark.gpu

K_SMALL = 0.01


@pytest.fixture(scope="module")
def rr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_08500_amd as rr
    return rr


@pytest.fixture(scope="module")
def setup():
    w = wl.loglik_walkers(npv=8, npt=6000, nss=3)
    w["times"] = np.linspace(0.0, 25.0, 6000)
    pv = w["pv"].copy()
    pv[:, 6] = [0.004, 0.005, 0.006, 0.008, 0.02, 0.05, 0.0045, 0.03]
    truth = w["truth"].copy()
    truth[6] = 0.005
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    kw = dict(nss=w["nss"], exptimes=w["exptimes"])
    f = orr.evaluate_small_planet(otab, w["times"], truth[None, :], K_SMALL, **kw)[0]
    assert (f < 1.0).sum() > 50
    obs = f + w["noise"]
    return w, pv, otab, obs, kw


def oracle_loglik(otab, w, pv, obs, kw):
    f = orr.evaluate_small_planet(otab, w["times"], pv, K_SMALL, **kw)
    return -0.5 * (((obs[None, :] - f) / w["sigma"]) ** 2).sum(axis=1)


def test_loglik_matches_oracle(rr, setup):
    w, pv, otab, obs, kw = setup
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    oll = oracle_loglik(otab, w, pv, obs, kw)
    ll, g = rr.loglik_grad_small_planet(tab, ser, pv, obs, w["sigma"], K_SMALL, "fp64")
    np.testing.assert_allclose(ll.cpu().numpy(), oll, rtol=1e-11)
    assert np.isfinite(g.cpu().numpy()).all()
    o32 = obs.astype(np.float32).astype(np.float64)
    ll32, _ = rr.loglik_grad_small_planet(tab, ser, pv, o32, w["sigma"], K_SMALL, "mixed")
    np.testing.assert_allclose(ll32.cpu().numpy(), oracle_loglik(otab, w, pv, o32, kw),
                               rtol=1e-6)


def test_gradient_matches_central_differences(rr, setup):
    w, pv, otab, obs, kw = setup
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    _, g64 = rr.loglik_grad_small_planet(tab, ser, pv, obs, w["sigma"], K_SMALL, "fp64")
    o32 = obs.astype(np.float32).astype(np.float64)
    _, g32 = rr.loglik_grad_small_planet(tab, ser, pv, o32, w["sigma"], K_SMALL, "mixed")
    g64, g32 = g64.cpu().numpy(), g32.cpu().numpy()
    h = np.array([1e-6, 1e-7, 1e-6, 1e-6, 1e-6, 1e-6, 1e-7])
    for i in (0, 3, 6):                                  # below the threshold
        fd = ogr.finite_difference(
            lambda r: oracle_loglik(otab, w, r[None, :], obs, kw)[0], pv[i], h)
        scale = np.abs(fd).max()
        np.testing.assert_allclose(g64[i], fd, rtol=2e-4, atol=1e-5 * scale)
        np.testing.assert_allclose(g32[i], g64[i], rtol=0, atol=3e-3 * scale)


def test_rows_above_threshold_equal_loglik_grad(rr, setup):
    w, pv, otab, obs, kw = setup
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    big = pv[[4, 5, 7]]
    for prec in ("fp64", "mixed"):
        a_ll, a_g = rr.loglik_grad_small_planet(tab, ser, big, obs, w["sigma"], K_SMALL, prec)
        b_ll, b_g, _ = rr.loglik_grad(tab, ser, big, obs, w["sigma"], prec)
        np.testing.assert_allclose(a_ll.cpu().numpy(), b_ll.cpu().numpy(), rtol=1e-12)
        np.testing.assert_allclose(a_g.cpu().numpy(), b_g.cpu().numpy(), rtol=1e-10,
                                   atol=1e-12 * np.abs(b_g.cpu().numpy()).max())


def test_invalid_rows_and_threshold(rr, setup):
    w, pv, otab, obs, kw = setup
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    bad = pv[:3].copy()
    bad[0, 6] = 0.0                     # k = 0
    bad[1, 6] = 0.009                   # above a threshold of 0.008, below k0
    ll, g = rr.loglik_grad_small_planet(tab, ser, bad, obs, w["sigma"], 0.008, "fp64")
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    assert np.isnan(ll[0]) and np.isnan(ll[1]) and np.isfinite(ll[2])
    assert np.isnan(g[0]).all() and np.isfinite(g[2]).all()
    with pytest.raises(rr.RRError):
        rr.loglik_grad_small_planet(tab, ser, pv, obs, w["sigma"], -1.0, "fp64")
