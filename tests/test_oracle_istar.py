"""Pins of the oracle's fixed normaliser (Tables(..., istar=...)), the
mirror of rr_set_istar: a law normalised by its own disk integral instead
of the profile interpolant's (Sect. 3.2.1, Sect. 3.2.2).

* I_star enters Eq. 5 as one factor: every flux deficit scales by
  I_star / I_star' (to rounding) and nothing else changes;
* for the linear law the interpolant is the law itself, so its integral is
  the closed form pi (1 - u/3) and setting that changes nothing;
* with the quadratic law's exact integral (adaptive quadrature of Eq. 2,
  Oracle-B) the single-light-curve configuration stays within 1 ppm of the
  analytic model (Mandel & Agol 2002);
* d logL / d I_star (what rr_loglik_grad_istar returns) against central
  differences of logL in I_star, and the profile gradient with I_star held
  fixed against differences in the samples (exactly linear then)."""

import numpy as np

import workloads as wl
from oracle import analytic as an
from oracle import exact as ex
from oracle import gradient as ogr
from oracle import orbit
from oracle import roadrunner as orr


def small_case():
    w = wl.population(npv=6, npt=600, seed_extra=40)
    w["pv"][:, 0] = np.linspace(0.05, 1.1, 6)          # transits inside the 0.83-d span
    w["pv"][:, 1] = np.linspace(1.0, 1.6, 6)
    return w


def test_fixed_istar_scales_every_deficit():
    w = small_case()
    t0 = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    new = t0.istar * 1.0137
    t1 = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID, istar=new)
    d0 = 1.0 - orr.evaluate(t0, w["times"], w["pv"])
    d1 = 1.0 - orr.evaluate(t1, w["times"], w["pv"])
    assert (d0 > 0).sum() > 100
    # the deficits come back as 1 - F, so each carries ~1e-16 of absolute rounding
    assert np.abs(d1 * new[0] - d0 * t0.istar[0]).max() <= 1e-15 * new[0]
    # the samples can change under a fixed normaliser; it stays
    t2 = orr.with_profile(t1, w["I_s"] * 0.9)
    assert t2.istar_fixed and np.array_equal(t2.istar, new)


def test_linear_law_closed_form_changes_nothing():
    mu = np.linspace(0.0, 1.0, 37)
    u = 0.55
    prof = 1.0 - u * (1.0 - mu)
    closed = np.pi * (1.0 - u / 3.0)
    t0 = orr.Tables(mu, prof, **wl.TEST_GRID)
    assert abs(t0.istar[0] - closed) <= 1e-15 * closed
    t1 = orr.Tables(mu, prof, **wl.TEST_GRID, istar=[closed])
    w = small_case()
    f0 = orr.evaluate(t0, w["times"], w["pv"])
    f1 = orr.evaluate(t1, w["times"], w["pv"])
    assert np.abs(f0 - f1).max() <= 1e-15


def test_quadratic_law_exact_istar_against_analytic():
    w = wl.single_light_curve()
    row = w["pv"][0]
    u1, u2 = 0.4, 0.25
    law = lambda mu: 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2   # noqa: E731
    ist = ex.istar_exact(law)
    assert abs(ist - np.pi * (1 - u1 / 3 - u2 / 6)) <= 1e-13
    tab = orr.Tables(w["mu_s"], w["I_s"], **wl.DEFAULT_GRID, istar=[ist])
    fa = orr.evaluate(tab, w["times"], w["pv"])[0]
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    fm = np.where(front, an.quadratic_flux(z, row[6], u1, u2), 1.0)
    assert np.abs(fa - fm).max() <= 1e-6


def test_istar_gradient_and_fixed_profile_gradient():
    w = small_case()
    base = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ist = base.istar * 1.002
    tab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID, istar=ist)
    truth = orr.evaluate(tab, w["times"], w["pv"][:1])[0]
    obs = truth + 2e-4 * np.random.default_rng(41).standard_normal(truth.size)
    sigma = 2e-4
    pv = w["pv"]
    logl, grad, gprof, gist = ogr.loglik_grad(tab, w["times"], pv, obs, sigma,
                                             want_profile=True, want_istar=True)

    def total(t):
        return ogr.loglik_grad(t, w["times"], pv, obs, sigma, want_profile=False)[0].sum()

    h = 1e-6 * ist[0]
    tp, tm = orr.with_profile(tab, w["I_s"]), orr.with_profile(tab, w["I_s"])
    tp.istar = ist + h
    tm.istar = ist - h
    fd = (total(tp) - total(tm)) / (2 * h)
    assert abs(gist[0] - fd) <= 1e-6 * abs(fd), (gist[0], fd)
    # samples with I_star fixed: logL depends on them only through T (linear)
    for s in (0, 57, 150, 199):
        hs = 1e-4
        ip, im = w["I_s"].copy(), w["I_s"].copy()
        ip[0, s] += hs
        im[0, s] -= hs
        fds = (total(orr.with_profile(tab, ip)) - total(orr.with_profile(tab, im))) / (2 * hs)
        scale = np.abs(gprof).max()
        assert abs(gprof[0, s] - fds) <= 1e-6 * scale, (s, gprof[0, s], fds)
