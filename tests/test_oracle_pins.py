"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against mathematics or the paper: closed forms,
textbook special cases, an independent 2-D brute-force integral, an
independent bisection Kepler solver, invariants, and the worked example of
Sect. 4.2.  A plausible slip in the oracle (a dropped term, a wrong sign or
index, a transposed operand) fails at least one of them.
"""

import json
import os
import warnings

import numpy as np
import pytest

from oracle import exact as ex
from oracle import orbit as orb
from oracle import roadrunner as rr
import workloads as wl

warnings.filterwarnings("ignore", category=UserWarning)
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def quad_prof(u1, u2):
    return lambda mu: wl.profile_quadratic(np.asarray(mu), u1, u2)


def p2_prof(c, al):
    return lambda mu: wl.profile_power2(np.asarray(mu), c, al)


def p2_concentric(k, c, al):
    """Closed form of 2 pi int_{mu_k}^1 mu I(mu) dmu for the power-2 law,
    mu_k = sqrt(1 - k^2): the light blocked by a planet centred on the star."""
    mk = np.sqrt(1.0 - k * k)
    return 2 * np.pi * ((1 - c) * (1 - mk ** 2) / 2 + c * (1 - mk ** (al + 2)) / (al + 2))


def quad_concentric(k, u1, u2):
    """Same for I = (1-u1-u2) + (u1+2u2) mu - u2 mu^2."""
    mk = np.sqrt(1.0 - k * k)
    c = [1 - u1 - u2, u1 + 2 * u2, -u2]
    return 2 * np.pi * sum(cn * (1 - mk ** (n + 2)) / (n + 2) for n, cn in enumerate(c))


# ------------------------------------------------------------------ z-grid
@pytest.mark.parametrize("zcut,nzin,nzlimb", [(0.7, 20, 30), (0.8, 60, 120), (0.5, 3, 7)])
def test_z_grid_structure(zcut, nzin, nzlimb):
    """Sect. 3.1.1: constant dz inside z_cut, constant dmu outside."""
    ze, zm, mu = rr.z_grid(zcut, nzin, nzlimb)
    assert ze.size == nzin + nzlimb + 1
    assert ze[0] == 0.0 and ze[-1] == 1.0
    assert ze[nzin] == pytest.approx(zcut, abs=1e-15)
    assert np.all(np.diff(ze) > 0)
    np.testing.assert_allclose(np.diff(ze[: nzin + 1]), zcut / nzin, rtol=1e-12)
    mue = np.sqrt(1 - ze[nzin:] ** 2)
    np.testing.assert_allclose(np.diff(mue), -np.sqrt(1 - zcut ** 2) / nzlimb,
                               rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(zm, 0.5 * (ze[1:] + ze[:-1]), rtol=0, atol=0)
    np.testing.assert_allclose(mu ** 2 + zm ** 2, 1.0, atol=1e-15)


# ------------------------------------------------------------------ lens area
def test_lens_area_textbook_values():
    """Closed-form lens areas: two unit circles at distance 1 overlap in
    2 pi/3 - sqrt(3)/2; at distance sqrt(2) in pi/2 - 1."""
    assert rr.lens_area(1.0, 1.0, 1.0) == pytest.approx(2 * np.pi / 3 - np.sqrt(3) / 2, abs=1e-14)
    assert rr.lens_area(1.0, 1.0, np.sqrt(2.0)) == pytest.approx(np.pi / 2 - 1, abs=1e-14)
    # R=2, k=1, centres 2 apart: segments of angles 2 acos(1/4)... known form
    R, k, c = 2.0, 1.0, 2.0
    a1 = np.arccos((c * c + R * R - k * k) / (2 * c * R))
    a2 = np.arccos((c * c + k * k - R * R) / (2 * c * k))
    seg = R * R * (a1 - np.sin(2 * a1) / 2) + k * k * (a2 - np.sin(2 * a2) / 2)
    assert rr.lens_area(R, k, c) == pytest.approx(seg, abs=1e-14)


def test_lens_area_special_cases_and_symmetry():
    assert rr.lens_area(1.0, 0.1, 0.0) == pytest.approx(np.pi * 0.01)
    assert rr.lens_area(1.0, 0.1, 0.5) == pytest.approx(np.pi * 0.01)     # inside
    assert rr.lens_area(0.3, 0.1, 0.0) == pytest.approx(np.pi * 0.01)
    assert rr.lens_area(0.05, 0.1, 0.02) == pytest.approx(np.pi * 0.0025)  # R inside k
    assert rr.lens_area(1.0, 0.1, 1.1) == 0.0
    assert rr.lens_area(1.0, 0.1, 5.0) == 0.0
    assert rr.lens_area(0.0, 0.1, 0.05) == 0.0
    rng = np.random.default_rng(1)
    R, k, c = rng.uniform(0.1, 1, 50), rng.uniform(0.01, 0.5, 50), rng.uniform(0, 1.5, 50)
    np.testing.assert_allclose(rr.lens_area(R, k, c), rr.lens_area(k, R, c), atol=1e-14)


def test_lens_area_brute_force_grid():
    """Cartesian cell counting (midpoint, 4000^2 cells) on two cases."""
    n = 4000
    for R, k, c in [(1.0, 0.3, 0.9), (0.6, 0.25, 0.5)]:
        x = np.linspace(c - k, c + k, n + 1)
        xm = 0.5 * (x[1:] + x[:-1])
        h = x[1] - x[0]
        X, Y = np.meshgrid(xm, xm - c)
        inside = ((X - c) ** 2 + Y ** 2 < k * k) & (X ** 2 + Y ** 2 < R * R)
        assert rr.lens_area(R, k, c) == pytest.approx(inside.sum() * h * h, rel=2e-4)


# ------------------------------------------------------------------ weights
def test_weights_rows_sum_to_one_and_limits():
    """Sect. 2: weights are annulus areas over the total occluded area, so
    each vector sums to one; at g = 1 the limit puts all weight in the limb
    annulus; weights are non-negative."""
    ze, _, _ = rr.z_grid(0.7, 10, 14)
    dk, dg, W = rr.weights_3d(ze, 9, 0.01, 0.3, 33)
    np.testing.assert_allclose(W.sum(-1), 1.0, atol=1e-12)
    assert W.min() >= -1e-13
    np.testing.assert_array_equal(W[:, -1, :-1], 0.0)
    np.testing.assert_array_equal(W[:, -1, -1], 1.0)
    assert dk == pytest.approx(0.29 / 8) and dg == pytest.approx(1 / 32)


def test_weights_concentric_closed_form():
    """At g = 0 the planet is centred: annulus j holds
    (min(ze_{j+1}, k)^2 - min(ze_j, k)^2) / k^2 of the occluded area."""
    ze, _, _ = rr.z_grid(0.7, 10, 14)
    k0, k1, nk = 0.01, 0.3, 9
    _, _, W = rr.weights_3d(ze, nk, k0, k1, 17)
    for i in range(nk):
        k = k0 + i * (k1 - k0) / (nk - 1)
        want = np.diff(np.minimum(ze, k) ** 2) / k ** 2
        np.testing.assert_allclose(W[i, 0], want, atol=1e-13)


def test_weights_match_direct_area_ratio():
    """The k index is the first axis and g the second (a transposed table
    fails): compare one entry against the area ratio computed by hand."""
    ze, _, _ = rr.z_grid(0.7, 10, 14)
    nk, ng, k0, k1 = 7, 11, 0.05, 0.25
    _, _, W = rr.weights_3d(ze, nk, k0, k1, ng)
    i, m, j = 5, 7, 18
    k = k0 + i * (k1 - k0) / (nk - 1)
    c = m / (ng - 1) * (1 + k)
    a_hi = rr.lens_area(ze[j + 1], k, c)
    a_lo = rr.lens_area(ze[j], k, c)
    assert W[i, m, j] == pytest.approx((a_hi - a_lo) / rr.lens_area(1.0, k, c), abs=1e-14)


# ------------------------------------------------------------------ I_star
def test_istar_exact_for_polynomials_of_degree_one():
    """The interpolant of a linear profile is the profile itself, so
    I_star is exact: I = 1 -> pi, I = mu -> 2 pi/3, I = 1 - 0.6(1 - mu) ->
    pi (1 - 0.6/3)."""
    mu = np.sort(np.concatenate([[0.0, 1.0], np.random.default_rng(3).uniform(0, 1, 37)]))
    assert rr.istar_of_profile(mu, np.ones_like(mu))[0] == pytest.approx(np.pi, abs=1e-14)
    assert rr.istar_of_profile(mu, mu)[0] == pytest.approx(2 * np.pi / 3, abs=1e-14)
    assert rr.istar_of_profile(mu, 1 - 0.6 * (1 - mu))[0] == pytest.approx(np.pi * 0.8, abs=1e-14)


def test_istar_matches_adaptive_quadrature_and_analytic():
    mu = np.linspace(0, 1, 200)
    I = wl.profile_power2(mu, 0.65, 0.6)
    a = rr.istar_of_profile(mu, I)[0]
    b = ex.istar_exact(ex.tabulated_profile(mu, I))
    assert a == pytest.approx(b, abs=1e-12)
    # the analytic power-2 normaliser differs only by the sampling error
    assert a == pytest.approx(p2_concentric(1.0, 0.65, 0.6), rel=2e-4)
    # samples not reaching mu = 0 or 1: constant extension
    mu2 = np.linspace(0.1, 0.9, 50)
    I2 = 0.3 + mu2
    want = 2 * np.pi * (0.4 * 0.1 ** 2 / 2 + ((0.9 ** 3 - 0.1 ** 3) / 3 + 0.3 * (0.9 ** 2 - 0.1 ** 2) / 2)
                        + 1.2 * (1 - 0.81) / 2)
    assert rr.istar_of_profile(mu2, I2)[0] == pytest.approx(want, abs=1e-14)


# ------------------------------------------------------------------ Eq. 5
@pytest.mark.parametrize("grid", [wl.TEST_GRID, dict(zcut=0.5, nzin=4, nzlimb=5, ng=7, nk=3, k0=0.02, k1=0.25)])
def test_uniform_disk_is_exact_at_any_resolution(grid):
    """With I = 1 every LD-weighted table entry is 1, so Eq. 5 reduces to the
    uniform-disk model 1 - a(z, k)/pi, whatever the resolution."""
    mu = np.linspace(0, 1, 11)
    tab = rr.Tables(mu, np.ones_like(mu), **grid)
    np.testing.assert_allclose(tab.T, 1.0, atol=1e-13)
    assert tab.istar[0] == pytest.approx(np.pi, abs=1e-14)
    for k in [0.03, 0.1, 0.17, 0.25]:
        z = np.linspace(0, 1.3, 301)
        want = 1 - rr.lens_area(1.0, k, z) / np.pi
        np.testing.assert_allclose(rr.flux_at_z(tab, 0, k, z), want, atol=1e-14)


def test_uniform_disk_independent_geometry():
    """The uniform-disk depth at full overlap is k^2 and at z = 1 (planet
    centre on the limb) is the lens of Eq. 5 -- cross-check with the 2-D
    brute force rather than the lens formula."""
    k = 0.1
    one = lambda mu: np.ones_like(np.asarray(mu, float))
    assert 1 - ex.occulted_bruteforce(0.0, k, one) / np.pi == pytest.approx(1 - k * k, abs=1e-14)
    bf = ex.occulted_bruteforce(1.0, k, one)
    assert bf == pytest.approx(rr.lens_area(1.0, k, 1.0), abs=1e-12)


ZK_CASES = [(0.0, 0.1), (0.3, 0.1), (0.75, 0.2), (0.89, 0.1), (0.95, 0.1), (1.0, 0.1),
            (1.05, 0.1), (1.09, 0.1), (0.5, 0.05), (0.97, 0.05), (1.2, 0.25), (0.8, 0.3),
            (0.05, 0.2), (0.15, 0.2), (0.65, 0.4), (1.3, 0.5), (0.6, 0.5), (0.999, 0.01),
            (0.2, 0.01), (1.005, 0.01)]


@pytest.mark.parametrize("z,k", ZK_CASES)
def test_exact_1d_reduction_matches_2d_brute_force(z, k):
    """Oracle-B's 1-D radial reduction (Eq. 1-2) against a 2-D integral over
    the planet disk, for quadratic and power-2 profiles."""
    for prof in (quad_prof(0.4, 0.25), p2_prof(0.7, 0.5)):
        a = ex.occulted_exact(z, k, prof)
        b = ex.occulted_bruteforce(z, k, prof, n_theta=256, n_rho=256)
        assert a == pytest.approx(b, abs=1e-12)


@pytest.mark.parametrize("k", [0.01, 0.1, 0.3, 0.6])
def test_exact_concentric_closed_forms(k):
    """Planet centred on the star: closed forms for quadratic and power-2."""
    assert ex.occulted_exact(0.0, k, quad_prof(0.4, 0.25)) == pytest.approx(
        quad_concentric(k, 0.4, 0.25), abs=1e-13)
    assert ex.occulted_exact(0.0, k, p2_prof(0.6, 0.45)) == pytest.approx(
        p2_concentric(k, 0.6, 0.45), abs=1e-13)


def test_oracle_a_close_to_exact_and_converges():
    """Sect. 3.3: the discretised model has no bias and its error shrinks
    with resolution; at modest resolution the error is a few ppm (the paper
    quotes ~5 ppm at its lowest setting)."""
    mu = np.linspace(0, 1, 200)
    I = wl.profile_quadratic(mu, 0.4, 0.25)
    prof = ex.tabulated_profile(mu, I)
    ist = ex.istar_exact(prof)
    k = 0.1
    z = np.concatenate([np.linspace(0, 1.1, 45, endpoint=False), [0.895, 0.9, 0.905]])
    ref = np.array([1 - ex.occulted_exact(zz, k, prof) / ist for zz in z])
    errs = []
    for g in [dict(zcut=0.7, nzin=10, nzlimb=15, ng=50, nk=16),
              dict(zcut=0.7, nzin=20, nzlimb=30, ng=100, nk=32),
              dict(zcut=0.8, nzin=60, nzlimb=120, ng=512, nk=128)]:
        tab = rr.Tables(mu, I, k0=0.01, k1=0.3, **g)
        errs.append(np.abs(rr.flux_at_z(tab, 0, k, z) - ref).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 30e-6 and errs[2] < 5e-6


# ------------------------------------------------------------------ orbit
def test_kepler_newton_matches_bisection():
    rng = np.random.default_rng(7)
    M = rng.uniform(-np.pi, np.pi, 2000)
    for e in [0.0, 0.1, 0.3, 0.7, 0.95]:
        E1 = orb.solve_kepler(M, e)
        E2 = orb.solve_kepler_bisection(M, e)
        np.testing.assert_allclose(E1, E2, atol=2e-14)
        np.testing.assert_allclose(E1 - e * np.sin(E1), M, atol=2e-15)


def test_circular_orbit_closed_form():
    """e = 0: z = a sqrt(sin^2 phi + cos^2 i cos^2 phi), phi = 2 pi dt / P,
    and cos i = b / a."""
    a, b, P = 8.0, 0.3, 3.0
    dt = np.linspace(-0.6, 0.6, 301)
    z, front, cosi = orb.projected_separation(dt, P, a, b, 0.0, 0.7)
    assert cosi == pytest.approx(b / a)
    ph = 2 * np.pi * dt / P
    np.testing.assert_allclose(z, a * np.sqrt(np.sin(ph) ** 2 + (b / a) ** 2 * np.cos(ph) ** 2), rtol=1e-13)
    assert front.all()
    z2, front2, _ = orb.projected_separation(np.array([P / 2]), P, a, b, 0.0, 0.0)
    assert not front2[0]


@pytest.mark.parametrize("e,w", [(0.1, 0.3), (0.3, 2.0), (0.6, 4.5), (0.25, 0.0)])
def test_eccentric_orbit_geometry(e, w):
    """z(t0) = b (t0 is the conjunction); and for a chosen true anomaly f the
    time from conjunction follows in closed form from E(f), M(f) without any
    Kepler solve, while the separation follows from r(f) = a(1-e^2)/(1+e cos f)."""
    a, b, P = 9.0, 0.4, 4.0
    z0, fr0, cosi = orb.projected_separation(np.array([0.0]), P, a, b, e, w)
    assert z0[0] == pytest.approx(b, abs=1e-13) and fr0[0]
    f = (0.5 * np.pi - w) + np.linspace(-0.5, 0.5, 41)
    E = orb.eccentric_from_true(f, e)
    M = E - e * np.sin(E)
    dM = np.mod(M - orb.conjunction_mean_anomaly(e, w) + np.pi, 2 * np.pi) - np.pi
    z, front, _ = orb.projected_separation(dM * P / (2 * np.pi), P, a, b, e, w)
    r = a * (1 - e * e) / (1 + e * np.cos(f))
    zgeo = r * np.sqrt(1 - np.sin(w + f) ** 2 * (1 - cosi ** 2))
    np.testing.assert_allclose(z, zgeo, rtol=1e-11)
    assert front.all()


def test_phase_offset_periodicity():
    """The offset is in [-P/2, P/2] and differs from t - t0 by whole periods."""
    t = np.linspace(-50, 50, 1001)
    dt = orb.phase_offset(t, 1.3, 2.7)
    assert np.all(np.abs(dt) <= 1.35 + 1e-12)
    n = (t - 1.3 - dt) / 2.7
    np.testing.assert_allclose(n, np.round(n), atol=1e-12)


# ------------------------------------------------------------------ light curves
def test_single_light_curve_contacts():
    """Circular orbit: the planet overlaps the star for |t - t0| < T14/2,
    T14 = P/pi asin(sqrt((1+k)^2 - b^2) / (a sin i)), and is fully inside
    for |t - t0| < T23/2 with (1-k) in place of (1+k)."""
    w = wl.single_light_curve()
    mu, I = w["mu_s"], w["I_s"]
    tab = rr.Tables(mu, I, **wl.TEST_GRID)
    f = rr.evaluate(tab, w["times"], w["pv"])[0]
    P, a, b, k = 3.0, 8.0, 0.3, 0.1
    sini = np.sqrt(1 - (b / a) ** 2)
    t14 = P / np.pi * np.arcsin(np.sqrt((1 + k) ** 2 - b ** 2) / (a * sini))
    t23 = P / np.pi * np.arcsin(np.sqrt((1 - k) ** 2 - b ** 2) / (a * sini))
    t = w["times"]
    assert t14 == pytest.approx(0.126786, abs=2e-6) and t23 == pytest.approx(0.101548, abs=2e-6)
    inside = np.abs(t) < t14 / 2
    assert np.all(f[~inside] == 1.0)
    assert np.all(f[inside] < 1.0)
    assert inside.sum() == 316 and (np.abs(t) < t23 / 2).sum() == 254
    # symmetry about mid-transit for a circular orbit
    np.testing.assert_allclose(f, f[::-1], atol=1e-13)


def test_mid_transit_against_exact_and_small_planet():
    """Single light curve at mid-transit (z = b = 0.3): exact flux from the
    quadratic law and the small-planet limit 1 - pi k^2 I(mu_c)/I_star."""
    mu = np.linspace(0, 1, 100)
    I = wl.profile_quadratic(mu, 0.4, 0.25)
    prof = quad_prof(0.4, 0.25)
    ist = np.pi * (1 - 0.4 / 3 - 0.25 / 6)
    exact = 1 - ex.occulted_exact(0.3, 0.1, prof) / ist
    assert exact == pytest.approx(0.988123463154, abs=1e-11)
    small = 1 - np.pi * 0.01 * prof(np.sqrt(1 - 0.09)) / ist
    assert exact - small == pytest.approx(0.0, abs=2 * 0.1 ** 4)
    tab = rr.Tables(mu, I, **wl.DEFAULT_GRID)
    fa = rr.flux_at_z(tab, 0, 0.1, np.array([0.3]))[0]
    assert fa == pytest.approx(exact, abs=2e-6)


def test_depth_monotone_in_k():
    mu = np.linspace(0, 1, 200)
    tab = rr.Tables(mu, wl.profile_power2(mu, 0.7, 0.5), **wl.TEST_GRID)
    ks = np.linspace(0.02, 0.29, 40)
    for z in [0.0, 0.4, 0.8]:
        f = np.array([rr.flux_at_z(tab, 0, k, np.array([z]))[0] for k in ks])
        assert np.all(np.diff(f) < 0)


def test_supersampling_is_mean_of_subsample_evaluations():
    """Sect. 4.1: an exposure is the mean over nss subsamples spread over the
    exposure (midpoint rule); nss = 1 with any exposure time is the plain
    evaluation at the mid-exposure time."""
    w = wl.population(npv=3, npt=400)
    tab = rr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    pv = w["pv"].copy()
    pv[:, 0] = 0.1
    t = np.linspace(-0.3, 0.3, 37)
    exp = 0.05
    base = rr.evaluate(tab, t, pv)
    one = rr.evaluate(tab, t, pv, nss=1, exptimes=exp)
    np.testing.assert_array_equal(base, one)
    ss = rr.evaluate(tab, t, pv, nss=7, exptimes=exp)
    offs = exp * ((np.arange(7) + 0.5) / 7 - 0.5)
    manual = np.mean([rr.evaluate(tab, t + o, pv) for o in offs], axis=0)
    np.testing.assert_allclose(ss, manual, atol=1e-15)


def test_supersampling_converges_to_exposure_average():
    from scipy import integrate
    w = wl.single_light_curve()
    tab = rr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    pv = w["pv"]
    t, exp = 0.055, 0.02
    f = lambda tt: rr.evaluate(tab, np.array([tt]), pv)[0, 0]
    avg = integrate.quad(f, t - exp / 2, t + exp / 2, epsabs=1e-13, limit=200, points=[0.0634])[0] / exp
    errs = [abs(rr.evaluate(tab, np.array([t]), pv, nss=n, exptimes=exp)[0, 0] - avg) for n in (2, 8, 32)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-7


def test_invalid_rows_are_nan():
    w = wl.population(npv=6, npt=50)
    tab = rr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    pv = w["pv"].copy()
    pv[1, 6] = 0.5       # k above k1
    pv[2, 4] = 1.0       # e = 1
    pv[3, 3] = -0.1      # b < 0
    pv[4, 2] = 0.1       # a so small that |cos i| > 1
    out = rr.evaluate(tab, w["times"], pv)
    assert np.isnan(out[1:5]).all()
    assert np.isfinite(out[[0, 5]]).all()


def test_worked_example_mid_transit():
    """Sect. 4.2 example: t0 = 0, P = 1, i = pi/2, so every integer time is a
    mid-transit with z = 0 and the flux is 1 - (closed-form concentric
    occultation)/I_star of each passband's power-2 profile; light curves map
    to passbands through pbids, and chromatic radius ratios follow."""
    ex_ = json.load(open(os.path.join(GOLD, "worked_example.json")))
    times = np.array(ex_["times"], float)
    lcids, pbids = np.array(ex_["lcids"]), np.array(ex_["pbids"])
    ldc = np.array(ex_["ldc"] if "ldc" in ex_ else ex_["achromatic"]["ldc"])[0]
    mu = np.linspace(0, 1, 400)
    coeffs = [(ldc[0], ldc[1]), (ldc[2], ldc[3])]
    I_s = np.stack([wl.profile_power2(mu, c, al) for c, al in coeffs])
    tab = rr.Tables(mu, I_s, **wl.DEFAULT_GRID)
    for case in ("achromatic", "chromatic"):
        c_ = ex_[case]
        kk = np.broadcast_to(np.asarray(c_["k"], float), (2,))
        a, P, t0, inc = c_["a"], c_["p"], c_["t0"], np.pi * c_["i_over_pi"]
        b = a * np.cos(inc)
        pv = np.array([[t0, P, a, b, 0.0, 0.0, kk[0], kk[1]]])
        f = rr.evaluate(tab, times, pv, lcids=lcids, pbids=pbids)[0]
        for it in range(times.size):
            pb = pbids[lcids[it]]
            c, al = coeffs[pb]
            want = 1 - p2_concentric(kk[pb], c, al) / p2_concentric(1.0, c, al)
            assert f[it] == pytest.approx(want, abs=3e-6)
    # the population call: shapes (npv, npt) and per-row parameters
    c_ = ex_["population"]
    k2 = np.array(c_["k"])
    rows = []
    for i in range(2):
        inc = np.pi * c_["i_over_pi"][i]
        rows.append([c_["t0"][i], c_["p"][i], c_["a"][i], c_["a"][i] * np.cos(inc), 0, 0, *k2[i]])
    f = rr.evaluate(tab, times, np.array(rows), lcids=lcids, pbids=pbids)
    assert f.shape == (2, 6) and np.all(f <= 1.0)
