"""Pins of the oracle's per-vector limb darkening (every parameter vector with
its own LD profile, as when LD coefficients are sampled with the orbit), and
of the named LD laws:

* a vector given the tables' own profile reproduces ``evaluate`` exactly;
* the oracle's reuse of the weight table agrees with tables built from
  scratch for the vector's profile (catches a stale LD-dependent step);
* the flux is invariant under scaling of the profile (I_star and w . l scale
  together, Eq. 5);
* a uniform profile gives 1 - a(z, k)/pi, the closed form of the uniform
  source (Mandel & Agol's lambda_e);
* per-vector quadratic profiles at the default grid are within 5 ppm (the
  accuracy level the paper quotes, Sect. 3.3) of the
  analytic quadratic model with each vector's own coefficients;
* each named law's closed-form I_star equals adaptive quadrature of
  2 pi int mu I dmu, and the oracle's integral of a finely sampled profile
  converges to it."""

import numpy as np
import pytest
from scipy.integrate import quad

import workloads as wl
from oracle import analytic as an
from oracle import orbit
from oracle import roadrunner as orr
from paper_2009_08500_amd import ldlaws


@pytest.fixture(scope="module")
def small():
    w = wl.population_ld(npv=6, npt=4000)
    tab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    return w, tab


def test_own_profile_reduces_to_shared_tables(small):
    w, tab = small
    prof = np.broadcast_to(tab.I_s, (6,) + tab.I_s.shape)
    a = orr.evaluate_ld(tab, w["times"], w["pv"], prof)
    b = orr.evaluate(tab, w["times"], w["pv"])
    assert np.array_equal(a, b)


def test_weight_reuse_matches_fresh_tables(small):
    w, tab = small
    for i in (0, 3):
        fresh = orr.Tables(w["mu_s"], w["prof_pv"][i], **wl.TEST_GRID)
        a = orr.evaluate_ld(tab, w["times"], w["pv"][i:i + 1], w["prof_pv"][i:i + 1])
        b = orr.evaluate(fresh, w["times"], w["pv"][i:i + 1])
        assert np.abs(a - b).max() <= 1e-14
        assert np.abs(a - orr.evaluate(tab, w["times"], w["pv"][i:i + 1])).max() > 1e-6


def test_flux_invariant_under_profile_scaling(small):
    w, tab = small
    a = orr.evaluate_ld(tab, w["times"], w["pv"], w["prof_pv"])
    b = orr.evaluate_ld(tab, w["times"], w["pv"], 2.7 * w["prof_pv"])
    assert np.abs(a - b).max() <= 1e-14


def test_uniform_profile_is_the_uniform_source(small):
    w, tab = small
    ones = np.ones((6, 1, w["mu_s"].size))
    f = orr.evaluate_ld(tab, w["times"], w["pv"], ones)
    for i, row in enumerate(w["pv"]):
        dt = orbit.phase_offset(w["times"], row[0], row[1])
        z, front, _ = orbit.projected_separation(dt, *row[1:6])
        ref = np.where(front, an.quadratic_flux(z, row[6], 0.0, 0.0), 1.0)
        assert np.abs(f[i] - ref).max() <= 1e-13


def test_per_vector_quadratic_within_five_ppm_of_analytic():
    w = wl.single_light_curve()
    tab = orr.Tables(w["mu_s"], w["I_s"], **wl.DEFAULT_GRID)
    coef = [(0.4, 0.25), (0.1, 0.6), (0.8, -0.1)]
    pv = np.repeat(w["pv"], 3, axis=0)
    pv[1, 6], pv[2, 6] = 0.05, 0.2
    prof = np.stack([wl.profile_quadratic(w["mu_s"], u1, u2) for u1, u2 in coef])[:, None, :]
    f = orr.evaluate_ld(tab, w["times"], pv, prof)
    for i, (u1, u2) in enumerate(coef):
        row = pv[i]
        z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
        ref = np.where(front, an.quadratic_flux(z, row[6], u1, u2), 1.0)
        assert np.abs(f[i] - ref).max() <= 5e-6, (i, np.abs(f[i] - ref).max())


LAWS = {"uniform": [], "linear": [0.4], "quadratic": [0.4, 0.25],
        "triangular-quadratic": [0.3, 0.35], "general": [0.3, 0.2, -0.1],
        "nonlinear": [0.6, -0.3, 0.5, -0.2], "logarithmic": [0.5, 0.2],
        "power-2": [0.6, 0.55], "power-2-pm": [0.75, 0.5]}


@pytest.mark.parametrize("law", sorted(LAWS))
def test_law_istar_closed_form(law):
    c = np.array(LAWS[law], float)
    f = lambda mu: float(ldlaws.profile(law, np.array([mu]), c).reshape(-1)[0])  # noqa: E731
    num = 2.0 * np.pi * quad(lambda mu: mu * f(mu), 0.0, 1.0, epsabs=1e-14, limit=400)[0]
    assert float(ldlaws.istar(law, c)) == pytest.approx(num, abs=1e-9)
    mu = np.linspace(0.0, 1.0, 20001)
    I = ldlaws.profile(law, mu, c).numpy().reshape(1, -1)
    assert orr.istar_of_profile(mu, I)[0] == pytest.approx(float(ldlaws.istar(law, c)), abs=2e-6)
    assert float(ldlaws.profile(law, np.array([1.0]), c).reshape(-1)[0]) == pytest.approx(1.0)


def test_law_reparametrisations():
    q1, q2 = 0.3, 0.35
    a, b = 2 * np.sqrt(q1) * q2, np.sqrt(q1) * (1 - 2 * q2)
    mu = np.linspace(0, 1, 11)
    assert np.allclose(ldlaws.profile("triangular-quadratic", mu, [q1, q2]).numpy(),
                       wl.profile_quadratic(mu, a, b), atol=1e-15)
    c, al = 0.6, 0.55
    h1, h2 = 1 - c * (1 - 2 ** -al), c * 2 ** -al
    assert np.allclose(ldlaws.profile("power-2-pm", mu, [h1, h2]).numpy(),
                       ldlaws.profile("power-2", mu, [c, al]).numpy(), atol=1e-14)
    # coefficient batches broadcast: (3, 2) coefficients -> (3, nmu) profiles
    cs = np.array([[0.4, 0.25], [0.1, 0.6], [0.8, -0.1]])
    P = ldlaws.profile("quadratic", mu, cs).numpy()
    assert P.shape == (3, mu.size)
    for i, (u1, u2) in enumerate(cs):
        assert np.allclose(P[i], wl.profile_quadratic(mu, u1, u2), atol=1e-15)
    with pytest.raises(ValueError):
        ldlaws.profile("quadratic", mu, [0.1])
