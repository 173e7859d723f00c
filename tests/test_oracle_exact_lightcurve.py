"""Pins of Oracle-B's light curve (``oracle.exact.evaluate_exact``): the
plain definition (Eq. 1-2) evaluated along the orbit with the supersampling
reading, checked against computations that share none of its steps.

* A circular orbit with the exact quadratic law: the sky separation is the
  closed form z = a sqrt(sin^2 phi + cos^2 i cos^2 phi), phi = 2 pi (t - t0)/P
  (written out here, not taken from the oracle's orbit module), and the flux
  is the analytic quadratic model of Mandel & Agol (2002), the model the
  paper measures its accuracy against (Sect. 3.3).  Agreement to 1e-10.
* Supersampling (Sect. 4.1, reading R10): the exposure value equals the mean
  of the analytic model at the midpoint-rule subsample times.
* Light-curve and passband bookkeeping (Sect. 4.2): each point uses its own
  light curve's passband, radius ratio, profile and normaliser.
* Against Oracle-A (the tabulated method, Sect. 3.1) on the same tabulated
  profile: within the accuracy class the paper quotes for its grids
  (Sect. 3.3: a few ppm), and closer on a finer grid.
"""

import numpy as np
import pytest

from oracle import analytic as an
from oracle import exact as ex
from oracle import roadrunner as orr


def quad_profile(u1, u2):
    def prof(mu):
        return 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2
    return prof


def quad_istar(u1, u2):
    # 2 pi int_0^1 mu I(mu) dmu for I = 1 - u1 (1 - mu) - u2 (1 - mu)^2
    return np.pi * (1.0 - u1 / 3.0 - u2 / 6.0)


def circular_z(t, t0, P, a, b):
    cosi = b / a
    phi = 2.0 * np.pi * (t - t0) / P
    return a * np.sqrt(np.sin(phi) ** 2 + (cosi * np.cos(phi)) ** 2), np.cos(phi) > 0.0


@pytest.mark.parametrize("k,b", [(0.1, 0.3), (0.05, 0.8), (0.2, 0.0)])
def test_circular_orbit_equals_analytic_quadratic_model(k, b):
    u1, u2 = 0.4, 0.25
    t0, P, a = 0.3, 3.0, 8.0
    times = np.linspace(t0 - 0.12, t0 + 0.12, 41)
    row = np.array([t0, P, a, b, 0.0, 0.0, k])
    f = ex.evaluate_exact(times, row, [quad_profile(u1, u2)], [quad_istar(u1, u2)])
    z, front = circular_z(times, t0, P, a, b)
    ref = np.where(front, an.quadratic_flux(z, k, u1, u2), 1.0)
    assert np.abs(f - ref).max() <= 1e-10
    assert f.min() < 1.0 - 0.5 * k * k          # the window covers the transit


def test_supersampled_exposures_are_subsample_means():
    u1, u2 = 0.3, 0.2
    t0, P, a, b, k = 0.0, 2.5, 7.0, 0.4, 0.12
    nss, ex_t = 5, 0.02
    times = np.linspace(-0.1, 0.1, 17)
    row = np.array([t0, P, a, b, 0.0, 0.0, k])
    f = ex.evaluate_exact(times, row, [quad_profile(u1, u2)], [quad_istar(u1, u2)],
                          nss=[nss], exptimes=[ex_t])
    offs = ((np.arange(nss) + 0.5) / nss - 0.5) * ex_t
    ts = times[:, None] + offs[None, :]
    z, front = circular_z(ts, t0, P, a, b)
    sub = np.where(front, an.quadratic_flux(z.ravel(), k, u1, u2).reshape(z.shape), 1.0)
    assert np.abs(f - sub.mean(axis=1)).max() <= 1e-10
    # and it differs from the unsupersampled curve in ingress/egress
    f1 = ex.evaluate_exact(times, row, [quad_profile(u1, u2)], [quad_istar(u1, u2)])
    assert np.abs(f - f1).max() > 1e-5


def test_light_curves_use_their_own_passband():
    """Two light curves on passbands 1 and 0 (swapped order), each with its
    own k and quadratic coefficients."""
    t0, P, a, b = 0.0, 3.0, 9.0, 0.2
    times = np.concatenate([np.linspace(-0.08, 0.08, 9), np.linspace(-0.08, 0.08, 9)])
    lcids = np.repeat([0, 1], 9)
    ld = [(0.5, 0.1), (0.2, 0.3)]
    ks = [0.09, 0.14]
    row = np.array([t0, P, a, b, 0.0, 0.0, ks[0], ks[1]])
    f = ex.evaluate_exact(times, row, [quad_profile(*ld[0]), quad_profile(*ld[1])],
                          [quad_istar(*ld[0]), quad_istar(*ld[1])], lcids=lcids, pbids=[1, 0])
    z, front = circular_z(times, t0, P, a, b)
    for lc, pb in ((0, 1), (1, 0)):
        sel = lcids == lc
        ref = np.where(front[sel], an.quadratic_flux(z[sel], ks[pb], *ld[pb]), 1.0)
        assert np.abs(f[sel] - ref).max() <= 1e-10


def test_close_to_the_tabulated_method():
    """An eccentric orbit and a power-2 profile tabulated at 200 mu samples:
    Oracle-A (tables, k on a node) within a few ppm of the exact definition
    on a coarse grid and closer on a fine one; both share only the orbit and
    supersampling readings."""
    mu = np.linspace(0.0, 1.0, 200)
    I_s = 1.0 - 0.6 * (1.0 - mu ** 0.6)
    prof = ex.tabulated_profile(mu, I_s)
    istar = ex.istar_exact(prof)
    k = 0.1
    row = np.array([0.2, 4.0, 10.0, 0.5, 0.2, 1.1, k])
    # conjunction +- 0.09 d: ingress, egress and the flat bottom
    times = 0.2 + np.linspace(-0.09, 0.09, 25)
    fe = ex.evaluate_exact(times, row, [prof], [istar], nss=[3], exptimes=[0.01])
    errs = []
    for nzin, nzlimb, ng in ((20, 40, 128), (100, 200, 1024)):
        # k sits on node 9 of the k-grid, so no k-interpolation
        tab = orr.Tables(mu, I_s, zcut=0.8, nzin=nzin, nzlimb=nzlimb, ng=ng, nk=19,
                         k0=0.01, k1=0.19)
        fa = orr.evaluate(tab, times, row[None, :], nss=3, exptimes=0.01)[0]
        errs.append(np.abs(fa - fe).max())
    assert fe.min() < 0.99
    assert errs[0] <= 10e-6 and errs[1] <= 0.5e-6 and errs[1] < errs[0], errs
