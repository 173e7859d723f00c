"""Keplerian orbit -> projected planet-star separation, FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper evaluates the model for the orbital elements zero epoch t0, period
P, scaled semi-major axis a, inclination i, eccentricity e and argument of
periastron w (Sect. 4.1), and notes that the orbit computation dominates the
cost (Sect. 3.1.2, Sect. 5), but gives no orbit algorithm.  The readings used
here are the standard ones for transiting planets:

* the planet transits at true anomaly f_tr = pi/2 - w, with +Z towards the
  observer, so the planet is in front of the star when sin(w + f) > 0;
* t0 is the time of inferior conjunction (f = f_tr);
* the parameter vector carries the conjunction impact parameter
  b = a cos(i) (1 - e^2) / (1 + e sin w) instead of i, so
  cos(i) = b (1 + e sin w) / (a (1 - e^2));
* the sky-plane separation is z = r sqrt(cos^2(w+f) + sin^2(w+f) cos^2 i),
  algebraically the same as r sqrt(1 - sin^2(w+f) sin^2 i) but without the
  cancellation near mid-transit.
"""

import numpy as np

TWO_PI = 2.0 * np.pi


def cos_inclination(a, b, e, w):
    """cos(i) from the conjunction impact parameter b (reading, see module doc)."""
    return b * (1.0 + e * np.sin(w)) / (a * (1.0 - e * e))


def eccentric_from_true(f, e):
    """Eccentric anomaly for true anomaly f (textbook half-angle relation)."""
    return 2.0 * np.arctan2(np.sqrt(1.0 - e) * np.sin(0.5 * f),
                            np.sqrt(1.0 + e) * np.cos(0.5 * f))


def true_from_eccentric(E, e):
    """True anomaly for eccentric anomaly E (textbook half-angle relation)."""
    return 2.0 * np.arctan2(np.sqrt(1.0 + e) * np.sin(0.5 * E),
                            np.sqrt(1.0 - e) * np.cos(0.5 * E))


def conjunction_mean_anomaly(e, w):
    """Mean anomaly at inferior conjunction, M_tr = E_tr - e sin E_tr."""
    f_tr = 0.5 * np.pi - w
    E_tr = eccentric_from_true(f_tr, e)
    return E_tr - e * np.sin(E_tr)


def solve_kepler(M, e, tol=1e-15, maxiter=60):
    """Solve E - e sin E = M by Newton's method from E0 = M + e sin M.

    Points that have not converged after ``maxiter`` steps (none are expected
    for e < 1) are finished by bisection on [M - e, M + e], which always
    brackets the root because |E - M| = e |sin E| <= e.
    """
    M = np.asarray(M, dtype=np.float64)
    e = np.broadcast_to(np.asarray(e, dtype=np.float64), M.shape)
    E = M + e * np.sin(M)
    done = np.zeros(M.shape, dtype=bool)
    for _ in range(maxiter):
        dE = (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        E = np.where(done, E, E - dE)
        done |= np.abs(dE) <= tol * np.maximum(1.0, np.abs(E))
        if done.all():
            break
    bad = np.abs(E - e * np.sin(E) - M) > 1e-12 * np.maximum(1.0, np.abs(M))
    if bad.any():
        E[bad] = solve_kepler_bisection(M[bad], e[bad])
    return E


def solve_kepler_bisection(M, e, iters=200):
    """Solve E - e sin E = M by plain bisection (slow, unconditionally safe).

    Used as an independent pin for :func:`solve_kepler`.
    """
    M = np.asarray(M, dtype=np.float64)
    e = np.broadcast_to(np.asarray(e, dtype=np.float64), M.shape)
    lo = M - e
    hi = M + e
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        f = mid - e * np.sin(mid) - M
        lo = np.where(f < 0.0, mid, lo)
        hi = np.where(f < 0.0, hi, mid)
    return 0.5 * (lo + hi)


def phase_offset(t, t0, P):
    """Time since the nearest conjunction, in [-P/2, P/2].

    Done in FP64 on the mid-exposure or subsample time; this is the step the
    mixed-precision GPU path keeps in FP64 (the paper's closing discussion of
    mixed CPU/GPU precision, Sect. 6).
    """
    x = t - t0
    return x - P * np.round(x / P)


def projected_separation(dt, P, a, b, e, w):
    """Projected separation z and the in-front flag for time offsets ``dt``
    from conjunction.  Scalars P, a, b, e, w; ``dt`` any shape.

    Returns (z, front, cos_i); z is in units of the stellar radius.
    """
    dt = np.asarray(dt, dtype=np.float64)
    cosi = cos_inclination(a, b, e, w)
    M = conjunction_mean_anomaly(e, w) + TWO_PI * dt / P
    if e == 0.0:
        E = M
    else:
        E = solve_kepler(M, e)
    f = true_from_eccentric(E, e)
    r = a * (1.0 - e * np.cos(E))
    s = np.sin(w + f)
    c = np.cos(w + f)
    z = r * np.sqrt(c * c + s * s * cosi * cosi)
    return z, s > 0.0, cosi


def subsample_times(t, nss, exptime):
    """Subsample times for exposures centred on ``t`` (shape (npt, nss)).

    Midpoint rule over the exposure (Sect. 4.1, supersampling after Kipping
    2010): t_s = t + exptime * ((s + 1/2)/nss - 1/2), s = 0..nss-1.
    """
    t = np.asarray(t, dtype=np.float64)
    s = np.arange(nss, dtype=np.float64)
    off = exptime * ((s + 0.5) / nss - 0.5)
    return t[:, None] + off[None, :]
