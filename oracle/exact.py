"""Oracle-B: the transit signal from its plain definition, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 1-2 define the transit signal as the stellar surface brightness
integrated over the disk minus its integral over the occluded area.  With a
radially symmetric profile the occluded integral reduces to one dimension:

    int_{A_p} I dA = int_0^1 I(r) 2 r phi(r) dr,

where 2 phi(r) is the angle of the circle of radius r (centred on the star)
that lies inside the planet disk.  ``occulted_exact`` integrates this with
adaptive quadrature (scipy's QUADPACK), split at every point where the
integrand is not smooth.  ``occulted_bruteforce`` integrates the same
brightness over the planet disk in 2-D (planet-centred polar coordinates,
Gauss-Legendre in both directions) and serves as the independent check of the
1-D reduction on tiny inputs.  Neither uses any of the method's tables.
"""

import numpy as np
from scipy import integrate

from . import orbit as _orbit


def tabulated_profile(mu_s, I_s):
    """I(mu) as the piecewise-linear interpolant of samples (constant beyond
    the end samples) -- the same reading of a tabulated profile as Oracle-A."""
    mu_s = np.asarray(mu_s, float)
    I_s = np.asarray(I_s, float)

    def prof(mu):
        return np.interp(mu, mu_s, I_s)

    prof.knots = mu_s
    return prof


def _phi(r, z, k):
    """Half-angle of the star-centred circle of radius r inside the planet."""
    if z == 0.0:
        return np.where(r < k, np.pi, 0.0)
    x = (r * r + z * z - k * k) / (2.0 * r * z)
    return np.arccos(np.clip(x, -1.0, 1.0))


def occulted_exact(z, k, prof, epsabs=1e-15, epsrel=1e-13):
    """int_0^1 I(mu(r)) 2 r phi(r) dr for one (z, k); ``prof`` maps mu -> I.

    Split at r = |z - k|, z + k, the unit limb and every profile knot so that
    each piece is smooth inside.
    """
    if z >= 1.0 + k:
        return 0.0
    upper = min(1.0, z + k)
    pts = {0.0, upper}
    if z < k:
        pts.add(k - z)
    else:
        pts.add(z - k)
    for mu_k in getattr(prof, "knots", ()):
        r = np.sqrt(max(0.0, 1.0 - mu_k * mu_k))
        if 0.0 < r < upper:
            pts.add(float(r))
    pts = sorted(p for p in pts if 0.0 <= p <= upper)
    total = 0.0

    def f(r):
        mu = np.sqrt(max(0.0, 1.0 - r * r))
        return float(prof(mu)) * 2.0 * r * float(_phi(r, z, k))

    for lo, hi in zip(pts[:-1], pts[1:]):
        if hi <= lo:
            continue
        val, _ = integrate.quad(f, lo, hi, epsabs=epsabs, epsrel=epsrel,
                                limit=400)
        total += val
    return total


def istar_exact(prof, epsabs=1e-15, epsrel=1e-13):
    """I_star = 2 pi int_0^1 mu I(mu) dmu (Eq. 2, Eq. 4), adaptive quadrature."""
    pts = sorted({0.0, 1.0, *[float(m) for m in getattr(prof, "knots", ())
                              if 0.0 < m < 1.0]})
    total = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        val, _ = integrate.quad(lambda m: m * float(prof(m)), lo, hi,
                                epsabs=epsabs, epsrel=epsrel, limit=200)
        total += val
    return 2.0 * np.pi * total


def flux_exact(z, k, prof, istar=None):
    """Normalised flux 1 - (occluded integral)/I_star (Eq. 1-4) at each z."""
    istar = istar_exact(prof) if istar is None else istar
    z = np.atleast_1d(np.asarray(z, float))
    return np.array([1.0 - occulted_exact(zz, k, prof) / istar for zz in z])


# ---------------------------------------------------------------- 2-D check
def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def occulted_bruteforce(z, k, prof, n_theta=256, n_rho=256):
    """2-D integral of I over the part of the planet disk inside the star.

    Planet-centred polar coordinates (rho, theta); the point is at
    (z + rho cos theta, rho sin theta) from the star centre.  For each theta
    the ray is clipped to the stellar disk and the clipped segment is split
    at its midpoint.  On a half that ends on the stellar limb (where
    mu ~ sqrt(distance)) the radial variable is substituted rho = end -/+ s^2
    so the integrand is smooth; other halves use plain Gauss-Legendre.
    theta is split where the two limbs cross and where a ray grazes the limb.
    Symmetric in theta, so [0, pi] is integrated and doubled.  Intended for
    smooth analytic profiles on tiny inputs.
    """
    breaks = {0.0, np.pi}
    if z > 0.0:
        cth = (1.0 - z * z - k * k) / (2.0 * z * k)
        if -1.0 < cth < 1.0:
            breaks.add(float(np.arccos(cth)))
        if z >= 1.0:
            breaks.add(float(np.pi - np.arcsin(1.0 / z)))
    breaks = sorted(breaks)
    xg, wg = np.polynomial.legendre.leggauss(n_rho)
    u, wu = 0.5 * (xg + 1.0), 0.5 * wg                      # nodes on [0, 1]
    total = 0.0
    for t0, t1 in zip(breaks[:-1], breaks[1:]):
        th, wth = _gl(n_theta, t0, t1)
        ct, st = np.cos(th), np.sin(th)
        disc = 1.0 - z * z * st * st
        ok = disc > 0.0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        rp, rm = -z * ct + sq, -z * ct - sq
        lo, hi = np.maximum(0.0, rm), np.minimum(k, rp)
        ok &= hi > lo
        if not ok.any():
            continue
        ct, st, lo, hi, wth = ct[ok], st[ok], lo[ok], hi[ok], wth[ok]
        lo_limb, hi_limb = (lo == rm[ok]), (hi == rp[ok])
        mid = 0.5 * (lo + hi)
        half = (mid - lo)[:, None]
        # lower half [lo, mid]
        s_lo = np.sqrt(half) * u[None, :]
        rho_a = np.where(lo_limb[:, None], lo[:, None] + s_lo * s_lo,
                         lo[:, None] + half * u[None, :])
        jac_a = np.where(lo_limb[:, None], 2.0 * s_lo * np.sqrt(half), half)
        # upper half [mid, hi]
        s_hi = np.sqrt(half) * u[None, :]
        rho_b = np.where(hi_limb[:, None], hi[:, None] - s_hi * s_hi,
                         mid[:, None] + half * u[None, :])
        jac_b = np.where(hi_limb[:, None], 2.0 * s_hi * np.sqrt(half), half)
        acc = 0.0
        for rho, jac in ((rho_a, jac_a), (rho_b, jac_b)):
            x = z + rho * ct[:, None]
            y = rho * st[:, None]
            mu = np.sqrt(np.maximum(0.0, 1.0 - x * x - y * y))
            acc = acc + np.sum(wu[None, :] * jac * rho * prof(mu), axis=1)
        total += np.sum(wth * acc)
    return 2.0 * total


# ---------------------------------------------------------------- light curves
def evaluate_exact(times, row, prof_by_pb, istar_by_pb, lcids=None, pbids=None,
                   nss=None, exptimes=None):
    """Exact-definition light curve for one parameter row (slow; tiny inputs).

    Same orbit and supersampling readings as Oracle-A; only the occultation
    step differs (the plain integral instead of the tables).
    """
    times = np.asarray(times, float)
    npt = times.size
    lcids = np.zeros(npt, np.int64) if lcids is None else np.asarray(lcids)
    if pbids is None:
        pbids = np.zeros(int(lcids.max()) + 1, np.int64)
    nlc = len(pbids)
    nss = np.ones(nlc, np.int64) if nss is None else np.broadcast_to(nss, (nlc,))
    exptimes = (np.zeros(nlc) if exptimes is None
                else np.broadcast_to(np.asarray(exptimes, float), (nlc,)))
    t0, P, a, b, e, w = row[:6]
    out = np.empty(npt)
    for it in range(npt):
        lc = int(lcids[it])
        pb = int(pbids[lc])
        k = row[6 + pb]
        ts = _orbit.subsample_times(times[it:it + 1], int(nss[lc]), exptimes[lc])[0]
        dt = _orbit.phase_offset(ts, t0, P)
        z, front, _ = _orbit.projected_separation(dt, P, a, b, e, w)
        d = [occulted_exact(zz, k, prof_by_pb[pb]) / istar_by_pb[pb] if fr else 0.0
             for zz, fr in zip(z, front)]
        out[it] = 1.0 - np.mean(d)
    return out
