"""Analytic transit light curve for quadratic limb darkening, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper checks its model's accuracy against the analytic quadratic-LD
transit model of Mandel & Agol (2002) (Sect. 3.2, the accuracy figure).  This
module restates that published model so the oracles can be pinned to it:

* the uniform source occults the lens area a(z, p)/pi (``lambda_e``);
* a brightness linear in mu occults an integral that reduces to complete
  elliptic integrals of the first, second and third kind (``lambda_d``):
  one form while the planet crosses the limb, another while it is inside the
  disk, an elementary form at z = 0;
* a brightness linear in mu^2 = 1 - r^2 occults an elementary integral
  (``eta_d``).

With I(mu) = 1 - u1 (1 - mu) - u2 (1 - mu)^2 = c0 + c2 mu + c4 mu^2
(c2 = u1 + 2 u2, c4 = -u2, c0 = 1 - c2 - c4) and the disk integral
4 Omega = c0 + 2 c2 / 3 + c4 / 2 (in units of pi I(1)), the normalised flux is

    F = 1 - [(1 - c2) lambda_e + c2 (lambda_d + 2/3 [p > z]) - c4 eta_d] / (4 Omega).

Complete elliptic integrals use the modulus k; Pi(n, k) is
int_0^{pi/2} dphi / ((1 - n sin^2 phi) sqrt(1 - k^2 sin^2 phi)), evaluated
with Carlson's symmetric forms, Pi = R_F(0, 1 - k^2, 1) +
(n / 3) R_J(0, 1 - k^2, 1, 1 - n).  Valid for 0 < p < 1/2 (the population's
radius ratios); the configurations z = 0, z = p and z = 1 - p, where the
general forms are singular, have their own closed forms.
"""

import numpy as np
from scipy import special


def _K(k):
    return special.ellipk(k * k)


def _E(k):
    return special.ellipe(k * k)


def _Pi(n, k):
    return special.elliprf(0.0, 1.0 - k * k, 1.0) + n / 3.0 * special.elliprj(
        0.0, 1.0 - k * k, 1.0, 1.0 - n)


def lambda_e(p, z):
    """Fraction of the uniform disk occulted: lens area / pi."""
    if z >= 1.0 + p:
        return 0.0
    if z <= 1.0 - p:
        return p * p
    kap0 = np.arccos((p * p + z * z - 1.0) / (2.0 * p * z))
    kap1 = np.arccos((1.0 - p * p + z * z) / (2.0 * z))
    return (p * p * kap0 + kap1 - 0.5 * np.sqrt(4.0 * z * z - (1.0 + z * z - p * p) ** 2)) / np.pi


def lambda_d_eta_d(p, z):
    """(lambda_d, eta_d): the occulted parts of the mu and mu^2 terms."""
    if z >= 1.0 + p:
        return 0.0, 0.0
    a = (z - p) ** 2
    b = (z + p) ** 2
    q = p * p - z * z
    eta2 = 0.5 * p * p * (p * p + 2.0 * z * z)
    if z > 1.0 - p:
        # the planet crosses the limb
        k = np.sqrt((1.0 - a) / (4.0 * z * p))
        lam = (((1.0 - b) * (2.0 * b + a - 3.0) - 3.0 * q * (b - 2.0)) * _K(k)
               + 4.0 * p * z * (z * z + 7.0 * p * p - 4.0) * _E(k)
               - 3.0 * q / a * _Pi((a - 1.0) / a, k)) / (9.0 * np.pi * np.sqrt(p * z))
        kap0 = np.arccos((p * p + z * z - 1.0) / (2.0 * p * z))
        kap1 = np.arccos((1.0 - p * p + z * z) / (2.0 * z))
        eta = (kap1 + 2.0 * eta2 * kap0
               - 0.25 * (1.0 + 5.0 * p * p + z * z) * np.sqrt((1.0 - a) * (b - 1.0))) / (2.0 * np.pi)
        return lam, eta
    if z == 0.0:
        return -2.0 / 3.0 * (1.0 - p * p) ** 1.5, eta2
    if z == p:
        # the planet's limb passes through the stellar centre (p < 1/2)
        m = 4.0 * p * p
        lam = 1.0 / 3.0 + 2.0 / (9.0 * np.pi) * (
            4.0 * (2.0 * p * p - 1.0) * special.ellipe(m) + (1.0 - 4.0 * p * p) * special.ellipk(m))
        return lam, eta2
    if z == 1.0 - p:
        # the planet touches the limb from inside (p < 1/2)
        lam = (2.0 / (3.0 * np.pi) * np.arccos(1.0 - 2.0 * p)
               - 4.0 / (9.0 * np.pi) * (3.0 + 2.0 * p - 8.0 * p * p) * np.sqrt(p * (1.0 - p)))
        return lam, eta2
    # the planet is inside the disk
    kinv = np.sqrt(4.0 * z * p / (1.0 - a))
    lam = 2.0 / (9.0 * np.pi * np.sqrt(1.0 - a)) * (
        (1.0 - 5.0 * z * z + p * p + q * q) * _K(kinv)
        + (1.0 - a) * (z * z + 7.0 * p * p - 4.0) * _E(kinv)
        - 3.0 * q / a * _Pi((a - b) / a, kinv))
    return lam, eta2


def quadratic_flux(z, p, u1, u2):
    """Normalised flux for separations z (array) of a planet with radius
    ratio p in front of a star with quadratic limb darkening (u1, u2)."""
    z = np.atleast_1d(np.asarray(z, float))
    c2 = u1 + 2.0 * u2
    c4 = -u2
    c0 = 1.0 - c2 - c4
    four_omega = c0 + 2.0 * c2 / 3.0 + c4 / 2.0
    out = np.empty(z.shape)
    for i, zz in enumerate(z):
        le = lambda_e(p, zz)
        ld, ed = lambda_d_eta_d(p, zz)
        th = 1.0 if p > zz else 0.0
        out[i] = 1.0 - ((1.0 - c2) * le + c2 * (ld + 2.0 / 3.0 * th) - c4 * ed) / four_omega
    return out
