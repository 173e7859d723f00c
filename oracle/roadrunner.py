"""Oracle-A: the RoadRunner model step by step, FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's method in its own order:

1. z-grid of annulus edges and means, constant dz inside z_cut and constant
   dmu outside it (Sect. 3.1.1);
2. limb-darkening profile at the bin means (Sect. 2, Sect. 3.1.1); the
   profile is given as samples I_s at mu_s and read as their piecewise-linear
   interpolant (the custom-profile case of Sect. 3.2.2);
3. normalising integral I_star = 2 pi int_0^1 z I dz (Eq. 2, Eq. 4), here the
   exact integral of that interpolant;
4. the 3-D weight table w[k][g][z-bin]: area of each annulus occluded by the
   planet over the total occluded area (Sect. 2), on a (k, g) grid with
   g = c/(1+k) (Sect. 3.1, Sect. 3.1.2);
5. LD-weighted tables T = w . l over (k, g) (Sect. 3.1.2);
6. per radius ratio, linear interpolation of T in k (Sect. 3.1.2);
7. per separation z, linear interpolation in g and Eq. 5:
   F = (I_star - (w . l) a(z, k)) / I_star (Sect. 2, Sect. 3.1.1);
8. orbit and supersampling for populations of parameter vectors and
   heterogeneous light curves (Sect. 4.1, Sect. 4.2).

Also the per-row LD form (each row's own profile through steps 2-5), the
direct model (weights for a row's own k, Sect. 3.1.1) and the small-planet
approximation (the LD value at the planet's centre below a radius-ratio
threshold, Sect. 3.4.2).

Readings of points the paper leaves open (listed with reasons in the design
notes): n_g and n_k count grid points including both ends; the g index is
clamped to n_g - 2 and the k index to n_k - 2; the weight vector at g = 1
(zero overlap, 0/0) is its limit, all weight in the outermost annulus; a k
outside [k0, k1] or a non-physical orbit gives a NaN row.
"""

import numpy as np

from . import orbit as _orbit

PAR_T0, PAR_P, PAR_A, PAR_B, PAR_E, PAR_W = range(6)
NPAR_ORBIT = 6


# ---------------------------------------------------------------- step 1
def z_grid(zcut, nzin, nzlimb):
    """Annulus edges ``ze`` (nz+1), means ``zm`` (nz) and ``mu`` at the means.

    Sect. 3.1.1: bins of constant width in z on [0, z_cut] and of constant
    width in mu on [z_cut, 1].  The outer edges are spaced uniformly in mu
    from mu(z_cut) down to 0 and mapped back to z.
    """
    ze_in = np.linspace(0.0, zcut, nzin + 1)
    mu_cut = np.sqrt(1.0 - zcut * zcut)
    mu_edges = np.linspace(mu_cut, 0.0, nzlimb + 1)
    ze_out = np.sqrt(1.0 - mu_edges * mu_edges)
    ze = np.concatenate([ze_in, ze_out[1:]])
    zm = 0.5 * (ze[:-1] + ze[1:])
    mu = np.sqrt(1.0 - zm * zm)
    return ze, zm, mu


# ---------------------------------------------------------------- areas
def lens_area(R, k, c):
    """Area of the intersection of a disk of radius R centred at the origin
    and a disk of radius k centred at distance c (textbook circle-circle
    intersection; a(c, k) of Eq. 5 is ``lens_area(1, k, c)``)."""
    R, k, c = np.broadcast_arrays(np.asarray(R, float), np.asarray(k, float),
                                  np.asarray(c, float))
    out = np.zeros(R.shape)
    inside = c <= np.abs(R - k)
    out[inside] = np.pi * np.minimum(R[inside], k[inside]) ** 2
    part = (~inside) & (c < R + k)
    Rp, kp, cp = R[part], k[part], c[part]
    a1 = np.clip((cp * cp + Rp * Rp - kp * kp) / (2.0 * cp * Rp), -1.0, 1.0)
    a2 = np.clip((cp * cp + kp * kp - Rp * Rp) / (2.0 * cp * kp), -1.0, 1.0)
    rad = (-cp + Rp + kp) * (cp + Rp - kp) * (cp - Rp + kp) * (cp + Rp + kp)
    out[part] = (Rp * Rp * np.arccos(a1) + kp * kp * np.arccos(a2)
                 - 0.5 * np.sqrt(np.maximum(rad, 0.0)))
    return out


# ---------------------------------------------------------------- step 4
def grid_steps(nk, k0, k1, ng):
    """(dk, dg): n_k and n_g count points including both ends."""
    return (k1 - k0) / (nk - 1), 1.0 / (ng - 1)


def weights_3d(ze, nk, k0, k1, ng):
    """Weight table W[nk][ng][nz] (Sect. 2, Sect. 3.1.2).

    W[i, m, j] = (A(ze[j+1], k_i, c) - A(ze[j], k_i, c)) / A(1, k_i, c),
    with k_i = k0 + i dk, g_m = m / (ng - 1) (so the last node is exactly
    g = 1) and c = g_m (1 + k_i): the area of annulus j covered by the planet
    over the total covered area.  At g = 1 the overlap is zero and W is its
    limit, the unit vector of the outermost annulus.
    """
    dk, dg = grid_steps(nk, k0, k1, ng)
    nz = ze.size - 1
    k = k0 + dk * np.arange(nk)
    g = np.arange(ng) / (ng - 1.0)
    c = g[None, :] * (1.0 + k[:, None])                    # (nk, ng)
    A = lens_area(ze[None, None, :], k[:, None, None], c[:, :, None])
    total = A[:, :, -1]
    W = np.zeros((nk, ng, nz))
    ok = total > 0.0
    W[ok] = np.diff(A, axis=-1)[ok] / total[ok][:, None]
    W[~ok] = 0.0
    W[~ok, nz - 1] = 1.0
    return dk, dg, W


# ---------------------------------------------------------------- steps 2-3
def profile_on_grid(mu_s, I_s, mu):
    """LD profile at the bin means: the piecewise-linear interpolant of the
    samples (constant beyond the end samples).  I_s may be (nmu,) or
    (npb, nmu)."""
    I_s = np.atleast_2d(np.asarray(I_s, float))
    return np.stack([np.interp(mu, mu_s, row) for row in I_s])


def istar_of_profile(mu_s, I_s):
    """I_star = 2 pi int_0^1 mu I(mu) dmu (Eq. 2 with z dz = -mu dmu, Eq. 4)
    for the piecewise-linear interpolant with constant end extension.

    On a segment where I is linear, mu I(mu) is quadratic and
    int mu I dmu = h/6 [I_a (2 mu_a + mu_b) + I_b (mu_a + 2 mu_b)] exactly.
    """
    mu_s = np.asarray(mu_s, float)
    I_s = np.atleast_2d(np.asarray(I_s, float))
    ma, mb = mu_s[:-1], mu_s[1:]
    h = mb - ma
    seg = (h / 6.0) * (I_s[:, :-1] * (2 * ma + mb) + I_s[:, 1:] * (ma + 2 * mb))
    lo = I_s[:, 0] * 0.5 * mu_s[0] ** 2
    hi = I_s[:, -1] * 0.5 * (1.0 - mu_s[-1] ** 2)
    return 2.0 * np.pi * (seg.sum(axis=1) + lo + hi)


# ---------------------------------------------------------------- step 5
def ld_tables(W, ldp):
    """T[pb][i][m] = sum_j W[i][m][j] ldp[pb][j] (Sect. 3.1.2)."""
    return np.einsum("imj,pj->pim", W, ldp)


class Tables:
    """Everything Oracle-A precomputes for one grid and one set of profiles.

    ``istar`` (one value per passband) replaces the interpolant's integral
    as the normaliser, for a law whose disk integral is known in closed form
    (Sect. 3.2.1: the named laws are normalised by their analytic integral;
    Sect. 3.2.2: a callable may come with its normalising integral); it then
    stays fixed when the profile samples change."""

    def __init__(self, mu_s, I_s, zcut, nzin, nzlimb, ng, nk, k0, k1, istar=None):
        self.mu_s = np.asarray(mu_s, float)
        self.I_s = np.atleast_2d(np.asarray(I_s, float))
        self.zcut, self.nzin, self.nzlimb = zcut, nzin, nzlimb
        self.ng, self.nk, self.k0, self.k1 = ng, nk, k0, k1
        self.ze, self.zm, self.mu = z_grid(zcut, nzin, nzlimb)
        self.dk, self.dg, self.W = weights_3d(self.ze, nk, k0, k1, ng)
        self.ldp = profile_on_grid(self.mu_s, self.I_s, self.mu)
        self.istar_fixed = istar is not None
        self.istar = (np.broadcast_to(np.asarray(istar, float), (self.npb,)).copy()
                      if self.istar_fixed else istar_of_profile(self.mu_s, self.I_s))
        self.T = ld_tables(self.W, self.ldp)

    @property
    def npb(self):
        return self.I_s.shape[0]


# ---------------------------------------------------------------- step 6
def ldw_for_k(tab, pb, k):
    """k-interpolated LD-weighted vector over g for passband ``pb``
    (Sect. 3.1.2): u = (k - k0)/dk, ik = floor(u) clamped to nk-2,
    ldw = (1 - ak) T[ik] + ak T[ik+1]."""
    u = (k - tab.k0) / tab.dk
    ik = min(int(np.floor(u)), tab.nk - 2)
    ak = u - ik
    return (1.0 - ak) * tab.T[pb, ik] + ak * tab.T[pb, ik + 1]


# ---------------------------------------------------------------- step 7
def occulted(tab, pb, k, z, front):
    """delta = (w . l) a(z, k) / I_star for each separation (Eq. 5 without
    the leading 1), zero when the planet is behind the star or the disks do
    not overlap.  g-interpolation as in Sect. 3.1.1, index clamped to
    ng - 2."""
    return occulted_with(tab, ldw_for_k(tab, pb, k), pb, k, z, front)


def occulted_with(tab, ldw, pb, k, z, front):
    """``occulted`` for a given LD-weighted vector ldw over g."""
    z = np.asarray(z, float)
    delta = np.zeros(z.shape)
    hit = front & (z < 1.0 + k)
    if not hit.any():
        return delta
    zz = z[hit]
    v = (zz / (1.0 + k)) / tab.dg
    m = np.minimum(np.floor(v).astype(np.int64), tab.ng - 2)
    al = v - m
    ip = (1.0 - al) * ldw[m] + al * ldw[m + 1]
    ap = lens_area(1.0, k, zz)
    delta[hit] = ip * ap / tab.istar[pb]
    return delta


def flux_at_z(tab, pb, k, z):
    """Eq. 5 for separations z of a planet in front of the star."""
    z = np.asarray(z, float)
    return 1.0 - occulted(tab, pb, k, z, np.ones(z.shape, bool))


# ---------------------------------------------------------------- step 8
def pv_is_valid(row, tab):
    """Physical and in-table parameter vector (NaN row otherwise)."""
    t0, P, a, b, e, w = row[:NPAR_ORBIT]
    ks = row[NPAR_ORBIT:]
    if not np.all(np.isfinite(row)):
        return False
    if not (P > 0.0 and a > 0.0 and b >= 0.0 and 0.0 <= e < 1.0):
        return False
    if np.any(ks < tab.k0) or np.any(ks > tab.k1):
        return False
    return abs(_orbit.cos_inclination(a, b, e, w)) <= 1.0


def evaluate(tab, times, pv, lcids=None, pbids=None, nss=None, exptimes=None):
    """Fluxes out[npv][npt] for parameter rows pv[npv][6 + npb].

    Row layout: [t0, P, a, b, e, w, k_0 .. k_{npb-1}].  ``lcids`` maps each
    time to a light curve, ``pbids`` each light curve to a passband, and
    ``nss``/``exptimes`` give each light curve's supersampling (Sect. 4.2).
    Every subsample is solved in full; the exposure flux is the mean of the
    subsample fluxes.
    """
    times = np.asarray(times, float)
    pv = np.atleast_2d(np.asarray(pv, float))
    npt = times.size
    lcids = np.zeros(npt, np.int64) if lcids is None else np.asarray(lcids)
    if pbids is None:
        nlc = int(lcids.max()) + 1 if npt else 1
        pbids = np.zeros(nlc, np.int64)
    else:
        pbids = np.asarray(pbids)
        nlc = pbids.size
    nss = np.ones(nlc, np.int64) if nss is None else np.broadcast_to(nss, (nlc,))
    exptimes = (np.zeros(nlc) if exptimes is None
                else np.broadcast_to(np.asarray(exptimes, float), (nlc,)))
    out = np.empty((pv.shape[0], npt))
    for ipv, row in enumerate(pv):
        if not pv_is_valid(row, tab):
            out[ipv] = np.nan
            continue
        t0, P, a, b, e, w = row[:NPAR_ORBIT]
        for lc in range(nlc):
            sel = np.nonzero(lcids == lc)[0]
            if sel.size == 0:
                continue
            pb = int(pbids[lc])
            k = row[NPAR_ORBIT + pb]
            ts = _orbit.subsample_times(times[sel], int(nss[lc]), exptimes[lc])
            dt = _orbit.phase_offset(ts, t0, P)
            z, front, _ = _orbit.projected_separation(dt, P, a, b, e, w)
            out[ipv, sel] = 1.0 - occulted(tab, pb, k, z, front).mean(axis=1)
    return out


# ------------------------------------------------- per-vector limb darkening
def with_profile(tab, I_s):
    """The same grid and weight table for other profile samples I_s[npb][nmu]
    on the same mu samples: only the LD-dependent steps 2, 3 and 5 are
    redone (T = w . l is linear in the profile at the bin means, Sect. 3.1.2),
    W is shared."""
    t = object.__new__(Tables)
    t.__dict__.update(tab.__dict__)
    t.I_s = np.atleast_2d(np.asarray(I_s, float))
    if t.I_s.shape != tab.I_s.shape:
        raise ValueError("profile samples must have the tables' shape")
    t.ldp = profile_on_grid(t.mu_s, t.I_s, t.mu)
    if not getattr(t, "istar_fixed", False):
        t.istar = istar_of_profile(t.mu_s, t.I_s)
    t.T = ld_tables(t.W, t.ldp)
    return t


def evaluate_ld(tab, times, pv, prof, lcids=None, pbids=None, nss=None, exptimes=None):
    """Fluxes with a limb-darkening profile per parameter row (the model's LD
    coefficients given per evaluation, Sect. 4.2): row i is evaluated as in
    ``evaluate`` with the tables rebuilt for prof[i] ([npb][nmu] samples on
    the tables' mu samples)."""
    pv = np.atleast_2d(np.asarray(pv, float))
    prof = np.asarray(prof, float).reshape(pv.shape[0], tab.npb, tab.mu_s.size)
    out = np.empty((pv.shape[0], np.asarray(times).size))
    for i in range(pv.shape[0]):
        out[i] = evaluate(with_profile(tab, prof[i]), times, pv[i:i + 1], lcids=lcids,
                          pbids=pbids, nss=nss, exptimes=exptimes)[0]
    return out


# ------------------------------------------------------------ direct model
def weights_for_k(ze, k, ng):
    """The direct model's weights W[ng][nz] for one radius ratio k: the
    formula of ``weights_3d`` at that k alone, so no k-grid, no
    k-interpolation and no k limits (Sect. 3.1.1)."""
    nz = ze.size - 1
    g = np.arange(ng) / (ng - 1.0)
    c = g * (1.0 + k)
    A = lens_area(ze[None, :], k, c[:, None])
    total = A[:, -1]
    W = np.zeros((ng, nz))
    ok = total > 0.0
    W[ok] = np.diff(A, axis=-1)[ok] / total[ok][:, None]
    W[~ok, nz - 1] = 1.0
    return W


def pv_is_valid_direct(row):
    """Physical parameter vector for the direct model: any k in (0, 1]."""
    ks = row[NPAR_ORBIT:]
    if not np.all(np.isfinite(row)):
        return False
    t0, P, a, b, e, w = row[:NPAR_ORBIT]
    if not (P > 0.0 and a > 0.0 and b >= 0.0 and 0.0 <= e < 1.0):
        return False
    if np.any(ks <= 0.0) or np.any(ks > 1.0):
        return False
    return abs(_orbit.cos_inclination(a, b, e, w)) <= 1.0


def evaluate_direct(tab, times, pv, lcids=None, pbids=None, nss=None, exptimes=None):
    """Fluxes of the direct model (Sect. 3.1.1): as ``evaluate``, but each
    row's LD-weighted vector comes from weights built for its own k
    (``weights_for_k``) and the tables' profile at the bin means, with no
    interpolation in k."""
    times = np.asarray(times, float)
    pv = np.atleast_2d(np.asarray(pv, float))
    npt = times.size
    lcids = np.zeros(npt, np.int64) if lcids is None else np.asarray(lcids)
    if pbids is None:
        nlc = int(lcids.max()) + 1 if npt else 1
        pbids = np.zeros(nlc, np.int64)
    else:
        pbids = np.asarray(pbids)
        nlc = pbids.size
    nss = np.ones(nlc, np.int64) if nss is None else np.broadcast_to(nss, (nlc,))
    exptimes = (np.zeros(nlc) if exptimes is None
                else np.broadcast_to(np.asarray(exptimes, float), (nlc,)))
    out = np.empty((pv.shape[0], npt))
    for ipv, row in enumerate(pv):
        if not pv_is_valid_direct(row):
            out[ipv] = np.nan
            continue
        t0, P, a, b, e, w = row[:NPAR_ORBIT]
        for lc in range(nlc):
            sel = np.nonzero(lcids == lc)[0]
            if sel.size == 0:
                continue
            pb = int(pbids[lc])
            k = row[NPAR_ORBIT + pb]
            ldw = weights_for_k(tab.ze, k, tab.ng) @ tab.ldp[pb]
            ts = _orbit.subsample_times(times[sel], int(nss[lc]), exptimes[lc])
            dt = _orbit.phase_offset(ts, t0, P)
            z, front, _ = _orbit.projected_separation(dt, P, a, b, e, w)
            out[ipv, sel] = 1.0 - occulted_with(tab, ldw, pb, k, z, front).mean(axis=1)
    return out


# ---------------------------------------------------------------- Sect. 3.4.2
def small_planet_ldw(tab, pb, k):
    """Small-planet approximation (Sect. 3.4.2) as an LD vector over g: at
    each g node the LD-weighted mean over the planet's disk is replaced by
    the profile at the planet's centre, c = g (1 + k), i.e. the interpolant
    of the samples at mu = sqrt(1 - c^2).  A centre off the disk (c > 1,
    limb overlap only) takes the limb value I(mu = 0).  The g-interpolation
    of ``occulted_with`` is then applied unchanged."""
    g = np.arange(tab.ng) / (tab.ng - 1.0)
    c = np.minimum(g * (1.0 + k), 1.0)
    return np.interp(np.sqrt(1.0 - c * c), tab.mu_s, tab.I_s[pb])


def pv_is_valid_small_planet(row, tab, k_small):
    """Physical parameter vector where every k is either below the
    small-planet threshold (and positive) or inside the table's [k0, k1]."""
    ks = row[NPAR_ORBIT:]
    if not np.all(np.isfinite(row)):
        return False
    t0, P, a, b, e, w = row[:NPAR_ORBIT]
    if not (P > 0.0 and a > 0.0 and b >= 0.0 and 0.0 <= e < 1.0):
        return False
    for k in ks:
        if k < k_small:
            if not k > 0.0:
                return False
        elif k < tab.k0 or k > tab.k1:
            return False
    return abs(_orbit.cos_inclination(a, b, e, w)) <= 1.0


def evaluate_small_planet(tab, times, pv, k_small, lcids=None, pbids=None, nss=None,
                          exptimes=None):
    """Fluxes as ``evaluate``, except that a passband whose radius ratio is
    below ``k_small`` uses ``small_planet_ldw`` instead of the table
    interpolated in k (Sect. 3.4.2); such a k may lie below the table's k0.
    I_star is the same normaliser in both cases."""
    times = np.asarray(times, float)
    pv = np.atleast_2d(np.asarray(pv, float))
    npt = times.size
    lcids = np.zeros(npt, np.int64) if lcids is None else np.asarray(lcids)
    if pbids is None:
        nlc = int(lcids.max()) + 1 if npt else 1
        pbids = np.zeros(nlc, np.int64)
    else:
        pbids = np.asarray(pbids)
        nlc = pbids.size
    nss = np.ones(nlc, np.int64) if nss is None else np.broadcast_to(nss, (nlc,))
    exptimes = (np.zeros(nlc) if exptimes is None
                else np.broadcast_to(np.asarray(exptimes, float), (nlc,)))
    out = np.empty((pv.shape[0], npt))
    for ipv, row in enumerate(pv):
        if not pv_is_valid_small_planet(row, tab, k_small):
            out[ipv] = np.nan
            continue
        t0, P, a, b, e, w = row[:NPAR_ORBIT]
        for lc in range(nlc):
            sel = np.nonzero(lcids == lc)[0]
            if sel.size == 0:
                continue
            pb = int(pbids[lc])
            k = row[NPAR_ORBIT + pb]
            ldw = small_planet_ldw(tab, pb, k) if k < k_small else ldw_for_k(tab, pb, k)
            ts = _orbit.subsample_times(times[sel], int(nss[lc]), exptimes[lc])
            dt = _orbit.phase_offset(ts, t0, P)
            z, front, _ = _orbit.projected_separation(dt, P, a, b, e, w)
            out[ipv, sel] = 1.0 - occulted_with(tab, ldw, pb, k, z, front).mean(axis=1)
    return out
