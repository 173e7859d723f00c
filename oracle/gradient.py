"""Gradient of the Gaussian log-likelihood of Oracle-A light curves, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

logL(pv) = -1/2 sum_t ((d_t - F_t)/sigma)^2 (constant dropped), with F_t the
Oracle-A flux (supersampled mean of Eq. 5 over the exposure).  The gradient
with respect to every entry of the parameter row [t0, P, a, b, e, w, k_pb]
and to the tabulated LD profile samples is written out by the chain rule
through each step of the model, in the model's own order:

  phase   dt = x - P round(x/P), x = t_s - t0; M = M_tr(e, w) + (2 pi/P) dt
          dM/dt0 = -2 pi/P, dM/dP = -2 pi x / P^2 (round() is locally
          constant), dM/de = dM_tr/de, dM/dw = dM_tr/dw;
  Kepler  E - e sin E = M: dE/dM = 1/(1 - e cos E), dE/de|_M = sin E/(1 - e cos E);
  orbit   X = -a[(cos E - e) cos w - q sin E sin w],
          rho = a[(cos E - e) sin w + q sin E cos w] (= r sin(w+f)),
          Y = -rho cos i, z = sqrt(X^2 + Y^2), q = sqrt(1 - e^2),
          cos i = b (1 + e sin w)/(a (1 - e^2));
  area    da/dz = -(chord length), da/dk = 2 k kappa_0 (the planet's arc
          inside the star);
  tables  ip = (1-alpha) ldw[m] + alpha ldw[m+1], ldw = (1-ak) T[ik] + ak T[ik+1],
          dip/dz through g = z/(1+k), dip/dk through g and ak;
  Eq. 5   delta = ip a / I_star, F = 1 - mean_s delta.
Profile samples enter only through T = W . ldp (ldp = R I_s, linear
interpolation) and I_star = q . I_s; both maps are linear, so their
transposes carry the gradient back (R and q are built by applying the
forward maps to unit vectors).

``finite_difference`` provides the central-difference check.
"""

import numpy as np

from . import orbit as _orbit
from . import roadrunner as _rr


def _lens_parts(k, z):
    """(area, d area/dz, d area/dk) of a(z, k) (unit star), elementwise."""
    k = np.broadcast_to(np.asarray(k, float), np.shape(z))
    A = _rr.lens_area(1.0, k, z)
    Az = np.zeros(np.shape(z))
    Ak = np.zeros(np.shape(z))
    inside = z <= np.abs(1.0 - k)
    Ak[inside] = 2.0 * np.pi * k[inside]
    part = (~inside) & (z < 1.0 + k)
    zp, kp = z[part], k[part]
    rad = (-zp + 1 + kp) * (zp + 1 - kp) * (zp - 1 + kp) * (zp + 1 + kp)
    h = np.sqrt(np.maximum(rad, 0.0)) / (2.0 * zp)
    kap0 = np.arccos(np.clip((zp * zp + kp * kp - 1.0) / (2.0 * zp * kp), -1.0, 1.0))
    Az[part] = -2.0 * h
    Ak[part] = 2.0 * kp * kap0
    return A, Az, Ak


def profile_maps(tab):
    """R[nz][nmu] (profile samples -> values at the bin means) and q[nmu]
    (samples -> I_star), by applying the forward maps to unit vectors."""
    nmu = tab.mu_s.size
    eye = np.eye(nmu)
    R = np.stack([np.interp(tab.mu, tab.mu_s, eye[s]) for s in range(nmu)], axis=1)
    q = _rr.istar_of_profile(tab.mu_s, eye)
    return R, q


def _pv_terms(tab, row, ts, pb):
    """Per-subsample delta and its derivatives for one parameter row.
    Returns delta, ddelta/dtheta for theta in (t0, P, a, b, e, w, k), and
    the table-gradient pieces (hit mask, ik, ak, m, alpha, A)."""
    t0, P, a, b, e, w = row[:6]
    k = row[6 + pb]
    sw, cw = np.sin(w), np.cos(w)
    q = np.sqrt(1.0 - e * e)
    ci = _orbit.cos_inclination(a, b, e, w)
    # conjunction (f_tr = pi/2 - w)
    den = 1.0 + e * sw
    cEt, sEt = (e + sw) / den, q * cw / den
    Mtr = _orbit.conjunction_mean_anomaly(e, w)
    dEtr_dw = -(1.0 - e * cEt) / q
    dEtr_de = -cw / (den * q)
    dMtr_dw = (1.0 - e * cEt) * dEtr_dw
    dMtr_de = (1.0 - e * cEt) * dEtr_de - sEt
    # phase and Kepler
    n = 2.0 * np.pi / P
    x = ts - t0
    dt = _orbit.phase_offset(ts, t0, P)
    M = Mtr + n * dt
    E = M if e == 0.0 else _orbit.solve_kepler(M, e)
    cE, sE = np.cos(E), np.sin(E)
    iE = 1.0 / (1.0 - e * cE)
    dE = {"t0": -n * iE, "P": -n * (x / P) * iE, "e": (dMtr_de + sE) * iE,
          "w": dMtr_dw * iE, "a": 0.0, "b": 0.0}
    X = -a * ((cE - e) * cw - q * sE * sw)
    rho = a * ((cE - e) * sw + q * sE * cw)
    Y = -rho * ci
    z = np.sqrt(X * X + Y * Y)
    X_E = a * (sE * cw + q * cE * sw)
    rho_E = a * (q * cE * cw - sE * sw)
    dq = -e / q
    X_e = a * (cw + dq * sE * sw)
    rho_e = a * (dq * sE * cw - sw)
    dci = {"a": -ci / a, "b": (1.0 + e * sw) / (a * (1.0 - e * e)),
           "e": b / a * (sw * (1.0 - e * e) + 2.0 * e * den) / (1.0 - e * e) ** 2,
           "w": b * e * cw / (a * (1.0 - e * e)), "t0": 0.0, "P": 0.0}
    dz = {}
    for th in ("t0", "P", "a", "b", "e", "w"):
        dX = X_E * dE[th]
        drho = rho_E * dE[th]
        if th == "a":
            dX = dX + X / a
            drho = drho + rho / a
        elif th == "e":
            dX = dX + X_e
            drho = drho + rho_e
        elif th == "w":
            dX = dX + rho
            drho = drho - X
        dY = -ci * drho - rho * dci[th]
        dz[th] = (X * dX + Y * dY) / z
    # occultation
    hit = (rho > 0.0) & (z < 1.0 + k)
    delta = np.zeros(z.shape)
    dd = {th: np.zeros(z.shape) for th in ("t0", "P", "a", "b", "e", "w", "k")}
    u = (k - tab.k0) / tab.dk
    ik = min(int(np.floor(u)), tab.nk - 2)
    ak = u - ik
    T0, T1 = tab.T[pb, ik], tab.T[pb, ik + 1]
    ldw = (1.0 - ak) * T0 + ak * T1
    zz = z[hit]
    g = zz / (1.0 + k)
    v = g / tab.dg
    m = np.minimum(np.floor(v).astype(np.int64), tab.ng - 2)
    al = v - m
    ip = (1.0 - al) * ldw[m] + al * ldw[m + 1]
    slope = (ldw[m + 1] - ldw[m]) / tab.dg
    ip_z = slope / (1.0 + k)
    ip_k = slope * (-zz / (1.0 + k) ** 2) + \
        ((1.0 - al) * (T1[m] - T0[m]) + al * (T1[m + 1] - T0[m + 1])) / tab.dk
    A, Az, Ak = _lens_parts(k, zz)
    ist = tab.istar[pb]
    delta[hit] = ip * A / ist
    dz_del = (ip_z * A + ip * Az) / ist
    for th in ("t0", "P", "a", "b", "e", "w"):
        dd[th][hit] = dz_del * dz[th][hit]
    dd["k"][hit] = (ip_k * A + ip * Ak) / ist
    return delta, dd, (hit, ik, ak, m, al, A)


def loglik_grad(tab, times, pv, obs, sigma, lcids=None, pbids=None, nss=None,
                exptimes=None, want_profile=True, want_istar=False):
    """(logL[npv], grad[npv][npar], grad_profile[npb][nmu] or None), and with
    ``want_istar`` a fourth entry: d(sum_pv logL)/d I_star[npb].

    grad_profile is the gradient of sum_pv logL with respect to the profile
    samples I_s of the tables, through I_star as well unless the tables hold
    a fixed normaliser (``Tables(..., istar=...)``).  Invalid rows give NaN
    logL and gradients and do not contribute to grad_profile."""
    times = np.asarray(times, float)
    obs = np.asarray(obs, float)
    pv = np.atleast_2d(np.asarray(pv, float))
    npv, npar = pv.shape
    npt = times.size
    lcids = np.zeros(npt, np.int64) if lcids is None else np.asarray(lcids)
    if pbids is None:
        pbids = np.zeros(int(lcids.max()) + 1 if npt else 1, np.int64)
    pbids = np.asarray(pbids)
    nlc = pbids.size
    nss = np.ones(nlc, np.int64) if nss is None else np.broadcast_to(nss, (nlc,))
    exptimes = (np.zeros(nlc) if exptimes is None
                else np.broadcast_to(np.asarray(exptimes, float), (nlc,)))
    logl = np.zeros(npv)
    grad = np.zeros((npv, npar))
    GT = np.zeros_like(tab.T)
    Gist = np.zeros(tab.npb)
    names = ("t0", "P", "a", "b", "e", "w")
    for ipv, row in enumerate(pv):
        if not _rr.pv_is_valid(row, tab):
            logl[ipv] = np.nan
            grad[ipv] = np.nan
            continue
        for lc in range(nlc):
            sel = np.nonzero(lcids == lc)[0]
            if sel.size == 0:
                continue
            pb = int(pbids[lc])
            ns = int(nss[lc])
            ts = _orbit.subsample_times(times[sel], ns, exptimes[lc])
            delta, dd, (hit, ik, ak, m, al, A) = _pv_terms(tab, row, ts, pb)
            F = 1.0 - delta.mean(axis=1)
            r = obs[sel] - F
            psi = r / sigma ** 2                       # dlogL/dF
            logl[ipv] += -0.5 * np.sum((r / sigma) ** 2)
            wgt = (-psi / ns)[:, None]                 # dlogL/ddelta per subsample
            for j, th in enumerate(names):
                grad[ipv, j] += np.sum(wgt * dd[th])
            grad[ipv, 6 + pb] += np.sum(wgt * dd["k"])
            if want_profile:
                c = np.broadcast_to(wgt, delta.shape)[hit] * A / tab.istar[pb]
                np.add.at(GT[pb, ik], m, (1 - ak) * (1 - al) * c)
                np.add.at(GT[pb, ik], m + 1, (1 - ak) * al * c)
                np.add.at(GT[pb, ik + 1], m, ak * (1 - al) * c)
                np.add.at(GT[pb, ik + 1], m + 1, ak * al * c)
                Gist[pb] += np.sum(wgt * (-delta / tab.istar[pb]))
    gprof = None
    if want_profile:
        R, q = profile_maps(tab)
        Gldp = np.einsum("imj,pim->pj", tab.W, GT)
        gprof = Gldp @ R
        if not getattr(tab, "istar_fixed", False):
            gprof = gprof + Gist[:, None] * q[None, :]
    if want_istar:
        return logl, grad, gprof, (Gist if want_profile else None)
    return logl, grad, gprof


def finite_difference(fun, x, h):
    """Central differences of a scalar function along each coordinate of x
    with per-coordinate steps h."""
    x = np.asarray(x, float)
    h = np.broadcast_to(np.asarray(h, float), x.shape)
    g = np.zeros(x.shape)
    for i in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[i] += h[i]
        xm[i] -= h[i]
        g[i] = (fun(xp) - fun(xm)) / (2.0 * h[i])
    return g
