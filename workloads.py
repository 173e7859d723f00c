"""Seeded synthetic inputs for the RoadRunner light-curve workloads.

This module only draws inputs: times, light-curve/passband maps,
supersampling settings, parameter vectors and radial limb-darkening profiles
sampled on a mu grid.  It contains none of the transit model's arithmetic and
is shared by the tests, the benchmark and the smoke check, which pass the
same arrays to the HIP library and to the CPU oracle.

The shapes follow the paper's use cases: light curves at TESS-like 2-min and
Kepler-like 30-min cadences over ~27-d sectors (Sect. 4.1, supersampling of
long-cadence data), populations of parameter vectors as in MCMC sampling
(Sect. 3.4.4, Sect. 4.1), heterogeneous multi-passband time series
(Sect. 4.2).  No mission data are used; every array is synthetic.

Parameter-vector row layout: [t0, P, a, b, e, w, k_0 .. k_{npb-1}] with
t0, P in days, a in stellar radii, b the conjunction impact parameter, w in
radians and k_pb the radius ratio in passband pb.
"""

import numpy as np

SEED_BASE = 2009085000
MINUTE = 1.0 / 1440.0

# Table resolution used by default (z-grid cut, inner and limb bin counts,
# g and k node counts, k range).
DEFAULT_GRID = dict(zcut=0.8, nzin=60, nzlimb=120, ng=512, nk=256,
                    k0=0.01, k1=0.30)
# Small grid for tests where the oracle must build the tables quickly.
TEST_GRID = dict(zcut=0.7, nzin=20, nzlimb=30, ng=96, nk=24, k0=0.01, k1=0.30)


def rng_for(config, extra=0):
    return np.random.default_rng(SEED_BASE + 100 * extra + config)


# ------------------------------------------------------------ LD profiles
def profile_quadratic(mu, u1, u2):
    return 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2


def profile_power2(mu, c, alpha):
    return 1.0 - c * (1.0 - mu ** alpha)


def profile_power2_quadratic(mu, c, alpha, d):
    """Smooth profile decreasing to the limb (power-2 plus a quadratic term)."""
    return 1.0 - c * (1.0 - mu ** alpha) - d * (1.0 - mu) ** 2


# ------------------------------------------------------------ orbits
def draw_orbits(rng, npv, npb=1, chromatic=0.0):
    """Parameter rows drawn as in the population workload:
    k ~ U(0.05, 0.2), a ~ U(5, 20), b ~ U(0, 0.9), e ~ U(0, 0.3),
    w ~ U(0, 2 pi), P ~ U(1, 10) d, t0 ~ U(0, P); per-passband
    k_pb = k (1 + U(-chromatic, chromatic))."""
    k = rng.uniform(0.05, 0.2, npv)
    a = rng.uniform(5.0, 20.0, npv)
    b = rng.uniform(0.0, 0.9, npv)
    e = rng.uniform(0.0, 0.3, npv)
    w = rng.uniform(0.0, 2.0 * np.pi, npv)
    P = rng.uniform(1.0, 10.0, npv)
    t0 = rng.uniform(0.0, 1.0, npv) * P
    pv = np.empty((npv, 6 + npb))
    pv[:, 0], pv[:, 1], pv[:, 2], pv[:, 3], pv[:, 4], pv[:, 5] = t0, P, a, b, e, w
    for pb in range(npb):
        pv[:, 6 + pb] = k * (1.0 + rng.uniform(-chromatic, chromatic, npv)) \
            if chromatic > 0.0 else k
    return pv


def _workload(times, pv, mu_s, I_s, lcids=None, pbids=None, nss=None,
              exptimes=None, name=""):
    times = np.ascontiguousarray(times, dtype=np.float64)
    nlc = 1 if pbids is None else len(pbids)
    return dict(
        name=name,
        times=times,
        lcids=(np.zeros(times.size, np.int32) if lcids is None
               else np.ascontiguousarray(lcids, dtype=np.int32)),
        pbids=(np.zeros(nlc, np.int32) if pbids is None
               else np.ascontiguousarray(pbids, dtype=np.int32)),
        nss=(np.ones(nlc, np.int32) if nss is None
             else np.ascontiguousarray(nss, dtype=np.int32)),
        exptimes=(np.zeros(nlc) if exptimes is None
                  else np.ascontiguousarray(exptimes, dtype=np.float64)),
        pv=np.ascontiguousarray(pv, dtype=np.float64),
        mu_s=np.ascontiguousarray(mu_s, dtype=np.float64),
        I_s=np.ascontiguousarray(np.atleast_2d(I_s), dtype=np.float64),
    )


# ------------------------------------------------------------ configurations
def single_light_curve():
    """One circular-orbit light curve: P = 3 d, a = 8, b = 0.3, k = 0.1,
    t0 = 0; quadratic LD (0.4, 0.25) sampled at 100 mu points; 1000 times
    uniform in [-0.2, 0.2] d; no supersampling."""
    mu = np.linspace(0.0, 1.0, 100)
    pv = np.array([[0.0, 3.0, 8.0, 0.3, 0.0, 0.0, 0.1]])
    return _workload(np.linspace(-0.2, 0.2, 1000), pv, mu,
                     profile_quadratic(mu, 0.4, 0.25), name="single_lc_fp64")


def population(npv=512, npt=20000, seed_extra=0):
    """Population evaluation: npv parameter vectors (see ``draw_orbits``),
    one power-2 profile with c ~ U(0.5, 0.8), alpha ~ U(0.4, 0.8) at 200 mu,
    npt times at 2-min cadence from t = 0; no supersampling."""
    rng = rng_for(2, seed_extra)
    pv = draw_orbits(rng, npv)
    c, alpha = rng.uniform(0.5, 0.8), rng.uniform(0.4, 0.8)
    mu = np.linspace(0.0, 1.0, 200)
    times = np.arange(npt) * (2.0 * MINUTE)
    return _workload(times, pv, mu, profile_power2(mu, c, alpha),
                     name=f"population_npv{npv}_npt{npt}")


def population_ld(npv=512, npt=20000, seed_extra=0):
    """Population evaluation with a profile per parameter vector (LD sampled
    with the orbit): the orbits, times and mu samples of ``population``, and
    for every vector its own power-2 profile with c ~ U(0.5, 0.8),
    alpha ~ U(0.4, 0.8) at 200 mu.  ``prof_pv`` is (npv, 1, 200); the shared
    ``I_s`` (the tables' own profile) is the population's."""
    w = population(npv, npt, seed_extra)
    rng = rng_for(6, seed_extra)
    c = rng.uniform(0.5, 0.8, npv)
    alpha = rng.uniform(0.4, 0.8, npv)
    w["prof_pv"] = np.stack([profile_power2(w["mu_s"], c[i], alpha[i])
                             for i in range(npv)])[:, None, :]
    w["ld_c_pv"], w["ld_alpha_pv"] = c, alpha
    w["name"] = f"population_ld_npv{npv}_npt{npt}"
    return w


def population_small(npv=512, npt=20000, seed_extra=0, k_lo=0.003, k_hi=0.03):
    """Population with small planets: the orbits, profile and times of
    ``population`` with k ~ logU(k_lo, k_hi), so that about half the vectors
    fall below a small-planet threshold of 0.01 (Earth- to Neptune-size
    planets around a Sun-like star)."""
    w = population(npv, npt, seed_extra)
    rng = rng_for(7, seed_extra)
    w["pv"][:, 6] = np.exp(rng.uniform(np.log(k_lo), np.log(k_hi), npv))
    w["name"] = f"population_small_npv{npv}_npt{npt}"
    return w


def heterogeneous(npv=256, days=27.0, seed_extra=0):
    """Four passbands with their own profiles and chromatic k; two 30-min
    light curves with nss = 10 and two 2-min light curves with nss = 1, all
    spanning ``days``."""
    rng = rng_for(3, seed_extra)
    mu = np.linspace(0.0, 1.0, 200)
    I_s = np.stack([profile_power2_quadratic(mu, rng.uniform(0.3, 0.6),
                                             rng.uniform(0.4, 0.8),
                                             rng.uniform(0.0, 0.2))
                    for _ in range(4)])
    n_long = int(round(days / (30.0 * MINUTE)))
    n_short = int(round(days / (2.0 * MINUTE)))
    t_long = np.arange(n_long) * (30.0 * MINUTE)
    t_short = np.arange(n_short) * (2.0 * MINUTE)
    times = np.concatenate([t_long, t_long, t_short, t_short])
    lcids = np.concatenate([np.full(n_long, 0), np.full(n_long, 1),
                            np.full(n_short, 2), np.full(n_short, 3)])
    pv = draw_orbits(rng, npv, npb=4, chromatic=0.05)
    return _workload(times, pv, mu, I_s, lcids=lcids, pbids=[0, 1, 2, 3],
                     nss=[10, 10, 1, 1],
                     exptimes=[30.0 * MINUTE, 30.0 * MINUTE, 2 * MINUTE,
                               2 * MINUTE],
                     name=f"heterogeneous_npv{npv}")


def serving_mix(nreq, nseries=12, seed_extra=0, max_npv=2048, max_npt=100000,
                min_npt=1000):
    """Request mix for the serving loop.  ``nseries`` resident time series,
    each with npt ~ logU(min_npt, max_npt), nss in {1, 5, 10} and npb in
    {1..4} passbands (the resident passbands 0..npb-1), its times split
    evenly into one 2-min-cadence light curve per passband with
    exptime = cadence.  ``nreq`` requests, each picking a series at random
    with npv ~ logU(1, max_npv) parameter rows drawn as in ``population``
    (chromatic k within 5 %).  Returns (series, requests)."""
    rng = rng_for(4, seed_extra)
    series = []
    for _ in range(nseries):
        npt = int(np.exp(rng.uniform(np.log(min_npt), np.log(max_npt))))
        nss = int(rng.choice([1, 5, 10]))
        npb = int(rng.integers(1, 5))
        per = max(1, npt // npb)
        times = np.concatenate([np.arange(per) * (2.0 * MINUTE) for _ in range(npb)])
        lcids = np.repeat(np.arange(npb), per).astype(np.int32)
        series.append(dict(times=times, lcids=lcids, pbids=np.arange(npb, dtype=np.int32),
                           nss=np.full(npb, nss, np.int32),
                           exptimes=np.full(npb, 2.0 * MINUTE), npb=npb))
    reqs = []
    for _ in range(nreq):
        sid = int(rng.integers(0, nseries))
        npv = int(np.exp(rng.uniform(0.0, np.log(max_npv))))
        pv = draw_orbits(rng, npv, npb=4, chromatic=0.05)
        reqs.append(dict(series=sid, pv=pv))
    return series, reqs


def serving_stream(nreq, seed_extra=0, max_npv=2048, max_npt=100000, min_npt=1000):
    """Request stream for the serving protocol: every request has its own
    time series, with npt ~ logU(min_npt, max_npt), nss in {1, 5, 10} and
    npb in {1..4} (the resident passbands 0..npb-1), its times split evenly
    into one 2-min-cadence light curve per passband with exptime = cadence,
    and npv ~ logU(1, max_npv) parameter rows drawn as in ``population``
    (chromatic k within 5 %).  Returns (series, requests) with request i on
    series i."""
    rng = rng_for(8, seed_extra)
    series, reqs = [], []
    for i in range(nreq):
        npt = int(np.exp(rng.uniform(np.log(min_npt), np.log(max_npt))))
        nss = int(rng.choice([1, 5, 10]))
        npb = int(rng.integers(1, 5))
        per = max(1, npt // npb)
        times = np.concatenate([np.arange(per) * (2.0 * MINUTE) for _ in range(npb)])
        lcids = np.repeat(np.arange(npb), per).astype(np.int32)
        series.append(dict(times=times, lcids=lcids, pbids=np.arange(npb, dtype=np.int32),
                           nss=np.full(npb, nss, np.int32),
                           exptimes=np.full(npb, 2.0 * MINUTE), npb=npb))
        npv = int(np.exp(rng.uniform(0.0, np.log(max_npv))))
        reqs.append(dict(series=i, pv=draw_orbits(rng, npv, npb=4, chromatic=0.05)))
    return series, reqs


def loglik_walkers(npv=1024, npt=50000, nss=5, seed_extra=0):
    """Walkers around a truth vector for the log-likelihood workload:
    the truth is drawn as in ``population``; walkers are the truth plus
    small seeded perturbations, so all of them transit.  Times at 2-min
    cadence, supersampled nss times over a 2-min exposure.  Also returns
    seeded Gaussian noise (sigma = 200 ppm) for the synthetic data and the
    power-2 LD coefficients."""
    rng = rng_for(5, seed_extra)
    truth = draw_orbits(rng, 1)[0]
    c, alpha = rng.uniform(0.5, 0.8), rng.uniform(0.4, 0.8)
    pv = np.repeat(truth[None, :], npv, axis=0)
    n = rng.standard_normal((npv, 7))
    pv[:, 0] += 1e-4 * truth[1] * n[:, 0]
    pv[:, 1] *= 1.0 + 1e-6 * n[:, 1]
    pv[:, 2] *= 1.0 + 1e-3 * n[:, 2]
    pv[:, 3] = np.abs(pv[:, 3] + 1e-3 * n[:, 3])
    pv[:, 4] = np.abs(pv[:, 4] + 1e-3 * n[:, 4])
    pv[:, 5] += 1e-3 * n[:, 5]
    pv[:, 6] *= 1.0 + 1e-3 * n[:, 6]
    times = np.arange(npt) * (2.0 * MINUTE)
    sigma = 200e-6
    noise = sigma * rng.standard_normal(npt)
    mu = np.linspace(0.0, 1.0, 200)
    wl = _workload(times, pv, mu, profile_power2(mu, c, alpha),
                   nss=[nss], exptimes=[2.0 * MINUTE],
                   name=f"loglik_npv{npv}_npt{npt}_nss{nss}")
    wl.update(truth=truth, noise=noise, sigma=sigma, ld_c=c, ld_alpha=alpha)
    return wl
