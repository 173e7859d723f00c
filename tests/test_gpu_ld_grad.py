"""GPU parity of the log-likelihood with a profile per parameter vector
(rr_loglik_grad_ld) against the oracle: each row's logL, parameter gradient
and gradient with respect to its own profile equal the oracle's analytic
gradient for tables rebuilt with that row's profile (which the oracle's own
pins tie to central differences).  Tolerances as the shared-profile adjoint
tests: FP64 1e-11 (logL) and 1e-7 of each row's largest component; mixed
1e-6 and 2e-4."""

import numpy as np
import pytest

import workloads as wl
from oracle import gradient as ogr
from oracle import roadrunner as orr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_08500_amd as rr
    return rr


def make(npv=6, npt=4000, nss=2, span=15.0):
    w = wl.loglik_walkers(npv=npv, npt=npt, nss=nss)
    w["times"] = np.linspace(0.0, span, npt)
    grid = wl.TEST_GRID
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    obs = orr.evaluate(otab, w["times"], w["truth"][None, :], nss=w["nss"],
                       exptimes=w["exptimes"])[0] + w["noise"]
    rng = np.random.default_rng(21)
    c = rng.uniform(0.4, 0.8, npv)
    al = rng.uniform(0.4, 0.8, npv)
    prof = (1.0 - c[:, None] * (1.0 - w["mu_s"][None, :] ** al[:, None]))[:, None, :]
    return w, grid, otab, obs, prof


def rowwise_close(a, b, rel):
    scale = np.abs(b).max(axis=-1, keepdims=True)
    assert np.all(np.abs(a - b) <= rel * scale), np.max(np.abs(a - b) / scale)


@pytest.mark.parametrize("precision,rel_ll,rel_g", [("fp64", 1e-11, 1e-7), ("mixed", 1e-6, 2e-4)])
def test_per_row_profile_gradients_match_oracle(rr, precision, rel_ll, rel_g):
    w, grid, otab, obs, prof = make()
    pv = w["pv"].copy()
    pv[3, 4] = 1.5                                   # invalid row
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    ll, g, gp = [x.cpu().numpy() for x in rr.loglik_grad_ld(tab, ser, pv, prof, obs, w["sigma"],
                                                            precision)]
    o = obs.astype(np.float32).astype(np.float64) if precision == "mixed" else obs
    assert np.isnan(ll[3]) and np.isnan(g[3]).all() and np.all(gp[3] == 0.0)
    for i in (0, 1, 2, 4, 5):
        oll, og, ogp = ogr.loglik_grad(orr.with_profile(otab, prof[i]), w["times"], pv[i:i + 1],
                                       o, w["sigma"], nss=w["nss"], exptimes=w["exptimes"])
        np.testing.assert_allclose(ll[i], oll[0], rtol=rel_ll)
        rowwise_close(g[i:i + 1], og, rel_g)
        rowwise_close(gp[i], ogp, rel_g)


def test_own_profile_reduces_to_shared(rr):
    w, grid, otab, obs, _ = make(npv=12, npt=6000)
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    prof = np.broadcast_to(w["I_s"], (12,) + w["I_s"].shape).copy()
    a = [x.cpu().numpy() for x in rr.loglik_grad_ld(tab, ser, w["pv"], prof, obs, w["sigma"],
                                                    "fp64")]
    b = [x.cpu().numpy() for x in rr.loglik_grad(tab, ser, w["pv"], obs, w["sigma"], "fp64",
                                                 grad=True, profile=True)]
    np.testing.assert_allclose(a[0], b[0], rtol=1e-12)
    rowwise_close(a[1], b[1], 1e-10)
    rowwise_close(a[2].sum(axis=0), b[2], 1e-10)


def test_autograd_through_per_row_coefficients(rr):
    """RRLogLikLD inside torch autograd, with per-row power-2 coefficients
    generating the profiles in torch: the gradient of sum logL with respect
    to each row's (c, alpha) against central differences of the GPU
    log-likelihood."""
    import torch
    w, grid, otab, obs, _ = make(npv=4, npt=3000)
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    mu = torch.tensor(w["mu_s"], device="cuda")
    coef = torch.tensor([[0.6, 0.5], [0.55, 0.7], [0.7, 0.45], [0.5, 0.6]], device="cuda",
                        dtype=torch.float64, requires_grad=True)
    pv = torch.tensor(w["pv"], device="cuda")
    obs_t = torch.tensor(obs, device="cuda")

    def loss(cf):
        prof = rr.ldlaws.profile("power-2", mu, cf)[:, None, :]
        return rr.RRLogLikLD.apply(pv, prof, tab, ser, obs_t, w["sigma"], "fp64").sum()

    L = loss(coef)
    L.backward()
    h = 1e-6
    for i in range(4):
        for q in range(2):
            cp = coef.detach().clone()
            cm = coef.detach().clone()
            cp[i, q] += h
            cm[i, q] -= h
            fd = (loss(cp).item() - loss(cm).item()) / (2 * h)
            assert coef.grad[i, q].item() == pytest.approx(fd, rel=2e-5, abs=1e-3)


def test_per_row_profiles_four_passbands(rr):
    """Four passbands, supersampled light curves, each row with four
    profiles of its own: logL, parameter gradients and every row's profile
    gradient against the oracle (FP64)."""
    w = wl.heterogeneous(npv=5, days=4.0)
    kw = dict(lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"], exptimes=w["exptimes"])
    grid = wl.TEST_GRID
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    obs = orr.evaluate(otab, w["times"], w["pv"][:1], **kw)[0] + \
        200e-6 * np.random.default_rng(8).standard_normal(w["times"].size)
    rng = np.random.default_rng(9)
    c = rng.uniform(0.3, 0.7, (5, 4))
    al = rng.uniform(0.4, 0.8, (5, 4))
    prof = 1.0 - c[..., None] * (1.0 - w["mu_s"][None, None, :] ** al[..., None])
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], w["lcids"], w["pbids"], w["nss"], w["exptimes"])
    ll, g, gp = [x.cpu().numpy() for x in rr.loglik_grad_ld(tab, ser, w["pv"], prof, obs, 2e-4,
                                                            "fp64")]
    for i in range(5):
        oll, og, ogp = ogr.loglik_grad(orr.with_profile(otab, prof[i]), w["times"],
                                       w["pv"][i:i + 1], obs, 2e-4, **kw)
        np.testing.assert_allclose(ll[i], oll[0], rtol=1e-11)
        rowwise_close(g[i:i + 1], og, 1e-7)
        rowwise_close(gp[i], ogp, 1e-7)
