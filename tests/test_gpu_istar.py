"""rr_set_istar and rr_loglik_grad_istar on the GPU against the oracle's
fixed normaliser (Tables(..., istar=...)), through the C ABI.

Forward: 1e-9 (FP64) and 1 ppm (mixed) of the oracle, on the registered-
series and the per-tile launches; clearing the override gives the tables'
own values back bit for bit; a new profile keeps the override.  Gradients:
logL and the parameter gradient as in the adjoint tests (mixed logL to
3e-6, see below), the profile
gradient with I_star held fixed and d logL / d I_star against the oracle
(1e-7 of scale in FP64, 2e-4 in mixed precision).  A named law through its
closed-form I_star (the quadratic law, Sect. 3.2.1) stays within 1 ppm of
the analytic model on the single-light-curve configuration."""

import numpy as np
import pytest

import workloads as wl
from oracle import analytic as an
from oracle import gradient as ogr
from oracle import orbit
from oracle import roadrunner as orr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_08500_amd as rr
    return rr


def test_forward_with_fixed_istar(rr):
    w = wl.population(npv=40, npt=5000, seed_extra=50)
    otab0 = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    new = otab0.istar * 1.0137
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID, istar=new)
    ref = orr.evaluate(otab, w["times"], w["pv"])
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    plain = {p: rr.evaluate(tab, ser, w["pv"], p).cpu().numpy() for p in ("fp64", "mixed")}
    tab.set_istar(new)
    for prec, tol in (("fp64", 1e-9), ("mixed", 1e-6)):
        for fn in (rr.evaluate, rr.evaluate_unregistered):
            got = fn(tab, ser, w["pv"], prec).cpu().numpy().astype(np.float64)
            assert np.abs(got - ref).max() <= tol, (prec, fn.__name__)
    assert np.allclose(tab.copy("istar"), new, rtol=0, atol=0)
    tab.set_istar(None)
    for prec in ("fp64", "mixed"):
        assert np.array_equal(rr.evaluate(tab, ser, w["pv"], prec).cpu().numpy(), plain[prec])
    # the override stays in force over a new profile
    tab.set_istar(new)
    prof2 = w["I_s"] * 0.97
    tab.set_profile(prof2)
    ref2 = orr.evaluate(orr.with_profile(otab, prof2), w["times"], w["pv"])
    got = rr.evaluate(tab, ser, w["pv"], "fp64").cpu().numpy()
    assert np.abs(got - ref2).max() <= 1e-9
    # an invalid normaliser gives NaN fluxes in transit, never a wrong number
    tab.set_istar([-1.0])
    bad = rr.evaluate(tab, ser, w["pv"], "fp64").cpu().numpy()
    assert np.all(np.isnan(bad[ref < 1.0])) and np.all(bad[ref == 1.0] == 1.0)
    tab.close()


# mixed logL: the walkers sit ~2000 in logL from their 4000 x 3 samples, so a
# float-level flux error (~0.1 ppm per in-transit point) can move logL by a
# few 1e-6 relative; the adjoint tests' 1e-6 is for walkers at the truth
@pytest.mark.parametrize("precision,rel_ll,rel_g", [("fp64", 1e-11, 1e-7), ("mixed", 3e-6, 2e-4)])
def test_gradients_with_fixed_istar(rr, precision, rel_ll, rel_g):
    w = wl.loglik_walkers(npv=16, npt=4000, nss=3, seed_extra=51)
    w["times"] = np.linspace(0.0, 20.0, 4000)
    base = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ist = base.istar * 1.003
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID, istar=ist)
    obs = orr.evaluate(otab, w["times"], w["truth"][None, :], nss=w["nss"],
                       exptimes=w["exptimes"])[0] + w["noise"]
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    tab.set_istar(ist)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    ll, g, gp, gi = rr.loglik_grad(tab, ser, w["pv"], obs, w["sigma"], precision, grad=True,
                                   profile=True, istar_grad=True)
    ll, g, gp, gi = (x.cpu().numpy() for x in (ll, g, gp, gi))
    if precision == "mixed":
        obs = obs.astype(np.float32).astype(np.float64)
    oll, og, ogp, ogi = ogr.loglik_grad(otab, w["times"], w["pv"], obs, w["sigma"],
                                       nss=w["nss"], exptimes=w["exptimes"], want_istar=True)
    np.testing.assert_allclose(ll, oll, rtol=rel_ll)
    scale = np.abs(og).max(axis=1, keepdims=True)
    assert np.all(np.abs(g - og) <= rel_g * scale)
    assert np.abs(gp - ogp).max() <= rel_g * np.abs(ogp).max()
    assert np.abs(gi - ogi).max() <= rel_g * np.abs(ogi).max()
    # without the profile gradient the I_star gradient alone
    _, _, gp2, gi2 = rr.loglik_grad(tab, ser, w["pv"], obs if precision == "fp64" else
                                    obs.astype(np.float32), w["sigma"], precision, grad=False,
                                    profile=False, istar_grad=True)
    assert gp2 is None and np.array_equal(gi2.cpu().numpy(), gi)
    tab.close()


def test_named_law_with_closed_form_istar_against_analytic(rr):
    import torch
    w = wl.single_light_curve()
    row = w["pv"][0]
    coeffs = torch.tensor([0.4, 0.25], dtype=torch.float64)
    prof = rr.ldlaws.profile("quadratic", w["mu_s"], coeffs)
    tab = rr.Tables(w["mu_s"], prof.cpu().numpy(), wl.DEFAULT_GRID)
    tab.set_istar(rr.ldlaws.istar("quadratic", coeffs).reshape(1))
    ser = rr.TimeSeries(w["times"])
    got = rr.evaluate(tab, ser, w["pv"], "fp64").cpu().numpy()[0]
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    fm = np.where(front, an.quadratic_flux(z, row[6], 0.4, 0.25), 1.0)
    assert np.abs(got - fm).max() <= 1e-6
    tab.close()


def test_autograd_through_law_and_its_closed_form_istar(rr):
    """RRLogLik with the power-2 profile and its closed-form I_star both
    generated from (c, alpha) in torch: the gradient with respect to (c,
    alpha) -- through the samples with I_star held fixed, plus through I_star
    -- against central differences of the GPU log-likelihood."""
    import torch
    w = wl.loglik_walkers(npv=8, npt=4000, nss=2, seed_extra=52)
    w["times"] = np.linspace(0.0, 15.0, 4000)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    obs = orr.evaluate(otab, w["times"], w["truth"][None, :], nss=w["nss"],
                       exptimes=w["exptimes"])[0] + w["noise"]
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], nss=w["nss"], exptimes=w["exptimes"])
    mu = torch.tensor(w["mu_s"], device="cuda")
    c = torch.tensor(w["ld_c"], device="cuda", dtype=torch.float64, requires_grad=True)
    al = torch.tensor(w["ld_alpha"], device="cuda", dtype=torch.float64, requires_grad=True)
    pv = torch.tensor(w["pv"], device="cuda")
    obs_t = torch.tensor(obs, device="cuda")
    weights = torch.linspace(0.5, 1.5, 8, device="cuda", dtype=torch.float64)

    def loss_fn(c_, al_):
        coeffs = torch.stack([c_, al_])
        prof = rr.ldlaws.profile("power-2", mu, coeffs)[None, :]
        ist = rr.ldlaws.istar("power-2", coeffs).reshape(1).to("cuda")
        ll = rr.RRLogLik.apply(pv, prof, tab, ser, obs_t, w["sigma"], "fp64", ist)
        return (weights * ll).sum()

    loss = loss_fn(c, al)
    loss.backward()
    with torch.no_grad():
        h = 1e-6
        fd_c = (loss_fn(c + h, al) - loss_fn(c - h, al)).item() / (2 * h)
        fd_a = (loss_fn(c, al + h) - loss_fn(c, al - h)).item() / (2 * h)
    assert c.grad.item() == pytest.approx(fd_c, rel=1e-4)
    assert al.grad.item() == pytest.approx(fd_a, rel=1e-4)
    # I_star's own part is not negligible: the gradient without it differs
    c2 = c.detach().clone().requires_grad_(True)
    coeffs = torch.stack([c2, al.detach()])
    prof = rr.ldlaws.profile("power-2", mu, coeffs)[None, :]
    ist = rr.ldlaws.istar("power-2", coeffs).reshape(1).to("cuda").detach()
    ((weights * rr.RRLogLik.apply(pv, prof, tab, ser, obs_t, w["sigma"], "fp64", ist))
     .sum()).backward()
    assert abs(c2.grad.item() - fd_c) > 1e-3 * abs(fd_c)
    tab.close()
