"""GPU parity of the direct model (rr_evaluate_direct: weights built for
each row's own k, Sect. 3.1.1) against the oracle's evaluate_direct, through
the C ABI: 1e-9 (FP64) / 1 ppm (mixed), exactly 1.0 where the oracle has no
occultation, NaN rows for k outside (0, 1]."""

import numpy as np
import pytest

import workloads as wl
from oracle import roadrunner as orr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_08500_amd as rr
    return rr


def check(ref, f64, f32):
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(f64)) and np.array_equal(nan, np.isnan(f32))
    r, a, b = ref[~nan], f64[~nan], f32[~nan]
    assert np.abs(a - r).max(initial=0.0) <= 1e-9
    assert np.abs(b - r).max(initial=0.0) <= 1e-6
    out = r == 1.0
    assert np.all(a[out] == 1.0) and np.all(b[out] == 1.0)


@pytest.mark.parametrize("npt", [700, 2049])
def test_direct_model_matches_oracle(rr, npt):
    """k inside and outside the tables' [0.01, 0.3] (0.004, 0.45, 0.8), an
    invalid k, ragged time tails."""
    w = wl.population(npv=8, npt=npt)
    w["times"] = np.linspace(0.0, 10.0, npt)
    pv = w["pv"].copy()
    pv[:, 6] = [0.004, 0.05, 0.1, 0.45, 0.8, 0.2, 1.3, 0.15]
    pv[:, 3] = np.minimum(pv[:, 3], 0.5)                    # keep the big planets transiting
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    f64 = rr.evaluate_direct(tab, ser, pv, "fp64").cpu().numpy()
    f32 = rr.evaluate_direct(tab, ser, pv, "mixed").cpu().numpy().astype(np.float64)
    ref = orr.evaluate_direct(otab, w["times"], pv)
    assert np.isnan(ref[6]).all()
    check(ref, f64, f32)


def test_node_k_equals_interpolated_model(rr):
    """With every k on a node of the tables' k-grid the direct model and
    rr_evaluate agree to rounding (the same weights and bin order)."""
    w = wl.population(npv=16, npt=5000)
    g = wl.DEFAULT_GRID
    dk = (g["k1"] - g["k0"]) / (g["nk"] - 1)
    pv = w["pv"].copy()
    pv[:, 6] = g["k0"] + dk * np.arange(20, 20 + 16 * 9, 9)
    tab = rr.Tables(w["mu_s"], w["I_s"], g)
    ser = rr.TimeSeries(w["times"])
    for prec, tol in (("fp64", 1e-13), ("mixed", 2e-7)):
        a = rr.evaluate_direct(tab, ser, pv, prec).cpu().numpy().astype(np.float64)
        b = rr.evaluate(tab, ser, pv, prec).cpu().numpy().astype(np.float64)
        assert np.abs(a - b).max() <= tol, (prec, np.abs(a - b).max())


def test_heterogeneous_direct(rr):
    w = wl.heterogeneous(npv=4, days=3.0)
    kw = dict(lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"], exptimes=w["exptimes"])
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], w["lcids"], w["pbids"], w["nss"], w["exptimes"])
    f64 = rr.evaluate_direct(tab, ser, w["pv"], "fp64").cpu().numpy()
    f32 = rr.evaluate_direct(tab, ser, w["pv"], "mixed").cpu().numpy().astype(np.float64)
    check(orr.evaluate_direct(otab, w["times"], w["pv"], **kw), f64, f32)


@pytest.mark.parametrize("k", [0.005, 0.1, 0.5])
def test_direct_model_against_analytic_model(rr, k):
    """The direct model on the single light curve's orbit with quadratic LD
    (2001 mu samples), at k below, inside and above the tables' k range:
    within 5 ppm of the analytic quadratic-LD model (Mandel & Agol 2002) in
    both precisions, as the paper's accuracy figure shows for the direct
    model up to k = 0.5."""
    from oracle import analytic as an
    from oracle import orbit
    w = wl.single_light_curve()
    mu = np.linspace(0.0, 1.0, 2001)
    tab = rr.Tables(mu, wl.profile_quadratic(mu, 0.4, 0.25), wl.DEFAULT_GRID)
    pv = w["pv"].copy()
    pv[0, 6] = k
    ser = rr.TimeSeries(w["times"])
    f64 = rr.evaluate_direct(tab, ser, pv, "fp64").cpu().numpy()[0]
    f32 = rr.evaluate_direct(tab, ser, pv, "mixed").cpu().numpy()[0]
    row = pv[0]
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    fm = np.where(front, an.quadratic_flux(z, k, 0.4, 0.25), 1.0)
    assert (fm < 1.0).sum() > 100
    assert np.abs(f64 - fm).max() <= 5e-6
    assert np.abs(f32.astype(np.float64) - fm).max() <= 6e-6
