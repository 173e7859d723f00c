"""GPU parity of per-vector limb darkening (rr_evaluate_ld: every parameter
vector with its own LD profile) against the oracle's evaluate_ld, through the
C ABI.  Tolerances as the shared-table parity tests: 1e-9 absolute for the
FP64 path (a logic check), 1 ppm for the mixed path, and exactly 1.0 where
the oracle has no occultation."""

import numpy as np
import pytest

import workloads as wl
from oracle import roadrunner as orr

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL_MIXED = 1e-6


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
    assert np.abs(a - r).max(initial=0.0) <= TOL64
    assert np.abs(b - r).max(initial=0.0) <= TOL_MIXED
    out = r == 1.0
    assert np.all(a[out] == 1.0) and np.all(b[out] == 1.0)


@pytest.mark.parametrize("npt", [1, 511, 513, 1537, 5000])
def test_population_ld_matches_oracle(rr, npt):
    """Ragged time tails around the 512-time tiles, one invalid row."""
    w = wl.population_ld(npv=10, npt=npt)
    w["times"] = np.linspace(0.0, 12.0, npt)
    pv = w["pv"].copy()
    pv[4, 6] = 0.5                                          # k outside the table: NaN row
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    f64 = rr.evaluate_ld(tab, ser, pv, w["prof_pv"], "fp64").cpu().numpy()
    f32 = rr.evaluate_ld(tab, ser, pv, w["prof_pv"], "mixed").cpu().numpy().astype(np.float64)
    ref = orr.evaluate_ld(otab, w["times"], pv, w["prof_pv"])
    assert np.isnan(ref[4]).all()
    check(ref, f64, f32)


def test_clustered_radius_ratios(rr):
    """Rows whose k fall on few k-rows (walkers): after sorting, 16-row tiles
    with one or two k-rows run on the matrix cores and tiles spanning more
    run per row; 45 rows give tiles of both kinds and a ragged last tile."""
    w = wl.population_ld(npv=45, npt=3000)
    w["times"] = np.linspace(0.0, 12.0, 3000)
    pv = w["pv"].copy()
    dk = (wl.TEST_GRID["k1"] - wl.TEST_GRID["k0"]) / (wl.TEST_GRID["nk"] - 1)
    base = wl.TEST_GRID["k0"] + 8 * dk
    pattern = [0.3] * 20 + [1.4] * 8 + [2.6, 3.5, 4.2, 5.1, 6.3, 7.7, 8.2, 9.9] + [11.3] * 9
    pv[:, 6] = base + dk * np.asarray(pattern)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    f64 = rr.evaluate_ld(tab, ser, pv, w["prof_pv"], "fp64").cpu().numpy()
    f32 = rr.evaluate_ld(tab, ser, pv, w["prof_pv"], "mixed").cpu().numpy().astype(np.float64)
    check(orr.evaluate_ld(otab, w["times"], pv, w["prof_pv"]), f64, f32)


def test_heterogeneous_passbands_and_supersampling(rr):
    """Four passbands, each vector with four profiles of its own, chromatic k,
    nss 10 and 1 light curves."""
    w = wl.heterogeneous(npv=6, days=4.0)
    rng = np.random.default_rng(11)
    c = rng.uniform(0.3, 0.7, (6, 4))
    al = rng.uniform(0.4, 0.8, (6, 4))
    prof = 1.0 - c[..., None] * (1.0 - w["mu_s"][None, None, :] ** al[..., None])
    kw = dict(lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"], exptimes=w["exptimes"])
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], w["lcids"], w["pbids"], w["nss"], w["exptimes"])
    f64 = rr.evaluate_ld(tab, ser, w["pv"], prof, "fp64").cpu().numpy()
    f32 = rr.evaluate_ld(tab, ser, w["pv"], prof, "mixed").cpu().numpy().astype(np.float64)
    ref = orr.evaluate_ld(otab, w["times"], w["pv"], prof, **kw)
    check(ref, f64, f32)


def test_own_profile_equals_shared_tables(rr):
    """Every vector given the tables' own profile: rr_evaluate_ld and
    rr_evaluate agree to rounding (each vector's two table rows are the
    shared rows up to the order of the FP64 additions over bins, then
    interpolated in k the same way; in mixed precision the rows are summed
    from the FP32 copy of the weights, so the float outputs may differ by
    an ulp)."""
    w = wl.population(npv=64, npt=6000)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.DEFAULT_GRID)
    ser = rr.TimeSeries(w["times"])
    prof = np.broadcast_to(w["I_s"], (64,) + w["I_s"].shape).copy()
    for prec, tol in (("fp64", 1e-14), ("mixed", 1.2e-7)):
        a = rr.evaluate_ld(tab, ser, w["pv"], prof, prec).cpu().numpy().astype(np.float64)
        b = rr.evaluate(tab, ser, w["pv"], prec).cpu().numpy().astype(np.float64)
        assert np.abs(a - b).max() <= tol, (prec, np.abs(a - b).max())


def test_full_size_sampled_rows(rr):
    """The per-vector LD population at full size (512 x 20 000, default
    grid), in the launch configuration the benchmark times; six sampled rows
    against the oracle."""
    w = wl.population_ld()
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.DEFAULT_GRID)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.DEFAULT_GRID)
    ser = rr.TimeSeries(w["times"])
    f64 = rr.evaluate_ld(tab, ser, w["pv"], w["prof_pv"], "fp64").cpu().numpy()
    f32 = rr.evaluate_ld(tab, ser, w["pv"], w["prof_pv"], "mixed").cpu().numpy()
    rows = np.random.default_rng(5).choice(512, 6, replace=False)
    ref = orr.evaluate_ld(otab, w["times"], w["pv"][rows], w["prof_pv"][rows])
    check(ref, f64[rows], f32[rows].astype(np.float64))
    assert np.isfinite(f64).all() and np.isfinite(f32).all()


def test_arguments(rr):
    import torch
    w = wl.population_ld(npv=3, npt=100)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    with pytest.raises(ValueError):
        rr.evaluate_ld(tab, ser, w["pv"], w["prof_pv"][:2], "fp64")
    out = rr.evaluate_ld(tab, ser, w["pv"][:0], w["prof_pv"][:0], "fp64")
    assert out.shape == (0, 100)
    from paper_2009_08500_amd import _lib
    pv = torch.as_tensor(w["pv"], device="cuda")
    lc, npt, pb, nss, ex, nlc = ser.lc_args()
    import ctypes
    o = torch.empty((3, 100), dtype=torch.float64, device="cuda")
    rc = _lib.lib().rr_evaluate_ld(tab.handle, ctypes.c_void_p(ser.times.data_ptr()), lc, npt,
                                   pb, nss, ex, nlc, ctypes.c_void_p(pv.data_ptr()), 3, 7, None,
                                   0, ctypes.c_void_p(o.data_ptr()), None)
    assert rc == _lib.RR_EINVAL and "prof" in _lib.last_error()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_deterministic_and_independent_of_batch(rr, precision):
    """The rows are sorted stably by k-row and both table kernels read the
    same weights, so two identical calls agree bitwise, and a row's fluxes do
    not depend on which rows share its call beyond rounding: row 50 sits in a
    32-row cluster on one k-row (a matrix-core tile) in one call and among
    rows spread over many k-rows (the per-row kernel) in another.  Only the
    order of the FP64 additions over bins differs between the two kernels;
    in mixed precision that can move a table value by one float ulp when the
    two sums round to different sides of a float, so the bound there is a
    few float ulps of the flux deficit."""
    w = wl.population_ld(npv=96, npt=4000)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    pv, prof = w["pv"].copy(), w["prof_pv"].copy()
    pv[40:72, 6] = pv[40, 6]                 # a cluster on one k-row
    a = rr.evaluate_ld(tab, ser, pv, prof, precision).cpu().numpy()
    b = rr.evaluate_ld(tab, ser, pv, prof, precision).cpu().numpy()
    assert np.array_equal(a, b)
    rows = [50] + list(range(31))            # two 16-row tiles over many k-rows
    c = rr.evaluate_ld(tab, ser, pv[rows], prof[rows], precision).cpu().numpy()
    if precision == "fp64":
        assert np.abs(c[0] - a[50]).max() <= 1e-13
    else:
        assert np.abs(c[0].astype(np.float64) - a[50]).max() <= 2e-7


def test_more_rows_than_the_sort_keeps_in_lds(rr):
    """8300 rows: the sorting workgroup keeps the keys of the first 8192 rows
    in LDS and reads the rest from memory.  Two identical calls agree
    bitwise (a stable sort), rows on both sides of that bound match the oracle,
    and the last rows alone give the same fluxes to rounding."""
    w = wl.population_ld(npv=8300, npt=64)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    otab = orr.Tables(w["mu_s"], w["I_s"], **wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    pv, prof = w["pv"], w["prof_pv"]
    f64 = rr.evaluate_ld(tab, ser, pv, prof, "fp64").cpu().numpy()
    f32 = rr.evaluate_ld(tab, ser, pv, prof, "mixed").cpu().numpy()
    assert np.array_equal(f64, rr.evaluate_ld(tab, ser, pv, prof, "fp64").cpu().numpy())
    rows = np.array([0, 4097, 8191, 8192, 8250, 8299])
    ref = orr.evaluate_ld(otab, w["times"], pv[rows], prof[rows])
    check(ref, f64[rows], f32[rows].astype(np.float64))
    tail = rr.evaluate_ld(tab, ser, pv[8192:], prof[8192:], "fp64").cpu().numpy()
    assert np.abs(tail - f64[8192:]).max() <= 1e-13
