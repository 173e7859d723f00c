"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (absolute, in flux):
* RR_FP64 path: 1e-9 (a logic check; the observed gap is ~1e-14, rounding
  order only), and exactly 1.0 wherever the oracle has no occultation.
* RR_MIXED path: 1 ppm (1e-6), the contract for FP32 bulk arithmetic with an
  FP64 time reduction.
Tables: see test_tables_match_oracle (the oracle's textbook lens formula is
ill-conditioned near tangencies; exact 40-digit values settle those).
"""

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


def both(rr, tab, series, pv):
    f64 = rr.evaluate(tab, series, pv, "fp64").cpu().numpy()
    f32 = rr.evaluate(tab, series, pv, "mixed").cpu().numpy().astype(np.float64)
    return f64, f32


def check_parity(ref, f64, f32, tol32=TOL_MIXED):
    assert f64.shape == ref.shape
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(f64)) and np.array_equal(nan, np.isnan(f32))
    r, a, b = ref[~nan], f64[~nan], f32[~nan]
    err64 = np.abs(a - r).max(initial=0.0)
    err32 = np.abs(b - r).max(initial=0.0)
    assert err64 <= TOL64, err64
    assert err32 <= tol32, err32
    out = r == 1.0
    assert np.all(a[out] == 1.0)                  # exactly 1 out of transit
    assert np.all(b[out] == 1.0)
    return err64, err32


def _lens_mp(R, k, c):
    """Lens area in 40-digit arithmetic (textbook formula)."""
    import mpmath as mp
    mp.mp.dps = 40
    R, k, c = mp.mpf(R), mp.mpf(k), mp.mpf(c)
    if c >= R + k:
        return mp.mpf(0)
    if c <= abs(R - k):
        return mp.pi * min(R, k) ** 2
    return (R * R * mp.acos((c * c + R * R - k * k) / (2 * c * R))
            + k * k * mp.acos((c * c + k * k - R * R) / (2 * c * k))
            - mp.sqrt((-c + R + k) * (c + R - k) * (c - R + k) * (c + R + k)) / 2)


def test_tables_match_oracle(rr):
    """Tables against the oracle.  W and T are FP64 on both sides, but the
    oracle's textbook arccos lens formula is ill-conditioned where an annulus
    edge is nearly tangent to the planet disk or the planet is small (its
    error there reaches ~sqrt(machine epsilon) of the area), so W is
    compared with the oracle at 1e-8 and, on the entries where the two differ
    most plus a random sample, against 40-digit arithmetic at 1e-13."""
    w = wl.heterogeneous(npv=1)
    grid = wl.TEST_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    o = orr.Tables(w["mu_s"], w["I_s"], **grid)
    np.testing.assert_allclose(tab.copy("ze"), o.ze, rtol=0, atol=1e-15)
    np.testing.assert_allclose(tab.copy("zm"), o.zm, rtol=0, atol=1e-15)
    kk = grid["k0"] + o.dk * np.arange(grid["nk"])
    W = tab.copy("W").transpose(0, 2, 1)            # device layout [nk][nz][ng]
    diff = np.abs(W - o.W)
    assert diff.max() <= 1e-8, diff.max()
    ng = grid["ng"]
    worst = np.argsort(diff, axis=None)[-5:]
    rnd = np.random.default_rng(11).choice(W.size, 20, replace=False)
    for flat in np.concatenate([worst, rnd]):
        i, m, j = np.unravel_index(flat, W.shape)
        c = m / (ng - 1.0) * (1 + kk[i])
        tot = _lens_mp(1.0, kk[i], c)
        if tot == 0:
            exact = 1.0 if j == W.shape[2] - 1 else 0.0
        else:
            exact = float((_lens_mp(o.ze[j + 1], kk[i], c) - _lens_mp(o.ze[j], kk[i], c)) / tot)
        assert abs(W[i, m, j] - exact) <= 1e-13, (i, m, j, W[i, m, j], exact)
    np.testing.assert_allclose(tab.copy("ldp"), o.ldp, rtol=0, atol=1e-14)
    np.testing.assert_allclose(tab.copy("istar"), o.istar, rtol=1e-14)
    T64 = tab.copy("T64")
    assert np.abs(T64 - o.T).max() <= 1e-8 * np.abs(o.ldp).max()
    np.testing.assert_allclose(tab.copy("T32"), T64, rtol=6e-8, atol=0)


def test_single_light_curve(rr):
    w = wl.single_light_curve()
    for grid in (wl.TEST_GRID, wl.DEFAULT_GRID):
        tab = rr.Tables(w["mu_s"], w["I_s"], grid)
        ref = orr.evaluate(orr.Tables(w["mu_s"], w["I_s"], **grid), w["times"], w["pv"])
        f64, f32 = both(rr, tab, rr.TimeSeries(w["times"]), w["pv"])
        check_parity(ref, f64, f32)
        assert (f64 < 1).sum() == 316


def test_single_light_curve_against_analytic_model(rr):
    """The single light curve (quadratic LD sampled at 100 mu) at the default
    grid, both precisions, within 1 ppm of the analytic quadratic-LD model
    (Mandel & Agol 2002) that the paper measures its accuracy against."""
    from oracle import analytic as an
    from oracle import orbit
    w = wl.single_light_curve()
    row = w["pv"][0]
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.DEFAULT_GRID)
    f64, f32 = both(rr, tab, rr.TimeSeries(w["times"]), w["pv"])
    z, front, _ = orbit.projected_separation(w["times"] - row[0], *row[1:6])
    fm = np.where(front, an.quadratic_flux(z, row[6], 0.4, 0.25), 1.0)
    assert np.abs(f64[0] - fm).max() <= 1e-6
    assert np.abs(f32[0].astype(np.float64) - fm).max() <= 1e-6


@pytest.mark.parametrize("npt", [1, 7, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 5000])
def test_population_ragged_sizes(rr, npt):
    """Tiles of 512 (forward) and 1024 (log-likelihood) times per workgroup,
    and the vector fast path's whole-span condition: sizes around the edges."""
    w = wl.population(npv=24, npt=npt)
    grid = wl.TEST_GRID
    pv = w["pv"].copy()
    pv[:, 0] = np.linspace(0.0, 0.02 * max(npt, 1), pv.shape[0])   # transits inside the window
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ref = orr.evaluate(orr.Tables(w["mu_s"], w["I_s"], **grid), w["times"], pv)
    f64, f32 = both(rr, tab, rr.TimeSeries(w["times"]), pv)
    check_parity(ref, f64, f32)


def test_population_full_size(rr):
    """The population workload at full size (512 x 20000, default grid), the
    launch configuration the benchmark times; every output is compared."""
    w = wl.population()
    grid = wl.DEFAULT_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ref = orr.evaluate(orr.Tables(w["mu_s"], w["I_s"], **grid), w["times"], w["pv"])
    f64, f32 = both(rr, tab, rr.TimeSeries(w["times"]), w["pv"])
    e64, e32 = check_parity(ref, f64, f32)
    print(f"population 512x20000: max|fp64-oracle| {e64:.2e}, max|mixed-oracle| {e32 * 1e6:.3f} ppm,"
          f" in-transit fraction {np.mean(ref < 1):.4f}")


def test_more_rows_than_one_grid_dimension(rr):
    """70 000 rows (the kernels put rows on the grid's y dimension, at most
    65 535 per launch, so this takes two launches) x 300 times: 100 distinct
    rows tiled 700 times must give bitwise-identical outputs wherever a row
    repeats, and the distinct rows match the oracle."""
    grid = wl.TEST_GRID
    w = wl.population(npv=100, npt=300)
    pv = w["pv"].copy()
    pv[:, 0] = np.linspace(0.0, 0.4, pv.shape[0])      # transits inside the 0.42-d span
    big = np.tile(pv, (700, 1))
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"])
    for prec in ("fp64", "mixed"):
        out = rr.evaluate(tab, ser, big, prec).cpu().numpy()
        assert out.shape == (70000, 300)
        rows = out.reshape(700, 100, 300)
        assert np.array_equal(rows, np.broadcast_to(rows[0], rows.shape))
    ref = orr.evaluate(orr.Tables(w["mu_s"], w["I_s"], **grid), w["times"], pv)
    assert (ref < 1.0).sum() > 500
    f64, f32 = both(rr, tab, ser, pv)
    check_parity(ref, f64, f32)
    # the 70 000-row call takes the per-tile kernel: bitwise equal to it on
    # the 100 rows; the 100-row call may take the split launch (one rounding)
    last64 = rr.evaluate(tab, ser, big, "fp64").cpu().numpy()[-100:]
    assert np.array_equal(last64, rr.evaluate_unregistered(tab, ser, pv, "fp64").cpu().numpy())
    assert np.abs(last64 - f64).max() <= 1e-15


def test_population_bjd_offset(rr):
    """Times near BJD 2.459e6: the FP64 time reduction keeps the mixed path
    within 1 ppm."""
    w = wl.population(npv=64, npt=8000)
    off = 2459000.0
    times = w["times"] + off
    pv = w["pv"].copy()
    pv[:, 0] += off
    grid = wl.TEST_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ref = orr.evaluate(orr.Tables(w["mu_s"], w["I_s"], **grid), times, pv)
    f64, f32 = both(rr, tab, rr.TimeSeries(times), pv)
    check_parity(ref, f64, f32)


def test_heterogeneous_supersampled(rr):
    """Four passbands, chromatic k, two supersampled 30-min light curves and
    two 2-min light curves (Sect. 4.2); 6 days, 48 parameter vectors."""
    w = wl.heterogeneous(npv=48, days=6.0)
    grid = wl.TEST_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ref = orr.evaluate(orr.Tables(w["mu_s"], w["I_s"], **grid), w["times"], w["pv"],
                       lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"], exptimes=w["exptimes"])
    ser = rr.TimeSeries(w["times"], w["lcids"], w["pbids"], w["nss"], w["exptimes"])
    f64, f32 = both(rr, tab, ser, w["pv"])
    check_parity(ref, f64, f32)


def test_heterogeneous_full_size_sampled(rr):
    """The heterogeneous workload at full size (256 x 41472, default grid);
    32 sampled parameter rows are compared with the oracle."""
    w = wl.heterogeneous()
    grid = wl.DEFAULT_GRID
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], w["lcids"], w["pbids"], w["nss"], w["exptimes"])
    f64, f32 = both(rr, tab, ser, w["pv"])
    rows = np.random.default_rng(5).choice(w["pv"].shape[0], 32, replace=False)
    ref = orr.evaluate(orr.Tables(w["mu_s"], w["I_s"], **grid), w["times"], w["pv"][rows],
                       lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"], exptimes=w["exptimes"])
    check_parity(ref, f64[rows], f32[rows])
    assert np.all(f64 <= 1.0) and np.all(f64 > 0.9)


def test_orbit_edge_cases(rr):
    """Circular, grazing, central, boundary radius ratios, high eccentricity,
    orbits whose transit window covers the whole period, and invalid rows."""
    grid = wl.TEST_GRID
    mu = np.linspace(0, 1, 50)
    I = wl.profile_power2(mu, 0.7, 0.5)
    t = np.linspace(-1.0, 1.0, 4001)
    rows = [
        [0.0, 3.0, 8.0, 0.0, 0.0, 0.0, 0.1],           # central
        [0.0, 3.0, 8.0, 1.05, 0.0, 0.0, 0.1],          # grazing
        [0.0, 3.0, 8.0, 1.1, 0.0, 0.0, 0.1],           # exactly touching
        [0.0, 3.0, 8.0, 1.2, 0.0, 0.0, 0.1],           # miss
        [0.0, 3.0, 8.0, 0.3, 0.0, 0.0, grid["k0"]],    # k at the table edges
        [0.0, 3.0, 8.0, 0.3, 0.0, 0.0, grid["k1"]],
        [0.1, 5.0, 30.0, 0.5, 0.9, 1.0, 0.1],          # high e
        [0.1, 5.0, 30.0, 0.5, 0.95, 4.0, 0.2],
        [0.0, 0.5, 1.3, 0.2, 0.0, 0.0, 0.25],          # window covers the whole period
        [0.0, 0.6, 2.0, 0.1, 0.3, 2.0, 0.2],           # a(1-e) < 1 + k
        [0.0, 3.0, 8.0, 0.3, 1.0, 0.0, 0.1],           # invalid: e = 1
        [0.0, 3.0, 8.0, 0.3, 0.0, 0.0, 0.5],           # invalid: k > k1
        [0.0, -3.0, 8.0, 0.3, 0.0, 0.0, 0.1],          # invalid: P < 0
        [0.0, 3.0, 0.2, 0.3, 0.0, 0.0, 0.1],           # invalid: |cos i| > 1
        [np.nan, 3.0, 8.0, 0.3, 0.0, 0.0, 0.1],        # invalid: NaN
    ]
    pv = np.array(rows)
    tab = rr.Tables(mu, I, grid)
    ref = orr.evaluate(orr.Tables(mu, I, **grid), t, pv)
    assert np.isnan(ref[10:]).all() and np.isfinite(ref[:10]).all()
    f64, f32 = both(rr, tab, rr.TimeSeries(t), pv)
    check_parity(ref, f64, f32)
    assert f64[3].min() == 1.0 and f64[0].min() < f64[1].min() < 1.0


def test_supersampling_long_exposures(rr):
    grid = wl.TEST_GRID
    w = wl.population(npv=16, npt=3000)
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    for nss, ex in [(2, 0.01), (30, 0.02), (200, 0.1), (1, 0.5)]:
        ref = orr.evaluate(otab, w["times"], w["pv"], nss=nss, exptimes=ex)
        f64, f32 = both(rr, tab, rr.TimeSeries(w["times"], nss=nss, exptimes=ex), w["pv"])
        check_parity(ref, f64, f32)


def test_supersample_lane_groups(rr):
    """Light curves whose nss select the lane-group path (2, 7: groups that
    leave idle lanes, 32: two groups) or the per-lane loop (33), interleaved
    so that some waves see mixed nss; every row transits inside the span."""
    grid = wl.TEST_GRID
    w = wl.population(npv=12, npt=6000)
    pv = w["pv"].copy()
    pv[:, 0] = np.linspace(0.0, 4.0, pv.shape[0])
    times = w["times"]
    lcids = (np.arange(times.size) // 700) % 4                 # blocks of 700 times
    nss = np.array([2, 7, 32, 33], np.int32)
    ex = np.array([0.004, 0.01, 0.02, 0.03])
    pbids = np.zeros(4, np.int32)
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    ref = orr.evaluate(otab, times, pv, lcids=lcids, pbids=pbids, nss=nss, exptimes=ex)
    ser = rr.TimeSeries(times, lcids.astype(np.int32), pbids, nss, ex)
    f64, f32 = both(rr, tab, ser, pv)
    assert (ref < 1.0).sum() > 1000
    check_parity(ref, f64, f32)


def test_invalid_light_curve_ids_give_nan(rr):
    grid = wl.TEST_GRID
    w = wl.population(npv=4, npt=100)
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    lcids = np.zeros(100, np.int32)
    lcids[[3, 50]] = [5, -1]
    out = rr.evaluate(tab, rr.TimeSeries(w["times"], lcids, [0, 0], [1, 1], [0.0, 0.0]),
                      w["pv"], "fp64").cpu().numpy()
    assert np.isnan(out[:, [3, 50]]).all()
    assert np.isfinite(np.delete(out, [3, 50], axis=1)).all()


def test_zero_sizes_and_errors(rr):
    import torch
    grid = wl.TEST_GRID
    w = wl.population(npv=4, npt=100)
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    out = rr.evaluate(tab, rr.TimeSeries(np.zeros(0)), w["pv"], "fp64")
    assert out.shape == (4, 0)
    out = rr.evaluate(tab, rr.TimeSeries(w["times"]), np.zeros((0, 7)), "mixed")
    assert out.shape == (0, 100)
    with pytest.raises(rr.RRError) as e:
        rr.evaluate(tab, rr.TimeSeries(w["times"]), np.zeros((2, 8)), "fp64")   # npar mismatch
    assert e.value.code == -1
    with pytest.raises(rr.RRError) as e:
        rr.evaluate(tab, rr.TimeSeries(w["times"], np.zeros(100, np.int32), np.zeros(65, np.int32)),
                    w["pv"], "fp64")
    assert e.value.code == -4
    with pytest.raises(rr.RRError):
        rr.evaluate(tab, rr.TimeSeries(w["times"], nss=0), w["pv"], "fp64")
    torch.cuda.synchronize()


def test_set_profile_on_device(rr):
    import torch
    grid = wl.TEST_GRID
    w = wl.population(npv=32, npt=4000)
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    I2 = wl.profile_quadratic(w["mu_s"], 0.5, 0.1)[None, :]
    tab.set_profile(torch.tensor(I2, device="cuda"))
    ref = orr.evaluate(orr.Tables(w["mu_s"], I2, **grid), w["times"], w["pv"])
    f64, f32 = both(rr, tab, rr.TimeSeries(w["times"]), w["pv"])
    check_parity(ref, f64, f32)


def test_deterministic(rr):
    w = wl.population(npv=64, npt=6000)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    s = rr.TimeSeries(w["times"])
    a = rr.evaluate(tab, s, w["pv"], "mixed").cpu().numpy()
    b = rr.evaluate(tab, s, w["pv"], "mixed").cpu().numpy()
    assert np.array_equal(a, b)
