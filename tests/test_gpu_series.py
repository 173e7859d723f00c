"""rr_evaluate_series (registered series, split launch) on the GPU.

Every case is checked two ways: against rr_evaluate on the same raw arrays
(the per-tile kernel: the same arithmetic per exposure, so within one
rounding of the flux), and against the FP64 oracle (1e-9 for the FP64 path, 1 ppm for the mixed path).  The cases
cover what the split launch depends on: the transit workgroups' index of
each light curve (uniform cadence, gaps, repeated times, an empty light
curve, several light curves), periods shorter than the cadence and windows
covering whole orbits, ragged and misaligned row lengths, invalid rows,
absolute (BJD-like) times, and series the split launch does not serve
(unsorted times, a light curve split into two runs, supersampled light
curves), which take the per-tile kernel.
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


def run_case(rr, w, pv=None, grid=wl.TEST_GRID, oracle_rows=None):
    pv = w["pv"] if pv is None else pv
    multi = len(w["pbids"]) > 1 or (w["lcids"] is not None and np.any(w["lcids"] != 0))
    lcids = w["lcids"] if multi else None
    tab = rr.Tables(w["mu_s"], w["I_s"], grid)
    ser = rr.TimeSeries(w["times"], lcids=lcids, pbids=w["pbids"], nss=w["nss"],
                        exptimes=w["exptimes"])
    otab = orr.Tables(w["mu_s"], w["I_s"], **grid)
    rows = slice(None) if oracle_rows is None else oracle_rows
    ref = orr.evaluate(otab, w["times"], pv[rows], lcids=lcids, pbids=w["pbids"],
                       nss=w["nss"], exptimes=w["exptimes"])
    for prec, tol in (("fp64", TOL64), ("mixed", TOL_MIXED)):
        print(f"series case {w.get('name', '')} {prec} npv={pv.shape[0]} npt={w['times'].size}",
              flush=True)
        a = rr.evaluate(tab, ser, pv, prec).cpu().numpy().astype(np.float64)
        b = rr.evaluate_unregistered(tab, ser, pv, prec).cpu().numpy().astype(np.float64)
        nan = np.isnan(b)
        assert np.array_equal(nan, np.isnan(a))
        # the same arithmetic per exposure; the two kernels' code may round
        # one multiply-add differently (a float or double ulp of the flux)
        assert np.abs(a[~nan] - b[~nan]).max(initial=0.0) <= (2e-7 if prec == "mixed"
                                                              else 1e-15)
        r = ref
        got = a[rows]
        rn = np.isnan(r)
        assert np.array_equal(rn, np.isnan(got))
        err = np.abs(got[~rn] - r[~rn]).max(initial=0.0)
        assert err <= tol, (prec, err)
        assert np.all(got[~rn][r[~rn] == 1.0] == 1.0)
    ser.close()
    tab.close()
    return a


def test_population(rr):
    w = wl.population(npv=48, npt=6000, seed_extra=21)
    f = run_case(rr, w)
    assert (f < 1).any()


def test_ragged_and_misaligned_rows(rr):
    # npt not a multiple of 4: float rows start off 16-B boundaries, so the
    # streaming tiles take their per-exposure path; a ragged last tile
    for npt in (5003, 517, 130):
        w = wl.population(npv=21, npt=npt, seed_extra=22)
        run_case(rr, w)


def test_absolute_times(rr):
    w = wl.population(npv=24, npt=4000, seed_extra=23)
    w["times"] = w["times"] + 2459000.0
    w["pv"][:, 0] += 2459000.0
    run_case(rr, w)


def test_invalid_rows_and_short_periods(rr):
    w = wl.population(npv=40, npt=3000, seed_extra=24)
    pv = w["pv"].copy()
    pv[3, 6] = 0.5            # k outside the table: NaN row
    pv[5, 1] = -1.0           # P <= 0: NaN row
    pv[7, 4] = 1.2            # e >= 1: NaN row
    pv[9, 1] = 1e-3           # period shorter than the 2-min cadence
    pv[9, 2] = 1.6
    pv[11, 1] = 0.05          # 36 exposures per orbit
    pv[11, 2] = 1.8
    pv[13, 1] = 0.4           # a = 1.3: the window covers much of the orbit
    pv[13, 2] = 1.3
    pv[13, 3] = 0.1
    f = run_case(rr, w, pv=pv)
    assert np.isnan(f[3]).all() and np.isnan(f[5]).all() and np.isnan(f[7]).all()
    assert (f[9] < 1).any() and (f[11] < 1).any()


def test_eccentric_orbits(rr):
    w = wl.population(npv=32, npt=5000, seed_extra=25)
    pv = w["pv"].copy()
    pv[:, 4] = np.linspace(0.0, 0.95, 32)
    pv[:, 2] = np.maximum(pv[:, 2], 6.0)
    run_case(rr, w, pv=pv)


def test_supersampled_passbands(rr):
    w = wl.heterogeneous(npv=40, days=8.0, seed_extra=26)
    w["name"] = "heterogeneous"
    run_case(rr, w)


def test_four_passbands_one_subsample(rr):
    """The heterogeneous workload's four light curves and passbands with one
    subsample each: the split launch (fused for these sizes) over several
    indexed light curves with their own passbands and exposure times, and
    rows with a radius ratio per passband."""
    w = wl.heterogeneous(npv=40, days=8.0, seed_extra=37)
    w["nss"] = np.ones_like(w["nss"])
    w["name"] = "four passbands, nss 1"
    multi = rr.TimeSeries(w["times"], lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"],
                          exptimes=w["exptimes"])
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    for prec in ("mixed", "fp64"):
        assert multi.kernel(tab, 40, prec) == "split_fused"
    multi.close()
    tab.close()
    run_case(rr, w)


def test_gaps_repeats_and_an_empty_light_curve(rr):
    rng = np.random.default_rng(27)
    base = wl.population(npv=24, npt=10, seed_extra=27)
    seg1 = np.arange(1500) * (2.0 / 1440.0)
    seg2 = 9.0 + np.arange(1200) * (2.0 / 1440.0)           # a 6-day gap
    t0 = np.concatenate([seg1, seg2])
    t1 = np.repeat(np.arange(300) * (30.0 / 1440.0), 3)     # each time three times
    t1 = np.concatenate([t1, np.full(50, 6.5)])              # and a run of one time
    times = np.concatenate([t0, t1])
    lcids = np.concatenate([np.zeros(t0.size, np.int32), np.full(t1.size, 2, np.int32)])
    w = dict(base)
    w["times"], w["lcids"] = times, lcids
    w["pbids"] = np.zeros(3, np.int32)                       # light curve 1 is empty
    w["nss"] = np.array([1, 1, 1], np.int32)
    w["exptimes"] = np.array([2.0, 2.0, 30.0]) / 1440.0
    w["name"] = "gaps"
    _ = rng
    run_case(rr, w)
    # the same with the last light curve supersampled (the per-tile kernel)
    w["nss"] = np.array([1, 1, 3], np.int32)
    w["name"] = "gaps supersampled"
    run_case(rr, w)


def test_series_without_index(rr):
    """Unsorted times, and a light curve in two runs: no index; the series
    is evaluated by the per-tile kernel with the same values."""
    w = wl.population(npv=16, npt=3000, seed_extra=28)
    perm = np.random.default_rng(28).permutation(3000)
    w1 = dict(w)
    w1["times"] = w["times"][perm]
    w1["name"] = "unsorted"
    run_case(rr, w1)
    w2 = wl.heterogeneous(npv=12, days=4.0, seed_extra=29)
    n = w2["times"].size
    order = np.concatenate([np.arange(0, n, 2), np.arange(1, n, 2)])   # interleaved runs
    w2["times"], w2["lcids"] = w2["times"][order], w2["lcids"][order]
    w2["name"] = "interleaved"
    run_case(rr, w2)


def test_many_rows_few_times(rr):
    w = wl.population(npv=700, npt=300, seed_extra=30)
    run_case(rr, w, oracle_rows=slice(0, 64))


def test_deterministic_and_errors(rr):
    import ctypes
    import torch
    from paper_2009_08500_amd import _lib
    w = wl.population(npv=20, npt=2000, seed_extra=31)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    for prec in ("mixed", "fp64"):
        a = rr.evaluate(tab, ser, w["pv"], prec).cpu().numpy()
        b = rr.evaluate(tab, ser, w["pv"], prec).cpu().numpy()
        assert np.array_equal(a, b)
    L = _lib.lib()
    pv = torch.as_tensor(w["pv"], device="cuda")
    out = torch.empty((20, 2000), dtype=torch.float32, device="cuda")
    rc = L.rr_evaluate_series(tab.handle, None, ctypes.c_void_p(pv.data_ptr()), 20, 7,
                              _lib.RR_MIXED, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == _lib.RR_EINVAL
    rc = L.rr_evaluate_series(tab.handle, ser.handle, ctypes.c_void_p(pv.data_ptr()), 20, 8,
                              _lib.RR_MIXED, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == _lib.RR_EINVAL
    rc = L.rr_evaluate_series(tab.handle, ser.handle, ctypes.c_void_p(pv.data_ptr()), 0, 7,
                              _lib.RR_MIXED, None, None)
    assert rc == _lib.RR_OK
    bad = rr.TimeSeries(w["times"], pbids=[3])            # passband beyond the tables
    rc = L.rr_evaluate_series(tab.handle, bad.handle, ctypes.c_void_p(pv.data_ptr()), 20, 7,
                              _lib.RR_MIXED, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == _lib.RR_EINVAL
    empty = rr.TimeSeries(np.zeros(0))
    rc = L.rr_evaluate_series(tab.handle, empty.handle, ctypes.c_void_p(pv.data_ptr()), 20, 7,
                              _lib.RR_MIXED, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == _lib.RR_OK
    tab.close()


def test_kernel_query(rr):
    """rr_series_kernel names the launch the documented rule picks: the split
    launch for an indexed series with one subsample per exposure, the
    per-tile kernel for supersampled, unindexed and the shortest series
    under more than 1024 rows; the two give the same fluxes either way."""
    w = wl.population(npv=8, npt=3000, seed_extra=32)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    for prec in ("mixed", "fp64"):
        # 8 rows: 128 transit + 24 streaming workgroups, all resident at once
        assert ser.kernel(tab, 8, prec) == "split_fused"
        assert ser.kernel(tab, 4096, prec) == "split"         # 6 tiles of 512
    short = rr.TimeSeries(w["times"][:1000])
    # (whether the split launch is fused depends on the device's capacity)
    assert short.kernel(tab, 1024, "mixed") in ("split", "split_fused")
    assert short.kernel(tab, 1025, "mixed") == "tiles"
    sup = rr.TimeSeries(w["times"], nss=[3], exptimes=[0.02])
    assert sup.kernel(tab, 8, "mixed") == "tiles"
    unsorted = rr.TimeSeries(w["times"][::-1].copy())
    assert unsorted.kernel(tab, 8, "mixed") == "tiles"
    import ctypes
    from paper_2009_08500_amd import _lib
    k = ctypes.c_int32(7)
    assert _lib.lib().rr_series_kernel(tab.handle, ser.handle, 1, 5, ctypes.byref(k)) == \
        _lib.RR_EINVAL
    for s_ in (ser, short, sup, unsorted):
        s_.close()
    tab.close()


def test_fused_launch_matches_setup_launch(rr):
    """The split launch gives the same bits whether its workgroups derive
    the rows' constants themselves (fewer rows) or read them from the
    per-row setup (many rows), and whatever its sizing: the first rows of a
    4096-row call equal 8-, 200-, 600- and 1000-row calls on the same rows,
    both precisions."""
    w = wl.population(npv=4096, npt=6000, seed_extra=35)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    for prec in ("mixed", "fp64"):
        assert ser.kernel(tab, 4096, prec) == "split"
        assert ser.kernel(tab, 8, prec) == "split_fused"
        print(f"fused vs setup launch {prec}", flush=True)
        full = rr.evaluate(tab, ser, w["pv"], prec).cpu().numpy()
        for n in (8, 200, 600, 1000):
            few = rr.evaluate(tab, ser, w["pv"][:n], prec).cpu().numpy()
            assert np.array_equal(full[:n], few, equal_nan=True), (prec, n, ser.kernel(tab, n, prec))
    ser.close()
    tab.close()


@pytest.mark.parametrize("npv,kind", [(64, "split_fused"), (4096, "split")])
def test_graph_replay_matches_eager(rr, npv, kind):
    """Evaluator.capture records one call (the fused split launch, or the
    per-row setup and the split launch) as a HIP graph; every replay, with
    eager evaluations and new rows written in place between replays, gives
    the eager call's fluxes bit for bit."""
    import torch
    w = wl.population(npv=npv, npt=6000, seed_extra=33)
    w2 = wl.population(npv=npv, npt=6000, seed_extra=34)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    for prec in ("mixed", "fp64"):
        assert ser.kernel(tab, npv, prec) == kind
        ev = rr.Evaluator(tab, ser, npv, prec)
        pv = torch.as_tensor(w["pv"], device="cuda").clone()
        ev.capture(pv)
        for it in range(5):
            rows = w["pv"] if it % 2 == 0 else w2["pv"]
            pv.copy_(torch.as_tensor(rows, device="cuda"))
            got = ev.replay().clone()
            torch.cuda.synchronize()
            ref = rr.evaluate(tab, ser, rows, prec)            # eager, between replays
            assert torch.equal(got, ref), (prec, it)
    ser.close()
    tab.close()
