"""rr_evaluate_noalloc (the entry point for callers that cannot allocate)
against rr_evaluate, both through the C ABI: same kernels, so the fluxes
agree bit for bit.  Two calls in a row, the second with fewer rows and
times, so that it runs over the first call's leftovers in the fixed device
array; both precisions; a supersampled four-passband series beside the
plain population; the size limit and empty calls."""

import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_08500_amd as rr
    return rr


def _call(rr, fn, tab, ser, pv, prec):
    import torch
    from paper_2009_08500_amd import _lib
    code = _lib.RR_FP64 if prec == "fp64" else _lib.RR_MIXED
    dtype = torch.float64 if prec == "fp64" else torch.float32
    pv = torch.as_tensor(np.ascontiguousarray(pv), dtype=torch.float64, device="cuda")
    npv, npar = pv.shape
    out = torch.full((npv, ser.npt), -7.0, dtype=dtype, device="cuda")
    lc, npt, pb, nss, ex, nlc = ser.lc_args()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(_lib.lib(), fn)(tab.handle, ctypes.c_void_p(ser.times.data_ptr()), lc, npt,
                                 pb, nss, ex, nlc, ctypes.c_void_p(pv.data_ptr()), npv, npar,
                                 code, ctypes.c_void_p(out.data_ptr()), stream)
    _lib.check(rc, fn)
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_equals_rr_evaluate(rr, prec):
    big = wl.population(npv=700, npt=9000, seed_extra=11)
    small = wl.population(npv=45, npt=2100, seed_extra=12)
    tab = rr.Tables(big["mu_s"], big["I_s"], wl.TEST_GRID)
    for w in (big, small):                       # the second call is smaller
        ser = rr.TimeSeries(w["times"])
        print(f"noalloc {prec}: npv={w['pv'].shape[0]} npt={ser.npt}", flush=True)
        a = _call(rr, "rr_evaluate_noalloc", tab, ser, w["pv"], prec)
        b = _call(rr, "rr_evaluate", tab, ser, w["pv"], prec)
        assert np.array_equal(a, b)
        assert np.isfinite(a).all() and (a < 1).any()
    tab.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_supersampled_passbands(rr, prec):
    w = wl.heterogeneous(npv=96, days=6.0, seed_extra=3)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"], lcids=w["lcids"], pbids=w["pbids"], nss=w["nss"],
                        exptimes=w["exptimes"])
    for rows in (slice(0, 96), slice(10, 30)):
        pv = w["pv"][rows]
        print(f"noalloc heterogeneous {prec}: npv={pv.shape[0]}", flush=True)
        a = _call(rr, "rr_evaluate_noalloc", tab, ser, pv, prec)
        b = _call(rr, "rr_evaluate", tab, ser, pv, prec)
        assert np.array_equal(a, b)
    tab.close()


def test_noalloc_limits(rr):
    import torch
    from paper_2009_08500_amd import _lib
    w = wl.population(npv=4, npt=300, seed_extra=13)
    tab = rr.Tables(w["mu_s"], w["I_s"], wl.TEST_GRID)
    ser = rr.TimeSeries(w["times"])
    L = _lib.lib()
    lc, npt, pb, nss, ex, nlc = ser.lc_args()
    n = _lib.RR_NOALLOC_MAX_PV + 1
    pv = torch.as_tensor(np.tile(w["pv"][:1], (n, 1)), device="cuda")
    out = torch.empty((n, ser.npt), dtype=torch.float32, device="cuda")
    rc = L.rr_evaluate_noalloc(tab.handle, ctypes.c_void_p(ser.times.data_ptr()), lc, npt, pb,
                               nss, ex, nlc, ctypes.c_void_p(pv.data_ptr()), n, 7,
                               _lib.RR_MIXED, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == _lib.RR_ELIMIT and "RR_NOALLOC_MAX_PV" in _lib.last_error()
    rc = L.rr_evaluate_noalloc(tab.handle, ctypes.c_void_p(ser.times.data_ptr()), lc, npt, pb,
                               nss, ex, nlc, ctypes.c_void_p(pv.data_ptr()), 0, 7,
                               _lib.RR_MIXED, None, None)
    assert rc == _lib.RR_OK
    # the largest allowed call works and matches rr_evaluate
    m = _lib.RR_NOALLOC_MAX_PV
    short = rr.TimeSeries(w["times"][:64])
    pvm = wl.population(npv=m, npt=64, seed_extra=14)["pv"]
    a = _call(rr, "rr_evaluate_noalloc", tab, short, pvm, "mixed")
    b = _call(rr, "rr_evaluate", tab, short, pvm, "mixed")
    assert np.array_equal(a, b)
    tab.close()
