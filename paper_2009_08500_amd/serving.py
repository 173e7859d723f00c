"""Python binding of the continuous-batching server (include/rr_serve.h):
argument marshalling only; scheduling, batching and admission run in the
library's worker thread."""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import RR_FP64, check
from .api import PRECISIONS, _host, _ptr

REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2


def _declare(L):
    if getattr(L, "_rr_serve_declared", False):
        return
    v, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.rr_server_create.argtypes = [v, i64, i32, ctypes.POINTER(v)]
    L.rr_server_add_series.argtypes = [v, v, v, i32, v, v, v, i32, ctypes.POINTER(i32)]
    L.rr_server_submit.argtypes = [v, i32, v, i32, i32, i32, v, ctypes.POINTER(i64)]
    L.rr_server_submit_device.argtypes = [v, i32, v, i32, i32, i32, v, ctypes.POINTER(i64)]
    L.rr_server_fail_next_tick.argtypes = [v]
    L.rr_server_poll.argtypes = [v, i64, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.rr_server_wait.argtypes = [v, i64, dbl, ctypes.POINTER(dbl)]
    L.rr_server_release.argtypes = [v, i64]
    L.rr_server_stats.argtypes = [v, ctypes.POINTER(i64)]
    L.rr_server_destroy.argtypes = [v]
    L.rr_server_destroy.restype = None
    for f in ("rr_server_create", "rr_server_add_series", "rr_server_submit",
              "rr_server_submit_device", "rr_server_fail_next_tick", "rr_server_poll",
              "rr_server_wait", "rr_server_release", "rr_server_stats"):
        getattr(L, f).restype = ctypes.c_int
    L._rr_serve_declared = True


class Request:
    """A submitted request: its id and its output buffer (page-locked host
    memory, or a device tensor for ``submit(..., device_out=True)``)."""

    def __init__(self, rid, out, npv, npt):
        self.id, self.out, self.npv, self.npt = rid, out, npv, npt
        self.latency = None


class Server:
    """rr_server over resident tables (see include/rr_serve.h)."""

    def __init__(self, tables, budget_bytes=8 << 30, max_tick_blocks=4096):
        self.L = _lib.lib()
        _declare(self.L)
        self.tables = tables
        h = ctypes.c_void_p()
        check(self.L.rr_server_create(tables.handle, int(budget_bytes), int(max_tick_blocks),
                                      ctypes.byref(h)), "rr_server_create")
        self._h = h
        self.series_npt = {}

    def add_series(self, times, lcids=None, pbids=None, nss=None, exptimes=None):
        times = _host(times, np.float64)
        npt = times.size
        if lcids is None:
            lc = None
            nlc = 1 if pbids is None else len(np.atleast_1d(pbids))
        else:
            lc = _host(lcids, np.int32)
            nlc = len(np.atleast_1d(pbids)) if pbids is not None else int(lc.max()) + 1
        pb = _host(0 if pbids is None else pbids, np.int32, nlc)
        ns = _host(1 if nss is None else nss, np.int32, nlc)
        ex = _host(0.0 if exptimes is None else exptimes, np.float64, nlc)
        sid = ctypes.c_int32()
        check(self.L.rr_server_add_series(self._h, _ptr(times), _ptr(lc) if lc is not None else None,
                                          npt, _ptr(pb), _ptr(ns), _ptr(ex), nlc, ctypes.byref(sid)),
              "rr_server_add_series")
        self.series_npt[sid.value] = npt
        return sid.value

    def submit(self, series_id, pv, precision="mixed", device_out=False, out=None):
        """Queue rows ``pv`` against a registered series.  The output goes to
        host memory (rr_server_submit: ``out``, page-locked for an
        asynchronous copy, or a new page-locked tensor), or with
        ``device_out`` to a device tensor (``out``, or a new one) that the
        kernels write directly (rr_server_submit_device); read it only once
        the request is done."""
        prec = PRECISIONS[precision]
        pv = np.ascontiguousarray(np.atleast_2d(np.asarray(pv, np.float64)))
        npv, npar = pv.shape
        npt = self.series_npt.get(series_id, 1)
        dtype = torch.float64 if prec == RR_FP64 else torch.float32
        rid = ctypes.c_int64()
        if device_out:
            if out is None:
                out = torch.empty((npv, npt), dtype=dtype, device="cuda")
            elif (not out.is_cuda or out.dtype != dtype or not out.is_contiguous()
                  or out.numel() != npv * npt):
                raise ValueError("out must be a contiguous device tensor of npv x npt")
            check(self.L.rr_server_submit_device(self._h, series_id, _ptr(pv), npv, npar, prec,
                                                 ctypes.c_void_p(out.data_ptr()),
                                                 ctypes.byref(rid)),
                  "rr_server_submit_device")
        else:
            if out is None:
                out = torch.empty((npv, npt), dtype=dtype, pin_memory=True)
            elif (out.is_cuda or out.dtype != dtype or not out.is_contiguous()
                  or out.numel() != npv * npt):
                raise ValueError("out must be a contiguous host tensor of npv x npt")
            check(self.L.rr_server_submit(self._h, series_id, _ptr(pv), npv, npar, prec,
                                          ctypes.c_void_p(out.data_ptr()), ctypes.byref(rid)),
                  "rr_server_submit")
        return Request(rid.value, out, npv, npt)

    def fail_next_tick(self):
        """Test hook: the next grouped launch is treated as failed on the
        host (rr_server_fail_next_tick)."""
        check(self.L.rr_server_fail_next_tick(self._h), "rr_server_fail_next_tick")

    def poll(self, req):
        st, lat = ctypes.c_int32(), ctypes.c_double()
        check(self.L.rr_server_poll(self._h, req.id, ctypes.byref(st), ctypes.byref(lat)),
              "rr_server_poll")
        if st.value == REQ_DONE:
            req.latency = lat.value
        return st.value

    def wait(self, req, timeout=120.0):
        lat = ctypes.c_double()
        check(self.L.rr_server_wait(self._h, req.id, float(timeout), ctypes.byref(lat)),
              "rr_server_wait")
        req.latency = lat.value
        return req.out

    def release(self, req):
        check(self.L.rr_server_release(self._h, req.id), "rr_server_release")

    def stats(self):
        a = (ctypes.c_int64 * 5)()
        check(self.L.rr_server_stats(self._h, a), "rr_server_stats")
        return dict(completed=a[0], points=a[1], ticks=a[2], incoming=a[3], last_error=a[4])

    def close(self):
        if getattr(self, "_h", None) is not None:
            self.L.rr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
