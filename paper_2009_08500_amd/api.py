"""Python binding of librr.so: argument marshalling only.

PyTorch supplies device memory and streams; every step of the light-curve
path runs in the library's HIP kernels.  Arrays given as NumPy are copied to
the current CUDA/HIP device; device tensors of the right dtype and layout are
passed through without copies.
"""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import RR_FP64, RR_MIXED, RRGrid, check

# Default table resolution: z-grid cut, inner and limb bins, g and k nodes,
# k range (Sect. 3.1.1, Sect. 3.1.2, Sect. 3.3).
DEFAULT_GRID = dict(zcut=0.8, nzin=60, nzlimb=120, ng=512, nk=256, k0=0.01, k1=0.30)

TABLE_IDS = {"ze": 0, "W": 1, "ldp": 2, "istar": 3, "T64": 4, "T32": 5, "zm": 6}

PRECISIONS = {"fp64": RR_FP64, "mixed": RR_MIXED, RR_FP64: RR_FP64, RR_MIXED: RR_MIXED}


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(x, dtype):
    """A contiguous device tensor of ``dtype`` holding ``x``."""
    if isinstance(x, torch.Tensor):
        if x.is_cuda and x.dtype == dtype and x.is_contiguous():
            return x
        return x.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _host(x, dtype, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=dtype))
    if n is not None:
        a = np.ascontiguousarray(np.broadcast_to(a, (n,)))
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_grid(**kw):
    g = dict(DEFAULT_GRID)
    g.update(kw)
    return RRGrid(float(g["zcut"]), int(g["nzin"]), int(g["nzlimb"]), int(g["ng"]),
                  int(g["nk"]), float(g["k0"]), float(g["k1"]))


class Tables:
    """LD tables on the device (rr_prepare_ld): z-grid, weights, I_star and
    the LD-weighted tables for ``npb`` radial profiles sampled at ``mu``."""

    def __init__(self, mu, prof, grid=None):
        L = _lib.lib()
        mu = _host(mu, np.float64)
        prof = np.ascontiguousarray(np.atleast_2d(np.asarray(prof, np.float64)))
        self.npb, self.nmu = prof.shape
        if mu.size != self.nmu:
            raise ValueError("prof must have shape (npb, len(mu))")
        self.grid = make_grid(**(grid or {}))
        h = ctypes.c_void_p()
        check(L.rr_prepare_ld(_ptr(mu), _ptr(prof), self.nmu, self.npb,
                              ctypes.byref(self.grid), ctypes.byref(h)), "rr_prepare_ld")
        self._h = h
        self.mu = mu

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("tables already freed")
        return self._h

    @property
    def npar(self):
        return 6 + self.npb

    def set_profile(self, prof_d, stream=None):
        """Rebuild I_star and T from device profile samples [npb][nmu]."""
        prof_d = _dev(prof_d, torch.float64)
        if prof_d.numel() != self.npb * self.nmu:
            raise ValueError("profile has the wrong size")
        check(_lib.lib().rr_set_profile(self.handle, ctypes.c_void_p(prof_d.data_ptr()),
                                        _stream(stream)), "rr_set_profile")
        return prof_d

    def set_istar(self, istar=None, stream=None):
        """Normalise passband pb by istar[pb] instead of the profile
        interpolant's integral (rr_set_istar), e.g. a named law's analytic
        integral from ``ldlaws.istar``; None goes back to the integral."""
        if istar is None:
            check(_lib.lib().rr_set_istar(self.handle, None, _stream(stream)), "rr_set_istar")
            return None
        istar = _dev(istar, torch.float64).reshape(-1)
        if istar.numel() != self.npb:
            raise ValueError("istar needs one value per passband")
        check(_lib.lib().rr_set_istar(self.handle, ctypes.c_void_p(istar.data_ptr()),
                                      _stream(stream)), "rr_set_istar")
        return istar

    def copy(self, name):
        """Copy one device table to a NumPy array (synchronous)."""
        L = _lib.lib()
        which = TABLE_IDS[name]
        n = ctypes.c_int64()
        check(L.rr_tables_copy(self.handle, which, None, 0, ctypes.byref(n)), "rr_tables_copy")
        out = np.empty(n.value, np.float32 if name == "T32" else np.float64)
        check(L.rr_tables_copy(self.handle, which, _ptr(out), n.value, ctypes.byref(n)),
              "rr_tables_copy")
        sizes = self.sizes()
        nz, ng, nk, npb = sizes[0], sizes[1], sizes[2], sizes[3]
        shapes = {"W": (nk, nz, ng), "ldp": (npb, nz), "T64": (npb, nk, ng),
                  "T32": (npb, nk, ng)}
        return out.reshape(shapes.get(name, out.shape))

    def sizes(self):
        arr = (ctypes.c_int32 * 6)()
        check(_lib.lib().rr_tables_info(self.handle, None, arr), "rr_tables_info")
        return list(arr)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.lib().rr_free_tables(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TimeSeries:
    """Device-resident description of a (heterogeneous) time series
    (Sect. 4.2): mid-exposure times, light-curve ids, and per light curve
    the passband, supersampling factor and exposure time."""

    def __init__(self, times, lcids=None, pbids=None, nss=None, exptimes=None):
        self.times = _dev(times, torch.float64)
        self.npt = self.times.numel()
        if lcids is None:
            self.lcids = None
            nlc = 1 if pbids is None else len(np.atleast_1d(pbids))
        else:
            self.lcids = _dev(lcids, torch.int32)
            if pbids is None:
                nlc = int(self.lcids.max().item()) + 1 if self.npt else 1
            else:
                nlc = len(np.atleast_1d(pbids))
        self.nlc = nlc
        self.pbids = _host(0 if pbids is None else pbids, np.int32, nlc)
        self.nss = _host(1 if nss is None else nss, np.int32, nlc)
        self.exptimes = _host(0.0 if exptimes is None else exptimes, np.float64, nlc)
        # the registered form (rr_series_create, from host copies), which
        # rr_evaluate_series reads
        t_h = self.times.cpu().numpy()
        ids_h = None if self.lcids is None else self.lcids.cpu().numpy()
        h = ctypes.c_void_p()
        check(_lib.lib().rr_series_create(_ptr(t_h), None if ids_h is None else _ptr(ids_h),
                                          self.npt, _ptr(self.pbids), _ptr(self.nss),
                                          _ptr(self.exptimes), self.nlc, ctypes.byref(h)),
              "rr_series_create")
        self._series = h

    @property
    def handle(self):
        """The rr_series handle of this series."""
        if self._series is None:
            raise ValueError("series already freed")
        return self._series

    def kernel(self, tables, npv, precision="mixed"):
        """The forward kernel ``evaluate`` launches on this series for npv
        rows (rr_series_kernel): "tiles" (per-tile kernel after the per-row
        setup), "split" (split launch after the per-row setup) or
        "split_fused" (the split launch alone, deriving the rows' constants
        itself)."""
        k = ctypes.c_int32(-1)
        check(_lib.lib().rr_series_kernel(tables.handle, self.handle, int(npv),
                                          PRECISIONS[precision], ctypes.byref(k)),
              "rr_series_kernel")
        return {_lib.RR_KERNEL_SPLIT: "split",
                _lib.RR_KERNEL_SPLIT_FUSED: "split_fused"}.get(k.value, "tiles")

    def lc_args(self):
        lc = ctypes.c_void_p(self.lcids.data_ptr()) if self.lcids is not None else None
        return (lc, self.npt, _ptr(self.pbids), _ptr(self.nss), _ptr(self.exptimes), self.nlc)

    def close(self):
        if getattr(self, "_series", None) is not None:
            _lib.lib().rr_series_free(self._series)
            self._series = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NUM_VARIANTS = 6


def evaluate(tables, series, pv, precision="fp64", out=None, stream=None, variant=None):
    """Fluxes (npv, npt) for parameter rows ``pv`` (npv, 6 + npb):
    [t0, P, a, b, e, w, k_0 .. k_{npb-1}] (rr_evaluate).  Returns a device
    tensor, float64 for "fp64" and float32 for "mixed".  ``variant`` (0-5,
    see ``select_variant``) picks a forward-kernel variant
    (rr_evaluate_variant); every variant gives the same values (to float
    rounding for supersampled series in mixed precision)."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    dtype = torch.float64 if prec == RR_FP64 else torch.float32
    if out is None:
        out = torch.empty((npv, series.npt), dtype=dtype, device=pv.device)
    elif out.dtype != dtype or not out.is_contiguous() or out.numel() != npv * series.npt:
        raise ValueError("out has the wrong dtype, layout or size")
    if variant is None:
        check(_lib.lib().rr_evaluate_series(tables.handle, series.handle,
                                            ctypes.c_void_p(pv.data_ptr()), npv, npar, prec,
                                            ctypes.c_void_p(out.data_ptr()), _stream(stream)),
              "rr_evaluate_series")
        return out
    lc, npt, pb, nss, ex, nlc = series.lc_args()
    if variant is not None:
        check(_lib.lib().rr_evaluate_variant(
            tables.handle, ctypes.c_void_p(series.times.data_ptr()), lc, npt, pb, nss, ex, nlc,
            ctypes.c_void_p(pv.data_ptr()), npv, npar, prec, int(variant),
            ctypes.c_void_p(out.data_ptr()), _stream(stream)), "rr_evaluate_variant")
        return out
    check(_lib.lib().rr_evaluate(tables.handle, ctypes.c_void_p(series.times.data_ptr()),
                                 lc, npt, pb, nss, ex, nlc,
                                 ctypes.c_void_p(pv.data_ptr()), npv, npar, prec,
                                 ctypes.c_void_p(out.data_ptr()), _stream(stream)),
          "rr_evaluate")
    return out


def evaluate_unregistered(tables, series, pv, precision="fp64", out=None, stream=None):
    """rr_evaluate on the series' raw arrays (no registered index): the same
    values as ``evaluate``, through the per-tile kernel."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    dtype = torch.float64 if prec == RR_FP64 else torch.float32
    if out is None:
        out = torch.empty((npv, series.npt), dtype=dtype, device=pv.device)
    elif out.dtype != dtype or not out.is_contiguous() or out.numel() != npv * series.npt:
        raise ValueError("out has the wrong dtype, layout or size")
    lc, npt, pb, nss, ex, nlc = series.lc_args()
    check(_lib.lib().rr_evaluate(tables.handle, ctypes.c_void_p(series.times.data_ptr()),
                                 lc, npt, pb, nss, ex, nlc,
                                 ctypes.c_void_p(pv.data_ptr()), npv, npar, prec,
                                 ctypes.c_void_p(out.data_ptr()), _stream(stream)),
          "rr_evaluate")
    return out


def select_variant(tables, series, pv, precision="mixed", reps=20, stream=None):
    """Trial-run selection of the forward-kernel variant (rr_select_variant,
    the GPU form of Sect. 3.4.1's choice among implementations): times
    every variant on these inputs (``reps`` launches each, after one
    untimed) and returns (best, ms) with ms[v] the mean milliseconds per
    forward launch of variant v.  Variants 0, 1, 2 give each lane 4, 8, 16
    exposures (1 is rr_evaluate's), spreading the subsamples of
    supersampled exposures over lanes where a wave's flags are sparse enough
    for that to pay; 3, 4, 5 are the same with supersampled exposures always
    evaluated one per lane.  Waits
    for the stream."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    dtype = torch.float64 if prec == RR_FP64 else torch.float32
    out = torch.empty((npv, series.npt), dtype=dtype, device=pv.device)
    lc, npt, pb, nss, ex, nlc = series.lc_args()
    best = ctypes.c_int32(-1)
    ms = (ctypes.c_float * NUM_VARIANTS)()
    check(_lib.lib().rr_select_variant(
        tables.handle, ctypes.c_void_p(series.times.data_ptr()), lc, npt, pb, nss, ex, nlc,
        ctypes.c_void_p(pv.data_ptr()), npv, npar, prec, ctypes.c_void_p(out.data_ptr()),
        int(reps), ctypes.byref(best), ms, _stream(stream)), "rr_select_variant")
    return best.value, [float(x) for x in ms]


def evaluate_direct(tables, series, pv, precision="fp64", out=None, stream=None):
    """Fluxes of the direct model (rr_evaluate_direct): weights built for
    each row's own k, no k-interpolation, any k in (0, 1].  Arguments and
    result as ``evaluate``."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    dtype = torch.float64 if prec == RR_FP64 else torch.float32
    if out is None:
        out = torch.empty((npv, series.npt), dtype=dtype, device=pv.device)
    elif out.dtype != dtype or not out.is_contiguous() or out.numel() != npv * series.npt:
        raise ValueError("out has the wrong dtype, layout or size")
    lc, npt, pb, nss, ex, nlc = series.lc_args()
    check(_lib.lib().rr_evaluate_direct(tables.handle, ctypes.c_void_p(series.times.data_ptr()),
                                        lc, npt, pb, nss, ex, nlc,
                                        ctypes.c_void_p(pv.data_ptr()), npv, npar, prec,
                                        ctypes.c_void_p(out.data_ptr()), _stream(stream)),
          "rr_evaluate_direct")
    return out


def evaluate_small_planet(tables, series, pv, k_small, precision="fp64", out=None,
                          stream=None):
    """Fluxes with the small-planet approximation (rr_evaluate_small_planet,
    Sect. 3.4.2): a passband whose k is below ``k_small`` uses the LD value
    at the planet's centre instead of the mean over its disk, and may lie
    below the tables' k0; the others are evaluated as ``evaluate``.
    Arguments and result as ``evaluate``."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    dtype = torch.float64 if prec == RR_FP64 else torch.float32
    if out is None:
        out = torch.empty((npv, series.npt), dtype=dtype, device=pv.device)
    elif out.dtype != dtype or not out.is_contiguous() or out.numel() != npv * series.npt:
        raise ValueError("out has the wrong dtype, layout or size")
    lc, npt, pb, nss, ex, nlc = series.lc_args()
    check(_lib.lib().rr_evaluate_small_planet(
        tables.handle, ctypes.c_void_p(series.times.data_ptr()), lc, npt, pb, nss, ex, nlc,
        ctypes.c_void_p(pv.data_ptr()), npv, npar, float(k_small), prec,
        ctypes.c_void_p(out.data_ptr()), _stream(stream)), "rr_evaluate_small_planet")
    return out


def flux_at_z(tables, z, k, pb=0, precision="fp64", stream=None):
    """Eq. 5 at separations ``z`` for radius ratio ``k`` (a scalar or one per
    separation), planet in front of the star (rr_flux_at_z).  Returns a
    device tensor shaped like ``z``."""
    prec = PRECISIONS[precision]
    z = _dev(z, torch.float64)
    kd = None
    if isinstance(k, (int, float)):
        kc = float(k)
    else:
        kd = _dev(k, torch.float64)
        if kd.numel() != z.numel():
            raise ValueError("k must be a scalar or have one value per separation")
        kc = 0.0
    out = torch.empty(z.shape, dtype=torch.float64 if prec == RR_FP64 else torch.float32,
                      device=z.device)
    check(_lib.lib().rr_flux_at_z(tables.handle, ctypes.c_void_p(z.data_ptr()),
                                  ctypes.c_void_p(kd.data_ptr()) if kd is not None else None,
                                  kc, z.numel(), int(pb), prec,
                                  ctypes.c_void_p(out.data_ptr()), _stream(stream)),
          "rr_flux_at_z")
    return out


def evaluate_ld(tables, series, pv, prof, precision="fp64", out=None, stream=None):
    """Fluxes (npv, npt) with a limb-darkening profile per parameter row
    (rr_evaluate_ld).  ``prof`` holds the radial profile samples of every
    row and passband on the tables' mu samples, shape (npv, npb, nmu) (or
    (npv, nmu) with one passband), e.g. from :mod:`ldlaws`.  Returns a
    device tensor, float64 for "fp64" and float32 for "mixed"."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    prof = _dev(prof, torch.float64)
    if prof.numel() != npv * tables.npb * tables.nmu:
        raise ValueError("prof must have npv * npb * nmu samples")
    dtype = torch.float64 if prec == RR_FP64 else torch.float32
    if out is None:
        out = torch.empty((npv, series.npt), dtype=dtype, device=pv.device)
    elif out.dtype != dtype or not out.is_contiguous() or out.numel() != npv * series.npt:
        raise ValueError("out has the wrong dtype, layout or size")
    lc, npt, pb, nss, ex, nlc = series.lc_args()
    check(_lib.lib().rr_evaluate_ld(tables.handle, ctypes.c_void_p(series.times.data_ptr()),
                                    lc, npt, pb, nss, ex, nlc,
                                    ctypes.c_void_p(pv.data_ptr()), npv, npar,
                                    ctypes.c_void_p(prof.data_ptr()), prec,
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)),
          "rr_evaluate_ld")
    return out


class Evaluator:
    """rr_evaluate for repeated calls with populations of one size over one
    time series (the MCMC pattern): every argument except the parameter
    rows is marshalled once, and the output buffer is reused.  Calls enqueue
    on the stream current at construction (or ``stream``).  ``variant``
    fixes a forward-kernel variant (``select_variant``); ``select(pv)``
    chooses it by a trial run on the given rows, and ``auto_select=True``
    runs that trial on the first call's rows, as the paper's model does
    after set-up (Sect. 3.4.1)."""

    def __init__(self, tables, series, npv, precision="mixed", stream=None, variant=None,
                 auto_select=False):
        if not isinstance(series, TimeSeries):
            series = TimeSeries(series)
        self.tables, self.series, self.npv = tables, series, int(npv)
        self.prec = PRECISIONS[precision]
        self.npar = tables.npar
        dtype = torch.float64 if self.prec == RR_FP64 else torch.float32
        self.out = torch.empty((self.npv, series.npt), dtype=dtype, device="cuda")
        lc, npt, pb, nss, ex, nlc = series.lc_args()
        s = torch.cuda.current_stream() if stream is None else stream
        self._stream = s
        self._base = [tables.handle, series.times.data_ptr(), lc, npt, pb, nss, ex, nlc,
                      None, self.npv, self.npar, self.prec]
        self._set_variant(variant)
        self._auto = bool(auto_select) and variant is None

    def _set_variant(self, variant):
        self.variant = variant
        if variant is None:
            self._fn = _lib.lib().rr_evaluate_series
            self._args = [self.tables.handle, self.series.handle, None, self.npv, self.npar,
                          self.prec, self.out.data_ptr(), self._stream.cuda_stream]
            self._pv_arg = 2
        else:
            if not 0 <= int(variant) < NUM_VARIANTS:
                raise ValueError("variant must lie in [0, 6)")
            self._fn = _lib.lib().rr_evaluate_variant
            self._args = self._base + [int(variant), self.out.data_ptr(),
                                       self._stream.cuda_stream]
            self._pv_arg = 8

    def select(self, pv, reps=20):
        """Trial run of every variant on rows ``pv`` (``select_variant``);
        later calls use the fastest.  Returns (best, ms)."""
        with torch.cuda.stream(self._stream):
            best, ms = select_variant(self.tables, self.series, pv,
                                      "fp64" if self.prec == RR_FP64 else "mixed", reps)
        self._set_variant(best)
        return best, ms

    def __call__(self, pv):
        """Fluxes (npv, npt) for a contiguous float64 device tensor of rows."""
        if (pv.dtype is not torch.float64 or not pv.is_cuda or not pv.is_contiguous()
                or pv.numel() != self.npv * self.npar):
            raise ValueError("pv must be a float64 device tensor of shape (npv, npar)")
        if self._auto:
            self._auto = False
            self.select(pv)
        a = self._args
        a[self._pv_arg] = pv.data_ptr()
        rc = self._fn(*a)
        if rc:
            check(rc, "rr_evaluate")
        return self.out

    def capture(self, pv):
        """Record one call on rows ``pv`` as a HIP graph (torch.cuda.CUDAGraph)
        on a private stream, after a warm-up call there.  ``replay()`` then
        runs the same kernels from one graph launch: the graph reads the rows
        from ``pv``'s memory (write new rows into that tensor in place
        between replays) and writes ``self.out``.  For callers that work
        under graph capture or build larger graphs around the evaluation; a
        replay is not faster than an eager call here (on one MI355X, 512
        rows x 20 000 times: 33.7 us per replay against 28.9 us per call).
        Nothing the graph records allocates or fills memory."""
        if (pv.dtype is not torch.float64 or not pv.is_cuda or not pv.is_contiguous()
                or pv.numel() != self.npv * self.npar):
            raise ValueError("pv must be a float64 device tensor of shape (npv, npar)")
        s = torch.cuda.Stream()
        args = list(self._args)
        args[self._pv_arg] = pv.data_ptr()
        args[-1] = s.cuda_stream
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):           # workspace for this stream, cached choices
                check(self._fn(*args), "rr_evaluate (graph warm-up)")
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            rc = self._fn(*args)
        check(rc, "rr_evaluate (graph capture)")
        self._graph, self._graph_pv = g, pv
        return g

    def replay(self):
        """Run the captured call (``capture``); returns ``self.out``."""
        if getattr(self, "_graph", None) is None:
            raise RuntimeError("capture(pv) first")
        self._graph.replay()
        return self.out


def loglik_grad(tables, series, pv, obs, sigma, precision="fp64", grad=True, profile=False,
                wprof=None, stream=None, istar_grad=False):
    """Gaussian log-likelihood of ``obs`` under each parameter row and its
    gradients (rr_loglik_grad).  Returns (logl[npv], grad[npv, npar] or None,
    grad_profile[npb, nmu] or None), float64 device tensors; grad_profile is
    the gradient of sum(wprof * logl) (wprof = ones if None) with respect to
    the tables' LD profile samples.  With ``istar_grad`` (rr_loglik_grad_istar)
    a fourth tensor, the gradient of the same sum with respect to each
    passband's I_star, follows."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    obs = _dev(obs, torch.float64 if prec == RR_FP64 else torch.float32)
    if obs.numel() != series.npt:
        raise ValueError("obs must have one value per time")
    logl = torch.empty(npv, dtype=torch.float64, device=pv.device)
    g = torch.empty((npv, npar), dtype=torch.float64, device=pv.device) if grad else None
    gp = (torch.empty((tables.npb, tables.nmu), dtype=torch.float64, device=pv.device)
          if profile else None)
    w = _dev(wprof, torch.float64) if wprof is not None else None

    def p(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    lc, npt, pb, nss, ex, nlc = series.lc_args()
    if istar_grad:
        gi = torch.empty(tables.npb, dtype=torch.float64, device=pv.device)
        check(_lib.lib().rr_loglik_grad_istar(tables.handle, p(series.times), lc, npt, pb, nss,
                                              ex, nlc, p(pv), npv, npar, prec, p(obs),
                                              float(sigma), p(w), p(logl), p(g), p(gp), p(gi),
                                              _stream(stream)),
              "rr_loglik_grad_istar")
        return logl, g, gp, gi
    check(_lib.lib().rr_loglik_grad(tables.handle, p(series.times), lc, npt, pb, nss, ex, nlc,
                                    p(pv), npv, npar, prec, p(obs), float(sigma), p(w),
                                    p(logl), p(g), p(gp), _stream(stream)),
          "rr_loglik_grad")
    return logl, g, gp


def loglik_grad_small_planet(tables, series, pv, obs, sigma, k_small, precision="fp64",
                             grad=True, stream=None):
    """rr_loglik_grad_small_planet: the log-likelihood of ``obs`` under the
    small-planet approximation below ``k_small`` (Sect. 3.4.2) and its
    parameter gradient.  Returns (logl[npv], grad[npv, npar] or None),
    float64 device tensors."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    obs = _dev(obs, torch.float64 if prec == RR_FP64 else torch.float32)
    if obs.numel() != series.npt:
        raise ValueError("obs must have one value per time")
    logl = torch.empty(npv, dtype=torch.float64, device=pv.device)
    g = torch.empty((npv, npar), dtype=torch.float64, device=pv.device) if grad else None

    def p(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    lc, npt, pb, nss, ex, nlc = series.lc_args()
    check(_lib.lib().rr_loglik_grad_small_planet(
        tables.handle, p(series.times), lc, npt, pb, nss, ex, nlc, p(pv), npv, npar,
        float(k_small), prec, p(obs), float(sigma), p(logl), p(g), _stream(stream)),
        "rr_loglik_grad_small_planet")
    return logl, g


def loglik_grad_ld(tables, series, pv, prof, obs, sigma, precision="fp64", grad=True,
                   profile=True, stream=None):
    """rr_loglik_grad_ld: the log-likelihood with a profile per parameter row
    ``prof`` (npv, npb, nmu).  Returns (logl[npv], grad[npv, npar] or None,
    grad_profile[npv, npb, nmu] or None), float64 device tensors;
    grad_profile[i] is d logl[i] / d prof[i]."""
    prec = PRECISIONS[precision]
    if not isinstance(series, TimeSeries):
        series = TimeSeries(series)
    pv = _dev(pv, torch.float64)
    if pv.dim() == 1:
        pv = pv.unsqueeze(0)
    npv, npar = pv.shape
    prof = _dev(prof, torch.float64)
    if prof.numel() != npv * tables.npb * tables.nmu:
        raise ValueError("prof must have npv * npb * nmu samples")
    obs = _dev(obs, torch.float64 if prec == RR_FP64 else torch.float32)
    if obs.numel() != series.npt:
        raise ValueError("obs must have one value per time")
    logl = torch.empty(npv, dtype=torch.float64, device=pv.device)
    g = torch.empty((npv, npar), dtype=torch.float64, device=pv.device) if grad else None
    gp = (torch.empty((npv, tables.npb, tables.nmu), dtype=torch.float64, device=pv.device)
          if profile else None)

    def p(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    lc, npt, pb, nss, ex, nlc = series.lc_args()
    check(_lib.lib().rr_loglik_grad_ld(tables.handle, p(series.times), lc, npt, pb, nss, ex,
                                       nlc, p(pv), npv, npar, p(prof), prec, p(obs),
                                       float(sigma), p(logl), p(g), p(gp), _stream(stream)),
          "rr_loglik_grad_ld")
    return logl, g, gp


class RRLogLikLD(torch.autograd.Function):
    """logL[npv] = rr_loglik_grad_ld(...) as a differentiable function of the
    parameter rows ``pv`` [npv, npar] and the per-row LD profiles ``prof``
    [npv, npb, nmu]; backward returns the hand-written adjoint's gradients."""

    @staticmethod
    def forward(ctx, pv, prof, tables, series, obs, sigma, precision):
        want_prof = prof.requires_grad
        logl, g, gp = loglik_grad_ld(tables, series, pv.detach(), prof.detach(), obs, sigma,
                                     precision, grad=True, profile=want_prof)
        ctx.save_for_backward(g, gp if gp is not None else torch.empty(0))
        ctx.want_prof = want_prof
        return logl

    @staticmethod
    def backward(ctx, gout):
        g, gp = ctx.saved_tensors
        gpv = gout[:, None] * g
        gprof = gout[:, None, None] * gp if ctx.want_prof else None
        return gpv, gprof, None, None, None, None, None


class RRLogLik(torch.autograd.Function):
    """logL[npv] = rr_loglik_grad(...) as a differentiable function of the
    parameter rows ``pv`` [npv, npar], the LD profile samples ``profile``
    [npb, nmu] and, optionally, the normalisers ``istar`` [npb] (a law's
    closed-form disk integral, e.g. ``ldlaws.istar``; None: the profile
    interpolant's integral).  Backward returns the hand-written adjoint's
    gradients (rr_loglik_grad_istar for ``istar``).

    The profile (and ``istar``) are written into ``tables`` on the current
    stream (rr_set_profile, rr_set_istar): the tables then hold them for
    every later use, and work on other streams must not read those tables
    meanwhile -- give the function a Tables object of its own."""

    @staticmethod
    def forward(ctx, pv, profile, tables, series, obs, sigma, precision, istar=None):
        if profile is not None:
            tables.set_profile(profile.detach())
        if istar is not None:
            tables.set_istar(istar.detach())
        want_prof = profile is not None and profile.requires_grad
        want_ist = istar is not None and istar.requires_grad
        out = loglik_grad(tables, series, pv.detach(), obs, sigma, precision,
                          grad=True, profile=want_prof, istar_grad=want_ist)
        logl, g, gp = out[:3]
        gi = out[3] if want_ist else None
        ctx.tables, ctx.series, ctx.sigma, ctx.precision = tables, series, sigma, precision
        ctx.want_prof, ctx.want_ist = want_prof, want_ist
        ctx.save_for_backward(pv.detach(), profile.detach() if profile is not None else None,
                              istar.detach() if istar is not None else None,
                              obs if isinstance(obs, torch.Tensor) else torch.as_tensor(obs),
                              g, gp, gi)
        return logl

    @staticmethod
    def backward(ctx, gout):
        pv, profile, istar, obs, g, gp, gi = ctx.saved_tensors
        gpv = gout[:, None] * g
        gprof = gist = None
        if ctx.want_prof or ctx.want_ist:
            if bool(torch.all(gout == gout[0])):
                gprof = gp * gout[0] if ctx.want_prof else None
                gist = gi * gout[0] if ctx.want_ist else None
            else:
                if profile is not None:
                    ctx.tables.set_profile(profile)
                if istar is not None:
                    ctx.tables.set_istar(istar)
                out = loglik_grad(ctx.tables, ctx.series, pv, obs, ctx.sigma, ctx.precision,
                                  grad=False, profile=ctx.want_prof, wprof=gout.detach(),
                                  istar_grad=ctx.want_ist)
                gprof = out[2] if ctx.want_prof else None
                gist = out[3] if ctx.want_ist else None
        return gpv, gprof, None, None, None, None, None, gist
