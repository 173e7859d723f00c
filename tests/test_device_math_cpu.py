"""The device math of rr_device.h, built for the host from the same template
code the kernels instantiate (tests/host/math_probe.hip supplies host
stand-ins of the GPU's reciprocal and square-root estimates), against
40-digit references (mpmath) over the domains the kernels use it on:

* atan2_poly, float: relative error <= 3e-7 (the polynomial's 1.14e-7 in
  exact arithmetic plus float evaluation); double: <= 5e-16 (2 ulp); the
  axes and octant boundaries exactly.
* rcp_nr: within 1 ulp of 1/x from any estimate within 2^-16.
* sincos_small, float, |x| <= 1/4 (the series): <= 6e-8 absolute.
* lens_area: absolute error <= 1e-6 min(1, k) in float (a flux error below
  1e-6 k / pi of the stellar intensity) and <= 1e-12 min(1, k)^2 in double,
  contact points included; exactly 0 without overlap, pi min(1, k)^2 inside.
* kepler_offset (transit-centred Kepler): the residual of Kepler's equation
  at the returned offset <= 3e-7 max(1, |d|) in float and 1e-15 max(1, |d|)
  in double for e up to 0.99, with sin(d/2), cos(d/2) consistent to 2e-7 /
  1e-15.
* the arctangent coefficients are the ones fit_atan_poly.py derives.
"""

import ctypes
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
mp.mp.dps = 40

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("mathprobe") / "libmathprobe.so")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-host-only",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2009_08500_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "math_probe.hip"), "-o", out],
                   check=True, capture_output=True)
    lib = ctypes.CDLL(out)
    f, d = ctypes.c_float, ctypes.c_double
    fp, dp = ctypes.POINTER(f), ctypes.POINTER(d)
    for name, res, args in (("probe_atan2f", f, [f, f]), ("probe_atan2d", d, [d, d]),
                            ("probe_rcp_nr", d, [d, d]), ("probe_sincos_small_f", None, [f, fp, fp]),
                            ("probe_lens_area_f", f, [f, f, f]), ("probe_lens_area_d", d, [d, d, d]),
                            ("probe_kepler_f", f, [f, f, f, f, fp, fp]),
                            ("probe_kepler_d", d, [d, d, d, d, dp, dp])):
        fn = getattr(lib, name)
        fn.argtypes, fn.restype = args, res
    return lib


def f32(x):
    return float(np.float32(x))


def test_atan2(L):
    rng = np.random.default_rng(11)
    ang = np.concatenate([np.linspace(-np.pi, np.pi, 2001), rng.uniform(-np.pi, np.pi, 2000)])
    rad = np.exp(rng.uniform(-5, 5, ang.size))
    wf = wd = 0.0
    for a, r in zip(ang, rad):
        y, x = r * np.sin(a), r * np.cos(a)
        yf, xf = f32(y), f32(x)
        ref = mp.atan2(yf, xf)
        if ref != 0:
            wf = max(wf, float(abs(L.probe_atan2f(yf, xf) - ref) / abs(ref)))
        ref = mp.atan2(y, x)
        if ref != 0:
            wd = max(wd, float(abs(L.probe_atan2d(y, x) - ref) / abs(ref)))
    assert wf <= 3e-7, wf
    assert wd <= 5e-16, wd
    # axes: exact zeros, and the quarter and half turns to the constants' rounding
    assert L.probe_atan2f(0.0, 1.0) == 0.0 and L.probe_atan2d(0.0, 2.0) == 0.0
    assert abs(L.probe_atan2d(1.0, 0.0) - np.pi / 2) <= 2.3e-16
    assert abs(L.probe_atan2d(0.0, -1.0) - np.pi) <= 4.5e-16
    assert abs(L.probe_atan2d(-1.0, -1e-300) + np.pi / 2) <= 2.3e-16
    assert abs(L.probe_atan2f(-1.0, 0.0) + np.pi / 2) <= 1.2e-7
    assert abs(L.probe_atan2f(1.0, 1.0) - np.pi / 4) <= 1e-7


def test_rcp_nr(L):
    rng = np.random.default_rng(12)
    xs = np.exp(rng.uniform(-60, 60, 2000)) * rng.choice([-1.0, 1.0], 2000)
    worst = 0.0
    for x in xs:
        for err in (0.0, 2.0 ** -16, -(2.0 ** -16), 2.0 ** -23, -(2.0 ** -30)):
            got = L.probe_rcp_nr(x, err)
            worst = max(worst, float(abs(got - 1 / mp.mpf(x)) / np.spacing(abs(1.0 / x))))
    assert worst <= 1.0, worst


def test_sincos_small(L):
    worst = 0.0
    for x in np.linspace(-0.25, 0.25, 4001):
        s, c = ctypes.c_float(), ctypes.c_float()
        xf = f32(x)
        L.probe_sincos_small_f(xf, ctypes.byref(s), ctypes.byref(c))
        worst = max(worst, float(max(abs(s.value - mp.sin(xf)), abs(c.value - mp.cos(xf)))))
    assert worst <= 6e-8, worst


def lens_exact(R, k, c):
    R, k, c = mp.mpf(R), mp.mpf(k), mp.mpf(c)
    if c >= R + k:
        return mp.mpf(0)
    if c <= abs(R - k):
        return mp.pi * min(R, k) ** 2
    a0 = mp.acos((c * c + k * k - R * R) / (2 * c * k))
    a1 = mp.acos((c * c + R * R - k * k) / (2 * c * R))
    return k * k * a0 + R * R * a1 - mp.sqrt(4 * c * c * R * R - (c * c + R * R - k * k) ** 2) / 2


def test_lens_area(L):
    wf = wd = 0.0
    for k in (0.001, 0.003, 0.01, 0.05, 0.1, 0.2, 0.3, 0.5, 0.9, 1.5):
        lo, hi = abs(1 - k), 1 + k
        cs = (list(np.linspace(lo, hi, 301)[1:-1]) + [hi - k * 10.0 ** -p for p in range(2, 9)]
              + [lo + k * 10.0 ** -p for p in range(2, 9)])
        for c in cs:
            kf, cf = f32(k), f32(c)
            wf = max(wf, float(abs(L.probe_lens_area_f(1.0, kf, cf) - lens_exact(1, kf, cf)))
                     / min(1.0, k))
            wd = max(wd, float(abs(L.probe_lens_area_d(1.0, k, c) - lens_exact(1, k, c)))
                     / min(1.0, k) ** 2)
        # no overlap, and the planet (or the star) entirely inside
        assert L.probe_lens_area_d(1.0, k, hi + 1e-9) == 0.0
        assert L.probe_lens_area_d(1.0, k, 1.0 + k + 0.5) == 0.0
        if k < 1:
            assert L.probe_lens_area_d(1.0, k, max(0.0, lo - 1e-9)) == np.pi * k * k
            assert L.probe_lens_area_d(1.0, k, 0.0) == np.pi * k * k
    assert wf <= 1e-6, wf
    assert wd <= 1e-12, wd


def kepler_residual(d, dM, e, Etr):
    d, dM, e = mp.mpf(d), mp.mpf(dM), mp.mpf(e)
    return d - e * (mp.sin(Etr) * (mp.cos(d) - 1) + mp.cos(Etr) * mp.sin(d)) - dM


def test_kepler(L):
    rng = np.random.default_rng(13)
    wf = wd = wsf = wsd = 0.0
    for e in (0.0, 0.01, 0.1, 0.3, 0.6, 0.9, 0.97, 0.99):
        for Etr in np.linspace(0.0, 2 * np.pi, 9)[:-1]:
            sE, cE = np.sin(Etr), np.cos(Etr)
            for dM in np.concatenate([np.linspace(-0.6, 0.6, 25), rng.uniform(-np.pi, np.pi, 6)]):
                s2, c2 = ctypes.c_float(), ctypes.c_float()
                df = L.probe_kepler_f(dM, e, sE, cE, ctypes.byref(s2), ctypes.byref(c2))
                ef, sEf, cEf, dMf = (f32(v) for v in (e, sE, cE, dM))
                r = kepler_residual(df, dMf, ef, mp.atan2(sEf, cEf))
                wf = max(wf, float(abs(r)) / max(1.0, abs(df)))
                wsf = max(wsf, float(max(abs(s2.value - mp.sin(mp.mpf(df) / 2)),
                                         abs(c2.value - mp.cos(mp.mpf(df) / 2)))))
                s2d, c2d = ctypes.c_double(), ctypes.c_double()
                dd = L.probe_kepler_d(dM, e, sE, cE, ctypes.byref(s2d), ctypes.byref(c2d))
                r = kepler_residual(dd, dM, e, mp.atan2(sE, cE))
                wd = max(wd, float(abs(r)) / max(1.0, abs(dd)))
                wsd = max(wsd, float(max(abs(s2d.value - mp.sin(mp.mpf(dd) / 2)),
                                         abs(c2d.value - mp.cos(mp.mpf(dd) / 2)))))
    assert wf <= 3e-7, wf
    assert wsf <= 2e-7, wsf
    assert wd <= 1e-15, wd
    assert wsd <= 1e-15, wsd


def test_arctangent_coefficients_are_the_fit():
    script = os.path.join(ROOT, "paper_2009_08500_amd", "csrc", "fit_atan_poly.py")
    r = subprocess.run([sys.executable, script, "--check"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
