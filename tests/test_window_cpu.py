"""The transit window of the library's per-row setup, built for the host:
every time offset at which the oracle's orbit puts the planet in front of
the star and closer than 1 + k must fall inside it (flux is written as
exactly 1 outside without solving the orbit), and it must stay tight.

The window logic (make_pv_const) is compiled from the library's own header
for the host; the orbit it is checked against is the oracle's."""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import orbit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
K_ALWAYS = 2


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("probe") / "libprobe.so")
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-host-only",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2009_08500_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "window_probe.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    lib = ctypes.CDLL(out)
    lib.probe_windows.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def windows(lib, rows, k0=0.01, k1=0.30, f32=0):
    """The setup's validity flags and window per row: FP64 (f32 = 0) or
    the mixed precision's setup (float sin w, cos w and sqrt(1 - e^2))."""
    rows = np.ascontiguousarray(rows, np.float64)
    n, npar = rows.shape
    flags = np.zeros(n, np.int32)
    flo = np.zeros(n)
    wn = np.zeros(n)
    lib.probe_windows(rows.ctypes.data, n, npar, k0, k1, int(f32), flags.ctypes.data,
                      flo.ctypes.data, wn.ctypes.data)
    return flags, flo, wn


def overlap_mask(row, dt):
    t0, P, a, b, e, w = row[:6]
    k = row[6:].max()
    z, front, _ = orbit.projected_separation(dt, P, a, b, e, w)
    return front & (z < 1.0 + k)


def inside(dt, P, flo, wn):
    g = dt / P - flo
    return (g - np.floor(g)) < wn


def random_rows(n, seed):
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        e = [0.0, 0.05, 0.3, 0.6, 0.9, 0.99][i % 6]
        amin = 1.05 / (1.0 - e)
        a = rng.uniform(amin, max(30.0, 3.0 * amin))
        k = rng.uniform(0.01, 0.30)
        rows.append([0.0, rng.uniform(0.5, 20.0), a, rng.uniform(0.0, 1.0 + k + 0.1), e,
                     rng.uniform(-10.0, 10.0), k])
    return np.array(rows)


@pytest.mark.parametrize("f32", [0, 1])
def test_window_contains_every_overlap(probe, f32):
    rows = random_rows(240, 11)
    flags, flo, wn = windows(probe, rows, f32=f32)
    checked = 0
    for row, f, lo, width in zip(rows, flags, flo, wn):
        if not f & 1:
            continue
        P = row[1]
        dt = np.linspace(-0.5 * P, 0.5 * P, 20001)
        ov = overlap_mask(row, dt)
        if not ov.any():
            continue
        # refine around the first and last overlapping offsets (the contacts)
        idx = np.flatnonzero(ov)
        h = dt[1] - dt[0]
        fine = np.concatenate([np.linspace(dt[i] - h, dt[i] + h, 401) for i in (idx[0], idx[-1])])
        dt_all = np.concatenate([dt, fine])
        ov_all = overlap_mask(row, dt_all)
        if f & K_ALWAYS:
            continue
        miss = ov_all & ~inside(dt_all, P, lo, width)
        assert not miss.any(), (row, lo, width, dt_all[miss][:5])
        checked += 1
    assert checked > 150


@pytest.mark.parametrize("f32", [0, 1])
def test_window_is_tight_for_the_population(probe, f32):
    import workloads as wl
    pv = wl.draw_orbits(np.random.default_rng(5), 64)
    flags, flo, wn = windows(probe, pv, f32=f32)
    assert np.all(flags & 1) and not np.any(flags & K_ALWAYS)
    for row, lo, width in zip(pv, flo, wn):
        P = row[1]
        dt = np.linspace(-0.5 * P, 0.5 * P, 40001)
        frac = overlap_mask(row, dt).mean()
        # the window exceeds the overlapping arc only by its margins and
        # by the r >= r_min bound
        assert frac <= width
        assert width <= 1.25 * frac + 1e-4, (row, frac, width)


def test_never_overlapping_and_invalid_rows(probe):
    rows = np.array([
        [0.0, 3.0, 8.0, 1.5, 0.0, 0.0, 0.1],     # b > 1 + k on a circular orbit
        [0.0, 3.0, 8.0, 0.3, 0.0, 0.0, 0.5],     # k outside [k0, k1]: invalid
        [0.0, -1.0, 8.0, 0.3, 0.0, 0.0, 0.1],    # P <= 0: invalid
        [0.0, 3.0, 1.01, 0.2, 0.0, 0.0, 0.1],    # a close to 1: the whole front half
    ])
    flags, flo, wn = windows(probe, rows)
    assert flags[0] & 1 and wn[0] == 0.0
    dt = np.linspace(-1.5, 1.5, 30001)
    assert not overlap_mask(rows[0], dt).any()
    assert not flags[1] & 1 and not flags[2] & 1
    ov = overlap_mask(rows[3], dt)
    assert flags[3] & 1 and ov.any()
    assert (flags[3] & K_ALWAYS) or not (ov & ~inside(dt, 3.0, flo[3], wn[3])).any()
