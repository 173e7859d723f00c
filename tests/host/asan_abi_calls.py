"""C-ABI calls whose host-side work needs no GPU, run by
tests/test_host_sanitized.py in a child process against a build of
librr.so whose host code carries AddressSanitizer:

* rr_prepare_ld's validation of the grid, the mu samples and every profile
  sample (then, with valid arguments, the device query fails on a host
  without a GPU);
* rr_series_create's validation and its time-index construction over
  sorted, unsorted, multi-light-curve, constant, empty and invalid series;
* every entry point's NULL-handle and NULL-argument paths, the serving
  calls included, and the error strings.

Usage: python asan_abi_calls.py <library> <path of paper_2009_08500_amd/_lib.py>
Prints a line per group; exits 1 on an unexpected return code (ASan itself
aborts the process on a memory error)."""

import ctypes
import importlib.util
import sys

import numpy as np


def main(lib_path, lib_py):
    spec = importlib.util.spec_from_file_location("rr_lib_decls", lib_py)
    decl = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(decl)
    L = ctypes.CDLL(lib_path)
    decl._declare(L)
    EINVAL, ELIMIT, EDEVICE, OK = decl.RR_EINVAL, decl.RR_ELIMIT, decl.RR_EDEVICE, decl.RR_OK
    bad = []

    def expect(name, rc, allowed):
        if rc not in allowed:
            bad.append((name, rc, L.rr_last_error().decode()))

    def ptr(a):
        return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None

    # error strings
    for code in range(-8, 2):
        assert L.rr_strerror(code) is not None
    # -- rr_prepare_ld
    good = (0.7, 10, 10, 32, 8, 0.01, 0.3)
    grids = [good, (0.0, 10, 10, 32, 8, 0.01, 0.3), (0.7, 0, 10, 32, 8, 0.01, 0.3),
             (0.7, 10, 10, 1, 8, 0.01, 0.3), (0.7, 10, 10, 32, 1, 0.01, 0.3),
             (0.7, 10, 10, 32, 8, 0.3, 0.01), (0.7, 3000, 3000, 32, 8, 0.01, 0.3),
             (float("nan"), 10, 10, 32, 8, 0.01, 0.3)]
    n = 0
    for gi, grid in enumerate(grids):
        for nmu, npb in ((2, 1), (37, 1), (200, 4), (11, 16), (11, 17), (1, 1), (11, 0)):
            mu = np.linspace(0.0, 1.0, max(nmu, 1))
            prof = np.ones((max(npb, 1), max(nmu, 1)))
            h = ctypes.c_void_p()
            g = decl.RRGrid(*grid)
            rc = L.rr_prepare_ld(ptr(mu), ptr(prof), nmu, npb, ctypes.byref(g), ctypes.byref(h))
            valid = gi == 0 and nmu >= 2 and 1 <= npb <= 16
            expect(f"prepare {grid} {nmu} {npb}", rc,
                   (OK, EDEVICE) if valid else (EINVAL, ELIMIT))
            if rc == OK:
                L.rr_free_tables(h)
            n += 1
        mu = np.linspace(0.0, 1.0, 11)
        for case in ("nan", "decreasing", "outside"):
            prof = np.ones(11)
            m = mu.copy()
            if case == "nan":
                prof[10] = np.nan
            elif case == "decreasing":
                m = m[::-1].copy()
            else:
                m[-1] = 1.5
            h = ctypes.c_void_p()
            rc = L.rr_prepare_ld(ptr(m), ptr(prof), 11, 1, ctypes.byref(decl.RRGrid(*good)),
                                 ctypes.byref(h))
            expect(f"prepare {case}", rc, (EINVAL,))
            n += 1
    expect("prepare null out", L.rr_prepare_ld(None, None, 2, 1, None, None), (EINVAL,))
    print(f"rr_prepare_ld: {n} argument sets")

    # -- rr_series_create (the index builder runs before the device query)
    rng = np.random.default_rng(7)
    n = 0

    def series(times, lcids, nlc, pb=None, nss=None, ex=None, npt=None):
        pb = np.zeros(nlc, np.int32) if pb is None else np.asarray(pb, np.int32)
        nss = np.ones(nlc, np.int32) if nss is None else np.asarray(nss, np.int32)
        ex = np.zeros(nlc) if ex is None else np.asarray(ex, np.float64)
        t = np.ascontiguousarray(times, np.float64)
        ids = None if lcids is None else np.ascontiguousarray(lcids, np.int32)
        h = ctypes.c_void_p()
        rc = L.rr_series_create(ptr(t), ptr(ids), t.size if npt is None else npt, ptr(pb),
                                ptr(nss), ptr(ex), nlc, ctypes.byref(h))
        if rc == OK:
            L.rr_series_free(h)
        return rc

    for it in range(120):
        nlc = int(rng.integers(1, 7))
        runs = []
        for _ in range(nlc):
            m = int(rng.integers(0, 400))
            runs.append(np.sort(2.46e6 + rng.uniform(0, 30, m)))
        order = rng.permutation(nlc)
        t = np.concatenate([runs[i] for i in order]) if nlc else np.zeros(0)
        ids = np.concatenate([np.full(runs[i].size, i) for i in order])
        for variant in ("sorted", "shuffled", "ids_out", "nan", "constant"):
            tt, ii = t.copy(), ids.copy()
            if variant == "shuffled" and tt.size:
                p = rng.permutation(tt.size)
                tt, ii = tt[p], ii[p]
            elif variant == "ids_out" and ii.size:
                ii[int(rng.integers(ii.size))] = nlc + 3
            elif variant == "nan" and tt.size:
                tt[int(rng.integers(tt.size))] = np.nan
            elif variant == "constant":
                tt[:] = 2.46e6
            expect(f"series {it} {variant}", series(tt, ii, nlc, nss=np.full(nlc, 3),
                                                    ex=np.full(nlc, 0.02)), (OK, EDEVICE))
            n += 1
        if nlc == 1:
            expect("series no ids", series(t, None, 1), (OK, EDEVICE))
    t = np.linspace(0, 1, 10)
    for name, kw, want in (("npt<0", dict(npt=-1), EINVAL), ("nlc 0", dict(nlc=0), EINVAL),
                           ("nlc>max", dict(nlc=65), ELIMIT), ("pb", dict(pb=[16]), EINVAL),
                           ("nss 0", dict(nss=[0]), EINVAL), ("nss>max", dict(nss=[2000]), ELIMIT),
                           ("ex nan", dict(ex=[np.nan]), EINVAL), ("ex<0", dict(ex=[-1.0]), EINVAL)):
        nlc = kw.pop("nlc", 1)
        args = dict(pb=[0] * nlc, nss=[1] * nlc, ex=[0.0] * nlc)
        args.update(kw)
        expect(f"series {name}", series(t, np.zeros(10, np.int32), nlc, **args), (want,))
        n += 1
    expect("series ids NULL, 2 lcs", series(t, None, 2), (EINVAL,))
    expect("series NULL out", L.rr_series_create(None, None, 0, None, None, None, 1, None),
           (EINVAL,))
    print(f"rr_series_create: {n} series")

    # -- NULL handles and arguments
    one = np.ones(1, np.int32)
    z = np.zeros(1)
    p1, pz = ptr(one), ptr(z)
    calls = [
        ("evaluate", lambda: L.rr_evaluate(None, None, None, 0, p1, p1, pz, 1, None, 0, 7, 0,
                                           None, None)),
        ("noalloc", lambda: L.rr_evaluate_noalloc(None, None, None, 0, p1, p1, pz, 1, None, 0,
                                                  7, 0, None, None)),
        ("series", lambda: L.rr_evaluate_series(None, None, None, 0, 7, 0, None, None)),
        ("series kernel", lambda: L.rr_series_kernel(None, None, 1, 0, None)),
        ("ld", lambda: L.rr_evaluate_ld(None, None, None, 0, p1, p1, pz, 1, None, 0, 7, None,
                                        0, None, None)),
        ("direct", lambda: L.rr_evaluate_direct(None, None, None, 0, p1, p1, pz, 1, None, 0, 7,
                                                0, None, None)),
        ("variant", lambda: L.rr_evaluate_variant(None, None, None, 0, p1, p1, pz, 1, None, 0,
                                                  7, 0, 1, None, None)),
        ("select", lambda: L.rr_select_variant(None, None, None, 0, p1, p1, pz, 1, None, 0, 7,
                                               0, None, 5, None, None, None)),
        ("small", lambda: L.rr_evaluate_small_planet(None, None, None, 0, p1, p1, pz, 1, None,
                                                     0, 7, 0.01, 0, None, None)),
        ("small grad", lambda: L.rr_loglik_grad_small_planet(None, None, None, 0, p1, p1, pz,
                                                             1, None, 0, 7, 0.01, 0, None, 1.0,
                                                             None, None, None)),
        ("flux at z", lambda: L.rr_flux_at_z(None, None, None, 0.1, 0, 0, 0, None, None)),
        ("loglik", lambda: L.rr_loglik_grad(None, None, None, 0, p1, p1, pz, 1, None, 0, 7, 0,
                                            None, 1.0, None, None, None, None, None)),
        ("loglik istar", lambda: L.rr_loglik_grad_istar(None, None, None, 0, p1, p1, pz, 1,
                                                        None, 0, 7, 0, None, 1.0, None, None,
                                                        None, None, None, None)),
        ("loglik ld", lambda: L.rr_loglik_grad_ld(None, None, None, 0, p1, p1, pz, 1, None, 0,
                                                  7, None, 0, None, 1.0, None, None, None,
                                                  None)),
        ("set profile", lambda: L.rr_set_profile(None, None, None)),
        ("set istar", lambda: L.rr_set_istar(None, None, None)),
        ("copy", lambda: L.rr_tables_copy(None, 0, None, 0, None)),
        ("info", lambda: L.rr_tables_info(None, None, None)),
        ("server create", lambda: L.rr_server_create(None, 1 << 30, 64, None)),
        ("server add", lambda: L.rr_server_add_series(None, None, None, 0, None, None, None, 0,
                                                      None)),
        ("server submit", lambda: L.rr_server_submit(None, 0, None, 1, 7, 0, None, None)),
        ("server submit dev", lambda: L.rr_server_submit_device(None, 0, None, 1, 7, 0, None,
                                                                None)),
        ("server poll", lambda: L.rr_server_poll(None, 1, None, None)),
        ("server wait", lambda: L.rr_server_wait(None, 1, 0.0, None)),
        ("server release", lambda: L.rr_server_release(None, 1)),
        ("server stats", lambda: L.rr_server_stats(None, None)),
        ("server fail", lambda: L.rr_server_fail_next_tick(None)),
    ]
    c_i64, c_dbl, c_i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int32
    vp = ctypes.c_void_p
    L.rr_server_create.argtypes = [vp, c_i64, c_i32, vp]
    L.rr_server_add_series.argtypes = [vp, vp, vp, c_i32, vp, vp, vp, c_i32, vp]
    L.rr_server_submit.argtypes = [vp, c_i32, vp, c_i32, c_i32, c_i32, vp, vp]
    L.rr_server_submit_device.argtypes = [vp, c_i32, vp, c_i32, c_i32, c_i32, vp, vp]
    L.rr_server_poll.argtypes = [vp, c_i64, vp, vp]
    L.rr_server_wait.argtypes = [vp, c_i64, c_dbl, vp]
    L.rr_server_release.argtypes = [vp, c_i64]
    L.rr_server_stats.argtypes = [vp, vp]
    L.rr_server_fail_next_tick.argtypes = [vp]
    L.rr_server_destroy.argtypes = [vp]
    L.rr_server_destroy.restype = None
    for name, fn in calls:
        expect(name, fn(), (EINVAL,))
    L.rr_series_free(None)
    L.rr_free_tables(None)
    L.rr_server_destroy(None)
    print(f"NULL paths: {len(calls)} entry points")
    if bad:
        for b in bad:
            print("unexpected:", b)
        return 1
    print("OK")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1], sys.argv[2]))
