#!/usr/bin/env python3
"""Derive the arctangent polynomials of rr_device.h.

Both are least-squares fits, weighted for relative error, of
atan(sqrt(u)) / sqrt(u) by a polynomial P(u) at Chebyshev nodes (first
kind) in u, computed in 40-digit arithmetic:

* float:  degree 7 in u = r^2 on [0, 1]          (atan r = r P(r^2), r <= 1)
* double: degree 10 in u = t^2 on [0, tan^2(pi/8)] (atan t = t P(t^2), |t| <= tan(pi/8))

The fit has converged (to every printed digit) from 16 nodes on; 64 are
used.  Printed highest degree first, the order of the Horner evaluation in
the header: the float coefficients rounded to 10 significant digits (each
then rounds to the same float), the double ones to 18.

  python3 fit_atan_poly.py           print both sets and their maximum
                                     relative error in exact arithmetic
  python3 fit_atan_poly.py --check   exit 1 unless rr_device.h holds them
"""

import os
import re
import sys

import mpmath as mp

mp.mp.dps = 40
NODES = 64


def fit(degree, umax):
    f = lambda u: mp.atan(mp.sqrt(u)) / mp.sqrt(u) if u > 0 else mp.mpf(1)
    us = [umax * (1 - mp.cos(mp.pi * (i + mp.mpf(1) / 2) / NODES)) / 2 for i in range(NODES)]
    A = mp.matrix(NODES, degree + 1)
    b = mp.matrix(NODES, 1)
    for i, u in enumerate(us):
        w = 1 / f(u)
        for j in range(degree + 1):
            A[i, j] = w * u ** j
        b[i] = w * f(u)
    c = mp.lu_solve(A.T * A, A.T * b)
    return [c[j] for j in range(degree + 1)]          # lowest degree first


def max_rel_error(coef, rmax, n=4000):
    worst = mp.mpf(0)
    for i in range(1, n + 1):
        r = rmax * i / n
        p = mp.mpf(0)
        for c in reversed(coef):
            p = p * r * r + c
        worst = max(worst, abs(r * p - mp.atan(r)) / mp.atan(r))
    return worst


def coefficients():
    f32 = [mp.mpf(mp.nstr(c, 10)) for c in fit(7, mp.mpf(1))]
    t8 = mp.tan(mp.pi / 8)
    f64 = [mp.mpf(mp.nstr(c, 18)) for c in fit(10, t8 * t8)]
    return f32, f64, t8


def header_coefficients(path):
    """The coefficients as written in rr_device.h: the float polynomial's
    Horner constants (p = -4.58e-03f; p = p * t + ...f;) and the double
    one's (p = 2.11e-02; p = fma(p, u, ...);), highest degree first."""
    src = open(path).read()
    fpart = src[src.index("__device__ inline float atan2_poly"):]
    fpart = fpart[:fpart.index("float a = r * p")]
    fl = [float(x) for x in re.findall(r"float p = ([-+]?\d\.\d+e[-+]\d+)f;", fpart)]
    fl += [float(sg + x) for sg, x in re.findall(r"p = p \* t ([-+]) (\d\.\d+e[-+]\d+)f;",
                                                 fpart)]
    dpart = src[src.index("__device__ inline double atan2_poly"):]
    dpart = dpart[:dpart.index("double a = fma(t, p")]
    db = [float(x) for x in re.findall(r"double p = ([-+]?\d\.\d+e[-+]\d+);", dpart)]
    db += [float(x) for x in re.findall(r"p = fma\(p, u, ([-+]?[\d.]+(?:e[-+]\d+)?)\);", dpart)]
    return fl, db


def main():
    f32, f64, t8 = coefficients()
    if "--check" in sys.argv:
        here = os.path.dirname(os.path.abspath(__file__))
        fl, db = header_coefficients(os.path.join(here, "rr_device.h"))
        want_f = [float(c) for c in reversed(f32)]
        want_d = [float(c) for c in reversed(f64)]
        ok = (len(fl) == 8 and len(db) == 11 and
              all(abs(a - b) <= 1e-9 * abs(b) for a, b in zip(fl, want_f)) and
              all(a == b for a, b in zip(db, want_d)))
        print("rr_device.h", "holds" if ok else "does NOT hold", "the fitted coefficients")
        sys.exit(0 if ok else 1)
    print("float, degree 7 in r^2 (highest first):")
    for c in reversed(f32):
        print(f"  {mp.nstr(c, 10, min_fixed=1, max_fixed=0)}f")
    print(f"  max relative error (exact arithmetic): {mp.nstr(max_rel_error(f32, 1), 3)}")
    print("double, degree 10 in t^2 (highest first):")
    for c in reversed(f64):
        print(f"  {mp.nstr(c, 18, min_fixed=1, max_fixed=0)}")
    print(f"  max relative error (exact arithmetic): {mp.nstr(max_rel_error(f64, t8, 2000), 3)}")


if __name__ == "__main__":
    main()
