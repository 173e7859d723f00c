// rr_device.h -- device math of the RoadRunner path, templated on the real
// type of the bulk arithmetic (double for RR_FP64, float for RR_MIXED).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "rr_internal.h"

namespace rr {

// The hardware primitives the device math is built on: the GPU's
// reciprocal and square-root estimates.  The functions below are written
// once against this interface (a template parameter defaulting to it), so
// that a host build for tests can instantiate the same code with host
// stand-ins of these three operations.
struct HwOps {
    __device__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static double rcp(double x) { return __builtin_amdgcn_rcp(x); }
};

template <typename R, class Ops = HwOps> struct Num;
// atan2 for float on the kernels' paths: r = min(|x|,|y|)/max(|x|,|y|) in
// [0, 1], atan r = r P(r^2) with P of degree 7 (a least-squares fit to
// atan(r)/r at 64 Chebyshev nodes in r^2, weighted for relative error;
// fit_atan_poly.py beside this file derives it: max relative error 1.14e-7
// in exact arithmetic), then the octant fix-ups.  About 20 instructions,
// half those of a correctly rounded atan2f; the lens areas need ~1e-6
// relative.
template <class Ops = HwOps>
__host__ __device__ inline float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float r = mx > 0.0f ? mn * Ops::rcp(mx) : 0.0f;
    const float t = r * r;
    float p = -4.583679842e-03f;
    p = p * t + 2.386548698e-02f;
    p = p * t - 5.894885931e-02f;
    p = p * t + 9.877179037e-02f;
    p = p * t - 1.400628610e-01f;
    p = p * t + 1.996748018e-01f;
    p = p * t - 3.333184671e-01f;
    p = p * t + 9.999998857e-01f;
    float a = r * p;
    a = ay > ax ? 1.57079632679f - a : a;
    a = x < 0.0f ? 3.14159265359f - a : a;
    return y < 0.0f ? -a : a;
}

// 1/x in double from the hardware estimate and two Newton steps
// (y <- y + y (1 - x y)), each doubling the correct bits: within ~1 ulp.
// For the normal, non-zero arguments of the kernels' paths only.
template <class Ops = HwOps>
__host__ __device__ inline double rcp_nr(double x) {
    double y = Ops::rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// atan2 for double on the kernels' paths: r = min/max in [0, 1]; above
// tan(pi/8) use atan r = pi/4 + atan((r - 1)/(r + 1)), so |t| <= tan(pi/8);
// atan t = t P(t^2) with P of degree 10 (a least-squares fit to atan(t)/t
// at 64 Chebyshev nodes in t^2 on [0, tan^2(pi/8)], done in 40-digit
// arithmetic and weighted for relative error, as fit_atan_poly.py beside
// this file derives it: 3.5e-17 in exact arithmetic, ~1 ulp in double).
template <class Ops = HwOps>
__host__ __device__ inline double atan2_poly(double y, double x) {
    const double ax = fabs(x), ay = fabs(y);
    const double mx = fmax(ax, ay), mn = fmin(ax, ay);
    const double r = mx > 0.0 ? mn * rcp_nr<Ops>(mx) : 0.0;
    const bool big = r > 0.41421356237309503;             // tan(pi/8)
    const double t = big ? (r - 1.0) * rcp_nr<Ops>(r + 1.0) : r;
    const double u = t * t;
    double p = 2.11428279540593587e-02;
    p = fma(p, u, -4.34869344380681838e-02);
    p = fma(p, u, 5.68858371271004082e-02);
    p = fma(p, u, -6.64028142107710717e-02);
    p = fma(p, u, 7.68995931129169419e-02);
    p = fma(p, u, -9.09077351572132597e-02);
    p = fma(p, u, 1.11111062008220365e-01);
    p = fma(p, u, -1.42857141815172506e-01);
    p = fma(p, u, 1.99999999988624111e-01);
    p = fma(p, u, -3.33333333333284743e-01);
    p = fma(p, u, 1.0);
    double a = fma(t, p, big ? 0.78539816339744831 : 0.0);  // + pi/4
    a = ay > ax ? 1.5707963267948966 - a : a;
    a = x < 0.0 ? 3.1415926535897932 - a : a;
    return y < 0.0 ? -a : a;
}

template <class Ops> struct Num<double, Ops> {
    static constexpr double pi = 3.14159265358979323846;
    __host__ __device__ static double sqrt_(double x) { return sqrt(x); }
    __host__ __device__ static double rcp_(double x) { return rcp_nr<Ops>(x); }
    __host__ __device__ static double atan2_(double y, double x) { return atan2_poly<Ops>(y, x); }
    __host__ __device__ static void sincos_(double x, double* s, double* c) { sincos(x, s, c); }
    __host__ __device__ static double abs_(double x) { return fabs(x); }
    // Halley iterations stop once a step is below this; the cubic rate then
    // leaves an error far below one ulp.
    static constexpr double kepler_stop = 1e-6;
    static constexpr int kepler_maxit = 24;
};
// Float: the hardware reciprocal and square root (1 ulp) stand in for the
// correctly rounded forms; every use tolerates a relative error of 1e-6.
template <class Ops> struct Num<float, Ops> {
    static constexpr float pi = 3.14159265358979323846f;
    __host__ __device__ static float sqrt_(float x) { return Ops::sqrt(x); }
    __host__ __device__ static float rcp_(float x) { return Ops::rcp(x); }
    __host__ __device__ static float atan2_(float y, float x) { return atan2_poly<Ops>(y, x); }
    __host__ __device__ static void sincos_(float x, float* s, float* c) { sincosf(x, s, c); }
    __host__ __device__ static float abs_(float x) { return fabsf(x); }
    static constexpr float kepler_stop = 2e-3f;
    static constexpr int kepler_maxit = 20;
};

// sin and cos of a half-angle x of the offset from conjunction, which is
// small inside a transit window.  In float, for |x| <= 1/4 the Maclaurin
// series through the x^7 and x^8 terms are summed by Horner's rule in x^2
// (truncation below 1e-11); larger float arguments and every double
// argument use the library sincos (a double series of the same accuracy
// measured slower).
__host__ __device__ inline void sincos_small(float x, float* s, float* c) {
    if (fabsf(x) > 0.25f) {
        sincosf(x, s, c);
        return;
    }
    const float x2 = x * x;
    float ps = -1.0f / 5040.0f;                          // -1/7!
    ps = ps * x2 + 1.0f / 120.0f;
    ps = ps * x2 - 1.0f / 6.0f;
    *s = x + x * x2 * ps;
    float pc = 1.0f / 40320.0f;                          // 1/8!
    pc = pc * x2 - 1.0f / 720.0f;
    pc = pc * x2 + 1.0f / 24.0f;
    pc = pc * x2 - 0.5f;
    *c = 1.0f + x2 * pc;
}
__host__ __device__ inline void sincos_small(double x, double* s, double* c) {
    sincos(x, s, c);
}

// (sin x, cos x) -> (sin(x + y), cos(x + y)) for |y| <= 1e-3, with
// sin y = y - y^3/6 and cos y = 1 - y^2/2 + y^4/24 (truncation below 1e-17).
template <typename R>
__host__ __device__ inline void rotate_small(R y, R* s, R* c) {
    const R y2 = y * y;
    const R sy = y - y * y2 * R(1.0 / 6.0);
    const R cy = R(1) - y2 * (R(0.5) - y2 * R(1.0 / 24.0));
    const R s0 = *s, c0 = *c;
    *s = s0 * cy + c0 * sy;
    *c = c0 * cy - s0 * sy;
}

// Area of the intersection of a disk of radius Rd centred at the origin and a
// disk of radius k centred at distance c (the lens a(c, k) of Eq. 5 when
// Rd = 1).  In the partial-overlap case the three centres-and-chord-end
// triangle has sides (Rd, k, c); its area D comes from Kahan's stable form of
// Heron's formula (sides sorted a >= b >= c), the half chord is h = 2D/c and
// the two half-angles are atan2(h, x) with x the signed distances from each
// centre to the chord.  A = Rd^2 k1 + k^2 k0 - c h.  Unlike the arccos form
// this keeps its accuracy at the contact points, where FP32 would otherwise
// lose several ppm: the host build against 40-digit arithmetic gives an
// absolute error below 5e-7 min(1, k) in float and 5e-13 min(1, k)^2 in
// double for k from 0.001 to 1.5.
template <typename R, class Ops = HwOps>
__host__ __device__ inline R lens_area(R Rd, R k, R c) {
    using N = Num<R, Ops>;
    if (c >= Rd + k) return R(0);
    const R dk = Rd - k;
    if (c <= N::abs_(dk)) {
        const R m = Rd < k ? Rd : k;
        return N::pi * m * m;
    }
    // sort the sides
    R a = Rd, b = k, s = c, tmp;
    if (a < b) { tmp = a; a = b; b = tmp; }
    if (b < s) { tmp = b; b = s; s = tmp; }
    if (a < b) { tmp = a; a = b; b = tmp; }
    R prod = (a + (b + s)) * (s - (a - b)) * (s + (a - b)) * (a + (b - s));
    prod = prod > R(0) ? prod : R(0);
    const R area2 = R(0.5) * N::sqrt_(prod);        // 2 D
    const R invc = N::rcp_(c);
    const R h = area2 * invc;                       // half chord
    const R x1 = (c * c + (Rd - k) * (Rd + k)) * (R(0.5) * invc);
    const R x0 = c - x1;
    const R k1 = N::atan2_(h, x1);
    const R k0 = N::atan2_(h, x0);
    return Rd * Rd * k1 + k * k * k0 - area2;
}

// Orbit constants of one parameter vector in the bulk precision.
template <typename R>
struct OrbitR {
    R n, e, sE, cE, q, a, cosw, sinw, rtr, cosi;
    __host__ __device__ explicit OrbitR(const PvConst& p)
        : n(R(p.n)), e(R(p.e)), sE(R(p.sE)), cE(R(p.cE)), q(R(p.q)),
          a(R(p.a)), cosw(R(p.cosw)), sinw(R(p.sinw)), rtr(R(p.rtr)),
          cosi(R(p.cosi)) {}
};

// Transit-centred Kepler solve: with E = E_tr + d and dM = n dt, Kepler's
// equation becomes h(d) = d - e [sin E_tr (cos d - 1) + cos E_tr sin d] - dM
// = 0.  h is increasing (h' = 1 - e cos E > 0) and its root lies in
// [dM - 2e, dM + 2e]; Halley's method starts from d = dM / (1 - e cos E_tr)
// and is safeguarded by that bracket (a step leaving the current bracket is
// replaced by bisection), so it converges for any e < 1.  Returns d and
// sin(d/2), cos(d/2) at d; after the last, small step they are rotated
// rather than recomputed.  cos d - 1 = -2 sin^2(d/2) keeps every quantity
// small near transit, so float keeps its relative precision there.
template <typename R, class Ops = HwOps>
__host__ __device__ inline R kepler_halley(R dM, R e, R sE, R cE, R* s2, R* c2) {
    using N = Num<R, Ops>;
    R lo = dM - R(2) * e, hi = dM + R(2) * e;
    R d = dM * N::rcp_(R(1) - e * cE);
    d = d < lo ? lo : (d > hi ? hi : d);
    for (int it = 0; it < N::kepler_maxit; ++it) {
        sincos_small(R(0.5) * d, s2, c2);
        const R sd = R(2) * *s2 * *c2;
        const R cm1 = R(-2) * *s2 * *s2;
        const R h = d - e * (sE * cm1 + cE * sd) - dM;
        if (h < R(0)) lo = d; else hi = d;
        const R hp = R(1) - e * (cE * (R(1) + cm1) - sE * sd);
        const R hpp = e * (sE * (R(1) + cm1) + cE * sd);
        // Halley: h / (h' - h h''/(2 h')) with a single division
        R dn = d - R(2) * h * hp * N::rcp_(R(2) * hp * hp - h * hpp);
        if (!(dn >= lo && dn <= hi)) dn = R(0.5) * (lo + hi);
        const R step = dn - d;
        d = dn;
        if (N::abs_(step) < N::kepler_stop) {
            rotate_small(R(0.5) * step, s2, c2);
            return d;
        }
    }
    sincos_small(R(0.5) * d, s2, c2);
    return d;
}

// Kepler solve of the bulk precision.  Double: the float solve's root (good
// to ~1e-7) and one Halley step in double, whose cubic rate leaves an error
// far below one ulp.  If that step is not small (float too coarse, e.g. e
// close to 1 near periapsis), the bracketed solve is repeated in double.
template <typename R, class Ops = HwOps>
__host__ __device__ inline R kepler_offset(R dM, R e, R sE, R cE, R* s2, R* c2) {
    if constexpr (std::is_same<R, double>::value) {
        float s2f, c2f;
        const double d = kepler_halley<float, Ops>(float(dM), float(e), float(sE), float(cE),
                                                   &s2f, &c2f);
        sincos_small(0.5 * d, s2, c2);
        const double sd = 2.0 * *s2 * *c2;
        const double cm1 = -2.0 * *s2 * *s2;
        const double h = d - e * (sE * cm1 + cE * sd) - dM;
        const double hp = 1.0 - e * (cE * (1.0 + cm1) - sE * sd);
        const double hpp = e * (sE * (1.0 + cm1) + cE * sd);
        const double step = -2.0 * h * hp / (2.0 * hp * hp - h * hpp);
        if (fabs(step) < 2e-6) {
            rotate_small(0.5 * step, s2, c2);
            return d + step;
        }
        return kepler_halley<double, Ops>(dM, e, sE, cE, s2, c2);
    } else {
        return kepler_halley<R, Ops>(dM, e, sE, cE, s2, c2);
    }
}

// Projected separation for a time offset dt from conjunction.  The sky
// coordinates are formed from the differences cos E - cos E_tr and
// sin E - sin E_tr, so every intermediate is small near transit:
//   X   = -a [(cos E - cos E_tr) cos w - q (sin E - sin E_tr) sin w]
//   rho = r sin(w + f) = r_tr + a [(cos E - cos E_tr) sin w
//                                  + q (sin E - sin E_tr) cos w]
//   Y   = -rho cos i,  z = sqrt(X^2 + Y^2),  in front iff rho > 0.
template <typename R, class Ops = HwOps>
__host__ __device__ inline R separation(R dt, const OrbitR<R>& o, bool* front) {
    using N = Num<R, Ops>;
    const R dM = o.n * dt;
    R s2, c2;
    if (o.e > R(0)) kepler_offset<R, Ops>(dM, o.e, o.sE, o.cE, &s2, &c2);
    else sincos_small(R(0.5) * dM, &s2, &c2);
    const R sd = R(2) * s2 * c2;
    const R cm1 = R(-2) * s2 * s2;
    const R dc = o.cE * cm1 - o.sE * sd;
    const R ds = o.sE * cm1 + o.cE * sd;
    const R X = -o.a * (dc * o.cosw - o.q * ds * o.sinw);
    const R rho = o.rtr + o.a * (dc * o.sinw + o.q * ds * o.cosw);
    const R Y = -rho * o.cosi;
    *front = rho > R(0);
    return N::sqrt_(X * X + Y * Y);
}

// x is neither infinite nor NaN (x - x is 0 exactly for every finite x).
__host__ __device__ inline bool is_finite(double x) { return (x - x) == 0.0; }

// Orbit constants and transit window of one parameter row
// [t0, P, a, b, e, w, k_0 .. k_{npb-1}] (FP64).  The row is invalid (NaN
// output) if any value is non-finite, P <= 0, a <= 0, b < 0, e outside
// [0, 1), a k outside [k0, k1] or |cos i| > 1.
// A radius ratio below k_small (small-planet rows, Sect. 3.4.2) only has to
// be positive; any other must lie in [k0, k1].
// kF32 (the mixed precision's setup, whose constants feed float orbit
// arithmetic): sin w, cos w (of w first reduced to [-pi, pi] in double) and
// sqrt(1 - e^2) in float; every forward path of one precision derives its
// constants with the same kF32, so they share their bits.
template <bool kF32 = false, class Ops = HwOps>
__host__ __device__ inline PvConst make_pv_const(const double* row, int npb, double k0,
                                                 double k1, double k_small = 0.0) {
    PvConst c = {};
    const double t0 = row[0], P = row[1], a = row[2], b = row[3], e = row[4],
                 w = row[5];
    bool ok = is_finite(t0) && is_finite(P) && is_finite(a) && is_finite(b) &&
              is_finite(e) && is_finite(w) && P > 0.0 && a > 0.0 && b >= 0.0 &&
              e >= 0.0 && e < 1.0;
    double kmax = 0.0;
    for (int pb = 0; pb < npb; ++pb) {
        const double k = row[6 + pb];
        ok = ok && is_finite(k) && (k < k_small ? k > 0.0 : (k >= k0 && k <= k1));
        kmax = k > kmax ? k : kmax;
    }
    // Few divisions, and most of them off the dependent chain: the
    // reciprocals of p = a (1 - e^2) and P do not wait for sin w.
    double sw = 0.0, cw = 1.0;
    const double ome2 = 1.0 - e * e;
    double q = 1.0;
    if (ok) {
        if (kF32) {
            const double inv2pi = 0.5 / Num<double>::pi;
            const double wr = w - 2.0 * Num<double>::pi * rint(w * inv2pi);
            float sf, cf;
            sincosf(float(wr), &sf, &cf);
            sw = sf;
            cw = cf;
            q = double(Ops::sqrt(float(ome2)));
        } else {
            sincos(w, &sw, &cw);
            q = sqrt(ome2);
        }
    }
    const double p = a * ome2;                       // semi-latus rectum
    const double inv_p = ok ? 1.0 / p : 0.0;
    // conjunction: f_tr = pi/2 - w, so cos f_tr = sin w and sin f_tr = cos w,
    // and r_tr = p / (1 + e sin w)
    const double den = 1.0 + e * sw;
    const double cosi = ok ? b * den * inv_p : 0.0;
    ok = ok && fabs(cosi) <= 1.0;
    c.t0 = t0; c.P = P; c.invP = 1.0 / P; c.n = 2.0 * Num<double>::pi * c.invP;
    c.a = a; c.e = e; c.cosw = cw; c.sinw = sw; c.q = q; c.cosi = cosi;
    const double inv_den = 1.0 / den;
    c.cE = (e + sw) * inv_den;
    c.sE = q * cw * inv_den;
    c.rtr = p * inv_den;
    c.kmax = kmax;
    int32_t flags = ok ? kValid : 0;
    c.flo = 0.0;
    c.wn = 2.0;                      // covers every phase unless narrowed below
    if (ok) {
        // With psi = f - f_tr (transit at psi = 0) the sky separation obeys
        // z^2 = r^2 (sin^2 psi sin^2 i + cos^2 i), and the planet is in front
        // for |psi| < pi/2.  Over any arc where r >= rmin, z < 1 + k needs
        // sin^2 psi < ((1 + k)^2 / rmin^2 - cos^2 i) / sin^2 i.  Starting from
        // rmin = a (1 - e), the arc |psi| < theta is narrowed once by taking
        // rmin as the smallest r = a (1 - e^2)/(1 + e cos f) over it (a
        // second pass narrows the population's windows by under 1 %).  An
        // empty arc means the planet never overlaps the star.
        //
        // The arc only has to contain the true one (margins below), so its
        // sin, cos (float square roots), the arctangents (the float
        // polynomial above, 1.1e-7 relative) and the reciprocals of sin^2 i
        // and 1 + e cos f run in float: their errors, a few 1e-7 rad, sit
        // far inside the margins, and the arc ends enter the arctangents
        // only through their direction.
        // Only sin and cos of theta are needed: the arc's ends f = f_tr +- theta
        // have cos f = sin w cos theta -+ cos w sin theta and
        // sin f = cos w cos theta +- sin w sin theta, their eccentric
        // anomalies follow from cos E = (e + cos f)/(1 + e cos f) and
        // sin E = q sin f/(1 + e cos f), and the mean-anomaly offsets from
        // conjunction are dM = dE - e (sin E - sin E_tr) with dE the angle from
        // E_tr to E (one atan2 each).  The arc contains periapsis iff
        // cos f_tr = sin w >= cos theta.  With r = p / g, g = 1 + e cos f,
        // (1 + k)^2 / r^2 = (1 + k)^2 g^2 / p^2: rmin = a (1 - e) is g = 1 + e,
        // and a larger rmin is a smaller g.
        const double ci2 = cosi * cosi, si2 = 1.0 - ci2;
        const double opk2 = (1.0 + kmax) * (1.0 + kmax) * (1.0 + 2e-6);
        const double opk2_p2 = opk2 * inv_p * inv_p;
        const double inv_si2 = si2 > 0.0 ? double(Ops::rcp(float(si2))) : 0.0;
        double gmax = 1.0 + e;
        double sth = 1.0, cth = 0.0;                 // theta = pi/2: the front half
        bool never = false;
        for (int it = 0; it < 2; ++it) {
            const double num = opk2_p2 * gmax * gmax - ci2;
            if (num <= 0.0) { never = true; break; }
            const double s2 = si2 > 0.0 ? num * inv_si2 : 2.0;
            if (s2 < 1.0) {
                sth = double(Ops::sqrt(float(s2)));
                cth = double(Ops::sqrt(float(1.0 - s2)));
            } else {
                sth = 1.0;
                cth = 0.0;
            }
            if (e == 0.0) break;
            const double cmax = sw >= cth ? 1.0 : fmax(sw * cth - cw * sth, sw * cth + cw * sth);
            const double gnew = 1.0 + e * cmax;
            if (gnew >= gmax) break;
            gmax = gnew;
        }
        if (never) {
            c.wn = 0.0;                  // no exposure is ever inside
        } else {
            // dE in float: its error (a few 1e-7 rad) is far inside the
            // margin of 2e-6 of a period added on each side.  The atan2
            // takes cos E and sin E times 1 + e cos f > 0 (the same angle),
            // so only sin E itself needs the division.
            auto dmean = [&](double sign) {
                const double cf = sw * cth - sign * cw * sth;
                const double sf = cw * cth + sign * sw * sth;
                const double cEu = e + cf, sEu = q * sf;
                const float dE = atan2_poly<Ops>(float(sEu * c.cE - cEu * c.sE),
                                                 float(cEu * c.cE + sEu * c.sE));
                const double sEx = sEu * double(Ops::rcp(float(1.0 + e * cf)));
                return double(dE) - e * (sEx - c.sE);
            };
            const double inv2pi = 0.5 / Num<double>::pi;
            const double dlo = dmean(-1.0), dhi = dmean(1.0);
            const double lo = dlo * inv2pi - 2e-6;
            const double hi = dhi * inv2pi + 2e-6;
            // |dE| < pi on both sides unless e is close to 1 and the arc is the
            // whole front half; a wrapped atan2 shows as a sign change
            if (dlo < 0.0 && dhi > 0.0 && hi - lo < 1.0) {
                c.flo = lo;
                c.wn = hi - lo;
            } else {
                flags |= kAlways;
            }
        }
    }
    c.flags = flags;
    return c;
}

// Is phase u = (t - t0)/P inside the transit window (repeated every
// period), widened by hw_phase (half an exposure, in periods) on each side?
__device__ inline bool in_phase_window(double u, const PvConst& p, double hw_phase) {
    const double g = u - (p.flo - hw_phase);
    return (g - floor(g)) < p.wn + 2.0 * hw_phase;
}

// Per-vector LD: a tile of 16 consecutive rows in k-row order goes to the
// matrix cores when its rows span at most kMfmaMaxRuns k-rows (each W value
// is then read once for the tile), else to the per-row kernels.  The
// matrix-core and per-row kernels apply this same test to the sorted keys.
constexpr int kMfmaMaxRuns = 2;
// Wave-level: lanes 0..15 each read one key, so it must be called by whole
// waves (the result is uniform).
__device__ inline bool tile_on_matrix_cores(const int32_t* __restrict__ ikr,
                                            const int32_t* __restrict__ perm, int64_t nr,
                                            int64_t tile) {
    const int lane = threadIdx.x & 63, q = lane & 15;
    const int64_t pos = tile * 16 + q;
    const bool in = pos < nr;
    const int ik = in ? ikr[perm[pos]] : -1;
    const int prev = __shfl(ik, (lane & 48) | ((q + 15) & 15), 64);
    const uint64_t starts = __ballot(lane < 16 && in && (q == 0 || ik != prev));
    return __popcll(starts) <= kMfmaMaxRuns;
}

}  // namespace rr
