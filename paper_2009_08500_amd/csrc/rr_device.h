// rr_device.h -- device math of the RoadRunner path, templated on the real
// type of the bulk arithmetic (double for RR_FP64, float for RR_MIXED).
#pragma once

#include <hip/hip_runtime.h>

#include "rr_internal.h"

namespace rr {

template <typename R> struct Num;
template <> struct Num<double> {
    static constexpr double pi = 3.14159265358979323846;
    __device__ static double sqrt_(double x) { return sqrt(x); }
    __device__ static double atan2_(double y, double x) { return atan2(y, x); }
    __device__ static void sincos_(double x, double* s, double* c) { sincos(x, s, c); }
    __device__ static double abs_(double x) { return fabs(x); }
    // Halley iterations stop once a step is below this; the cubic rate then
    // leaves an error far below one ulp.
    static constexpr double kepler_stop = 1e-6;
    static constexpr int kepler_maxit = 24;
};
template <> struct Num<float> {
    static constexpr float pi = 3.14159265358979323846f;
    __device__ static float sqrt_(float x) { return sqrtf(x); }
    __device__ static float atan2_(float y, float x) { return atan2f(y, x); }
    __device__ static void sincos_(float x, float* s, float* c) { sincosf(x, s, c); }
    __device__ static float abs_(float x) { return fabsf(x); }
    static constexpr float kepler_stop = 2e-3f;
    static constexpr int kepler_maxit = 20;
};

// Area of the intersection of a disk of radius Rd centred at the origin and a
// disk of radius k centred at distance c (the lens a(c, k) of Eq. 5 when
// Rd = 1).  In the partial-overlap case the three centres-and-chord-end
// triangle has sides (Rd, k, c); its area D comes from Kahan's stable form of
// Heron's formula (sides sorted a >= b >= c), the half chord is h = 2D/c and
// the two half-angles are atan2(h, x) with x the signed distances from each
// centre to the chord.  A = Rd^2 k1 + k^2 k0 - c h.  Unlike the arccos form
// this keeps full relative accuracy near contact points, where FP32 would
// otherwise lose several ppm.
template <typename R>
__device__ inline R lens_area(R Rd, R k, R c) {
    using N = Num<R>;
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
    const R h = area2 / c;                          // half chord
    const R x1 = (c * c + (Rd - k) * (Rd + k)) / (R(2) * c);
    const R x0 = c - x1;
    const R k1 = N::atan2_(h, x1);
    const R k0 = N::atan2_(h, x0);
    return Rd * Rd * k1 + k * k * k0 - area2;
}

// Orbit constants of one parameter vector in the bulk precision.
template <typename R>
struct OrbitR {
    R n, e, sE, cE, q, a, cosw, sinw, rtr, cosi;
    __device__ explicit OrbitR(const PvConst& p)
        : n(R(p.n)), e(R(p.e)), sE(R(p.sE)), cE(R(p.cE)), q(R(p.q)),
          a(R(p.a)), cosw(R(p.cosw)), sinw(R(p.sinw)), rtr(R(p.rtr)),
          cosi(R(p.cosi)) {}
};

// Projected separation for a time offset dt from conjunction.
//
// Transit-centred Kepler solve: with E = E_tr + d and dM = n dt, Kepler's
// equation becomes h(d) = d - e [sin E_tr (cos d - 1) + cos E_tr sin d] - dM
// = 0.  h is increasing (h' = 1 - e cos E > 0) and its root lies in
// [dM - 2e, dM + 2e]; Halley's method starts from d = dM / (1 - e cos E_tr)
// and is safeguarded by that bracket (a step leaving the current bracket is
// replaced by bisection), so it converges for any e < 1.  The sky
// coordinates are formed from the differences cos E - cos E_tr and
// sin E - sin E_tr (using cos d - 1 = -2 sin^2(d/2)), so every intermediate
// is small near transit and FP32 keeps its relative precision there:
//   X   = -a [(cos E - cos E_tr) cos w - q (sin E - sin E_tr) sin w]
//   rho = r sin(w + f) = r_tr + a [(cos E - cos E_tr) sin w
//                                  + q (sin E - sin E_tr) cos w]
//   Y   = -rho cos i,  z = sqrt(X^2 + Y^2),  in front iff rho > 0.
template <typename R>
__device__ inline R separation(R dt, const OrbitR<R>& o, bool* front) {
    using N = Num<R>;
    const R dM = o.n * dt;
    R d = dM;
    R s2, c2;
    if (o.e > R(0)) {
        R lo = dM - R(2) * o.e, hi = dM + R(2) * o.e;
        d = dM / (R(1) - o.e * o.cE);
        d = d < lo ? lo : (d > hi ? hi : d);
        for (int it = 0; it < N::kepler_maxit; ++it) {
            N::sincos_(R(0.5) * d, &s2, &c2);
            const R sd = R(2) * s2 * c2;
            const R cm1 = R(-2) * s2 * s2;
            const R h = d - o.e * (o.sE * cm1 + o.cE * sd) - dM;
            if (h < R(0)) lo = d; else hi = d;
            const R hp = R(1) - o.e * (o.cE * (R(1) + cm1) - o.sE * sd);
            const R hpp = o.e * (o.sE * (R(1) + cm1) + o.cE * sd);
            R dn = d - h / (hp - R(0.5) * h * hpp / hp);
            if (!(dn >= lo && dn <= hi)) dn = R(0.5) * (lo + hi);
            const R step = dn - d;
            d = dn;
            if (N::abs_(step) < N::kepler_stop) break;
        }
    }
    N::sincos_(R(0.5) * d, &s2, &c2);
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

// Orbit constants and transit window of one parameter row
// [t0, P, a, b, e, w, k_0 .. k_{npb-1}] (FP64).  The row is invalid (NaN
// output) if any value is non-finite, P <= 0, a <= 0, b < 0, e outside
// [0, 1), a k outside [k0, k1] or |cos i| > 1.
__device__ inline PvConst make_pv_const(const double* row, int npb, double k0,
                                        double k1) {
    PvConst c = {};
    const double t0 = row[0], P = row[1], a = row[2], b = row[3], e = row[4],
                 w = row[5];
    bool ok = isfinite(t0) && isfinite(P) && isfinite(a) && isfinite(b) &&
              isfinite(e) && isfinite(w) && P > 0.0 && a > 0.0 && b >= 0.0 &&
              e >= 0.0 && e < 1.0;
    double kmax = 0.0;
    for (int pb = 0; pb < npb; ++pb) {
        const double k = row[6 + pb];
        ok = ok && isfinite(k) && k >= k0 && k <= k1;
        kmax = k > kmax ? k : kmax;
    }
    double sw = 0.0, cw = 1.0;
    if (ok) sincos(w, &sw, &cw);
    const double q = ok ? sqrt(1.0 - e * e) : 1.0;
    const double cosi = ok ? b * (1.0 + e * sw) / (a * (1.0 - e * e)) : 0.0;
    ok = ok && fabs(cosi) <= 1.0;
    c.t0 = t0; c.P = P; c.invP = 1.0 / P; c.n = 2.0 * Num<double>::pi / P;
    c.a = a; c.e = e; c.cosw = cw; c.sinw = sw; c.q = q; c.cosi = cosi;
    // conjunction: f_tr = pi/2 - w, so cos f_tr = sin w and sin f_tr = cos w
    const double den = 1.0 + e * sw;
    c.cE = (e + sw) / den;
    c.sE = q * cw / den;
    c.rtr = a * (1.0 - e * e) / den;
    c.kmax = kmax;
    int32_t flags = ok ? kValid : 0;
    c.flo = 0.0;
    c.wn = 2.0;                      // covers every phase unless narrowed below
    if (ok) {
        // The planet can overlap the star only while r |cos(w + f)| < 1 + k
        // and sin(w + f) > 0.  With r >= a (1 - e) that confines f to
        // |f - f_tr| < theta = asin((1 + kmax) / (a (1 - e))).
        const double s = (1.0 + kmax) / (a * (1.0 - e)) * (1.0 + 1e-6) + 1e-12;
        if (s >= 1.0) {
            flags |= kAlways;
        } else {
            const double theta = asin(s);
            const double ftr = 0.5 * Num<double>::pi - w;
            const double beta = e / (1.0 + q);
            // mean anomaly as a continuous (unwrapped) function of the true
            // anomaly: E = f - 2 atan(beta sin f / (1 + beta cos f))
            auto mean_of_true = [&](double f) {
                double sf, cf;
                sincos(f, &sf, &cf);
                const double E = f - 2.0 * atan(beta * sf / (1.0 + beta * cf));
                return E - e * sin(E);
            };
            const double m0 = mean_of_true(ftr);
            const double inv2pi = 0.5 / Num<double>::pi;
            // window in phase units (mean anomaly / 2 pi) around conjunction,
            // widened by 1e-8 of a period on each side, more than the
            // rounding of a phase t/P - t0/P of up to 1e7 periods
            const double lo = (mean_of_true(ftr - theta) - m0) * inv2pi - 1e-8;
            const double hi = (mean_of_true(ftr + theta) - m0) * inv2pi + 1e-8;
            if (hi - lo < 1.0) {
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

}  // namespace rr
