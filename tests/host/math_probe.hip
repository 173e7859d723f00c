// Host build of the library's device math (rr_device.h) for CPU tests: the
// same template code as the kernels use, instantiated with host stand-ins of
// the GPU's reciprocal and square-root estimates (exact float division and
// square root; for the double reciprocal an estimate with a relative error
// the caller chooses, which the two Newton steps of rcp_nr must remove).
#include <cmath>

#include "rr_device.h"

namespace {
double g_rcp_rel_err = 0.0;   // relative error of the double reciprocal estimate

struct HostOps {
    static float rcp(float x) { return 1.0f / x; }
    static float sqrt(float x) { return std::sqrt(x); }
    static double rcp(double x) { return (1.0 / x) * (1.0 + g_rcp_rel_err); }
};
}  // namespace

extern "C" {
float probe_atan2f(float y, float x) { return rr::atan2_poly<HostOps>(y, x); }
double probe_atan2d(double y, double x) { return rr::atan2_poly<HostOps>(y, x); }
double probe_rcp_nr(double x, double est_rel_err) {
    g_rcp_rel_err = est_rel_err;
    const double r = rr::rcp_nr<HostOps>(x);
    g_rcp_rel_err = 0.0;
    return r;
}
void probe_sincos_small_f(float x, float* s, float* c) { rr::sincos_small(x, s, c); }
float probe_lens_area_f(float R, float k, float c) { return rr::lens_area<float, HostOps>(R, k, c); }
double probe_lens_area_d(double R, double k, double c) {
    return rr::lens_area<double, HostOps>(R, k, c);
}
// Kepler solve around conjunction: d = E - E_tr for mean-anomaly offset dM;
// also sin(d/2), cos(d/2) as returned with it.
float probe_kepler_f(float dM, float e, float sE, float cE, float* s2, float* c2) {
    return rr::kepler_offset<float, HostOps>(dM, e, sE, cE, s2, c2);
}
double probe_kepler_d(double dM, double e, double sE, double cE, double* s2, double* c2) {
    return rr::kepler_offset<double, HostOps>(dM, e, sE, cE, s2, c2);
}
}
