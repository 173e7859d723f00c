// Host build of the library's per-row setup (make_pv_const), so CPU tests
// can check the transit window it computes against the oracle's orbit.
#include <cmath>

#include "rr_device.h"

namespace {
// host stand-ins of the GPU's float reciprocal and square root (exact)
struct HostOps {
    static float rcp(float x) { return 1.0f / x; }
    static float sqrt(float x) { return std::sqrt(x); }
    static double rcp(double x) { return 1.0 / x; }
};
}  // namespace

extern "C" {
int probe_pvconst_size() { return int(sizeof(rr::PvConst)); }
// rows[n][npar] -> flags, window start and width (phase units) per row
// f32: the mixed precision's setup (float sin w, cos w and sqrt(1 - e^2))
void probe_windows(const double* rows, int n, int npar, double k0, double k1, int f32,
                   int* flags, double* flo, double* wn) {
    for (int i = 0; i < n; ++i) {
        const rr::PvConst c =
            f32 ? rr::make_pv_const<true, HostOps>(rows + size_t(i) * npar, npar - 6, k0, k1)
                : rr::make_pv_const<false, HostOps>(rows + size_t(i) * npar, npar - 6, k0, k1);
        flags[i] = c.flags;
        flo[i] = c.flo;
        wn[i] = c.wn;
    }
}
}
