// rr_capi.hip -- the C ABI: argument validation, handle lifetime, launches.
//
// Every argument check happens on the host before any HIP call, so invalid
// calls return an error code and enqueue nothing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "rr_internal.h"

namespace rr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

KernelEvents& kernel_events() {
    static thread_local KernelEvents ev;
    return ev;
}

int hip_fail(hipError_t err, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(err));
    return RR_EDEVICE;
}

// Device array behind rr_evaluate_noalloc: the orbit constants of at most
// RR_NOALLOC_MAX_PV rows, one copy per GPU for the life of the process.  In
// host code its name is not a device address: every use goes through the
// address hipGetSymbolAddress reports for the device (g_noalloc_scratch).
static __device__ __align__(256) PvConst scratch[RR_NOALLOC_MAX_PV];
constexpr int kMaxDevices = 256;
static std::mutex g_noalloc_mu;
static PvConst* g_noalloc_scratch[kMaxDevices] = {};

// Resolve `device`'s copy of the array once; `device` must be current.
static int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return RR_OK;   // entry point reports it
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_scratch[device]) return RR_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_noalloc_scratch[device] = static_cast<PvConst*>(ptr);
    return RR_OK;
}

static int einval(const char* msg) {
    set_error(msg);
    return RR_EINVAL;
}

static int elimit(const char* msg) {
    set_error(msg);
    return RR_ELIMIT;
}

static int check_grid(const rr_grid* g) {
    if (!g) return einval("grid is NULL");
    if (!(g->zcut > 0.0 && g->zcut < 1.0)) return einval("grid.zcut must be in (0, 1)");
    if (g->nzin < 1 || g->nzlimb < 1) return einval("grid.nzin and grid.nzlimb must be >= 1");
    if (int64_t(g->nzin) + g->nzlimb > 4096) return einval("grid.nzin + grid.nzlimb must be <= 4096");
    if (g->ng < 2 || g->ng > 4096) return einval("grid.ng must be in [2, 4096]");
    if (g->nk < 2 || g->nk > 4096) return einval("grid.nk must be in [2, 4096]");
    if (!(g->k0 > 0.0 && g->k0 < g->k1 && g->k1 < 1.0))
        return einval("grid k range must satisfy 0 < k0 < k1 < 1");
    return RR_OK;
}

hipError_t stream_workspace(rr_tables* t, hipStream_t stream, size_t bytes, void** out) {
    std::lock_guard<std::mutex> lk(t->ws_mu);
    auto& slot = t->ws[stream];
    if (slot.second < bytes) {
        if (slot.first) {
            hipError_t e = hipFree(slot.first);     // synchronising; growth only
            slot.first = nullptr;
            slot.second = 0;
            if (e != hipSuccess) return e;
        }
        const size_t nb = std::max(bytes, size_t(1) << 16);
        hipError_t e = hipMalloc(&slot.first, nb);
        if (e != hipSuccess) return e;
        slot.second = nb;
    }
    *out = slot.first;
    return hipSuccess;
}

static void free_tables(rr_tables* t) {
    if (!t) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    void* bufs[] = {t->mu_s, t->prof, t->ze, t->zm, t->ldp, t->istar,
                    t->W, t->W32, t->T64, t->T32, t->inv_istar, t->istar_user};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (auto& kv : t->ws)
        if (kv.second.first) (void)hipFree(kv.second.first);

    (void)hipSetDevice(cur);
    delete t;
}

// Common checks of rr_evaluate / rr_loglik_grad.
int check_eval_args(const rr_tables* t, const double* times_d,
                    const int32_t* lcids_d, int32_t npt, const int32_t* pbids,
                    const int32_t* nss, const double* exptimes, int32_t nlc,
                    const double* pv_d, int32_t npv, int32_t npar,
                    int32_t precision, LcInfo* lc) {
    if (!t) return einval("tables handle is NULL");
    if (npt < 0 || npv < 0) return einval("npt and npv must be >= 0");
    if (precision != RR_FP64 && precision != RR_MIXED)
        return einval("precision must be RR_FP64 or RR_MIXED");
    if (npar != 6 + t->npb) return einval("npar must equal 6 + npb of the tables");
    if (nlc < 1) return einval("nlc must be >= 1");
    if (nlc > RR_MAX_LC) return elimit("nlc exceeds RR_MAX_LC");
    if (!lcids_d && nlc != 1) return einval("lcids may be NULL only when nlc == 1");
    if (!pbids || !nss || !exptimes) return einval("pbids, nss and exptimes are required");
    lc->nlc = nlc;
    for (int i = 0; i < nlc; ++i) {
        if (pbids[i] < 0 || pbids[i] >= t->npb) return einval("pbids entry outside [0, npb)");
        if (nss[i] < 1) return einval("nss entries must be >= 1");
        if (nss[i] > RR_MAX_NSS) return elimit("nss entry exceeds RR_MAX_NSS");
        if (!(exptimes[i] >= 0.0) || !isfinite(exptimes[i]))
            return einval("exptimes entries must be finite and >= 0");
        lc->pb[i] = pbids[i];
        lc->nss[i] = nss[i];
        lc->exptime[i] = exptimes[i];
    }
    for (int i = nlc; i < RR_MAX_LC; ++i) {
        lc->pb[i] = 0;
        lc->nss[i] = 1;
        lc->exptime[i] = 0.0;
    }
    if (npt > 0 && npv > 0) {
        if (!times_d) return einval("times is NULL");
        if (!pv_d) return einval("pv is NULL");
    }
    const int64_t ntiles = (int64_t(npt) + adj_tile(true, false) - 1) /
                           adj_tile(true, false);            // the smaller tiles
    if (ntiles * npv * kAdjBlock >= (int64_t(1) << 32) ||
        ((int64_t(npt) + 4 * kFwdBlock - 1) / (4 * kFwdBlock)) * npv * kFwdBlock >=
            (int64_t(1) << 32))                  // the smallest forward tile (J = 4)
        return elimit("npv * npt too large for one launch");
    return RR_OK;
}

int check_device(const rr_tables* t) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != t->device) return einval("tables live on another device than the current one");
    return RR_OK;
}

}  // namespace rr

using namespace rr;

extern "C" {

RR_API const char* rr_strerror(int code) {
    switch (code) {
        case RR_OK: return "success";
        case RR_EINVAL: return "invalid argument";
        case RR_ENOMEM: return "out of memory";
        case RR_EDEVICE: return "HIP device error";
        case RR_ELIMIT: return "size exceeds a compiled-in limit";
        case RR_EBUSY: return "request does not fit the serving budget now";
        case RR_ENOTFOUND: return "unknown request id";
        default: return "unknown error code";
    }
}

RR_API const char* rr_last_error(void) { return g_last_error.c_str(); }

RR_API int rr_prepare_ld(const double* mu, const double* prof, int32_t nmu,
                         int32_t npb, const rr_grid* grid, rr_tables** out) {
    if (!out) return einval("out is NULL");
    *out = nullptr;
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!mu || !prof) return einval("mu and prof are required");
    if (nmu < 2 || nmu > 65536) return einval("nmu must be in [2, 65536]");
    if (npb < 1) return einval("npb must be >= 1");
    if (npb > RR_MAX_PB) return elimit("npb exceeds RR_MAX_PB");
    for (int i = 0; i < nmu; ++i) {
        if (!(mu[i] >= 0.0 && mu[i] <= 1.0)) return einval("mu samples must lie in [0, 1]");
        if (i && !(mu[i] > mu[i - 1])) return einval("mu samples must be strictly increasing");
    }
    for (int64_t i = 0; i < int64_t(npb) * nmu; ++i)
        if (!isfinite(prof[i])) return einval("profile samples must be finite");

    rr_tables* t = new (std::nothrow) rr_tables();
    if (!t) return RR_ENOMEM;
    t->grid = *grid;
    t->nz = grid->nzin + grid->nzlimb;
    t->npb = npb;
    t->nmu = nmu;
    t->dk = (grid->k1 - grid->k0) / (grid->nk - 1);
    hipError_t e = hipGetDevice(&t->device);
    if (e != hipSuccess) { delete t; return hip_fail(e, "hipGetDevice"); }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, t->device) !=
            hipSuccess || lds < kMinLdsBytes)
        lds = kMinLdsBytes;
    t->lds_max = size_t(lds);
    rc = noalloc_init(t->device);
    if (rc) { delete t; return rc; }

    const int64_t nz = t->nz, ng = grid->ng, nk = grid->nk;
    struct { void** p; size_t bytes; } allocs[] = {
        {(void**)&t->mu_s, sizeof(double) * nmu},
        {(void**)&t->prof, sizeof(double) * npb * nmu},
        {(void**)&t->ze, sizeof(double) * (nz + 1)},
        {(void**)&t->zm, sizeof(double) * nz},
        {(void**)&t->ldp, sizeof(double) * npb * nz},
        {(void**)&t->istar, sizeof(double) * npb},
        {(void**)&t->inv_istar, sizeof(double) * npb},
        {(void**)&t->W, sizeof(double) * nk * nz * ng},
        {(void**)&t->W32, sizeof(float) * nk * nz * ng},
        {(void**)&t->T64, sizeof(double) * npb * nk * ng},
        {(void**)&t->T32, sizeof(float) * npb * nk * ng},
    };
    for (auto& a : allocs) {
        e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) {
            free_tables(t);
            set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? RR_ENOMEM : RR_EDEVICE;
        }
    }
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) { free_tables(t); return hip_fail(e, "hipStreamCreate"); }
    auto fail = [&](hipError_t err, const char* what) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        free_tables(t);
        return hip_fail(err, what);
    };
    e = hipMemcpyAsync(t->mu_s, mu, sizeof(double) * nmu, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(e, "copy mu");
    e = hipMemcpyAsync(t->prof, prof, sizeof(double) * npb * nmu, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(e, "copy profile");
    e = launch_prepare_grid_weights(t, s);
    if (e != hipSuccess) return fail(e, "weight kernels");
    e = launch_prepare_profile(t, s);
    if (e != hipSuccess) return fail(e, "profile kernels");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(e, "table construction");
    (void)hipStreamDestroy(s);
    *out = t;
    return RR_OK;
}

RR_API int rr_set_profile(rr_tables* t, const double* prof_d, hipStream_t stream) {
    if (!t) return einval("tables handle is NULL");
    if (!prof_d) return einval("prof is NULL");
    int rc = check_device(t);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(t->prof, prof_d, sizeof(double) * t->npb * t->nmu,
                                  hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "copy profile");
    e = launch_prepare_profile(t, stream);
    if (e != hipSuccess) return hip_fail(e, "profile kernels");
    return RR_OK;
}

RR_API int rr_set_istar(rr_tables* t, const double* istar_d, hipStream_t stream) {
    if (!t) return einval("tables handle is NULL");
    int rc = check_device(t);
    if (rc) return rc;
    hipError_t e;
    if (!istar_d) {
        t->istar_fixed = false;
        e = launch_istar_from_profile(t, stream);
        if (e != hipSuccess) return hip_fail(e, "I_star kernel");
        return RR_OK;
    }
    if (!t->istar_user) {
        e = hipMalloc((void**)&t->istar_user, sizeof(double) * t->npb);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "hipMalloc");
    }
    e = launch_istar_set(t, istar_d, stream);
    if (e != hipSuccess) return hip_fail(e, "I_star kernel");
    t->istar_fixed = true;
    return RR_OK;
}

RR_API int rr_evaluate(const rr_tables* t, const double* times_d,
                       const int32_t* lcids_d, int32_t npt,
                       const int32_t* pbids, const int32_t* nss,
                       const double* exptimes, int32_t nlc,
                       const double* pv_d, int32_t npv, int32_t npar,
                       int32_t precision, void* out_d, hipStream_t stream) {
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    if (npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    rc = check_device(t);
    if (rc) return rc;
    void* ws = nullptr;
    hipError_t e = stream_workspace(const_cast<rr_tables*>(t), stream,
                                    sizeof(PvConst) * size_t(npv), &ws);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "workspace");
    PvConst* pvc = static_cast<PvConst*>(ws);
    e = launch_pv_setup(t, pv_d, npv, npar, pvc, precision, stream);
    if (e == hipSuccess)
        e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc,
                           precision, out_d, stream);
    if (e != hipSuccess) return hip_fail(e, "forward kernels");
    return RR_OK;
}

RR_API int rr_evaluate_noalloc(const rr_tables* t, const double* times_d,
                               const int32_t* lcids_d, int32_t npt,
                               const int32_t* pbids, const int32_t* nss,
                               const double* exptimes, int32_t nlc,
                               const double* pv_d, int32_t npv, int32_t npar,
                               int32_t precision, void* out_d, hipStream_t stream) {
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    if (npv > RR_NOALLOC_MAX_PV) return elimit("npv exceeds RR_NOALLOC_MAX_PV");
    if (npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    rc = check_device(t);
    if (rc) return rc;
    PvConst* pvc = nullptr;
    if (t->device >= 0 && t->device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        pvc = g_noalloc_scratch[t->device];
    }
    if (!pvc) return elimit("no fixed device array on this device");
    hipError_t e = launch_pv_setup(t, pv_d, npv, npar, pvc, precision, stream);
    if (e == hipSuccess)
        e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc,
                           precision, out_d, stream);
    if (e != hipSuccess) return hip_fail(e, "forward kernels");
    return RR_OK;
}

// ------------------------------------------------------------ time series
static void free_series(rr_series* se) {
    if (!se) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (se->device >= 0) (void)hipSetDevice(se->device);
    void* bufs[] = {se->times, se->lcids, se->lcs, se->buckets};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    (void)hipSetDevice(cur);
    delete se;
}

RR_API int rr_series_create(const double* times, const int32_t* lcids, int32_t npt,
                            const int32_t* pbids, const int32_t* nss,
                            const double* exptimes, int32_t nlc, rr_series** out) {
    if (!out) return einval("out is NULL");
    *out = nullptr;
    if (npt < 0) return einval("npt must be >= 0");
    if (npt > 0 && !times) return einval("times is NULL");
    if (nlc < 1) return einval("nlc must be >= 1");
    if (nlc > RR_MAX_LC) return elimit("nlc exceeds RR_MAX_LC");
    if (!lcids && nlc != 1) return einval("lcids may be NULL only when nlc == 1");
    if (!pbids || !nss || !exptimes) return einval("pbids, nss and exptimes are required");
    for (int i = 0; i < nlc; ++i) {
        if (pbids[i] < 0 || pbids[i] >= RR_MAX_PB) return einval("pbids entry outside [0, RR_MAX_PB)");
        if (nss[i] < 1) return einval("nss entries must be >= 1");
        if (nss[i] > RR_MAX_NSS) return elimit("nss entry exceeds RR_MAX_NSS");
        if (!(exptimes[i] >= 0.0) || !isfinite(exptimes[i]))
            return einval("exptimes entries must be finite and >= 0");
    }
    rr_series* se = new (std::nothrow) rr_series();
    if (!se) return RR_ENOMEM;
    se->npt = npt;
    se->nlc = nlc;
    se->pbids.assign(pbids, pbids + nlc);
    se->nss.assign(nss, nss + nlc);
    se->exptimes.assign(exptimes, exptimes + nlc);
    se->lc.nlc = nlc;
    for (int i = 0; i < RR_MAX_LC; ++i) {
        se->lc.pb[i] = i < nlc ? pbids[i] : 0;
        se->lc.nss[i] = i < nlc ? nss[i] : 1;
        se->lc.exptime[i] = i < nlc ? exptimes[i] : 0.0;
        if (i < nlc) se->max_nss = std::max(se->max_nss, nss[i]);
    }
    // Each light curve one contiguous run of finite, non-decreasing times?
    // Then the per-light-curve time index for the split launch.
    std::vector<SeriesLc> lcs;
    std::vector<int32_t> buckets;
    bool all_zero = true;
    const bool indexed = build_series_index(times, lcids, npt, nlc, &lcs, &buckets, &all_zero);
    se->indexed = indexed;
    hipError_t e = hipGetDevice(&se->device);
    if (e != hipSuccess) { delete se; return hip_fail(e, "hipGetDevice"); }
    // lcids are kept unless one light curve covers every exposure
    const bool keep_ids = lcids && !(nlc == 1 && all_zero && indexed);
    struct { void** p; const void* src; size_t bytes; } up[] = {
        {(void**)&se->times, times, sizeof(double) * size_t(npt)},
        {(void**)&se->lcids, keep_ids ? lcids : nullptr, keep_ids ? sizeof(int32_t) * size_t(npt) : 0},
        {(void**)&se->lcs, indexed ? lcs.data() : nullptr, indexed ? sizeof(SeriesLc) * lcs.size() : 0},
        {(void**)&se->buckets, indexed ? buckets.data() : nullptr,
         indexed ? sizeof(int32_t) * buckets.size() : 0},
    };
    for (auto& u : up) {
        if (!u.src || u.bytes == 0) continue;
        e = hipMalloc(u.p, u.bytes);
        if (e == hipSuccess) e = hipMemcpy(*u.p, u.src, u.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_series(se);
            set_error(std::string("series upload: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? RR_ENOMEM : RR_EDEVICE;
        }
    }
    *out = se;
    return RR_OK;
}

RR_API void rr_series_free(rr_series* s) { free_series(s); }

RR_API int rr_evaluate_series(const rr_tables* t, const rr_series* se, const double* pv_d,
                              int32_t npv, int32_t npar, int32_t precision, void* out_d,
                              hipStream_t stream) {
    if (!se) return einval("series is NULL");
    LcInfo lc;
    int rc = check_eval_args(t, se->times, se->lcids, se->npt, se->pbids.data(),
                             se->nss.data(), se->exptimes.data(), se->nlc, pv_d, npv, npar,
                             precision, &lc);
    if (rc) return rc;
    if (se->npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    rc = check_device(t);
    if (rc) return rc;
    if (se->device != t->device) return einval("series and tables live on different devices");
    const bool split = se->indexed && split_preferred(t, se, npv, precision);
    const SplitPlan sp = split ? plan_forward_split(se, npv, precision) : SplitPlan{};
    hipError_t e = hipSuccess;
    PvConst* pvc = nullptr;
    if (!(split && sp.self_setup)) {
        void* ws = nullptr;
        e = stream_workspace(const_cast<rr_tables*>(t), stream, sizeof(PvConst) * size_t(npv),
                             &ws);
        if (e != hipSuccess)
            return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "workspace");
        pvc = static_cast<PvConst*>(ws);
        e = launch_pv_setup(t, pv_d, npv, npar, pvc, precision, stream);
    }
    // Per-tile kernel on a supersampled series: 4 exposures per lane (twice
    // the waves) while the call has at most 16 384 waves of 8 exposures per
    // lane, where it measured faster (heterogeneous series of 64 rows 22.7
    // -> 15.6 us, 30-minute exposures at nss 10 over 256 x 20 000 48.7 ->
    // 42.8 us in float), else rr_evaluate's 8.
    const int64_t waves8 = int64_t(npv) * ((se->npt + kFwdBlock * 8 - 1) / (kFwdBlock * 8));
    const int variant = se->max_nss > 1 && waves8 <= 16384 ? 0 : kDefaultFwdVariant;
    if (e == hipSuccess)
        e = split ? launch_forward_split(t, se, sp, pv_d, npv, npar, pvc, precision, out_d,
                                         stream)
                  : launch_forward(t, se->times, se->lcids, se->npt, lc, pv_d, npv, npar, pvc,
                                   precision, out_d, stream, nullptr, nullptr, 0, variant);
    if (e != hipSuccess) return hip_fail(e, "forward kernels");
    return RR_OK;
}

RR_API int rr_series_kernel(const rr_tables* t, const rr_series* se, int32_t npv,
                            int32_t precision, int32_t* kind) {
    if (!kind) return einval("kind is NULL");
    *kind = RR_KERNEL_TILES;
    if (!t) return einval("tables handle is NULL");
    if (!se) return einval("series is NULL");
    if (npv < 0) return einval("npv must be >= 0");
    if (precision != RR_FP64 && precision != RR_MIXED) return einval("unknown precision");
    int rc = check_device(t);
    if (rc) return rc;
    if (se->indexed && split_preferred(t, se, npv, precision))
        *kind = plan_forward_split(se, npv, precision).self_setup ? RR_KERNEL_SPLIT_FUSED
                                                                  : RR_KERNEL_SPLIT;
    return RR_OK;
}

RR_API int rr_evaluate_variant(const rr_tables* t, const double* times_d,
                               const int32_t* lcids_d, int32_t npt,
                               const int32_t* pbids, const int32_t* nss,
                               const double* exptimes, int32_t nlc,
                               const double* pv_d, int32_t npv, int32_t npar,
                               int32_t precision, int32_t variant, void* out_d,
                               hipStream_t stream) {
    if (variant < 0 || variant >= RR_NUM_VARIANTS) return einval("unknown variant");
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    if (npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    rc = check_device(t);
    if (rc) return rc;
    void* ws = nullptr;
    hipError_t e = stream_workspace(const_cast<rr_tables*>(t), stream,
                                    sizeof(PvConst) * size_t(npv), &ws);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "workspace");
    PvConst* pvc = static_cast<PvConst*>(ws);
    e = launch_pv_setup(t, pv_d, npv, npar, pvc, precision, stream);
    if (e == hipSuccess)
        e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc, precision,
                           out_d, stream, nullptr, nullptr, 0, variant);
    if (e != hipSuccess) return hip_fail(e, "forward kernels");
    return RR_OK;
}

RR_API int rr_select_variant(const rr_tables* t, const double* times_d,
                             const int32_t* lcids_d, int32_t npt,
                             const int32_t* pbids, const int32_t* nss,
                             const double* exptimes, int32_t nlc,
                             const double* pv_d, int32_t npv, int32_t npar,
                             int32_t precision, void* out_d, int32_t reps,
                             int32_t* best, float* ms, hipStream_t stream) {
    if (!best) return einval("best is NULL");
    if (reps < 1 || reps > 1000) return einval("reps must lie in [1, 1000]");
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    *best = kDefaultFwdVariant;
    if (ms)
        for (int v = 0; v < RR_NUM_VARIANTS; ++v) ms[v] = 0.0f;
    if (npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    rc = check_device(t);
    if (rc) return rc;
    void* ws = nullptr;
    hipError_t e = stream_workspace(const_cast<rr_tables*>(t), stream,
                                    sizeof(PvConst) * size_t(npv), &ws);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "workspace");
    PvConst* pvc = static_cast<PvConst*>(ws);
    e = launch_pv_setup(t, pv_d, npv, npar, pvc, precision, stream);
    if (e != hipSuccess) return hip_fail(e, "setup kernel");
    // without supersampling the one-lane-per-exposure variants launch the
    // same kernels as the others: only J is tried
    bool sub = false;
    for (int l = 0; l < lc.nlc; ++l) sub = sub || lc.nss[l] > 1;
    const int nv = sub ? RR_NUM_VARIANTS : 3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float tbest = 0.0f;
    for (int v = 0; v < nv && e == hipSuccess; ++v) {
        // one untimed launch, then reps launches between two events
        e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc, precision,
                           out_d, stream, nullptr, nullptr, 0, v);
        if (e == hipSuccess) e = hipEventRecord(e0, stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc, precision,
                               out_d, stream, nullptr, nullptr, 0, v);
        if (e == hipSuccess) e = hipEventRecord(e1, stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float el = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&el, e0, e1);
        if (e != hipSuccess) break;
        el /= float(reps);
        if (ms) {
            ms[v] = el;
            if (!sub) ms[v + 3] = el;
        }
        if (v == 0 || el < tbest) {
            tbest = el;
            *best = v;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "variant trial");
    return RR_OK;
}

RR_API int rr_evaluate_direct(const rr_tables* t, const double* times_d,
                              const int32_t* lcids_d, int32_t npt,
                              const int32_t* pbids, const int32_t* nss,
                              const double* exptimes, int32_t nlc,
                              const double* pv_d, int32_t npv, int32_t npar,
                              int32_t precision, void* out_d, hipStream_t stream) {
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    if (npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    const int64_t nr = int64_t(npv) * t->npb;
    if (nr * ((t->grid.ng + kBlock - 1) / kBlock) >= (int64_t(1) << 31))
        return elimit("npv * npb too large");
    rc = check_device(t);
    if (rc) return rc;
    const size_t elt = precision == RR_FP64 ? sizeof(double) : sizeof(float);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    const size_t o_pvc = take(sizeof(PvConst) * size_t(npv));
    const size_t o_rows = take(elt * size_t(nr) * 2 * t->grid.ng);
    void* ws = nullptr;
    hipError_t e = stream_workspace(const_cast<rr_tables*>(t), stream, off, &ws);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "workspace");
    char* base = static_cast<char*>(ws);
    PvConst* pvc = reinterpret_cast<PvConst*>(base + o_pvc);
    void* rows = base + o_rows;
    // any k in (0, 1]: the smallest positive double as the lower bound
    e = launch_pv_setup_k(pv_d, npv, npar, 4.9406564584124654e-324, 1.0, pvc, precision,
                          stream);
    if (e == hipSuccess) e = launch_direct_rows(t, pv_d, npv, npar, precision, rows, stream);
    if (e == hipSuccess)
        e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc, precision,
                           out_d, stream, rows, nullptr, 1);
    if (e != hipSuccess) return hip_fail(e, "direct-model kernels");
    return RR_OK;
}

RR_API int rr_evaluate_small_planet(const rr_tables* t, const double* times_d,
                                    const int32_t* lcids_d, int32_t npt,
                                    const int32_t* pbids, const int32_t* nss,
                                    const double* exptimes, int32_t nlc,
                                    const double* pv_d, int32_t npv, int32_t npar,
                                    double k_small, int32_t precision, void* out_d,
                                    hipStream_t stream) {
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    if (!(k_small >= 0.0 && k_small <= 1.0)) return einval("k_small must lie in [0, 1]");
    if (npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    const int64_t nr = int64_t(npv) * t->npb;
    if (nr >= (int64_t(1) << 31)) return elimit("npv * npb too large");
    rc = check_device(t);
    if (rc) return rc;
    const size_t elt = precision == RR_FP64 ? sizeof(double) : sizeof(float);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    const size_t o_pvc = take(sizeof(PvConst) * size_t(npv));
    const size_t o_rows = take(elt * size_t(nr) * 2 * t->grid.ng);
    void* ws = nullptr;
    hipError_t e = stream_workspace(const_cast<rr_tables*>(t), stream, off, &ws);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "workspace");
    char* base = static_cast<char*>(ws);
    PvConst* pvc = reinterpret_cast<PvConst*>(base + o_pvc);
    void* rows = base + o_rows;
    e = launch_pv_setup_k(pv_d, npv, npar, t->grid.k0, t->grid.k1, pvc, precision, stream,
                          k_small);
    if (e == hipSuccess)
        e = launch_small_planet_rows(t, pv_d, npv, npar, k_small, precision, rows, stream);
    if (e == hipSuccess)
        e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc, precision,
                           out_d, stream, rows, nullptr, 1);
    if (e != hipSuccess) return hip_fail(e, "small-planet kernels");
    return RR_OK;
}

RR_API int rr_flux_at_z(const rr_tables* t, const double* z_d, const double* k_d,
                        double k, int64_t n, int32_t pb, int32_t precision, void* out_d,
                        hipStream_t stream) {
    if (!t) return einval("tables handle is NULL");
    if (n < 0) return einval("n must be >= 0");
    if (n >= (int64_t(1) << 40)) return elimit("n too large");
    if (pb < 0 || pb >= t->npb) return einval("pb out of range");
    if (precision != RR_FP64 && precision != RR_MIXED) return einval("unknown precision");
    if (n == 0) return RR_OK;
    if (!z_d || !out_d) return einval("z and out are required");
    int rc = check_device(t);
    if (rc) return rc;
    hipError_t e = launch_flux_at_z(t, z_d, k_d, k, n, pb, precision, out_d, stream);
    if (e != hipSuccess) return hip_fail(e, "flux kernel");
    return RR_OK;
}

RR_API int rr_evaluate_ld(const rr_tables* t, const double* times_d,
                          const int32_t* lcids_d, int32_t npt,
                          const int32_t* pbids, const int32_t* nss,
                          const double* exptimes, int32_t nlc,
                          const double* pv_d, int32_t npv, int32_t npar,
                          const double* prof_d, int32_t precision, void* out_d,
                          hipStream_t stream) {
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    if (npt == 0 || npv == 0) return RR_OK;
    if (!out_d) return einval("out is NULL");
    if (!prof_d) return einval("prof is NULL");
    const int64_t nr = int64_t(npv) * t->npb;
    if (nr * t->nz >= (int64_t(1) << 31))
        return elimit("npv * npb * nz must stay below 2^31");
    rc = check_device(t);
    if (rc) return rc;
    const size_t elt = precision == RR_FP64 ? sizeof(double) : sizeof(float);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    const size_t o_pvc = take(sizeof(PvConst) * size_t(npv));
    const size_t o_ldp = take(sizeof(double) * size_t(nr) * t->nz);
    const size_t o_is = take(sizeof(double) * size_t(nr));
    const size_t o_iis = take(sizeof(double) * size_t(nr));
    const size_t o_ldw = take(elt * size_t(nr) * 2 * t->grid.ng);
    const size_t o_ikr = take(sizeof(int32_t) * size_t(nr));
    const size_t o_perm = take(sizeof(int32_t) * size_t(nr));
    // the tables' per-stream workspace (as rr_evaluate): reused without
    // waiting by later calls on the same stream
    void* ws = nullptr;
    hipError_t e = stream_workspace(const_cast<rr_tables*>(t), stream, off, &ws);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "workspace");
    char* base = static_cast<char*>(ws);
    PvConst* pvc = reinterpret_cast<PvConst*>(base + o_pvc);
    double* inv_is = reinterpret_cast<double*>(base + o_iis);
    void* ldw = base + o_ldw;
    e = launch_pv_setup(t, pv_d, npv, npar, pvc, precision, stream);
    if (e == hipSuccess)
        e = launch_pv_ld(t, prof_d, pv_d, npv, npar, precision,
                         reinterpret_cast<double*>(base + o_ldp),
                         reinterpret_cast<double*>(base + o_is), inv_is,
                         reinterpret_cast<int32_t*>(base + o_ikr),
                         reinterpret_cast<int32_t*>(base + o_perm), ldw, stream,
                         precision == RR_MIXED);
    if (e == hipSuccess)
        e = launch_forward(t, times_d, lcids_d, npt, lc, pv_d, npv, npar, pvc, precision,
                           out_d, stream, ldw, inv_is);
    if (e != hipSuccess) return hip_fail(e, "per-vector LD kernels");
    return RR_OK;
}

// The log-likelihood and its adjoint; with per_row (per-vector LD) every
// vector uses its own profile prof_pv_d[npv][npb][nmu] and grad_prof_d is
// [npv][npb][nmu].
static int loglik_impl(const rr_tables* t, const double* times_d,
                       const int32_t* lcids_d, int32_t npt,
                       const int32_t* pbids, const int32_t* nss,
                       const double* exptimes, int32_t nlc,
                       const double* pv_d, int32_t npv, int32_t npar,
                       int32_t precision, const void* obs_d, double sigma,
                       const double* wprof_d, double* logl_d, double* grad_d,
                       double* grad_prof_d, bool per_row, const double* prof_pv_d,
                       hipStream_t stream, double k_small = -1.0,
                       double* grad_istar_d = nullptr) {
    LcInfo lc;
    int rc = check_eval_args(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc,
                             pv_d, npv, npar, precision, &lc);
    if (rc) return rc;
    if (!(sigma > 0.0) || !isfinite(sigma)) return einval("sigma must be finite and > 0");
    if (npt > 0 && npv > 0 && !obs_d) return einval("obs is NULL");
    if (npv > 0 && !logl_d && !grad_d && !grad_prof_d && !grad_istar_d)
        return einval("no output requested");
    if (adjoint_lds_bytes(precision, t->npb, t->grid.ng, grad_prof_d || grad_istar_d) +
            kAdjStaticLds > t->lds_max)
        return elimit("npb * ng adjoint LDS tables exceed the device's LDS per workgroup");
    rc = check_device(t);
    if (rc) return rc;
    hipError_t e;
    const int64_t nr = int64_t(npv) * t->npb;
    if (per_row && nr * std::max<int64_t>(t->nz, (t->grid.ng + kBlock - 1) / kBlock) >=
                       (int64_t(1) << 31))
        return elimit("npv * npb * nz must stay below 2^31");
    if (npv == 0) {
        if (grad_prof_d && !per_row) {
            e = launch_fill(grad_prof_d, int64_t(t->npb) * t->nmu, stream);
            if (e != hipSuccess) return hip_fail(e, "fill");
        }
        if (grad_istar_d) {
            e = launch_fill(grad_istar_d, t->npb, stream);
            if (e != hipSuccess) return hip_fail(e, "fill");
        }
        return RR_OK;
    }
    const bool prof = grad_prof_d != nullptr || grad_istar_d != nullptr;
    const int32_t tile = adj_tile(prof, precision == RR_FP64);
    const int32_t ntiles = npt > 0 ? (npt + tile - 1) / tile : 1;
    const int32_t nq = 7 + t->npb;
    const GridDev g = grid_dev(t);
    // With the profile gradient each workgroup runs tpp consecutive tiles of
    // one vector: enough workgroups to fill the chip (~16384), at most 256
    // MiB of per-workgroup profile partials.  Without it, one tile each.
    int64_t nseg = ntiles;
    int32_t tpp = 1;
    if (prof) {
        const size_t row_bytes = sizeof(double) * size_t(t->npb) * (size_t(g.ng) + 1);
        int64_t want = std::min<int64_t>(ntiles, (16384 + npv - 1) / npv);
        want = std::min<int64_t>(want, std::max<int64_t>(
                                           1, int64_t((size_t(256) << 20) / (row_bytes * npv))));
        tpp = int32_t((ntiles + want - 1) / std::max<int64_t>(1, want));
        nseg = (ntiles + tpp - 1) / tpp;
    }
    // one stream-ordered allocation for every temporary
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    const size_t o_pvc = take(sizeof(PvConst) * size_t(npv));
    const size_t o_part = take(sizeof(double) * size_t(npv) * nseg * nq);
    const size_t o_gldw = prof ? take(sizeof(double) * size_t(npv) * t->npb * g.ng) : 0;
    const size_t o_gist = prof ? take(sizeof(double) * size_t(npv) * t->npb) : 0;
    // shared-profile chain (table gradient) or per-vector LD temporaries
    const bool shared_prof = prof && !per_row;
    const size_t elt = precision == RR_FP64 ? sizeof(double) : sizeof(float);
    const size_t o_ldp = per_row ? take(sizeof(double) * size_t(nr) * t->nz) : 0;
    const size_t o_isr = per_row ? take(sizeof(double) * size_t(nr)) : 0;
    // small-planet rows (k_small >= 0): own row pairs and 1/I_star per row
    const bool sp = k_small >= 0.0;
    if (sp && nr >= (int64_t(1) << 31)) return elimit("npv * npb too large");
    const bool own_rows = per_row || sp;
    const size_t o_iisr = own_rows ? take(sizeof(double) * size_t(nr)) : 0;
    const size_t o_ikr = per_row ? take(sizeof(int32_t) * size_t(nr)) : 0;
    const size_t o_perm = per_row ? take(sizeof(int32_t) * size_t(nr)) : 0;
    const size_t o_rows = own_rows ? take(elt * size_t(nr) * 2 * g.ng) : 0;
    const size_t o_gldpr = per_row && prof ? take(sizeof(double) * size_t(nr) * t->nz) : 0;
    const size_t o_gt = shared_prof ? take(sizeof(double) * size_t(t->npb) * g.nk * g.ng) : 0;
    const size_t o_gldp = shared_prof ? take(sizeof(double) * size_t(t->npb) * t->nz) : 0;
    const size_t o_ldpp = shared_prof ? take(sizeof(double) * size_t(t->npb) * t->nz * 16) : 0;
    const size_t o_kidx = shared_prof ? take(sizeof(int32_t) * size_t(npv) * t->npb) : 0;
    const size_t o_kfrac = shared_prof ? take(sizeof(double) * size_t(npv) * t->npb) : 0;
    const size_t o_gist_sum = shared_prof ? take(sizeof(double) * size_t(t->npb)) : 0;
    // table-gradient row chunks: up to 32 rows each, at most 64 chunks and
    // 256 MiB of partial tables
    const size_t table_bytes = sizeof(double) * size_t(t->npb) * g.nk * g.ng;
    int32_t nchunks = std::max<int32_t>(1, std::min<int32_t>(64, (npv + 31) / 32));
    nchunks = int32_t(std::max<size_t>(1, std::min<size_t>(size_t(nchunks),
                                                           (size_t(256) << 20) / table_bytes)));
    const size_t o_gtp = shared_prof ? take(table_bytes * nchunks) : 0;
    const size_t o_gtf = shared_prof ? take(sizeof(int32_t) * size_t(nchunks) * t->npb * g.nk) : 0;
    const size_t o_gtr = shared_prof ? take(sizeof(int32_t) * size_t(t->npb) * g.nk) : 0;
    const bool segs = prof && nseg > 1;
    const size_t o_sgw = segs ? take(sizeof(double) * size_t(npv) * nseg * t->npb * g.ng) : 0;
    const size_t o_sgi = segs ? take(sizeof(double) * size_t(npv) * nseg * t->npb) : 0;
    const size_t o_sfl = segs ? take(sizeof(int32_t) * size_t(npv) * nseg) : 0;
    char* base = nullptr;
    e = hipMallocAsync((void**)&base, off, stream);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? RR_ENOMEM : hip_fail(e, "hipMallocAsync");
    AdjointArgs A;
    A.times = times_d; A.lcids = lcids_d; A.npt = npt; A.lc = &lc; A.pv = pv_d;
    A.npv = npv; A.npar = npar; A.pvc = reinterpret_cast<PvConst*>(base + o_pvc); A.g = g;
    A.T = precision == RR_FP64 ? static_cast<const void*>(t->T64) : static_cast<const void*>(t->T32);
    A.inv_istar = t->inv_istar; A.obs = obs_d; A.inv_sig2 = 1.0 / (sigma * sigma);
    A.rows_per_vector = own_rows ? 1 : 0;
    if (own_rows) {
        A.T = base + o_rows;
        A.inv_istar = reinterpret_cast<double*>(base + o_iisr);
    }
    A.ntiles = ntiles; A.want_grad = grad_d != nullptr; A.want_prof = prof; A.wprof = wprof_d;
    A.partials = reinterpret_cast<double*>(base + o_part);
    A.gldw_pv = prof ? reinterpret_cast<double*>(base + o_gldw) : nullptr;
    A.gist_pv = prof ? reinterpret_cast<double*>(base + o_gist) : nullptr;
    A.nparts = int32_t(nseg);
    A.tpp = tpp;
    A.seg_gw = segs ? reinterpret_cast<double*>(base + o_sgw) : nullptr;
    A.seg_gi = segs ? reinterpret_cast<double*>(base + o_sgi) : nullptr;
    A.seg_flag = segs ? reinterpret_cast<int32_t*>(base + o_sfl) : nullptr;
    A.logl = logl_d; A.grad = grad_d;
    e = sp ? launch_pv_setup_k(pv_d, npv, npar, t->grid.k0, t->grid.k1,
                               const_cast<PvConst*>(A.pvc), precision, stream, k_small)
           : launch_pv_setup(t, pv_d, npv, npar, const_cast<PvConst*>(A.pvc), precision,
                             stream);
    if (e == hipSuccess && sp)
        e = launch_small_planet_adj_rows(t, pv_d, npv, npar, k_small, precision, base + o_rows,
                                         reinterpret_cast<double*>(base + o_iisr), stream);
    if (e == hipSuccess && per_row)
        e = launch_pv_ld(t, prof_pv_d, pv_d, npv, npar, precision,
                         reinterpret_cast<double*>(base + o_ldp),
                         reinterpret_cast<double*>(base + o_isr),
                         reinterpret_cast<double*>(base + o_iisr),
                         reinterpret_cast<int32_t*>(base + o_ikr),
                         reinterpret_cast<int32_t*>(base + o_perm), base + o_rows, stream,
                         precision == RR_MIXED);     // the rows rr_evaluate_ld evaluates
    if (e == hipSuccess) e = launch_adjoint(A, precision, stream);
    if (e == hipSuccess && prof && per_row)
        e = launch_pv_prof_grad(t, A, reinterpret_cast<const int32_t*>(base + o_ikr),
                                reinterpret_cast<const int32_t*>(base + o_perm),
                                reinterpret_cast<double*>(base + o_gldpr), grad_prof_d, stream,
                                precision == RR_MIXED);
    if (e == hipSuccess && shared_prof) {
        ProfGradScratch w;
        w.kidx = reinterpret_cast<int32_t*>(base + o_kidx);
        w.kfrac = reinterpret_cast<double*>(base + o_kfrac);
        w.nchunks = nchunks;
        w.gt_part = reinterpret_cast<double*>(base + o_gtp);
        w.gt_flags = reinterpret_cast<int32_t*>(base + o_gtf);
        w.gt_rowflag = reinterpret_cast<int32_t*>(base + o_gtr);
        w.GT = reinterpret_cast<double*>(base + o_gt);
        w.ldp_part = reinterpret_cast<double*>(base + o_ldpp);
        w.gldp = reinterpret_cast<double*>(base + o_gldp);
        w.gist = reinterpret_cast<double*>(base + o_gist_sum);
        w.istar_fixed = t->istar_fixed ? 1 : 0;
        w.grad_istar = grad_istar_d;
        e = launch_profile_grad(t, A, w, grad_prof_d, stream);
    }
    hipError_t ef = hipFreeAsync(base, stream);
    if (e != hipSuccess) return hip_fail(e, "log-likelihood kernels");
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync");
    return RR_OK;
}

RR_API int rr_loglik_grad(const rr_tables* t, const double* times_d,
                          const int32_t* lcids_d, int32_t npt,
                          const int32_t* pbids, const int32_t* nss,
                          const double* exptimes, int32_t nlc,
                          const double* pv_d, int32_t npv, int32_t npar,
                          int32_t precision, const void* obs_d, double sigma,
                          const double* wprof_d, double* logl_d, double* grad_d,
                          double* grad_prof_d, hipStream_t stream) {
    return loglik_impl(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc, pv_d, npv, npar,
                       precision, obs_d, sigma, wprof_d, logl_d, grad_d, grad_prof_d, false,
                       nullptr, stream);
}

RR_API int rr_loglik_grad_istar(const rr_tables* t, const double* times_d,
                                const int32_t* lcids_d, int32_t npt,
                                const int32_t* pbids, const int32_t* nss,
                                const double* exptimes, int32_t nlc,
                                const double* pv_d, int32_t npv, int32_t npar,
                                int32_t precision, const void* obs_d, double sigma,
                                const double* wprof_d, double* logl_d, double* grad_d,
                                double* grad_prof_d, double* grad_istar_d,
                                hipStream_t stream) {
    return loglik_impl(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc, pv_d, npv, npar,
                       precision, obs_d, sigma, wprof_d, logl_d, grad_d, grad_prof_d, false,
                       nullptr, stream, -1.0, grad_istar_d);
}

RR_API int rr_loglik_grad_ld(const rr_tables* t, const double* times_d,
                             const int32_t* lcids_d, int32_t npt,
                             const int32_t* pbids, const int32_t* nss,
                             const double* exptimes, int32_t nlc,
                             const double* pv_d, int32_t npv, int32_t npar,
                             const double* prof_d, int32_t precision, const void* obs_d,
                             double sigma, double* logl_d, double* grad_d,
                             double* grad_prof_d, hipStream_t stream) {
    if (npv > 0 && !prof_d) return einval("prof is NULL");
    return loglik_impl(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc, pv_d, npv, npar,
                       precision, obs_d, sigma, nullptr, logl_d, grad_d, grad_prof_d, true,
                       prof_d, stream);
}

RR_API int rr_loglik_grad_small_planet(const rr_tables* t, const double* times_d,
                                       const int32_t* lcids_d, int32_t npt,
                                       const int32_t* pbids, const int32_t* nss,
                                       const double* exptimes, int32_t nlc,
                                       const double* pv_d, int32_t npv, int32_t npar,
                                       double k_small, int32_t precision, const void* obs_d,
                                       double sigma, double* logl_d, double* grad_d,
                                       hipStream_t stream) {
    if (!(k_small >= 0.0 && k_small <= 1.0)) return einval("k_small must lie in [0, 1]");
    return loglik_impl(t, times_d, lcids_d, npt, pbids, nss, exptimes, nlc, pv_d, npv, npar,
                       precision, obs_d, sigma, nullptr, logl_d, grad_d, nullptr, false,
                       nullptr, stream, k_small);
}

RR_API void rr_free_tables(rr_tables* t) { free_tables(t); }

RR_API int rr_set_kernel_events(hipEvent_t before, hipEvent_t after) {
    if ((before == nullptr) != (after == nullptr))
        return einval("rr_set_kernel_events needs both events or neither");
    kernel_events().before = before;
    kernel_events().after = after;
    return RR_OK;
}

RR_API int rr_tables_copy(const rr_tables* t, int32_t which, void* host_dst,
                          int64_t capacity, int64_t* count) {
    if (!t) return einval("tables handle is NULL");
    const int64_t nz = t->nz, ng = t->grid.ng, nk = t->grid.nk, npb = t->npb;
    const void* src = nullptr;
    int64_t n = 0;
    size_t elt = sizeof(double);
    switch (which) {
        case 0: src = t->ze; n = nz + 1; break;
        case 1: src = t->W; n = nk * nz * ng; break;
        case 2: src = t->ldp; n = npb * nz; break;
        case 3: src = t->istar; n = npb; break;
        case 4: src = t->T64; n = npb * nk * ng; break;
        case 5: src = t->T32; n = npb * nk * ng; elt = sizeof(float); break;
        case 6: src = t->zm; n = nz; break;
        default: return einval("unknown table id");
    }
    if (count) *count = n;
    if (!host_dst) return RR_OK;
    if (capacity < n) return einval("capacity smaller than the table");
    int rc = check_device(t);
    if (rc) return rc;
    hipError_t e = hipMemcpy(host_dst, src, elt * size_t(n), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy table to host");
    return RR_OK;
}

RR_API int rr_tables_info(const rr_tables* t, rr_grid* grid, int32_t* sizes) {
    if (!t) return einval("tables handle is NULL");
    if (grid) *grid = t->grid;
    if (sizes) {
        sizes[0] = t->nz;
        sizes[1] = t->grid.ng;
        sizes[2] = t->grid.nk;
        sizes[3] = t->npb;
        sizes[4] = t->nmu;
        sizes[5] = t->grid.nzin;
    }
    return RR_OK;
}

}  // extern "C"
