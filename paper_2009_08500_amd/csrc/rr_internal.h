// rr_internal.h -- structures shared by the translation units of librr.so.
//
// Not part of the public ABI.  Device-side layouts are plain structs of
// FP64/int32 so that host code can fill and launch them.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "rr.h"
#include "rr_host.h"

namespace rr {

#ifndef RR_TIMES_PER_THREAD
#define RR_TIMES_PER_THREAD 8
#endif
constexpr int kBlock = 256;          // threads per workgroup of the table,
                                     // setup and reduction kernels (4 wave64)
constexpr int kTimesPerThread = RR_TIMES_PER_THREAD;   // times per thread
// Forward kernels: one wave64 per workgroup (measured faster than 2 or 4:
// a finished wave frees its slot at once), each owning kFwdTile times.
constexpr int kFwdBlock = 64;
constexpr int kFwdTile = kFwdBlock * kTimesPerThread;
constexpr int kSplitRows = 4;       // rows per streaming workgroup of the split launch
// Log-likelihood kernel: two wave64 per workgroup share the LDS tables.
// Times per thread: 16, except 8 with the LD-profile gradient in mixed
// precision (measured fastest for each).
constexpr int kAdjBlock = 128;
constexpr int adj_times_per_thread(bool prof, bool f64) { return prof && !f64 ? 8 : 16; }
constexpr int adj_tile(bool prof, bool f64) { return kAdjBlock * adj_times_per_thread(prof, f64); }
constexpr int kMinLdsBytes = 64 * 1024;   // LDS a workgroup may use on any
                                          // device (the budget used if the
                                          // device does not report its own)

// Per-parameter-vector orbit constants, computed once per call (FP64).
struct PvConst {
    double t0, P, invP, n;        // n = 2 pi / P (mean motion)
    double a, e, cosw, sinw;
    double sE, cE, q, rtr;        // sin/cos of E at conjunction, sqrt(1-e^2),
                                  // star-planet distance at conjunction
    double cosi, flo, wn, kmax;   // transit window in phase units: inside iff
                                  // frac((t - t0)/P - flo) < wn
    int32_t flags;                // kValid | kAlways
    int32_t pad[3];
};
constexpr int32_t kValid = 1;     // physical and inside the table's k range
constexpr int32_t kAlways = 2;    // no usable transit window: evaluate every
                                  // subsample in full

// Per-light-curve description, passed by value to the kernels.
struct LcInfo {
    int32_t nlc;
    int32_t pb[RR_MAX_LC];
    int32_t nss[RR_MAX_LC];
    double exptime[RR_MAX_LC];
};

// One forward job: rows [pv0, pv0 + npv) of a population over one time
// series, workgroups [block0, block0 + npv * ntiles) of a launch.  pv, pvc
// and out are indexed by the population row; out is [rows][npt].
struct FwdJob {
    const double* times;
    const int32_t* lcids;
    const LcInfo* lc;          // device copy (serving); unused by rr_evaluate
    const double* pv;
    const PvConst* pvc;
    void* out;
    int32_t npt, npar, pv0, npv, ntiles, block0;
    int32_t max_nss;           // largest nss of the job's light curves
    // per-vector LD (rr_evaluate_ld), NULL with the shared tables: the
    // vector's own two table rows around its k, [npv][npb][2][ng] in the
    // evaluation precision, and 1/I_star [npv][npb]
    const void* ldw_pv;
    const double* inv_istar_pv;   // NULL: the tables' 1/I_star
    int32_t ldw_exact_k;          // 1: ldw_pv rows are for the row's exact k (direct model)
    int32_t spread;               // 1: supersampled exposures may spread over lanes
};
// Forward-kernel variants (rr_evaluate_variant): exposures per lane
// J = 4, 8, 16 for v = 0, 1, 2 with subsamples spread over lanes where
// possible, the same J with one lane per exposure for v = 3, 4, 5.
constexpr int kNumFwdVariants = 6;
static_assert(kTimesPerThread == 4 || kTimesPerThread == 8 || kTimesPerThread == 16,
              "the default forward variant has J = kTimesPerThread");
constexpr int kDefaultFwdVariant =        // rr_evaluate: J = kTimesPerThread, spreading
    kTimesPerThread == 4 ? 0 : (kTimesPerThread == 8 ? 1 : 2);
constexpr int kMaxJobs = 24;   // jobs per grouped launch (kernel arguments)
struct JobTable {
    int32_t njobs;
    FwdJob j[kMaxJobs];
};
struct SetupJob {
    const double* pv;
    PvConst* pvc;
    int32_t npv, npar, thread0, f32;   // f32: the mixed precision's setup
};
struct SetupTable {
    int32_t njobs;
    SetupJob j[kMaxJobs];
};

// SeriesLc (one light curve's run and time index) is in rr_host.h.
// What the split forward launch (rr_evaluate_series) needs beyond a FwdJob:
// the light curves' runs and index, and `shares` transit workgroups per
// parameter vector (the first npv * shares workgroups of the launch).
struct SplitInfo {
    const SeriesLc* lcs;       // [nlc], device
    const int32_t* buckets;    // device
    int32_t shares;
    int32_t rows_per;          // rows per streaming workgroup
    double k_lo, k_hi;         // accepted k range of the rows (the tables')
};

// Scalars of the table grid needed on the device.
struct GridDev {
    int32_t nz, ng, nk, npb;
    double k0, dk, inv_dk;        // k_i = k0 + i dk
    double gscale;                // ng - 1: grazing value -> node coordinate
};

// Arguments of the adjoint launch (rr_adjoint.hip).
struct AdjointArgs {
    const double* times;
    const int32_t* lcids;
    int32_t npt;
    const LcInfo* lc;
    const double* pv;
    int32_t npv, npar;
    const PvConst* pvc;
    GridDev g;
    const void* T;            // T64 or T32 by precision
    const double* inv_istar;
    const void* obs;          // double (RR_FP64) or float (RR_MIXED)
    double inv_sig2;
    int32_t ntiles, want_grad, want_prof;
    const double* wprof;      // per-vector weights of the profile gradient
    double* partials;         // [npv * nparts][7 + npb]
    double* gldw_pv;          // [npv][npb][ng]
    double* gist_pv;          // [npv][npb]
    int32_t rows_per_vector;  // 1: T holds each vector's own two rows [npv][npb][2][ng]
                              // and inv_istar is [npv][npb] (per-vector LD)
    int32_t nparts;           // workgroups per vector (ntiles without the profile gradient)
    int32_t tpp;              // tiles per workgroup
    double* seg_gw;           // [npv][nparts][npb][ng] (nparts > 1)
    double* seg_gi;           // [npv][nparts][npb]
    int32_t* seg_flag;        // [npv][nparts]
    double* logl;             // [npv] or null
    double* grad;             // [npv][npar] or null
};

}  // namespace rr

// Library-owned table handle (opaque in the ABI).
// A registered time series (rr_series_create).
struct rr_series {
    int device = -1;
    int32_t npt = 0, nlc = 0, max_nss = 1;
    rr::LcInfo lc;
    std::vector<int32_t> pbids, nss;   // host copies, [nlc]
    std::vector<double> exptimes;
    bool indexed = false;          // every light curve one sorted run: split launch
    double* times = nullptr;       // [npt] device
    int32_t* lcids = nullptr;      // [npt] device, or null for one light curve
    rr::SeriesLc* lcs = nullptr;   // [nlc] device (indexed only)
    int32_t* buckets = nullptr;    // device (indexed only)
};

struct rr_tables {
    rr_grid grid;
    int32_t nz, npb, nmu;
    int device;
    size_t lds_max = 0;          // LDS one workgroup may allocate on `device`
    double dk;
    // device buffers
    double* mu_s = nullptr;      // [nmu]
    double* prof = nullptr;      // [npb][nmu]
    double* ze = nullptr;        // [nz+1]
    double* zm = nullptr;        // [nz]
    double* ldp = nullptr;       // [npb][nz]
    double* istar = nullptr;     // [npb]
    double* W = nullptr;         // [nk][nz][ng]
    float* W32 = nullptr;        // [nk][nz][ng], FP32 copy (mixed per-vector tables)
    double* T64 = nullptr;       // [npb][nk][ng]
    float* T32 = nullptr;        // [npb][nk][ng]
    double* inv_istar = nullptr; // [npb]
    // rr_set_istar: normalisers given by the caller, [npb] device, used in
    // place of the profile interpolant's integral while istar_fixed
    double* istar_user = nullptr;
    bool istar_fixed = false;
    // Per-stream temporaries of rr_evaluate (grow-only; work on one stream is
    // ordered, so a stream's buffer is reused without waiting).
    std::mutex ws_mu;
    std::unordered_map<hipStream_t, std::pair<void*, size_t>> ws;

};

namespace rr {

void set_error(const std::string& msg);
// Events bracketing the next main-kernel launch of this thread (or null).
struct KernelEvents { hipEvent_t before = nullptr, after = nullptr; };
KernelEvents& kernel_events();

// Launches `kernel`; if st or sp is set they become the launch's own start
// and stop events (recorded at the kernel's execution, not around the
// launch call).
template <typename K, typename... Args>
inline void launch_timed(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                         hipEvent_t st, hipEvent_t sp, Args... args) {
    if (st || sp)
        hipExtLaunchKernelGGL(kernel, grid, block, uint32_t(lds), s, st, sp, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}
int hip_fail(hipError_t err, const char* what);
// Device workspace of at least `bytes` for `stream`, owned by the tables.
hipError_t stream_workspace(rr_tables* t, hipStream_t stream, size_t bytes, void** out);
rr::GridDev grid_dev(const rr_tables* t);

// Kernel launchers (rr_prep.hip, rr_forward.hip).
hipError_t launch_prepare_grid_weights(rr_tables* t, hipStream_t s);
hipError_t launch_prepare_profile(rr_tables* t, hipStream_t s);
// Per-row constants for the forward paths of `precision`; k must lie in
// [k_lo, k_hi] (the tables' k range by default; the direct model takes
// (0, 1]), or in (0, k_small) for small-planet rows.
hipError_t launch_pv_setup(const rr_tables* t, const double* pv, int32_t npv,
                           int32_t npar, PvConst* pvc, int32_t precision, hipStream_t s);
hipError_t launch_pv_setup_k(const double* pv, int32_t npv, int32_t npar, double k_lo,
                             double k_hi, PvConst* pvc, int32_t precision, hipStream_t s,
                             double k_small = 0.0);
// Dynamic LDS of one log-likelihood workgroup: the k-interpolated LD
// vectors and their k-derivatives, plus (prof) each wave's copy of
// d logL / d ldw and d logL / d I_star.
size_t adjoint_lds_bytes(int32_t precision, int32_t npb, int32_t ng, bool prof);
// What the log-likelihood kernel declares in LDS statically (an upper
// bound): the dynamic part must fit in lds_max less this.
constexpr size_t kAdjStaticLds = 512;
hipError_t launch_adjoint(const AdjointArgs& a, int32_t precision, hipStream_t s);
// Temporaries of the profile gradient.
struct ProfGradScratch {
    int32_t* kidx;        // [npv][npb]
    double* kfrac;        // [npv][npb]
    int32_t nchunks;      // row chunks of the table gradient
    double* gt_part;      // [nchunks][npb][nk][ng]
    int32_t* gt_flags;    // [nchunks][npb][nk]
    int32_t* gt_rowflag;  // [npb][nk]: k-row touched by any chunk
    double* GT;           // [npb][nk][ng]
    double* ldp_part;     // [npb][nz][16]
    double* gldp;         // [npb][nz]
    double* gist;         // [npb]
    int32_t istar_fixed;  // 1: I_star does not depend on the samples (rr_set_istar)
    double* grad_istar;   // [npb] output (d logL / d I_star) or null
};
// Per-vector LD: d logL / d prof[ipv][pb][s] from the adjoint's per-vector
// d logL / d ldw and d logL / d I_star; ikr and perm are launch_pv_ld's sort
// of the rows by k-row, gldp is [npv][npb][nz] scratch.
// w32: the weights are the FP32 copy (the mixed per-vector rows' own).
hipError_t launch_pv_prof_grad(const rr_tables* t, const AdjointArgs& A, const int32_t* ikr,
                               const int32_t* perm, double* gldp, double* out, hipStream_t s,
                               bool w32);
hipError_t launch_profile_grad(const rr_tables* t, const AdjointArgs& a,
                               const ProfGradScratch& w, double* out, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, hipStream_t s);
// I_star and 1/I_star from the caller's normalisers (rr_set_istar): copy
// src[npb] into the tables' istar and istar_user (when given) and set
// inv_istar; a value that is not finite and positive gives NaN fluxes.
hipError_t launch_istar_set(rr_tables* t, const double* src, hipStream_t s);
// I_star from the profile samples (the interpolant's exact integral).
hipError_t launch_istar_from_profile(rr_tables* t, hipStream_t s);
// Whether rr_evaluate_series takes the split launch for this size: series
// with one subsample per exposure, except two time tiles or fewer under
// more than 1024 rows (measured, both precisions); the per-tile kernel
// otherwise.
bool split_preferred(const rr_tables* t, const rr_series* se, int32_t npv, int32_t precision);
// Shape of a split launch over a registered, indexed series: transit
// workgroups per row, rows per streaming workgroup, the grid size, and
// whether the workgroups derive their rows' constants themselves (then no
// per-row setup precedes the launch).
struct SplitPlan {
    int32_t shares = 1, rows_per = 1;
    int64_t blocks = 0;
    bool self_setup = false;
};
SplitPlan plan_forward_split(const rr_series* se, int32_t npv, int32_t precision);
// The split launch (rr_evaluate_series); pvc (the per-row setup's output)
// is read unless sp.self_setup.
hipError_t launch_forward_split(const rr_tables* t, const rr_series* se, const SplitPlan& sp,
                                const double* pv, int32_t npv, int32_t npar,
                                const PvConst* pvc, int32_t precision, void* out,
                                hipStream_t s);
hipError_t launch_forward_jobs(const rr_tables* t, const JobTable& jt,
                               int32_t nblocks_total, int32_t precision, hipStream_t s);
hipError_t launch_pv_setup_jobs(const rr_tables* t, const SetupTable& st,
                                int32_t nthreads, hipStream_t s);
hipError_t launch_forward(const rr_tables* t, const double* times,
                          const int32_t* lcids, int32_t npt, const LcInfo& lc,
                          const double* pv, int32_t npv, int32_t npar,
                          const PvConst* pvc, int32_t precision, void* out,
                          hipStream_t s, const void* ldw_pv = nullptr,
                          const double* inv_istar_pv = nullptr, int32_t ldw_exact_k = 0,
                          int32_t variant = kDefaultFwdVariant);
// Direct model (rr_evaluate_direct): each (vector, passband) row's
// LD-weighted vector for its own k, rows [npv][npb][2][ng] by precision.
hipError_t launch_direct_rows(const rr_tables* t, const double* pv, int32_t npv, int32_t npar,
                              int32_t precision, void* rows, hipStream_t s);
// Small-planet approximation (rr_evaluate_small_planet): rows
// [npv][npb][2][ng] by precision; a row whose k is below k_small holds the
// profile at the planet's centre for each g node, any other the tables' two
// k-rows already interpolated at its k (read with zero k-weight).
hipError_t launch_small_planet_rows(const rr_tables* t, const double* pv, int32_t npv,
                                    int32_t npar, double k_small, int32_t precision,
                                    void* rows, hipStream_t s);
// The same for the log-likelihood's adjoint: row pairs whose k-lerp gives
// the centre values and whose difference over dk their k-derivative, and
// 1/I_star per row ([npv][npb]).
hipError_t launch_small_planet_adj_rows(const rr_tables* t, const double* pv, int32_t npv,
                                        int32_t npar, double k_small, int32_t precision,
                                        void* rows, double* inv_istar_rows, hipStream_t s);
// Eq. 5 at separations z[n] (rr_flux_at_z); kv[n] or, if NULL, kconst.
hipError_t launch_flux_at_z(const rr_tables* t, const double* z, const double* kv,
                           double kconst, int64_t n, int32_t pb, int32_t precision, void* out,
                           hipStream_t s);
// Per-vector LD (rr_evaluate_ld): from prof[npv][npb][nmu] on the tables'
// mu samples, the profile at the bin means (ldp, [npv][npb][nz]), I_star and
// 1/I_star ([npv][npb]) and the vector's own two table rows around its k
// (rows, [npv][npb][2][ng], double or float by precision); ikr and perm are
// [npv npb] int32 scratch.
// w32: the per-row kernel reads the FP32 copy of W (mixed precision only).
hipError_t launch_pv_ld(const rr_tables* t, const double* prof, const double* pv,
                        int32_t npv, int32_t npar, int32_t precision, double* ldp,
                        double* istar, double* inv_istar, int32_t* ikr, int32_t* perm,
                        void* rows, hipStream_t s, bool w32 = false);

}  // namespace rr
