/*
 * rr.h -- C ABI of the MI355X RoadRunner light-curve library (librr.so).
 *
 * RoadRunner (Parviainen 2020) evaluates limb-darkened transit light curves
 * as F = (I_star - (w . l) a(z, k)) / I_star (Eq. 5): the occluded area
 * a(z, k) of the stellar disk times the mean occluded surface brightness
 * w . l, which is precomputed over a grid of radius ratios k and grazing
 * values g = z / (1 + k) and interpolated (Sect. 3.1.2).  This library runs
 * the whole path on one AMD Instinct MI355X (gfx950):
 *
 *   rr_prepare_ld   z-grid, annulus weights W over (k, g), LD profile at the
 *                   bin means, I_star, LD-weighted tables T = W . l
 *                   (Sect. 2, Sect. 3.1.1, Sect. 3.1.2, Sect. 3.2.2);
 *   rr_evaluate     fluxes for a population of parameter vectors over a
 *                   heterogeneous, supersampled time series (Sect. 4.1,
 *                   Sect. 4.2): phase -> Kepler orbit -> separation z ->
 *                   g-interpolation x lens area -> supersample mean;
 *   rr_evaluate_ld  the same with a limb-darkening profile per parameter
 *                   vector (LD sampled with the orbit);
 *   rr_evaluate_variant / rr_select_variant  one forward-kernel variant,
 *                   and the trial run that picks the fastest for given
 *                   inputs (Sect. 3.4.1);
 *   rr_evaluate_direct  the direct model: weights for each vector's own k,
 *                   no k-interpolation and no k limits (Sect. 3.1.1);
 *   rr_evaluate_small_planet  the small-planet approximation below a
 *                   radius-ratio threshold (Sect. 3.4.2), and
 *                   rr_loglik_grad_small_planet its log-likelihood and
 *                   parameter gradient;
 *   rr_flux_at_z    Eq. 5 at given separations and radius ratios;
 *   rr_loglik_grad  Gaussian log-likelihood of observed fluxes and its
 *                   gradient with respect to every parameter and to the
 *                   LD profile samples (hand-written adjoint);
 *   rr_loglik_grad_ld  the same with a profile per parameter vector and
 *                   the gradient with respect to each one;
 *   rr_server_*     a continuous-batching request loop over resident tables.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * Pointers named *_d are device pointers (memory of the current HIP device);
 * others are host pointers.  The caller owns every buffer it passes; the
 * library owns rr_tables and rr_server objects.  Calls that take a stream
 * enqueue their device work on it and return without waiting, unless stated
 * otherwise.  Return values are RR_OK (0) or a negative RR_E* code; argument
 * errors are detected on the host before anything is enqueued.
 *
 * Parameter-vector rows (npar = 6 + npb doubles, row-major [npv][npar]):
 *   [t0, P, a, b, e, w, k_0, ..., k_{npb-1}]
 * t0  time of inferior conjunction (same unit as the times, normally days)
 * P   orbital period, a  semi-major axis in stellar radii,
 * b   impact parameter at conjunction, b = a cos(i) (1 - e^2)/(1 + e sin w),
 * e   eccentricity, w  argument of periastron (radians),
 * k_pb radius ratio in passband pb (chromatic radius ratios, Sect. 4.2).
 * The planet transits at true anomaly pi/2 - w and occults only while it is
 * in front of the star.  A row with a non-finite value, P <= 0, a <= 0,
 * b < 0, e outside [0, 1), |cos i| > 1 or any k_pb outside the table's
 * [k0, k1] produces a row of NaN; other rows are unaffected.
 */
#ifndef RR_H
#define RR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RR_API __attribute__((visibility("default")))

/* Return codes. */
#define RR_OK        0
#define RR_EINVAL   -1   /* an argument is out of its documented range     */
#define RR_ENOMEM   -2   /* a device or host allocation failed             */
#define RR_EDEVICE  -3   /* a HIP call failed (message via rr_last_error)  */
#define RR_ELIMIT   -4   /* a size exceeds a compiled-in limit below       */
#define RR_EBUSY    -5   /* serving: the request does not fit right now    */
#define RR_ENOTFOUND -6  /* serving: unknown request id                    */

/* Compiled-in limits. */
#define RR_MAX_PB    16   /* passbands per table set                        */
#define RR_MAX_LC    64   /* light curves per rr_evaluate call              */
#define RR_MAX_NSS   1024 /* subsamples per exposure                        */
#define RR_NUM_VARIANTS 6 /* forward-kernel variants (rr_evaluate_variant)  */

/* Precision policies for rr_evaluate / rr_loglik_grad. */
#define RR_FP64  0  /* every step in FP64; output double                  */
#define RR_MIXED 1  /* FP64 phase reduction, FP32 orbit/area/tables,
                       output float; held to 1 ppm (absolute flux) of the
                       FP64 model by the parity tests                      */

/* Table resolution (Sect. 3.1.1, Sect. 3.1.2, Sect. 3.3).
 * zcut   radius dividing the inner region (bins of constant dz) from the
 *        limb region (bins of constant dmu), 0 < zcut < 1;
 * nzin   bins in the inner region, >= 1;  nzlimb  bins in the limb region,
 *        >= 1 (nz = nzin + nzlimb <= 4096);
 * ng     grazing-value nodes g_m = m / (ng - 1), 2 <= ng <= 4096;
 * nk     radius-ratio nodes k_i = k0 + i (k1 - k0)/(nk - 1), 2 <= nk <= 4096;
 * k0,k1  radius-ratio range, 0 < k0 < k1 < 1. */
typedef struct rr_grid {
    double  zcut;
    int32_t nzin;
    int32_t nzlimb;
    int32_t ng;
    int32_t nk;
    double  k0;
    double  k1;
} rr_grid;

typedef struct rr_tables rr_tables;   /* opaque, owned by the library */

/* Build the LD tables for npb passbands from radial profiles given as
 * samples prof[npb][nmu] at mu[nmu] (host arrays, FP64).  mu must be
 * strictly increasing within [0, 1]; the profile is read as the
 * piecewise-linear interpolant of the samples, constant beyond the first and
 * last sample (the custom-profile case of Sect. 3.2.2), and I_star is that
 * interpolant's exact disk integral (Eq. 2, Eq. 4).
 * Builds, on the device: the z-grid, the weight table
 * W[nk][nz][ng] (area of annulus j occluded by a planet of radius k_i at
 * grazing value g_m over the total occluded area, Sect. 2), the profile at
 * the bin means, I_star and the LD-weighted tables T[npb][nk][ng] in FP64
 * and FP32.  Device memory ~ 12 nk nz ng + 12 npb nk ng bytes (W in FP64
 * and an FP32 copy for the mixed per-vector tables).
 * Synchronous: returns when the tables are ready for use on any stream.
 * 2 <= nmu <= 65536, 1 <= npb <= RR_MAX_PB.  On success *out receives a new
 * handle; release it with rr_free_tables. */
RR_API int rr_prepare_ld(const double* mu, const double* prof, int32_t nmu,
                         int32_t npb, const rr_grid* grid, rr_tables** out);

/* Replace the profile samples of an existing handle (same mu grid, same
 * npb) with prof_d[npb][nmu], a device array, and rebuild I_star and T on
 * `stream` without any host synchronisation.  W is reused.  Work enqueued
 * on other streams that reads the tables must be ordered after this call by
 * the caller. */
RR_API int rr_set_profile(rr_tables* t, const double* prof_d,
                          hipStream_t stream);

/* Set the normaliser I_star of every passband to istar_d[npb] (device
 * FP64, finite and > 0; other values give NaN fluxes), in place of the
 * exact integral of the profile interpolant, or with istar_d = NULL go
 * back to that integral.  For profiles that come from a law with a known
 * disk integral, such as the named laws, which the paper normalises by
 * their analytic integral (Sect. 3.2.1), or a callable with its own
 * normalising integral (Sect. 3.2.2).  The values stay in force across
 * rr_set_profile until changed or cleared; they apply wherever the
 * tables' own profile is used (rr_evaluate, rr_evaluate_series,
 * rr_evaluate_direct, rr_evaluate_small_planet, rr_flux_at_z,
 * rr_loglik_grad*), not to the per-vector profiles of rr_evaluate_ld and
 * rr_loglik_grad_ld, which are normalised by their own integrals.  Enqueued
 * on `stream` without a host synchronisation (the first call allocates
 * 8 npb bytes); work on other streams that reads the tables must be
 * ordered after it by the caller. */
RR_API int rr_set_istar(rr_tables* t, const double* istar_d, hipStream_t stream);

/* Fluxes for npv parameter vectors at npt mid-exposure times.
 * times_d[npt]   device FP64 mid-exposure times;
 * lcids_d[npt]   device int32 light-curve index of each time, each in
 *                [0, nlc) (values outside give NaN), or NULL for one light
 *                curve (then nlc must be 1);
 * pbids[nlc]     host int32 passband of each light curve, in [0, npb);
 * nss[nlc]       host int32 subsamples per exposure, 1..RR_MAX_NSS;
 * exptimes[nlc]  host FP64 exposure time of each light curve, >= 0;
 *                subsample s of an exposure at t is evaluated at
 *                t + exptime ((s + 1/2)/nss - 1/2) and the exposure flux is
 *                the mean over its subsamples (Sect. 4.1);
 * pv_d[npv][npar] device FP64 parameter rows (layout above),
 *                npar == 6 + npb of the tables;
 * precision      RR_FP64 (out_d is double[npv][npt]) or RR_MIXED
 *                (out_d is float[npv][npt]);
 * out_d          device output, row-major, times contiguous.
 * npt >= 0, npv >= 0 (zero sizes enqueue nothing), 1 <= nlc <= RR_MAX_LC.
 * Temporary device memory (144 bytes per parameter vector) is a per-stream
 * buffer kept by the tables handle: it grows (with a synchronising
 * reallocation) when a call needs more, is reused without waiting by later
 * calls on the same stream, and is freed by rr_free_tables. */
RR_API int rr_evaluate(const rr_tables* t, const double* times_d,
                       const int32_t* lcids_d, int32_t npt,
                       const int32_t* pbids, const int32_t* nss,
                       const double* exptimes, int32_t nlc,
                       const double* pv_d, int32_t npv, int32_t npar,
                       int32_t precision, void* out_d, hipStream_t stream);

/* A registered time series (the model's data set-up of Sect. 4.1 and
 * Sect. 4.2: mid-exposure times, light-curve ids, and per light curve the
 * passband, supersampling factor and exposure time), kept on the device
 * with an index that maps a time to the exposures around it, so that
 * rr_evaluate_series can hand each transit to its own workgroups.
 * Arguments as rr_evaluate's, but times[npt] and lcids[npt] (or NULL for
 * one light curve) are HOST arrays; ids outside [0, nlc) are allowed and
 * give NaN, as in rr_evaluate.  The index is used when every light curve's
 * exposures form one contiguous run of the arrays with finite,
 * non-decreasing times; otherwise the series is still valid and
 * rr_evaluate_series evaluates it as rr_evaluate does.  Device memory:
 * 12 npt bytes plus 4 per exposure of the index and 40 per light curve.
 * Synchronous; the series lives on the current device.  npt >= 0. */
typedef struct rr_series rr_series;   /* opaque, owned by the library */
RR_API int rr_series_create(const double* times, const int32_t* lcids, int32_t npt,
                            const int32_t* pbids, const int32_t* nss,
                            const double* exptimes, int32_t nlc, rr_series** out);

/* Release a series; no enqueued work may still read it.  NULL is ignored. */
RR_API void rr_series_free(rr_series* s);

/* Fluxes of npv parameter vectors over a registered series: the values of
 * rr_evaluate on the same times, computed with the same arithmetic per
 * exposure (the two kernels may round a multiply-add differently: within a
 * float ulp of the flux in RR_MIXED, a double ulp in RR_FP64).  With the
 * index and one subsample per exposure, one launch gives every parameter
 * vector up to 16 workgroups that evaluate only its transits -- each finds
 * a transit's exposures through the index, and they start first -- while
 * the other workgroups stream F = 1 over every other exposure; series
 * without the index, supersampled series and the shortest series under
 * more than 1024 vectors (two time tiles of 512 exposures or fewer) take
 * rr_evaluate's per-tile kernel.  pv_d, npv, npar, precision, out_d,
 * stream, errors and temporary memory as rr_evaluate; the series must live
 * on the tables' device. */
RR_API int rr_evaluate_series(const rr_tables* t, const rr_series* s, const double* pv_d,
                              int32_t npv, int32_t npar, int32_t precision, void* out_d,
                              hipStream_t stream);

/* Which forward kernel rr_evaluate_series launches for npv parameter
 * vectors in `precision` over this series: *kind = RR_KERNEL_TILES (0:
 * rr_evaluate's per-tile kernel, after the per-vector setup),
 * RR_KERNEL_SPLIT (1: the split launch of transit and streaming
 * workgroups, after the per-vector setup) or RR_KERNEL_SPLIT_FUSED (2: the
 * split launch alone, its workgroups deriving their vectors' constants
 * themselves; taken while the launch has at most twice as many workgroups
 * as the float kernel keeps resident, where it measured faster, so such a
 * call is one launch).  The two split launches give the same bits; the
 * per-tile kernel agrees with them within a rounding of the flux (see
 * rr_evaluate_series).  For benchmarks and profiles that name the kernel
 * they time.  Enqueues nothing (the choice may query the device's
 * occupancy once); errors as rr_evaluate_series's checks. */
#define RR_KERNEL_TILES 0
#define RR_KERNEL_SPLIT 1
#define RR_KERNEL_SPLIT_FUSED 2
RR_API int rr_series_kernel(const rr_tables* t, const rr_series* s, int32_t npv,
                            int32_t precision, int32_t* kind);

/* rr_evaluate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, and harnesses that forbid
 * hipMalloc.  Same arguments, kernels, results and argument errors as
 * rr_evaluate; the only difference is where the per-parameter-vector orbit
 * constants (144 bytes per row) live: instead of the tables' per-stream
 * workspace, a fixed device array of RR_NOALLOC_MAX_PV rows (2.25 MiB) that
 * the library holds on each GPU from the first rr_prepare_ld on it until
 * the process ends.  Nothing is allocated or freed by this call.
 * npv > RR_NOALLOC_MAX_PV returns RR_ELIMIT and enqueues nothing.
 * Every call on one GPU uses the same array, which keeps the last call's
 * contents (each call's setup kernel rewrites the rows it reads, so nothing
 * needs clearing).  Calls that overlap on one GPU -- on different streams or
 * threads, before an earlier call's kernels have finished -- race on the
 * array and can produce wrong fluxes: issue them on one stream, or order
 * them with events. */
#define RR_NOALLOC_MAX_PV 16384
RR_API int rr_evaluate_noalloc(const rr_tables* t, const double* times_d,
                               const int32_t* lcids_d, int32_t npt,
                               const int32_t* pbids, const int32_t* nss,
                               const double* exptimes, int32_t nlc,
                               const double* pv_d, int32_t npv, int32_t npar,
                               int32_t precision, void* out_d, hipStream_t stream);

/* rr_evaluate with a chosen forward-kernel variant.  The variants differ
 * only in how work maps onto the GPU, never in the arithmetic of an
 * exposure, so every variant writes the values of rr_evaluate (bit for bit
 * without supersampling; for supersampled series the compiler may contract
 * the arithmetic of the two subsample paths differently, so values may
 * differ by an ulp in FP64 and by float rounding in RR_MIXED):
 *   variant 0, 1, 2   each lane owns 4, 8, 16 exposures (a workgroup, one
 *                     wave64, owns 256, 512, 1024 consecutive times); the
 *                     subsamples of supersampled exposures are spread over
 *                     the lanes where a wave's flagged exposures share nss
 *                     and are few enough for that to be the cheaper
 *                     schedule (else summed by one lane, as below);
 *   variant 3, 4, 5   the same tiles with every exposure's subsamples
 *                     summed by one lane.
 * rr_evaluate is variant 1.  Smaller tiles give more waves for small
 * problems; larger ones amortise the per-tile work of long series.
 * variant outside [0, RR_NUM_VARIANTS) is RR_EINVAL; other arguments,
 * errors and memory as rr_evaluate. */
RR_API int rr_evaluate_variant(const rr_tables* t, const double* times_d,
                               const int32_t* lcids_d, int32_t npt,
                               const int32_t* pbids, const int32_t* nss,
                               const double* exptimes, int32_t nlc,
                               const double* pv_d, int32_t npv, int32_t npar,
                               int32_t precision, int32_t variant, void* out_d,
                               hipStream_t stream);

/* Trial-run selection of the implementation (Sect. 3.4.1, where the model
 * times each implementation once after set-up and keeps the fastest): runs
 * the per-vector set-up once, then for every variant one untimed forward
 * launch and `reps` timed ones between two HIP events on `stream`, and
 * writes the variant with the smallest mean time to *best (host int32) and,
 * if ms is not NULL, the mean milliseconds per launch of each variant to
 * ms[RR_NUM_VARIANTS] (host).  Without supersampling variants 3-5 launch
 * the same kernels as 0-2, so only 0-2 run and ms[v + 3] = ms[v].  out_d
 * (as rr_evaluate's) receives the fluxes.  Waits for `stream` to finish the
 * trial before returning.  reps outside [1, 1000] or best == NULL is
 * RR_EINVAL; other arguments, errors and memory as rr_evaluate; with
 * npt == 0 or npv == 0 nothing runs, *best = 1 and ms is zeroed. */
RR_API int rr_select_variant(const rr_tables* t, const double* times_d,
                             const int32_t* lcids_d, int32_t npt,
                             const int32_t* pbids, const int32_t* nss,
                             const double* exptimes, int32_t nlc,
                             const double* pv_d, int32_t npv, int32_t npar,
                             int32_t precision, void* out_d, int32_t reps,
                             int32_t* best, float* ms, hipStream_t stream);

/* The direct model (Sect. 3.1.1): fluxes as rr_evaluate, but every
 * (vector, passband) gets the LD-weighted vector built from annulus weights
 * for its own k instead of interpolating the tables in k, so k is not
 * limited to the tables' [k0, k1] (any k in (0, 1]) and carries no
 * k-interpolation error; the tables' z-grid, profile and I_star are used.
 * Costs ng (nz + 1) lens areas per vector and passband (about 0.5 ms for
 * 512 vectors at the default grid) before the forward kernel.  Arguments,
 * errors and invalid rows as rr_evaluate, except that the k limits are
 * (0, 1].  A k on a table node gives that node's row of the tables.
 * Temporary device memory (144 + 2 npb ng sizeof(real) bytes per vector)
 * is the per-stream buffer that rr_evaluate uses. */
RR_API int rr_evaluate_direct(const rr_tables* t, const double* times_d,
                              const int32_t* lcids_d, int32_t npt,
                              const int32_t* pbids, const int32_t* nss,
                              const double* exptimes, int32_t nlc,
                              const double* pv_d, int32_t npv, int32_t npar,
                              int32_t precision, void* out_d, hipStream_t stream);

/* The small-planet approximation (Sect. 3.4.2): fluxes as rr_evaluate,
 * except that a passband whose radius ratio k is below k_small replaces the
 * LD-weighted mean over the planet's disk with the LD value at the planet's
 * centre.  Per g node (centre distance c = g (1 + k), clamped to 1 off the
 * disk) that value is the tables' piecewise-linear profile at
 * mu = sqrt(1 - c^2); the g-interpolation, lens area and I_star of
 * rr_evaluate are kept.  Such a k needs only k > 0, so planets smaller than
 * the tables' k0 are evaluated without widening the tables; a k at or above
 * k_small takes the interpolated model and must lie in [k0, k1] (results
 * equal rr_evaluate's up to rounding).  k_small: host scalar in [0, 1]
 * (0: no row uses the approximation), else RR_EINVAL.  Other arguments,
 * errors and invalid rows as rr_evaluate.  Temporary device memory
 * (144 + 2 npb ng sizeof(real) bytes per vector) is the per-stream buffer
 * that rr_evaluate uses.  rr_loglik_grad_small_planet gives its
 * log-likelihood and parameter gradient (no LD-profile gradient). */
RR_API int rr_evaluate_small_planet(const rr_tables* t, const double* times_d,
                                    const int32_t* lcids_d, int32_t npt,
                                    const int32_t* pbids, const int32_t* nss,
                                    const double* exptimes, int32_t nlc,
                                    const double* pv_d, int32_t npv, int32_t npar,
                                    double k_small, int32_t precision, void* out_d,
                                    hipStream_t stream);

/* rr_loglik_grad with the small-planet approximation of
 * rr_evaluate_small_planet (Sect. 3.4.2): logl_d[npv] and, if grad_d is not
 * NULL, grad_d[npv][npar] for the same data arguments, obs_d and sigma as
 * rr_loglik_grad.  A passband whose k is below k_small (host scalar in
 * [0, 1], else RR_EINVAL) contributes the derivative of the centre values
 * with respect to k (the piecewise-linear profile's slope at each g node's
 * centre distance); the others are as rr_loglik_grad.  There is no
 * LD-profile gradient here.  Invalid rows give NaN.  Errors and memory as
 * rr_loglik_grad (its temporaries plus 2 npb ng sizeof(real) + 8 npb bytes
 * per vector). */
RR_API int rr_loglik_grad_small_planet(const rr_tables* t, const double* times_d,
                                       const int32_t* lcids_d, int32_t npt,
                                       const int32_t* pbids, const int32_t* nss,
                                       const double* exptimes, int32_t nlc,
                                       const double* pv_d, int32_t npv, int32_t npar,
                                       double k_small, int32_t precision, const void* obs_d,
                                       double sigma, double* logl_d, double* grad_d,
                                       hipStream_t stream);

/* The model as a function of the separation: out_d[i] = Eq. 5 for a planet
 * in front of the star at separation z_d[i] (in stellar radii) with radius
 * ratio k_d[i] (or the scalar k when k_d is NULL), passband pb of the
 * tables -- the k- and g-interpolated LD vector times the lens area over
 * I_star (Sect. 3.1.1, Sect. 3.1.2), without orbit or supersampling.
 * z_d, k_d: device FP64 arrays of n values; out_d: device double[n]
 * (RR_FP64) or float[n] (RR_MIXED).  A k outside [k0, k1] or a z that is
 * negative or not finite gives NaN for that point.  n >= 0 (zero enqueues
 * nothing); errors as rr_evaluate.  No temporary memory. */
RR_API int rr_flux_at_z(const rr_tables* t, const double* z_d, const double* k_d,
                        double k, int64_t n, int32_t pb, int32_t precision, void* out_d,
                        hipStream_t stream);

/* Fluxes as rr_evaluate, but with a limb-darkening profile of its own for
 * every parameter vector, as when the LD coefficients are sampled together
 * with the orbit (each row of the population carries its own stellar
 * profile; the paper's model takes LD coefficients per evaluation,
 * Sect. 4.2).  prof_d[npv][npb][nmu] is a device FP64 array of radial
 * profile samples of vector ipv in passband pb, on the tables' mu samples
 * (the mu grid given to rr_prepare_ld).  The tables' z-grid and annulus
 * weights W are reused; per vector and passband the library interpolates
 * the profile to the bin means, integrates I_star exactly for the
 * piecewise-linear profile (as rr_prepare_ld does) and contracts W with it
 * over the two k-rows around the vector's k (T = W . l of Sect. 3.1.2,
 * restricted to those rows, in the same bin order as the shared table) in
 * FP64, then interpolates them in k as the shared rows are; the
 * evaluation then follows rr_evaluate with those rows in place of the
 * shared ones.  With every vector given the tables' own profile the fluxes
 * equal rr_evaluate's bitwise.  Other arguments, errors and
 * invalid rows as rr_evaluate; non-finite profile samples give non-finite
 * in-transit fluxes of that vector only.  npv * npb * nz < 2^31
 * (RR_ELIMIT beyond).  Temporary device memory, ~(144 + npb (32 + 8 nz +
 * 2 ng sizeof(real))) bytes per vector, is the per-stream buffer that
 * rr_evaluate uses (same growth and reuse rules). */
RR_API int rr_evaluate_ld(const rr_tables* t, const double* times_d,
                          const int32_t* lcids_d, int32_t npt,
                          const int32_t* pbids, const int32_t* nss,
                          const double* exptimes, int32_t nlc,
                          const double* pv_d, int32_t npv, int32_t npar,
                          const double* prof_d, int32_t precision, void* out_d,
                          hipStream_t stream);

/* Gaussian log-likelihood of observed fluxes obs_d[npt] under each
 * parameter vector, and its gradient, with the same time-series and
 * parameter arguments as rr_evaluate:
 *   logl_d[ipv] = -1/2 sum_t ((obs_t - F_t)/sigma)^2     (constant dropped)
 * obs_d     device observed fluxes, double[npt] for RR_FP64 and float[npt]
 *           for RR_MIXED (the residual itself is always formed in FP64);
 * sigma     flux uncertainty, finite and > 0;
 * logl_d    device double[npv], or NULL;
 * grad_d    device double[npv][npar], or NULL: d logl_d[ipv] / d pv[ipv][*]
 *           in the row layout (t0, P, a, b, e, w, k_0 ..);
 * grad_prof_d device double[npb][nmu], or NULL: the gradient of
 *           sum_ipv wprof[ipv] logl[ipv] with respect to the tables' LD
 *           profile samples (through the profile interpolation, I_star and
 *           T = W . ldp; with I_star held at the caller's values while
 *           rr_set_istar is in force);
 * wprof_d   device double[npv] weights for grad_prof_d, or NULL for ones.
 * At least one output must be requested.  Invalid rows give NaN in logl
 * and grad and contribute nothing to grad_prof.  Every sum is formed in
 * FP64 in an order fixed by the inputs (grad_prof: each wave's partial sums
 * in its own LDS copy, the copies added in wave order, then the workgroups
 * in order), so all outputs are bitwise reproducible.  The adjoint keeps
 * npb * ng * (2 sizeof(real) + 8) bytes of tables in LDS (and with
 * grad_prof a copy of d logL / d ldw per wave), at most the device's LDS per
 * workgroup (RR_ELIMIT beyond).  Temporary device memory comes from the stream-ordered
 * allocator: ~(160 + 8 (7 + npb) npt / 1024) bytes per parameter vector,
 * and with grad_prof a further 8 npb ng bytes per vector plus at most
 * 512 MiB of partial sums. */
RR_API int rr_loglik_grad(const rr_tables* t, const double* times_d,
                          const int32_t* lcids_d, int32_t npt,
                          const int32_t* pbids, const int32_t* nss,
                          const double* exptimes, int32_t nlc,
                          const double* pv_d, int32_t npv, int32_t npar,
                          int32_t precision, const void* obs_d, double sigma,
                          const double* wprof_d, double* logl_d, double* grad_d,
                          double* grad_prof_d, hipStream_t stream);

/* rr_loglik_grad with one more output: grad_istar_d, device double[npb]
 * (or NULL), the gradient of sum_ipv wprof[ipv] logl[ipv] with respect to
 * each passband's normaliser I_star, for callers that set I_star
 * themselves (rr_set_istar) and carry its dependence on LD coefficients
 * (Sect. 3.2.1: named laws integrated analytically).  Arguments, errors
 * and memory otherwise as rr_loglik_grad. */
RR_API int rr_loglik_grad_istar(const rr_tables* t, const double* times_d,
                                const int32_t* lcids_d, int32_t npt,
                                const int32_t* pbids, const int32_t* nss,
                                const double* exptimes, int32_t nlc,
                                const double* pv_d, int32_t npv, int32_t npar,
                                int32_t precision, const void* obs_d, double sigma,
                                const double* wprof_d, double* logl_d, double* grad_d,
                                double* grad_prof_d, double* grad_istar_d,
                                hipStream_t stream);

/* rr_loglik_grad with a limb-darkening profile per parameter vector (as
 * rr_evaluate_ld; prof_d[npv][npb][nmu] device FP64 on the tables' mu
 * samples): logl_d and grad_d as rr_loglik_grad, and grad_prof_d, if not
 * NULL, a device double[npv][npb][nmu] holding d logl_d[ipv] / d
 * prof_d[ipv][pb][s] -- each vector's gradient with respect to its own
 * profile, through the profile at the bin means, I_star and its own two
 * table rows (the transpose of their contraction with W).  Invalid rows
 * give NaN in logl and grad and a zero profile gradient.  With every
 * vector given the tables' own profile, logl and grad equal
 * rr_loglik_grad's bitwise and the per-vector profile gradients sum to its
 * shared one (to rounding).  Other arguments, errors and limits as
 * rr_loglik_grad (no wprof); npv * npb * nz < 2^31. */
RR_API int rr_loglik_grad_ld(const rr_tables* t, const double* times_d,
                             const int32_t* lcids_d, int32_t npt,
                             const int32_t* pbids, const int32_t* nss,
                             const double* exptimes, int32_t nlc,
                             const double* pv_d, int32_t npv, int32_t npar,
                             const double* prof_d, int32_t precision, const void* obs_d,
                             double sigma, double* logl_d, double* grad_d,
                             double* grad_prof_d, hipStream_t stream);

/* Instrumentation: the next rr_evaluate / rr_loglik_grad calls made by the
 * calling thread launch their main kernel with `before` and `after` as the
 * launch's own start and stop events (hipExtLaunchKernel), so the pair times
 * that kernel's execution alone (the per-parameter-vector setup kernel that
 * precedes it is outside the pair; with more than 65 535 parameter vectors
 * the pair spans the consecutive launches of the main kernel).  Both events
 * must be created by the caller on the device of the tables; NULL, NULL
 * turns this off.  Returns RR_EINVAL if exactly one of them is NULL. */
RR_API int rr_set_kernel_events(hipEvent_t before, hipEvent_t after);

/* Release a handle (device and host memory).  The caller must make sure no
 * enqueued work still reads it.  NULL is ignored. */
RR_API void rr_free_tables(rr_tables* t);

/* Table introspection for tests and tools: copy one table to host memory.
 * which: 0 ze[nz+1], 1 W[nk][nz][ng], 2 ldp[npb][nz], 3 istar[npb],
 *        4 T64[npb][nk][ng], 5 T32[npb][nk][ng] (float), 6 zm[nz].
 * Writes at most `capacity` elements and stores the element count in *count.
 * Synchronous. */
RR_API int rr_tables_copy(const rr_tables* t, int32_t which, void* host_dst,
                          int64_t capacity, int64_t* count);

/* Grid and sizes of a handle: sizes[0..5] = nz, ng, nk, npb, nmu, nzin. */
RR_API int rr_tables_info(const rr_tables* t, rr_grid* grid, int32_t* sizes);

/* Static description of a return code. */
RR_API const char* rr_strerror(int code);

/* Text of the most recent RR_EDEVICE / RR_EINVAL condition of the calling
 * thread (empty if none). */
RR_API const char* rr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RR_H */
