// rr_forward.hip -- population light-curve evaluation (Sect. 2 Eq. 5,
// Sect. 3.1.1, Sect. 3.1.2, Sect. 4.1, Sect. 4.2).
//
// Two kernels per call:
//
//   k_pv_setup  one thread per parameter vector: validity, cos i from b,
//               sin/cos of the eccentric anomaly at conjunction, and the
//               transit window -- the range of time offsets outside which
//               the planet is either behind the star or farther than 1 + k
//               from its centre, so the flux is exactly 1 (kept in phase
//               units, so the test is frac(phase - lo) < width);
//   k_forward   one wave64 workgroup per (parameter vector, tile of 64 J
//               consecutive times; J = 8 by default, 4 or 16 in the variants
//               of rr_evaluate_variant), lanes along time so loads of the shared
//               time array and the stores of out[pv][t] are coalesced; each
//               wave runs alone (no LDS, no barrier).  Pass 1 reduces each
//               mid-exposure time to an offset from conjunction (FP64),
//               writes 1 for the exposures outside the window (on the
//               aligned fast path for all of them, with 16-B stores) and
//               flags the others; a wave with no flag ends there.
//               Pass 2 evaluates the flagged exposures: per subsample,
//               Kepler orbit -> z -> LD vector interpolated in k and g from
//               the resident table (Sect. 3.1.1, Sect. 3.1.2) x lens area
//               (Eq. 5) -> mean over subsamples.
//
// The kernels are templated on the bulk real type: double (RR_FP64) or float
// (RR_MIXED: the time reduction stays FP64, the rest is FP32).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "rr_device.h"

namespace rr {
namespace {

// Exposures per lane (J) of the forward kernel's variants: the tile of a
// workgroup is 64 J consecutive times.  J is a multiple of 4 (pass 1 packs
// 4 float or 2 double outputs per 16-B store) and at most 32 (a lane's
// flags fit one 32-bit mask).
constexpr int kFwdJ[3] = {4, 8, 16};
static_assert(kTimesPerThread % 4 == 0 && kTimesPerThread <= 32,
              "pass 1 packs 4 float or 2 double outputs per 16-B store");

template <bool kF32>
__global__ void k_pv_setup(const double* __restrict__ pv, int32_t npv,
                           int32_t npar, double k0, double k1, double k_small,
                           PvConst* __restrict__ out) {
    const int ipv = blockIdx.x * blockDim.x + threadIdx.x;
    if (ipv >= npv) return;
    out[ipv] = make_pv_const<kF32>(pv + int64_t(ipv) * npar, npar - 6, k0, k1, k_small);
}

// Per-row, per-passband constants of pass 2: the two k-rows of T that
// bracket k and the k-lerp weight (Sect. 3.1.2), 1 + k, I_star.
template <typename R>
struct PbConst {
    const R* t0r;          // T[pb][ik]; T[pb][ik+1] follows at + ng
    R ak, k, onepk, inv1pk, istar_inv;
};

template <typename R>
__device__ inline PbConst<R> pb_const(const double* __restrict__ pv, int ipv, int npar, int pb,
                                      const GridDev& g, const R* __restrict__ T,
                                      const double* __restrict__ inv_istar, const FwdJob& job) {
    PbConst<R> c;
    const double kd = pv[int64_t(ipv) * npar + 6 + pb];
    if (job.ldw_pv) {
        // per-vector LD: the vector's own copies of the two table rows
        // around its k, interpolated in k below as the shared rows are; or
        // (direct model) its LD vector for its exact k, stored twice and
        // read with zero k-weight
        const int64_t r = int64_t(ipv) * g.npb + pb;
        if (job.ldw_exact_k) {
            c.ak = R(0);
        } else {
            const double u = (kd - g.k0) / g.dk;
            int ik = int(floor(u));
            ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
            c.ak = R(u - ik);
        }
        c.t0r = static_cast<const R*>(job.ldw_pv) + r * 2 * g.ng;
        c.k = R(kd);
        c.onepk = R(1) + c.k;
        c.inv1pk = R(1) / c.onepk;
        c.istar_inv = R(job.inv_istar_pv ? job.inv_istar_pv[r] : inv_istar[pb]);
        return c;
    }
    const double u = (kd - g.k0) / g.dk;
    int ik = int(floor(u));
    ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
    c.ak = R(u - ik);
    c.t0r = T + (int64_t(pb) * g.nk + ik) * g.ng;
    c.k = R(kd);
    c.onepk = R(1) + c.k;
    c.inv1pk = R(1) / c.onepk;
    c.istar_inv = R(inv_istar[pb]);
    return c;
}

// Eq. 5 without the leading 1 at separation z for a planet in front of the
// star: zero without overlap, else the LD vector interpolated in k and g
// from the two table rows (Sect. 3.1.1, Sect. 3.1.2) times the lens area
// over I_star.
template <typename R>
__device__ inline R occulted_at(R z, const PbConst<R>& c, const GridDev& g) {
    if (!(z < c.onepk)) return R(0);
    const R v = z * c.inv1pk * R(g.gscale);
    int m = int(v);
    m = m > g.ng - 2 ? g.ng - 2 : m;
    const R al = v - R(m);
    const R* t0r = c.t0r;
    const R l0 = (R(1) - c.ak) * t0r[m] + c.ak * t0r[g.ng + m];
    const R l1 = (R(1) - c.ak) * t0r[m + 1] + c.ak * t0r[g.ng + m + 1];
    const R ip = (R(1) - al) * l0 + al * l1;
    return ip * lens_area<R>(R(1), c.k, z) * c.istar_inv;
}

// Occulted fraction of subsample s of an exposure at mid-time t (the term
// of Eq. 5 after the leading 1): the orbit (z), the LD vector interpolated
// in k and g from the resident table (Sect. 3.1.1, Sect. 3.1.2) and the lens
// area; 0 when the planet does not overlap the star.
template <typename R>
__device__ inline R subsample_delta(const PvConst& p, const OrbitR<R>& orb,
                                    const PbConst<R>& c, double t, double ex,
                                    double inv_nss, int s, const GridDev& g) {
    const double x = (t + ex * ((s + 0.5) * inv_nss - 0.5)) - p.t0;
    const double u = x * p.invP;
    if (!in_phase_window(u, p, 0.0)) return R(0);
    const double dt = x - p.P * rint(u);
    bool front;
    const R z = separation<R>(R(dt), orb, &front);
    if (!front) return R(0);
    return occulted_at<R>(z, c, g);
}

// Flux of one exposure: 1 - mean over its nss subsamples (Sect. 4.1),
// summed in subsample order.
template <typename R>
__device__ inline R exposure_flux(const PvConst& p, const OrbitR<R>& orb, const PbConst<R>& c,
                                  double t, double ex, int nss, const GridDev& g) {
    const double inv_nss = 1.0 / nss;
    R acc = R(0);
    for (int s = 0; s < nss; ++s) acc += subsample_delta<R>(p, orb, c, t, ex, inv_nss, s, g);
    return R(1) - acc * R(inv_nss);
}

// The work of one workgroup: population row ipv, time tile `tile`.  Each
// wave64 owns 64 J consecutive exposures of the tile and works
// on its own, with no workgroup barrier: a wave whose exposures all lie
// outside the transit window stores ones and ends.
template <typename R, bool kSubPar, int J>
__device__ inline void forward_block(const FwdJob& job, const LcInfo& lc, int ipv,
                                     int tile, const GridDev& g,
                                     const R* __restrict__ T,
                                     const double* __restrict__ inv_istar) {
    constexpr int kSpan = 64 * J;           // exposures per wave
    const int lane = threadIdx.x & 63;
    const int npt = job.npt, npar = job.npar;
    const double* __restrict__ times = job.times;
    const int32_t* __restrict__ lcids = job.lcids;
    const double* __restrict__ pv = job.pv;
    // exposure r of this lane (pass 2 order, and pass 1 off the fast path)
    const int w0 = tile * (kFwdBlock * J) + (threadIdx.x >> 6) * kSpan;
    const int t_base = w0 + lane;
    R* __restrict__ orow = static_cast<R*>(job.out) + int64_t(ipv) * npt;
    const PvConst p = job.pvc[ipv];

    if (!(p.flags & kValid)) {
        for (int r = 0; r < J; ++r) {
            const int it = t_base + 64 * r;
            if (it < npt) orow[it] = R(NAN);
        }
        return;
    }

    // Pass 1: exposures that cannot overlap the star get F = 1 now.  Bit r
    // of `todo` marks exposure t_base + 64 r as one that may overlap it.
    uint32_t todo = 0;
    constexpr int kVec = 16 / int(sizeof(R));            // outputs per 16-B store
    constexpr int kGroups = J / kVec;
    bool vec = w0 + kSpan <= npt &&
               ((reinterpret_cast<uintptr_t>(orow + w0) | reinterpret_cast<uintptr_t>(times) |
                 reinterpret_cast<uintptr_t>(lcids)) & 15) == 0;
    int lvec = 0;                                       // the span's light curve
    if (vec && lcids) {
        // The fast path also serves a span that lies in one light curve:
        // the lane reads its light-curve ids in the same grouping as its
        // times (kVec consecutive ids per group).
        typedef int IV __attribute__((ext_vector_type(kVec)));
        bool same = true;
        int first = 0;
#pragma unroll
        for (int q = 0; q < kGroups; ++q) {
            const IV ids = *reinterpret_cast<const IV*>(lcids + w0 + q * (64 * kVec) + lane * kVec);
#pragma unroll
            for (int v = 0; v < kVec; ++v) {
                if (q == 0 && v == 0) first = ids[0];
                same = same && ids[v] == first;
            }
        }
        lvec = __shfl(first, 0);
        vec = __all(same && first == lvec) && lvec >= 0 && lvec < lc.nlc;
    }
    if (vec) {
        // Whole span in range, in one light curve, 16-B aligned: in group q
        // the lane owns the kVec consecutive exposures w0 + 64 kVec q +
        // kVec lane + v (16-B loads of times, one 16-B store of ones), with
        // no bounds or light-curve checks.  Phase g = t/P + c0 with
        // c0 = -t0/P - (window start) by one FMA.
        typedef R RV __attribute__((ext_vector_type(kVec)));
        double tv[J];
#pragma unroll
        for (int q = 0; q < kGroups; ++q) {
            const double* tp = times + w0 + q * (64 * kVec) + lane * kVec;
#pragma unroll
            for (int v = 0; v < kVec; v += 2) {
                const double2 d = *reinterpret_cast<const double2*>(tp + v);
                tv[q * kVec + v] = d.x;
                tv[q * kVec + v + 1] = d.y;
            }
        }
        const double hw = 0.5 * lc.exptime[lvec] * p.invP;
        const double c0 = -p.t0 * p.invP - (p.flo - hw);
        const double wn = p.wn + 2.0 * hw;
        const RV ones = R(1);
        uint32_t bits = 0;                                // bit q kVec + v
#pragma unroll
        for (int q = 0; q < kGroups; ++q) {
#pragma unroll
            for (int v = 0; v < kVec; ++v) {
                const double gph = fma(tv[q * kVec + v], p.invP, c0);
                if (gph - floor(gph) < wn) bits |= 1u << (q * kVec + v);
            }
            *reinterpret_cast<RV*>(orow + w0 + q * (64 * kVec) + lane * kVec) = ones;
        }
        if (!__any(bits != 0)) return;
        // Regroup to pass 2's order: exposure w0 + 64 r + lane, r = q kVec + s,
        // is bit q kVec + lane % kVec of lane (64 s + lane) / kVec.
#pragma unroll
        for (int sidx = 0; sidx < kVec; ++sidx) {
            const uint32_t x = uint32_t(__shfl(int(bits), (64 * sidx + lane) / kVec));
#pragma unroll
            for (int q = 0; q < kGroups; ++q)
                todo |= ((x >> (q * kVec + lane % kVec)) & 1u) << (q * kVec + sidx);
        }
    } else {
        double tv[J];
        int lv[J];
#pragma unroll
        for (int r = 0; r < J; ++r) {
            const int it = t_base + 64 * r;
            tv[r] = it < npt ? times[it] : 0.0;
            lv[r] = (lcids && it < npt) ? lcids[it] : 0;
        }
        const double hw0 = 0.5 * lc.exptime[0] * p.invP;
#pragma unroll
        for (int r = 0; r < J; ++r) {
            const int it = t_base + 64 * r;
            if (it >= npt) continue;
            const int l = lv[r];
            if (l < 0 || l >= lc.nlc) { orow[it] = R(NAN); continue; }
            const double hw = lcids ? 0.5 * lc.exptime[l] * p.invP : hw0;
            if (in_phase_window((tv[r] - p.t0) * p.invP, p, hw)) todo |= 1u << r;
            else orow[it] = R(1);
        }
        if (!__any(todo != 0)) return;
    }

    const OrbitR<R> orb(p);
    int pb_cached = -1;
    PbConst<R> c = {};

    // Pass 2 when every flagged exposure of the wave has nss = 1: two
    // exposures of the same passband at a time, as two independent chains
    // the compiler interleaves (a lane with several exposures is
    // latency-bound, above all in the kernel's tail where few waves are left
    // to hide it).  Both kernel variants take this path for such waves, so
    // a series gives the same bits whichever variant a launch uses.
    auto pass2_pairs = [&]() {
        while (todo) {
            const int r1 = __builtin_ctz(todo);
            todo &= todo - 1;
            const int it1 = t_base + 64 * r1;
            const int l1 = lcids ? lcids[it1] : 0;
            const int pb1 = lc.pb[l1];
            if (pb1 != pb_cached) {
                pb_cached = pb1;
                c = pb_const<R>(pv, ipv, npar, pb1, g, T, inv_istar, job);
            }
            int it2 = -1, l2 = 0;
            if (todo) {
                const int r2 = __builtin_ctz(todo);
                const int cand = t_base + 64 * r2;
                l2 = lcids ? lcids[cand] : 0;
                if (lc.pb[l2] == pb1) {
                    it2 = cand;
                    todo &= todo - 1;
                }
            }
            const R d1 = subsample_delta<R>(p, orb, c, times[it1], lc.exptime[l1], 1.0, 0, g);
            if (it2 >= 0) {
                const R d2 = subsample_delta<R>(p, orb, c, times[it2], lc.exptime[l2], 1.0, 0, g);
                orow[it2] = R(1) - d2;
            }
            orow[it1] = R(1) - d1;
        }
    };

    if constexpr (kSubPar) {
        // Supersampled exposures: if every flagged exposure of the wave has
        // the same nss in [2, 32] and the wave's flags are sparse enough to
        // gain from it, spread the subsamples over the lanes --
        // G = 64 / nss exposures per round, lane L on subsample L % nss of
        // exposure L / nss -- and let the first lane of each group sum the
        // group's terms in subsample order (so the result is the same as
        // one lane's serial loop).  The flagged exposures are packed in
        // exposure order into this wave's own LDS region first.
        int nmin = 1 << 30, nmax = 0;
        for (uint32_t b = todo; b; b &= b - 1) {
            const int it = t_base + 64 * __builtin_ctz(b);
            const int n = lc.nss[lcids ? lcids[it] : 0];
            nmin = n < nmin ? n : nmin;
            nmax = n > nmax ? n : nmax;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const int a = __shfl_xor(nmin, off), b = __shfl_xor(nmax, off);
            nmin = a < nmin ? a : nmin;
            nmax = b > nmax ? b : nmax;
        }
        const int N = nmax;
        if (N == 1) {
            pass2_pairs();
            return;
        }
        // Spreading takes ceil(flagged / (64 / N)) rounds of one subsample
        // per lane, each with its gathers and an N-term reduction (measured
        // at ~1.5 subsamples of the per-lane loop); the per-lane loop N
        // times the largest number of flagged exposures of one lane.  The
        // wave takes the cheaper (both sum the same terms in the same order;
        // their values agree to an ulp, as the compiler may contract the two
        // copies of the subsample arithmetic differently).
        bool spread = job.spread && nmin == nmax && N >= 2 && N <= 32;
        if (spread) {
            int mine = __popc(todo), most = mine, flagged = mine;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const int a = __shfl_xor(most, off);
                most = a > most ? a : most;
                flagged += __shfl_xor(flagged, off);
            }
            const int G = 64 / N;
            spread = 3 * ((flagged + G - 1) / G) < 2 * most * N;
        }
        if (spread) {
            __shared__ uint16_t packed[kFwdBlock / 64][kSpan];
            uint16_t* pk = packed[threadIdx.x >> 6];
            const uint64_t below = __lanemask_lt();
            int total = 0;
#pragma unroll
            for (int r = 0; r < J; ++r) {
                const uint64_t m = __ballot((todo >> r) & 1u);
                if ((todo >> r) & 1u) pk[total + __popcll(m & below)] = uint16_t(64 * r + lane);
                total += __popcll(m);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int G = 64 / N;
            const int gi = lane / N, sub = lane - gi * N;
            const double inv_nss = 1.0 / N;
            for (int j0 = 0; j0 < total; j0 += G) {
                const int j = j0 + gi;
                const bool have = gi < G && j < total;
                int it = 0;
                R val = R(0);
                if (have) {
                    it = w0 + pk[j];
                    const int l = lcids ? lcids[it] : 0;
                    const int pb = lc.pb[l];
                    if (pb != pb_cached) {
                        pb_cached = pb;
                        c = pb_const<R>(pv, ipv, npar, pb, g, T, inv_istar, job);
                    }
                    val = subsample_delta<R>(p, orb, c, times[it], lc.exptime[l], inv_nss, sub, g);
                }
                R acc = R(0);
                const int src0 = gi < G ? gi * N : 0;         // idle lanes read lane 0..N-1
                for (int q = 0; q < N; ++q) acc += __shfl(val, src0 + q);
                if (have && sub == 0) orow[it] = R(1) - acc * R(inv_nss);
            }
            return;
        }
    }

    // Pass 2 in the wave: the flagged exposures, one per lane and bit.
    if constexpr (!kSubPar) {
        pass2_pairs();
        return;
    }
    while (todo) {
        const int r = __builtin_ctz(todo);
        todo &= todo - 1;
        const int it = t_base + 64 * r;
        const int l = lcids ? lcids[it] : 0;          // reloaded: keeps pass 1's
        const int pb = lc.pb[l];                      // registers free here
        if (pb != pb_cached) {
            pb_cached = pb;
            c = pb_const<R>(pv, ipv, npar, pb, g, T, inv_istar, job);
        }
        orow[it] = exposure_flux<R>(p, orb, c, times[it], lc.exptime[l], lc.nss[l], g);
    }
}

// ---------------------------------------------------------------------------
// Split launch over a registered series (rr_evaluate_series).
//
// The window test both roles apply to every exposure: with hw half the
// exposure time in periods, g = t/P - t0/P - (window start) + hw, and the
// exposure may overlap the star iff frac(g) < window width + 2 hw.  Every
// multiply-add is an explicit fma and nothing else can be contracted, so
// the streaming and transit workgroups reach the same decision bit for bit:
// each exposure is written by exactly one of them.  floor(g) numbers the
// transit (epoch) an exposure belongs to.
struct Win {
    double c0, wn;
};
__device__ inline Win lc_window(double t0, double invP, double flo, double wn, double exptime) {
    Win w;
    const double a = fma(-t0, invP, -flo);
    w.c0 = fma(0.5 * exptime, invP, a);
    w.wn = fma(exptime, invP, wn);
    return w;
}
__device__ inline double win_phase(double t, double invP, const Win& w) {
    return fma(t, invP, w.c0);
}
__device__ inline bool win_in(double gph, const Win& w) { return gph - floor(gph) < w.wn; }

// Constants of row ipv in the split launch: read from the per-row setup's
// output, or (kSelf) derived here from the parameter row by the same
// function, so both give the same bits.
template <typename R, bool kSelf>
__device__ inline PvConst split_row_const(const FwdJob& job, const SplitInfo& si, int ipv) {
    if (kSelf)
        return make_pv_const<std::is_same<R, float>::value>(job.pv + int64_t(ipv) * job.npar,
                                                            job.npar - 6, si.k_lo, si.k_hi);
    return job.pvc[ipv];
}

// Streaming role: tile `tile` of 64 J consecutive times for rows
// [r0, r1).  The lane loads its J times once and, row by row, writes F = 1
// to every exposure outside the row's window (NaN to every exposure of an
// invalid row), leaving the others to the transit workgroups.  Only four
// constants per row are used, so a row costs a handful of VALU operations
// per exposure and its stores.  On the aligned path (whole
// tile in one light curve, 16-B aligned rows) lane L owns the kVec
// consecutive exposures 64 kVec q + kVec L + v of group q and stores a
// group with one 16-B store when none of it is in the window.
template <typename R, int J, bool kSelf>
__device__ inline void stream_rows(const FwdJob& job, const LcInfo& lc, const SplitInfo& si,
                                   int r0, int r1, int tile) {
    constexpr int kSpan = 64 * J;
    constexpr int kVec = 16 / int(sizeof(R));
    constexpr int kGroups = J / kVec;
    typedef R RV __attribute__((ext_vector_type(kVec)));
    const int lane = threadIdx.x & 63;
    const int npt = job.npt;
    const double* __restrict__ times = job.times;
    const int32_t* __restrict__ lcids = job.lcids;
    const int w0 = tile * kSpan;
    const bool whole = w0 + kSpan <= npt && (reinterpret_cast<uintptr_t>(times) & 15) == 0;
    // rows start 16-B aligned when the base is and npt is a multiple of kVec
    const bool aligned = whole && npt % kVec == 0 &&
                         (reinterpret_cast<uintptr_t>(job.out) & 15) == 0;
    int lvec = 0;
    bool vec = aligned;
    if (vec && lcids) {
        // the light curves are contiguous runs: one id at both ends means
        // one light curve over the tile
        lvec = lcids[w0];
        vec = lvec == lcids[w0 + kSpan - 1] && lvec >= 0 && lvec < lc.nlc;
    }
    double tv[J];
    int lv[J];
    if (vec) {
#pragma unroll
        for (int q = 0; q < kGroups; ++q) {
            const double* tp = times + w0 + q * (64 * kVec) + lane * kVec;
#pragma unroll
            for (int v = 0; v < kVec; v += 2) {
                const double2 d = *reinterpret_cast<const double2*>(tp + v);
                tv[q * kVec + v] = d.x;
                tv[q * kVec + v + 1] = d.y;
            }
        }
    } else {
        // per exposure: it = w0 + 64 r + lane
#pragma unroll
        for (int r = 0; r < J; ++r) {
            const int it = w0 + 64 * r + lane;
            tv[r] = it < npt ? times[it] : 0.0;
            lv[r] = it < npt ? (lcids ? lcids[it] : 0) : -1;
        }
    }
    const double ex_vec = lc.exptime[lvec];
    // The rows' four window constants, 64 rows at a time (lane i takes row
    // r0 + 64 k + i), handed to the row loop by readlane.
    double c_t0 = 0.0, c_invP = 0.0, c_flo = 0.0, c_wn = 0.0;
    int c_ok = 0;
    for (int ipv = r0; ipv < r1; ++ipv) {
        const int k = (ipv - r0) & 63;
        if (k == 0) {
            const int rl = ipv + lane;
            if (rl < r1) {
                const PvConst pl = split_row_const<R, kSelf>(job, si, rl);
                c_t0 = pl.t0; c_invP = pl.invP; c_flo = pl.flo; c_wn = pl.wn;
                c_ok = pl.flags & kValid;
            }
        }
        R* __restrict__ orow = static_cast<R*>(job.out) + int64_t(ipv) * npt;
        const double t0 = __shfl(c_t0, k), invP = __shfl(c_invP, k);
        const double flo = __shfl(c_flo, k), pwn = __shfl(c_wn, k);
        if (!__shfl(c_ok, k)) {
#pragma unroll
            for (int r = 0; r < J; ++r) {
                const int it = w0 + 64 * r + lane;
                if (it < npt) orow[it] = R(NAN);
            }
            continue;
        }
        if (vec) {
            const Win w = lc_window(t0, invP, flo, pwn, ex_vec);
#pragma unroll
            for (int q = 0; q < kGroups; ++q) {
                const int base = w0 + q * (64 * kVec) + lane * kVec;
                bool in[kVec];
                bool any = false;
#pragma unroll
                for (int v = 0; v < kVec; ++v) {
                    in[v] = win_in(win_phase(tv[q * kVec + v], invP, w), w);
                    any = any || in[v];
                }
                if (!any) {
                    *reinterpret_cast<RV*>(orow + base) = RV(R(1));
                } else {
#pragma unroll
                    for (int v = 0; v < kVec; ++v)
                        if (!in[v]) orow[base + v] = R(1);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < J; ++r) {
                const int it = w0 + 64 * r + lane;
                const int l = lv[r];
                if (it >= npt) continue;
                if (l < 0 || l >= lc.nlc) { orow[it] = R(NAN); continue; }
                const Win w = lc_window(t0, invP, flo, pwn, lc.exptime[l]);
                if (!win_in(win_phase(tv[r], invP, w), w)) orow[it] = R(1);
            }
        }
    }
}

// Flat position j of a wave's candidate list -> the largest lane s with
// excl_s <= j (excl is the exclusive scan of the lanes' candidate counts,
// so s's run holds j whenever j < total).
__device__ inline int owner_lane(int excl, int j) {
    int s = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int c = s + step;
        if (__shfl(excl, c) <= j) s = c;
    }
    return s;
}

// Transit role: share `share` of row ipv's transit exposures.  Per light
// curve, 64 transits (epochs) at a time, one per lane: the lane turns its
// epoch's phase range [n, n + min(wn, 1)) into a time range and, through the
// light curve's index, into a run of candidate exposures (widened by a
// bucket on each side, so that it holds every exposure of the epoch); a
// scan across the wave concatenates the runs, and the row's shares take
// every shares-th chunk of 64 candidates, so each gets an equal part of the
// row's transits whatever their lengths.  A candidate is evaluated where it
// stands: one outside the window comes out as exactly 1 (each of its
// subsamples fails the window test), the value the streaming workgroups
// store there, and an exposure two runs share is written twice with the
// same bits; so nothing is compacted or staged.  One subsample per
// exposure (the launch serves such series only); two candidates per lane as
// independent chains.
template <typename R, bool kSelf>
__device__ inline void transit_share(const FwdJob& job, const LcInfo& lc, const SplitInfo& si,
                                     int ipv, int share, const GridDev& g,
                                     const R* __restrict__ T,
                                     const double* __restrict__ inv_istar) {
    const int lane = threadIdx.x & 63;
    const PvConst p = split_row_const<R, kSelf>(job, si, ipv);
    if (!(p.flags & kValid)) return;
    const double* __restrict__ times = job.times;
    R* __restrict__ orow = static_cast<R*>(job.out) + int64_t(ipv) * job.npt;
    const OrbitR<R> orb(p);
    const int E = si.shares;
    int64_t chunk0 = 0;              // candidate chunks dealt so far for this row
    for (int l = 0; l < lc.nlc; ++l) {
        const SeriesLc sl = si.lcs[l];
        if (sl.end <= sl.start) continue;
        const double ex = lc.exptime[l];
        const Win w = lc_window(p.t0, p.invP, p.flo, p.wn, ex);
        const double span = w.wn < 1.0 ? w.wn : 1.0;
        const double n_first = floor(win_phase(sl.t_first, p.invP, w));
        const double n_last = floor(win_phase(sl.t_last, p.invP, w));
        // more transits than exposures (a period shorter than the cadence),
        // or epoch numbers too large to step through exactly: every
        // exposure of the light curve is a candidate, in one batch
        const bool dense = n_last - n_first >= double(sl.end - sl.start) ||
                           !(fabs(n_first) < 1e15) || !(fabs(n_last) < 1e15);
        const PbConst<R> c = pb_const<R>(job.pv, ipv, job.npar, lc.pb[l], g, T, inv_istar, job);
        const int32_t* __restrict__ bk = si.buckets + sl.boff;
        for (double nb0 = n_first; dense || nb0 <= n_last; nb0 += 64.0) {
            int i0 = sl.start, excl = 0, total = sl.end - sl.start;
            if (!dense) {
                const double n = nb0 + double(lane);
                int cnt = 0;
                i0 = 0;
                if (n <= n_last) {
                    const double ta = (n - w.c0) * p.P;
                    const double tb = (n + span - w.c0) * p.P;
                    const double fa = floor((ta - sl.t_first) * sl.inv_bw) - 1.0;
                    const double fb = floor((tb - sl.t_first) * sl.inv_bw) + 2.0;
                    const int bl = !(fa > 0.0) ? 0 : (fa > double(sl.nb) ? sl.nb : int(fa));
                    const int bh = !(fb > 0.0) ? 0 : (fb > double(sl.nb) ? sl.nb : int(fb));
                    i0 = bk[bl];
                    cnt = bk[bh] - i0;
                }
                int incl = cnt;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int x = __shfl_up(incl, off);
                    if (lane >= off) incl += x;
                }
                total = __shfl(incl, 63);
                excl = incl - cnt;
            }
            const int64_t nchunks = (int64_t(total) + 63) / 64;
            const int64_t q0 = (share - chunk0 % E + E) % E;
            chunk0 += nchunks;
            // exposure of flat candidate position q * 64 + lane (-1 past the
            // end); every lane takes part in the shuffles
            auto cand = [&](int64_t q) -> int {
                const int j = int(q) * 64 + lane;
                if (dense) return j < total ? sl.start + j : -1;
                const int src = owner_lane(excl, j);
                const int it = __shfl(i0, src) + (j - __shfl(excl, src));
                return j < total ? it : -1;
            };
            for (int64_t q = q0; q < nchunks; q += 2 * int64_t(E)) {
                const int ia = cand(q);
                const int ib = q + E < nchunks ? cand(q + E) : -1;
                R da = R(0), db = R(0);
                if (ia >= 0) da = subsample_delta<R>(p, orb, c, times[ia], ex, 1.0, 0, g);
                if (ib >= 0) db = subsample_delta<R>(p, orb, c, times[ib], ex, 1.0, 0, g);
                if (ia >= 0) orow[ia] = R(1) - da;
                if (ib >= 0) orow[ib] = R(1) - db;
            }
            if (dense) break;
        }
    }
}

// The split launch: workgroups [0, npv * shares) take the transits (share
// b % shares of row b / shares); the others stream time tiles over blocks
// of rows (tile u % ntiles of rows [rows_per u / ntiles, ...)).  The
// transit workgroups are resident from the start, so their work runs beside
// the streaming stores instead of forming a tail.  kSelf: each workgroup
// derives its rows' constants itself (no setup launch before it).
template <typename R, bool kSelf>
__global__ __launch_bounds__(kFwdBlock) void k_forward_split(FwdJob job, LcInfo lc, GridDev g,
                                                          const R* __restrict__ T,
                                                          const double* __restrict__ inv_istar,
                                                          SplitInfo si) {
    const int b = int(blockIdx.x);
    const int n2 = job.npv * si.shares;
    if (b < n2) {
        const int ipv = b / si.shares;
        transit_share<R, kSelf>(job, lc, si, ipv, b - ipv * si.shares, g, T, inv_istar);
        return;
    }
    const int u = b - n2;
    const int rg = u / job.ntiles;
    const int r0 = rg * si.rows_per;
    const int r1 = r0 + si.rows_per < job.npv ? r0 + si.rows_per : job.npv;
    stream_rows<R, kTimesPerThread, kSelf>(job, lc, si, r0, r1, u - rg * job.ntiles);
}

// One population (rr_evaluate): workgroup (x, y) -> row pv0 + y, tile x of
// 64 J times.  kSubPar: some light curve has nss > 1.
template <typename R, bool kSubPar, int J>
__global__ __launch_bounds__(kFwdBlock) void k_forward(FwdJob job, LcInfo lc, GridDev g,
                                                    const R* __restrict__ T,
                                                    const double* __restrict__ inv_istar) {
    const int ipv = job.pv0 + blockIdx.y;
    const int tile = blockIdx.x;
    forward_block<R, kSubPar, J>(job, lc, ipv, tile, g, T, inv_istar);
}

// Grouped launch (serving): workgroup b belongs to the last job whose
// block0 <= b; jobs come from several requests and time series.
template <typename R, bool kSubPar>
__global__ __launch_bounds__(kFwdBlock) void k_forward_jobs(JobTable jt, GridDev g,
                                                         const R* __restrict__ T,
                                                         const double* __restrict__ inv_istar) {
    const int b = blockIdx.x;
    int jj = 0;
    for (int q = 1; q < jt.njobs; ++q)
        if (jt.j[q].block0 <= b) jj = q;
    const FwdJob& job = jt.j[jj];
    const int local = b - job.block0;
    const int ipv = job.pv0 + local / job.ntiles;
    const int tile = local - (local / job.ntiles) * job.ntiles;
    forward_block<R, kSubPar, kTimesPerThread>(job, *job.lc, ipv, tile, g, T, inv_istar);
}

// Eq. 5 at given separations (the model as a function of z and k, the
// form of the paper's listings): out[i] = 1 - occulted_at(z_i) for passband
// pb with k = kv[i] (or kconst); NaN for a k outside the table or a z that
// is negative or not finite.
template <typename R>
__global__ void k_flux_at_z(const double* __restrict__ z, const double* __restrict__ kv,
                            double kconst, int64_t n, int32_t pb, GridDev g, double k1,
                            const R* __restrict__ T, const double* __restrict__ inv_istar,
                            R* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double k = kv ? kv[i] : kconst;
    const double zi = z[i];
    if (!(k >= g.k0 && k <= k1) || !(zi >= 0.0) || !is_finite(zi)) {
        out[i] = R(NAN);
        return;
    }
    PbConst<R> c;
    const double u = (k - g.k0) / g.dk;
    int ik = int(floor(u));
    ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
    c.ak = R(u - ik);
    c.t0r = T + (int64_t(pb) * g.nk + ik) * g.ng;
    c.k = R(k);
    c.onepk = R(1) + c.k;
    c.inv1pk = R(1) / c.onepk;
    c.istar_inv = R(inv_istar[pb]);
    out[i] = R(1) - occulted_at<R>(R(zi), c, g);
}

__global__ void k_pv_setup_jobs(SetupTable st, double k0, double k1) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int jj = 0;
    for (int q = 1; q < st.njobs; ++q)
        if (st.j[q].thread0 <= t) jj = q;
    const SetupJob& sj = st.j[jj];
    const int ipv = t - sj.thread0;
    if (ipv < 0 || ipv >= sj.npv) return;
    sj.pvc[ipv] = sj.f32 ? make_pv_const<true>(sj.pv + int64_t(ipv) * sj.npar, sj.npar - 6, k0, k1)
                         : make_pv_const<false>(sj.pv + int64_t(ipv) * sj.npar, sj.npar - 6, k0, k1);
}

inline unsigned nblocks(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_pv_setup(const rr_tables* t, const double* pv, int32_t npv,
                           int32_t npar, PvConst* pvc, int32_t precision, hipStream_t s) {
    return launch_pv_setup_k(pv, npv, npar, t->grid.k0, t->grid.k1, pvc, precision, s);
}

hipError_t launch_pv_setup_k(const double* pv, int32_t npv, int32_t npar, double k_lo,
                             double k_hi, PvConst* pvc, int32_t precision, hipStream_t s,
                             double k_small) {
    if (precision == RR_FP64)
        hipLaunchKernelGGL(k_pv_setup<false>, dim3(nblocks(npv)), dim3(kBlock), 0, s, pv, npv,
                           npar, k_lo, k_hi, k_small, pvc);
    else
        hipLaunchKernelGGL(k_pv_setup<true>, dim3(nblocks(npv)), dim3(kBlock), 0, s, pv, npv,
                           npar, k_lo, k_hi, k_small, pvc);
    return hipGetLastError();
}

// One launch of k_forward for J exposures per lane.
template <typename R>
hipError_t launch_forward_j(int J, bool sub, dim3 grid, dim3 block, hipStream_t s,
                            hipEvent_t st, hipEvent_t sp, const FwdJob& job, const LcInfo& lc,
                            const GridDev& g, const R* T, const double* inv_istar) {
    switch (J * 2 + (sub ? 1 : 0)) {
        case 8: launch_timed(k_forward<R, false, 4>, grid, block, 0, s, st, sp, job, lc, g, T, inv_istar); break;
        case 9: launch_timed(k_forward<R, true, 4>, grid, block, 0, s, st, sp, job, lc, g, T, inv_istar); break;
        case 16: launch_timed(k_forward<R, false, 8>, grid, block, 0, s, st, sp, job, lc, g, T, inv_istar); break;
        case 17: launch_timed(k_forward<R, true, 8>, grid, block, 0, s, st, sp, job, lc, g, T, inv_istar); break;
        case 32: launch_timed(k_forward<R, false, 16>, grid, block, 0, s, st, sp, job, lc, g, T, inv_istar); break;
        case 33: launch_timed(k_forward<R, true, 16>, grid, block, 0, s, st, sp, job, lc, g, T, inv_istar); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward(const rr_tables* t, const double* times,
                          const int32_t* lcids, int32_t npt, const LcInfo& lc,
                          const double* pv, int32_t npv, int32_t npar,
                          const PvConst* pvc, int32_t precision, void* out,
                          hipStream_t s, const void* ldw_pv, const double* inv_istar_pv,
                          int32_t ldw_exact_k, int32_t variant) {
    const GridDev g = grid_dev(t);
    // variant (rr_evaluate_variant): J = kFwdJ[v % 3]; v >= 3 evaluates
    // supersampled exposures one per lane instead of spreading subsamples
    if (variant < 0 || variant >= kNumFwdVariants) variant = kDefaultFwdVariant;
    const int J = kFwdJ[variant % 3];
    FwdJob job;
    job.ldw_pv = ldw_pv; job.inv_istar_pv = inv_istar_pv; job.ldw_exact_k = ldw_exact_k;
    job.spread = variant < 3 ? 1 : 0;
    job.times = times; job.lcids = lcids; job.lc = nullptr; job.pv = pv; job.pvc = pvc;
    job.out = out; job.npt = npt; job.npar = npar; job.pv0 = 0; job.npv = npv;
    job.ntiles = (npt + kFwdBlock * J - 1) / (kFwdBlock * J); job.block0 = 0; job.max_nss = 1;
    for (int l = 0; l < lc.nlc; ++l) job.max_nss = lc.nss[l] > job.max_nss ? lc.nss[l] : job.max_nss;
    const KernelEvents ev = kernel_events();
    const bool sub = job.max_nss > 1;
    // rows along grid y, at most 65535 per launch
    for (int32_t r0 = 0; r0 < npv; r0 += 65535) {
        job.pv0 = r0;
        const dim3 grid(unsigned(job.ntiles), unsigned(npv - r0 < 65535 ? npv - r0 : 65535));
        const dim3 block(kFwdBlock);
        hipEvent_t st = r0 == 0 ? ev.before : nullptr;
        hipEvent_t sp = npv - r0 <= 65535 ? ev.after : nullptr;
        const hipError_t e =
            precision == RR_FP64
                ? launch_forward_j<double>(J, sub, grid, block, s, st, sp, job, lc, g, t->T64,
                                           t->inv_istar)
                : launch_forward_j<float>(J, sub, grid, block, s, st, sp, job, lc, g, t->T32,
                                          t->inv_istar);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// Workgroups of the split kernel (one wave each) resident at once on the
// current device; 0 if the query fails.
static int split_capacity(int32_t precision, bool self) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const auto key = std::make_tuple(dev, precision == RR_FP64 ? 0 : 1, self ? 1 : 0);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int ncu = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e;
    if (precision == RR_FP64)
        e = self ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &per_cu, k_forward_split<double, true>, kFwdBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &per_cu, k_forward_split<double, false>, kFwdBlock, 0);
    else
        e = self ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &per_cu, k_forward_split<float, true>, kFwdBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &per_cu, k_forward_split<float, false>, kFwdBlock, 0);
    if (e != hipSuccess || per_cu <= 0) return 0;
    cache[key] = per_cu * ncu;
    return per_cu * ncu;
}

bool split_preferred(const rr_tables* t, const rr_series* se, int32_t npv, int32_t precision) {
    (void)t;
    // Measured: the split launch wins on series with one subsample per
    // exposure except the shortest (two time tiles or fewer) under more than
    // 1024 rows; the per-tile kernel stays ahead on supersampled series.
    const int64_t ntiles = (int64_t(se->npt) + kFwdTile - 1) / kFwdTile;
    if (se->max_nss != 1 || (ntiles <= 2 && npv > 1024)) return false;
    return split_capacity(precision, false) > 0;
}

SplitPlan plan_forward_split(const rr_series* se, int32_t npv, int32_t precision) {
    SplitPlan sp;
    int cap = split_capacity(precision, false);
    if (cap <= 0) cap = 2048;
    const int cap_self = split_capacity(precision, true);
    const int64_t ntiles = (int64_t(se->npt) + kFwdTile - 1) / kFwdTile;
    const int64_t tiles_total = ntiles * npv;
    const int64_t max_sh = std::max<int64_t>(1, (int64_t(se->npt) + 63) / 64);
    // Streaming workgroups take kSplitRows rows of one time tile each (2
    // for small problems, so that there are enough of them).
    sp.rows_per = std::max<int32_t>(
        1, std::min<int32_t>(tiles_total < 2 * int64_t(cap) ? 2 : kSplitRows, npv));
    // Two regimes, from sweeps of both precisions over the population
    // workloads (16 to 4096 rows, 1000 to 50 000 times, 1 to 16 transit
    // workgroups per row, 4 to 16 rows per streaming workgroup).  With
    // `ref` the float fused kernel's resident workgroups (4096 here; the
    // double kernel holds half as many, yet measured best with the same
    // counts):
    //  * every workgroup derives its rows' constants itself and no setup
    //    launch precedes the kernel, as long as that launch has at most
    //    2 ref workgroups; beyond that too many of them pay the set-up's
    //    latency again behind the first.  Transit workgroups per row:
    //    ceil(sqrt(2 ref x min(tiles, 40) / (40 rows))), fewer for series
    //    shorter than 40 tiles (20 000 exposures), whose rows have fewer
    //    transits, and at least 1024 in all; over 40 tiles or more that is
    //    16 per row at 64 rows, 8 at 128, 6 at 256, 4 at 512, 3 at 1024.
    //    More queue behind each other or spend their time on set-up, fewer
    //    leave too much serial work per lane.  From 768 rows over 32 tiles
    //    or more the streaming workgroups take 8 rows, so that fewer of
    //    them pay the set-up.
    //  * otherwise the setup kernel runs first and, for 512 rows or more
    //    over 16 tiles or more, there are as many transit workgroups as are
    //    resident at once, else at most 2048.
    const int ref = split_capacity(RR_MIXED, true);
    if (cap_self > 0 && ref > 0) {
        const double len = double(std::min<int64_t>(ntiles, 40));
        const int64_t by_rows =
            int64_t(std::ceil(std::sqrt(2.0 * double(ref) * len / (40.0 * double(npv)))));
        const int64_t by_total = (1024 + int64_t(npv) - 1) / npv;
        const int64_t shares =
            std::min<int64_t>({16, max_sh, std::max<int64_t>({1, by_rows, by_total})});
        const int32_t rows =
            npv >= 768 && ntiles >= 32 ? std::min<int32_t>(2 * kSplitRows, npv) : sp.rows_per;
        const int64_t blocks = int64_t(npv) * shares + ntiles * ((npv + rows - 1) / rows);
        if (blocks <= 2 * int64_t(ref)) {
            sp.self_setup = true;
            sp.shares = int32_t(shares);
            sp.rows_per = rows;
        }
    }
    if (!sp.self_setup) {
        const int64_t n_transit =
            npv >= 512 && ntiles >= 16 ? int64_t(cap) : std::min<int64_t>(cap, 2048);
        sp.shares =
            int32_t(std::min<int64_t>({16, max_sh, std::max<int64_t>(1, n_transit / npv)}));
    }
    sp.blocks = int64_t(npv) * sp.shares + ntiles * ((npv + sp.rows_per - 1) / sp.rows_per);
    return sp;
}

hipError_t launch_forward_split(const rr_tables* t, const rr_series* se, const SplitPlan& sp,
                                const double* pv, int32_t npv, int32_t npar,
                                const PvConst* pvc, int32_t precision, void* out,
                                hipStream_t s) {
    const GridDev g = grid_dev(t);
    FwdJob job = {};
    job.times = se->times; job.lcids = se->lcids; job.pv = pv; job.pvc = pvc; job.out = out;
    job.npt = se->npt; job.npar = npar; job.pv0 = 0; job.npv = npv;
    job.ntiles = (se->npt + kFwdTile - 1) / kFwdTile; job.max_nss = se->max_nss; job.spread = 1;
    if (se->max_nss != 1) return hipErrorInvalidValue;    // see split_preferred
    if (!sp.self_setup && !pvc) return hipErrorInvalidValue;
    if (sp.shares < 1 || sp.rows_per < 1) return hipErrorInvalidValue;
    const int64_t ntiles = job.ntiles;
    const int64_t blocks =
        int64_t(npv) * sp.shares + ntiles * ((npv + sp.rows_per - 1) / sp.rows_per);
    if (blocks != sp.blocks || blocks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    SplitInfo si;
    si.lcs = se->lcs;
    si.buckets = se->buckets;
    si.shares = sp.shares;
    si.rows_per = sp.rows_per;
    si.k_lo = t->grid.k0;
    si.k_hi = t->grid.k1;
    const dim3 grid{unsigned(blocks), 1u, 1u};
    const dim3 block{unsigned(kFwdBlock), 1u, 1u};
    const KernelEvents ev = kernel_events();
    if (precision == RR_FP64) {
        if (sp.self_setup)
            launch_timed(k_forward_split<double, true>, grid, block, 0, s, ev.before, ev.after,
                         job, se->lc, g, t->T64, t->inv_istar, si);
        else
            launch_timed(k_forward_split<double, false>, grid, block, 0, s, ev.before, ev.after,
                         job, se->lc, g, t->T64, t->inv_istar, si);
    } else {
        if (sp.self_setup)
            launch_timed(k_forward_split<float, true>, grid, block, 0, s, ev.before, ev.after,
                         job, se->lc, g, t->T32, t->inv_istar, si);
        else
            launch_timed(k_forward_split<float, false>, grid, block, 0, s, ev.before, ev.after,
                         job, se->lc, g, t->T32, t->inv_istar, si);
    }
    return hipGetLastError();
}

hipError_t launch_forward_jobs(const rr_tables* t, const JobTable& jt, int32_t nblocks_total,
                               int32_t precision, hipStream_t s) {
    if (nblocks_total <= 0 || jt.njobs <= 0) return hipSuccess;
    const GridDev g = grid_dev(t);
    bool sub = false;
    for (int q = 0; q < jt.njobs; ++q) sub = sub || jt.j[q].max_nss > 1;
    const dim3 grid{unsigned(nblocks_total), 1u, 1u};
    if (precision == RR_FP64) {
        if (sub)
            hipLaunchKernelGGL((k_forward_jobs<double, true>), grid, dim3(kFwdBlock), 0, s, jt, g,
                               t->T64, t->inv_istar);
        else
            hipLaunchKernelGGL((k_forward_jobs<double, false>), grid, dim3(kFwdBlock), 0, s, jt, g,
                               t->T64, t->inv_istar);
    } else {
        if (sub)
            hipLaunchKernelGGL((k_forward_jobs<float, true>), grid, dim3(kFwdBlock), 0, s, jt, g,
                               t->T32, t->inv_istar);
        else
            hipLaunchKernelGGL((k_forward_jobs<float, false>), grid, dim3(kFwdBlock), 0, s, jt, g,
                               t->T32, t->inv_istar);
    }
    return hipGetLastError();
}

hipError_t launch_flux_at_z(const rr_tables* t, const double* z, const double* kv,
                           double kconst, int64_t n, int32_t pb, int32_t precision, void* out,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const GridDev g = grid_dev(t);
    const dim3 grid(unsigned((n + kBlock - 1) / kBlock));
    if (precision == RR_FP64)
        hipLaunchKernelGGL(k_flux_at_z<double>, grid, dim3(kBlock), 0, s, z, kv, kconst, n, pb,
                           g, t->grid.k1, t->T64, t->inv_istar, static_cast<double*>(out));
    else
        hipLaunchKernelGGL(k_flux_at_z<float>, grid, dim3(kBlock), 0, s, z, kv, kconst, n, pb,
                           g, t->grid.k1, t->T32, t->inv_istar, static_cast<float*>(out));
    return hipGetLastError();
}

hipError_t launch_pv_setup_jobs(const rr_tables* t, const SetupTable& st, int32_t nthreads,
                                hipStream_t s) {
    if (nthreads <= 0 || st.njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pv_setup_jobs, dim3(nblocks(nthreads)), dim3(kBlock), 0, s, st,
                       t->grid.k0, t->grid.k1);
    return hipGetLastError();
}

}  // namespace rr
