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

__global__ void k_pv_setup(const double* __restrict__ pv, int32_t npv,
                           int32_t npar, double k0, double k1, double k_small,
                           PvConst* __restrict__ out) {
    const int ipv = blockIdx.x * blockDim.x + threadIdx.x;
    if (ipv >= npv) return;
    out[ipv] = make_pv_const(pv + int64_t(ipv) * npar, npar - 6, k0, k1, k_small);
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
        // the same nss in [2, 32], spread the subsamples over the lanes --
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
        if (job.spread && nmin == nmax && N >= 2 && N <= 32) {
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
    sj.pvc[ipv] = make_pv_const(sj.pv + int64_t(ipv) * sj.npar, sj.npar - 6, k0, k1);
}

inline unsigned nblocks(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_pv_setup(const rr_tables* t, const double* pv, int32_t npv,
                           int32_t npar, PvConst* pvc, hipStream_t s) {
    return launch_pv_setup_k(pv, npv, npar, t->grid.k0, t->grid.k1, pvc, s);
}

hipError_t launch_pv_setup_k(const double* pv, int32_t npv, int32_t npar, double k_lo,
                             double k_hi, PvConst* pvc, hipStream_t s, double k_small) {
    hipLaunchKernelGGL(k_pv_setup, dim3(nblocks(npv)), dim3(kBlock), 0, s, pv, npv,
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
