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
//   k_forward   one workgroup per (parameter vector, tile of 2048 times),
//               lanes along time so loads of the shared time array and the
//               stores of out[pv][t] are coalesced.  Pass 1 reduces each
//               mid-exposure time to an offset from conjunction (FP64) and
//               writes 1 for exposures entirely outside the window; if any
//               exposure of the tile overlaps it, the workgroup builds the
//               k-interpolated LD vectors of its parameter vector in LDS
//               (Sect. 3.1.2) and pass 2 evaluates those exposures:
//               per subsample, Kepler orbit -> z -> g-interpolation in LDS
//               (Sect. 3.1.1) x lens area (Eq. 5) -> mean over subsamples.
//
// The kernels are templated on the bulk real type: double (RR_FP64) or float
// (RR_MIXED: the time reduction stays FP64, the rest is FP32).
#include "rr_device.h"

namespace rr {
namespace {

__global__ void k_pv_setup(const double* __restrict__ pv, int32_t npv,
                           int32_t npar, double k0, double k1,
                           PvConst* __restrict__ out) {
    const int ipv = blockIdx.x * blockDim.x + threadIdx.x;
    if (ipv >= npv) return;
    out[ipv] = make_pv_const(pv + int64_t(ipv) * npar, npar - 6, k0, k1);
}

// The work of one workgroup: population row ipv, time tile `tile`.
template <typename R>
__device__ inline void forward_block(const FwdJob& job, const LcInfo& lc, int ipv,
                                     int tile, const GridDev& g,
                                     const R* __restrict__ T,
                                     const double* __restrict__ inv_istar, R* ldw) {
    const int tid = threadIdx.x;
    const int npt = job.npt, npar = job.npar;
    const double* __restrict__ times = job.times;
    const int32_t* __restrict__ lcids = job.lcids;
    const double* __restrict__ pv = job.pv;
    const int t_base = tile * kTile + tid;
    R* __restrict__ orow = static_cast<R*>(job.out) + int64_t(ipv) * npt;
    const PvConst p = job.pvc[ipv];

    if (!(p.flags & kValid)) {
        for (int j = 0; j < kTimesPerThread; ++j) {
            const int it = t_base + j * kBlock;
            if (it < npt) orow[it] = R(NAN);
        }
        return;
    }

    // Pass 1: exposures that cannot overlap the star get F = 1 now.
    uint32_t todo = 0;
    const int tfirst = tile * kTile;
    if (!lcids && tfirst + kTile <= npt) {
        // Whole tile in range, one light curve: no bounds or light-curve
        // checks; phase g = t/P + c0 with c0 = -t0/P - (window start) by one
        // FMA; every output is written as 1 here and pass 2 overwrites the
        // exposures that overlap the star.
        const double* tp = times + tfirst + tid;
        R* op = orow + tfirst + tid;
        double tv[kTimesPerThread];
#pragma unroll
        for (int j = 0; j < kTimesPerThread; ++j) tv[j] = tp[j * kBlock];
        const double hw = 0.5 * lc.exptime[0] * p.invP;
        const double c0 = -p.t0 * p.invP - (p.flo - hw);
        const double wn = p.wn + 2.0 * hw;
#pragma unroll
        for (int j = 0; j < kTimesPerThread; ++j) {
            const double gph = fma(tv[j], p.invP, c0);
            if (gph - floor(gph) < wn) todo |= 1u << j;
            op[j * kBlock] = R(1);
        }
    } else {
        double tv[kTimesPerThread];
        int lv[kTimesPerThread];
#pragma unroll
        for (int j = 0; j < kTimesPerThread; ++j) {
            const int it = t_base + j * kBlock;
            tv[j] = it < npt ? times[it] : 0.0;
            lv[j] = (lcids && it < npt) ? lcids[it] : 0;
        }
        const double hw0 = 0.5 * lc.exptime[0] * p.invP;
#pragma unroll
        for (int j = 0; j < kTimesPerThread; ++j) {
            const int it = t_base + j * kBlock;
            if (it >= npt) continue;
            const int l = lv[j];
            if (l < 0 || l >= lc.nlc) { orow[it] = R(NAN); continue; }
            const double hw = lcids ? 0.5 * lc.exptime[l] * p.invP : hw0;
            if (in_phase_window((tv[j] - p.t0) * p.invP, p, hw)) todo |= 1u << j;
            else orow[it] = R(1);
        }
    }
    // Workgroup vote: does any exposure of the tile overlap the window?
    __shared__ int wave_any[kBlock / 64];
    const int wany = __any(todo != 0);
    if ((tid & 63) == 0) wave_any[tid >> 6] = wany;
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) any |= wave_any[w] != 0;
    if (!any) return;

    // k-interpolated LD-weighted vectors of this parameter vector, one per
    // passband (Sect. 3.1.2): ldw = (1 - ak) T[ik] + ak T[ik+1].
    for (int pb = 0; pb < g.npb; ++pb) {
        const double u = (pv[int64_t(ipv) * npar + 6 + pb] - g.k0) / g.dk;
        int ik = int(floor(u));
        ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
        const R ak = R(u - ik);
        const R* t0r = T + (int64_t(pb) * g.nk + ik) * g.ng;
        for (int m = tid; m < g.ng; m += kBlock)
            ldw[pb * g.ng + m] = (R(1) - ak) * t0r[m] + ak * t0r[g.ng + m];
    }
    __syncthreads();

    // Pass 2: exposures that may overlap the star.
    const OrbitR<R> orb(p);
    const R gscale = R(g.gscale);
    while (todo) {
        const int j = __builtin_ctz(todo);
        todo &= todo - 1;
        const int it = t_base + j * kBlock;
        const int l = lcids ? lcids[it] : 0;          // reloaded: keeps pass 1's
        const int pb = lc.pb[l];                      // registers free here
        const int nss = lc.nss[l];
        const double ex = lc.exptime[l];
        const double t = times[it];
        const R k = R(pv[int64_t(ipv) * npar + 6 + pb]);
        const R onepk = R(1) + k;
        const R inv1pk = R(1) / onepk;
        const R istar_inv = R(inv_istar[pb]);
        const R* lw = ldw + pb * g.ng;
        R acc = R(0);
        for (int s = 0; s < nss; ++s) {
            const double x = (t + ex * ((s + 0.5) / nss - 0.5)) - p.t0;
            const double u = x * p.invP;
            if (!in_phase_window(u, p, 0.0)) continue;
            const double dt = x - p.P * rint(u);
            bool front;
            const R z = separation<R>(R(dt), orb, &front);
            if (!front || !(z < onepk)) continue;
            const R v = z * inv1pk * gscale;
            int m = int(v);
            m = m > g.ng - 2 ? g.ng - 2 : m;
            const R al = v - R(m);
            const R ip = (R(1) - al) * lw[m] + al * lw[m + 1];
            acc += ip * lens_area<R>(R(1), k, z) * istar_inv;
        }
        orow[it] = R(1) - acc / R(nss);
    }
}

// One population (rr_evaluate): workgroup (x, y) -> row pv0 + y, tile x.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_forward(FwdJob job, LcInfo lc, GridDev g,
                                                    const R* __restrict__ T,
                                                    const double* __restrict__ inv_istar) {
    extern __shared__ unsigned char smem_raw[];
    const int ipv = job.pv0 + blockIdx.y;
    const int tile = blockIdx.x;
    forward_block<R>(job, lc, ipv, tile, g, T, inv_istar, reinterpret_cast<R*>(smem_raw));
}

// Grouped launch (serving): workgroup b belongs to the last job whose
// block0 <= b; jobs come from several requests and time series.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_forward_jobs(JobTable jt, GridDev g,
                                                         const R* __restrict__ T,
                                                         const double* __restrict__ inv_istar) {
    extern __shared__ unsigned char smem_raw[];
    const int b = blockIdx.x;
    int jj = 0;
    for (int q = 1; q < jt.njobs; ++q)
        if (jt.j[q].block0 <= b) jj = q;
    const FwdJob& job = jt.j[jj];
    const int local = b - job.block0;
    const int ipv = job.pv0 + local / job.ntiles;
    const int tile = local - (local / job.ntiles) * job.ntiles;
    forward_block<R>(job, *job.lc, ipv, tile, g, T, inv_istar, reinterpret_cast<R*>(smem_raw));
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
    hipLaunchKernelGGL(k_pv_setup, dim3(nblocks(npv)), dim3(kBlock), 0, s, pv, npv,
                       npar, t->grid.k0, t->grid.k1, pvc);
    return hipGetLastError();
}

hipError_t launch_forward(const rr_tables* t, const double* times,
                          const int32_t* lcids, int32_t npt, const LcInfo& lc,
                          const double* pv, int32_t npv, int32_t npar,
                          const PvConst* pvc, int32_t precision, void* out,
                          hipStream_t s) {
    const GridDev g = grid_dev(t);
    FwdJob job;
    job.times = times; job.lcids = lcids; job.lc = nullptr; job.pv = pv; job.pvc = pvc;
    job.out = out; job.npt = npt; job.npar = npar; job.pv0 = 0; job.npv = npv;
    job.ntiles = (npt + kTile - 1) / kTile; job.block0 = 0;
    const KernelEvents ev = kernel_events();
    if (ev.before) {
        hipError_t e = hipEventRecord(ev.before, s);
        if (e != hipSuccess) return e;
    }
    // rows along grid y, at most 65535 per launch
    for (int32_t r0 = 0; r0 < npv; r0 += 65535) {
        job.pv0 = r0;
        const dim3 grid(unsigned(job.ntiles), unsigned(npv - r0 < 65535 ? npv - r0 : 65535));
        if (precision == RR_FP64) {
            const size_t lds = sizeof(double) * size_t(g.npb) * g.ng;
            hipLaunchKernelGGL(k_forward<double>, grid, dim3(kBlock), lds, s, job, lc, g,
                               t->T64, t->inv_istar);
        } else {
            const size_t lds = sizeof(float) * size_t(g.npb) * g.ng;
            hipLaunchKernelGGL(k_forward<float>, grid, dim3(kBlock), lds, s, job, lc, g,
                               t->T32, t->inv_istar);
        }
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && ev.after) e = hipEventRecord(ev.after, s);
    return e;
}

hipError_t launch_forward_jobs(const rr_tables* t, const JobTable& jt, int32_t nblocks_total,
                               int32_t precision, hipStream_t s) {
    if (nblocks_total <= 0 || jt.njobs <= 0) return hipSuccess;
    const GridDev g = grid_dev(t);
    if (precision == RR_FP64) {
        const size_t lds = sizeof(double) * size_t(g.npb) * g.ng;
        hipLaunchKernelGGL(k_forward_jobs<double>, dim3(unsigned(nblocks_total)), dim3(kBlock),
                           lds, s, jt, g, t->T64, t->inv_istar);
    } else {
        const size_t lds = sizeof(float) * size_t(g.npb) * g.ng;
        hipLaunchKernelGGL(k_forward_jobs<float>, dim3(unsigned(nblocks_total)), dim3(kBlock),
                           lds, s, jt, g, t->T32, t->inv_istar);
    }
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
