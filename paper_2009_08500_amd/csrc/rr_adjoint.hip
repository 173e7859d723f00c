// rr_adjoint.hip -- Gaussian log-likelihood of the population light curves
// and its hand-written adjoint: gradients with respect to every parameter
// of each row and to the shared LD profile samples.
//
//   logL_pv = -1/2 sum_t ((d_t - F_t)/sigma)^2,   psi_t = (d_t - F_t)/sigma^2
//   dlogL/dtheta = sum_t psi_t dF_t/dtheta,       F_t = 1 - mean_s delta_s
//   delta = ip(g, k) a(z, k) / I_star                               (Eq. 5)
//
// k_adjoint     workgroups of two wave64 over tiles of 1024 times of one
//               parameter vector (one tile each without the profile
//               gradient), lanes along time.  Out-of-window exposures only
//               add their residual to logL.  For the others the subsample
//               loop evaluates delta together with d delta/dz and
//               d delta/dk, and z's derivatives through the transit-centred
//               Kepler solution (dE/dM = 1/(1 - e cos E),
//               dE/de = sin E/(1 - e cos E)); the lens area gives
//               da/dz = -chord and da/dk = 2 k kappa_0.  Per-lane sums are
//               FP64 and reduced in a fixed order (butterfly within the wave,
//               then waves in order) to one partial per workgroup.  With the
//               profile gradient requested each workgroup runs several
//               consecutive tiles, and a second subsample loop scatters
//               psi-weighted lerp weights into its wave's own LDS copy of
//               d logL / d ldw and d logL / d I_star (no two waves share an
//               address, and one wave's LDS additions complete in program
//               order); the copies are added in wave order and stored once
//               per workgroup, and k_prof_seg_sum adds a vector's workgroups
//               in order.  Every sum therefore has an order fixed by the
//               inputs alone: the gradient is bitwise reproducible.
//   k_adjoint_reduce   per parameter vector, the workgroup partials in a
//               fixed order (lanes over tiles, then a butterfly) -> logL and
//               the gradient row.
//   k_table_grad d logL / d T[pb][i][m] from the per-vector d logL / d ldw
//               through the k-interpolation weights: chunks of vectors in
//               parallel, each in order, then the chunks in order.
//   k_ldp_grad   d logL / d ldp = sum_{i,m} W[i][j][m] dT[i][m] (fixed tree).
//   k_prof_grad  back through the profile interpolation and I_star (both
//               linear in the samples) to d logL / d I_s.
#include <algorithm>

#include "rr_device.h"

namespace rr {
namespace {

constexpr int kNq = 7;   // logL + 6 orbit parameters (k gradients follow)

// Lens area and its partial derivatives for the unit star (R = 1).
template <typename R>
__device__ inline R lens_area_grad(R k, R z, R* Az, R* Ak) {
    using N = Num<R>;
    if (z >= R(1) + k) { *Az = R(0); *Ak = R(0); return R(0); }
    if (z <= R(1) - k) { *Az = R(0); *Ak = R(2) * N::pi * k; return N::pi * k * k; }
    if (z <= k - R(1)) { *Az = R(0); *Ak = R(0); return N::pi; }
    R a = R(1), b = k, s = z, tmp;
    if (a < b) { tmp = a; a = b; b = tmp; }
    if (b < s) { tmp = b; b = s; s = tmp; }
    if (a < b) { tmp = a; a = b; b = tmp; }
    R prod = (a + (b + s)) * (s - (a - b)) * (s + (a - b)) * (a + (b - s));
    prod = prod > R(0) ? prod : R(0);
    const R area2 = R(0.5) * N::sqrt_(prod);
    const R invz = N::rcp_(z);
    const R h = area2 * invz;
    const R x1 = (z * z + (R(1) - k) * (R(1) + k)) * (R(0.5) * invz);
    const R x0 = z - x1;
    const R k1 = N::atan2_(h, x1);
    const R k0 = N::atan2_(h, x0);
    *Az = R(-2) * h;
    *Ak = R(2) * k * k0;
    return k1 + k * k * k0 - area2;
}

// Per-vector derivative constants (FP64, from the row and its PvConst).
struct PvDeriv {
    double dMtr_de, dMtr_dw, dci_da, dci_db, dci_de, dci_dw, dq_de;
};

__device__ inline PvDeriv make_pv_deriv(const PvConst& p, double b) {
    PvDeriv d;
    const double e = p.e, sw = p.sinw, cw = p.cosw, q = p.q, a = p.a;
    const double den = 1.0 + e * sw, ome2 = 1.0 - e * e;
    const double dEtr_dw = -(1.0 - e * p.cE) / q;
    const double dEtr_de = -cw / (den * q);
    d.dMtr_dw = (1.0 - e * p.cE) * dEtr_dw;
    d.dMtr_de = (1.0 - e * p.cE) * dEtr_de - p.sE;
    d.dci_da = -p.cosi / a;
    d.dci_db = den / (a * ome2);
    d.dci_de = b / a * (sw * ome2 + 2.0 * e * den) / (ome2 * ome2);
    d.dci_dw = b * e * cw / (a * ome2);
    d.dq_de = -e / q;
    return d;
}

template <typename R>
struct DerivR {
    R dMtr_de, dMtr_dw, dci_da, dci_db, dci_de, dci_dw, dq_de;
    __device__ explicit DerivR(const PvDeriv& d)
        : dMtr_de(R(d.dMtr_de)), dMtr_dw(R(d.dMtr_dw)), dci_da(R(d.dci_da)),
          dci_db(R(d.dci_db)), dci_de(R(d.dci_de)), dci_dw(R(d.dci_dw)),
          dq_de(R(d.dq_de)) {}
};

// Separation and dz/d(t0, P, a, b, e, w) for one subsample.  x = t_s - t0
// (for dM/dP = -n x / P).  Same transit-centred solve as the forward path.
template <typename R>
__device__ inline R separation_grad(R dt, R x, const OrbitR<R>& o,
                                    const DerivR<R>& dv, R invP, bool* front,
                                    R dz[6]) {
    using N = Num<R>;
    const R dM = o.n * dt;
    R s2, c2;
    if (o.e > R(0)) kepler_offset<R>(dM, o.e, o.sE, o.cE, &s2, &c2);
    else sincos_small(R(0.5) * dM, &s2, &c2);
    const R sd = R(2) * s2 * c2;
    const R cm1 = R(-2) * s2 * s2;
    const R dc = o.cE * cm1 - o.sE * sd;
    const R ds = o.sE * cm1 + o.cE * sd;
    const R X = -o.a * (dc * o.cosw - o.q * ds * o.sinw);
    const R rho = o.rtr + o.a * (dc * o.sinw + o.q * ds * o.cosw);
    const R Y = -rho * o.cosi;
    *front = rho > R(0);
    const R z = N::sqrt_(X * X + Y * Y);
    // derivatives (absolute cos E, sin E are fine here)
    const R cE = o.cE + dc, sE = o.sE + ds;
    const R iE = N::rcp_(R(1) - o.e * cE);
    const R XE = o.a * (sE * o.cosw + o.q * cE * o.sinw);
    const R rE = o.a * (o.q * cE * o.cosw - sE * o.sinw);
    const R Xe = o.a * (o.cosw + dv.dq_de * sE * o.sinw);
    const R re = o.a * (dv.dq_de * sE * o.cosw - o.sinw);
    const R inva = N::rcp_(o.a);
    const R iz = z > R(0) ? N::rcp_(z) : R(0);
    // dE/dtheta for t0, P, e, w
    const R dE_t0 = -o.n * iE;
    const R dE_P = -o.n * (x * invP) * iE;
    const R dE_e = (dv.dMtr_de + sE) * iE;
    const R dE_w = dv.dMtr_dw * iE;
    auto dzdt = [&](R dX, R drho, R dci) {
        const R dY = -o.cosi * drho - rho * dci;
        return (X * dX + Y * dY) * iz;
    };
    dz[0] = dzdt(XE * dE_t0, rE * dE_t0, R(0));
    dz[1] = dzdt(XE * dE_P, rE * dE_P, R(0));
    dz[2] = dzdt(X * inva, rho * inva, dv.dci_da);
    dz[3] = dzdt(R(0), R(0), dv.dci_db);
    dz[4] = dzdt(XE * dE_e + Xe, rE * dE_e + re, dv.dci_de);
    dz[5] = dzdt(XE * dE_w + rho, rE * dE_w - X, dv.dci_dw);
    return z;
}

template <typename T>
__device__ inline T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup (ipv, c) = blockIdx.x = ipv nparts + c handles the time tiles
// [c tpp, (c + 1) tpp) of vector ipv (tpp = tiles per part, 1 without the
// profile gradient).  Per tile, pass 1 adds the residuals of exposures that
// cannot overlap the star; pass 2 runs the subsample loop of the others.
// The LDS tables (ldw and its k-derivative) are built at the first tile with
// in-window work.  Per-lane sums go to one partial per workgroup; with the
// profile gradient the workgroup's LDS sums of d logL / d ldw and
// d logL / d I_star are stored once at the end, to slot (ipv, c) of
// seg_gw / seg_gi with flag 1 (flag 0 and nothing else if no exposure was in
// the window), or, with seg_flag NULL (one part per vector), as the final
// per-vector sums.
// sum over c = 0 .. n-1, in order, of (flag(c) ? val(c) : 0), with eight
// flags and then eight values loaded at a time (their loads are independent,
// so a flagged sum over many parts costs n/8 memory round trips, not n)
template <typename F, typename V>
__device__ inline double flagged_sum(int n, F flag, V val, bool* any = nullptr) {
    double s = 0.0;
    bool a = false;
    for (int c0 = 0; c0 < n; c0 += 8) {
        bool f[8];
        double v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) f[b] = c0 + b < n && flag(c0 + b);
#pragma unroll
        for (int b = 0; b < 8; ++b) v[b] = f[b] ? val(c0 + b) : 0.0;
#pragma unroll
        for (int b = 0; b < 8; ++b) { s += v[b]; a = a || f[b]; }
    }
    if (any) *any = a;
    return s;
}

template <typename R, int NPBT, bool kProf>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint(
    const double* __restrict__ times, const int32_t* __restrict__ lcids,
    int32_t npt, LcInfo lc, const double* __restrict__ pv, int32_t npar,
    const PvConst* __restrict__ pvc, GridDev g, const R* __restrict__ T,
    const double* __restrict__ inv_istar, const R* __restrict__ obs,
    double inv_sig2, int32_t ntiles, int32_t nparts, int32_t tpp, int32_t want_grad,
    const double* __restrict__ wprof, double* __restrict__ partials,
    double* __restrict__ seg_gw, double* __restrict__ seg_gi, int32_t* __restrict__ seg_flag,
    int32_t rows_per_vector) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int kJ = adj_times_per_thread(kProf, sizeof(R) == 8);   // times per thread
    constexpr int kTile = kAdjBlock * kJ;
    constexpr int kWaves = kAdjBlock / 64;
    const int npb = g.npb, ng = g.ng;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    R* ldw = reinterpret_cast<R*>(smem_raw);                    // [npb][ng]
    R* dTk = ldw + npb * ng;                                    // [npb][ng]
    // per-wave copies of d logL / d ldw [kWaves][npb][ng] and
    // d logL / d I_star [kWaves][npb] (profile instantiation only)
    double* gw_all = reinterpret_cast<double*>(
        smem_raw + ((2 * sizeof(R) * npb * ng + 7) / 8) * 8);
    double* gi_all = gw_all + kWaves * npb * ng;
    double* gw = gw_all + wave * npb * ng;                      // this wave's copy
    double* gi = gi_all + wave * npb;
    __shared__ double red[kWaves][kNq + NPBT];
    __shared__ int wave_any[2][kWaves];                         // by tile parity
    static_assert(sizeof(red) + sizeof(wave_any) <= kAdjStaticLds,
                  "static LDS must fit the reserve the host budget assumes");

    const int64_t slot = blockIdx.x;
    const int ipv = int(slot / nparts);
    const int c = int(slot - int64_t(ipv) * nparts);
    const int nq = kNq + npb;
    double* part = partials + slot * nq;
    const PvConst p = pvc[ipv];

    if (!(p.flags & kValid)) {
        if (tid < nq) part[tid] = NAN;
        if (kProf) {
            if (seg_flag) {
                if (tid == 0) seg_flag[slot] = 0;
            } else {
                for (int idx = tid; idx < npb * ng; idx += kAdjBlock)
                    seg_gw[slot * npb * ng + idx] = 0.0;
                if (tid < npb) seg_gi[slot * npb + tid] = 0.0;
            }
        }
        return;
    }

    double ll = 0.0;
    double ga[6] = {0, 0, 0, 0, 0, 0};
    double gk[NPBT];
#pragma unroll
    for (int q = 0; q < NPBT; ++q) gk[q] = 0.0;
    bool ready = false;                  // LDS tables built (uniform)

    // without the profile gradient: exactly one tile, tile c
    const int tile0 = kProf ? c * tpp : c;
    const int tile_end = kProf ? min(ntiles, (c + 1) * tpp) : c + 1;
    for (int tile = tile0; tile < tile_end; ++tile) {
        const int t_base = tile * kTile + tid;
        // Pass 1: residuals of exposures that cannot overlap the star.
        uint32_t todo = 0;
        const int tfirst = tile * kTile;
        if (!lcids && tfirst + kTile <= npt) {
            // whole tile in range, one light curve (see forward_block)
            double tv[kJ], ov[kJ];
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                tv[j] = times[tfirst + tid + j * kAdjBlock];
                ov[j] = double(obs[tfirst + tid + j * kAdjBlock]);
            }
            const double hw = 0.5 * lc.exptime[0] * p.invP;
            const double c0 = -p.t0 * p.invP - (p.flo - hw);
            const double wn = p.wn + 2.0 * hw;
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const double gph = fma(tv[j], p.invP, c0);
                if (gph - floor(gph) < wn) {
                    todo |= 1u << j;
                } else {
                    const double r = ov[j] - 1.0;
                    ll -= 0.5 * r * r * inv_sig2;
                }
            }
        } else {
            for (int j = 0; j < kJ; ++j) {
                const int it = t_base + j * kAdjBlock;
                if (it >= npt) continue;
                const int l = lcids ? lcids[it] : 0;
                if (l < 0 || l >= lc.nlc) { ll = NAN; continue; }
                if (in_phase_window((times[it] - p.t0) * p.invP, p, 0.5 * lc.exptime[l] * p.invP)) {
                    todo |= 1u << j;
                } else {
                    const double r = double(obs[it]) - 1.0;
                    ll -= 0.5 * r * r * inv_sig2;
                }
            }
        }
        // wave_any is double-buffered by tile parity: a wave that runs ahead
        // to the next tile writes the other half while slower waves read
        const int par = tile & 1;
        const int wany = __any(todo != 0);
        if (lane == 0) wave_any[par][wave] = wany;
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int w = 0; w < kAdjBlock / 64; ++w) any |= wave_any[par][w] != 0;
        if (!any) continue;

        if (!ready) {
            for (int idx = tid; idx < npb * ng; idx += kAdjBlock) {
                const int pb = idx / ng, m = idx - pb * ng;
                const double u = (pv[int64_t(ipv) * npar + 6 + pb] - g.k0) / g.dk;
                int ik = int(floor(u));
                ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
                const R ak = R(u - ik);
                // the shared table's two rows, or the vector's own copies
                const R* t0r = rows_per_vector ? T + (int64_t(ipv) * npb + pb) * 2 * ng
                                               : T + (int64_t(pb) * g.nk + ik) * ng;
                ldw[idx] = (R(1) - ak) * t0r[m] + ak * t0r[ng + m];
                dTk[idx] = (t0r[ng + m] - t0r[m]) * R(g.inv_dk);
            }
            if (kProf) {
                for (int idx = tid; idx < kWaves * npb * ng; idx += kAdjBlock) gw_all[idx] = 0.0;
                if (tid < kWaves * npb) gi_all[tid] = 0.0;
            }
            __syncthreads();
            ready = true;
        }

        const OrbitR<R> orb(p);
        const DerivR<R> dv(make_pv_deriv(p, pv[int64_t(ipv) * npar + 3]));
        const R gscale = R(g.gscale);
        const R invP = R(p.invP);

        // Pass 2: the exposures that may overlap the star.
        while (todo) {
            const int j = __builtin_ctz(todo);
            todo &= todo - 1;
            const int it = t_base + j * kAdjBlock;
            const int l = lcids ? lcids[it] : 0;
            const int pb = lc.pb[l];
            const int nss = lc.nss[l];
            const double ex = lc.exptime[l];
            const double t = times[it];
            const R k = R(pv[int64_t(ipv) * npar + 6 + pb]);
            const R onepk = R(1) + k;
            const R inv1pk = R(1) / onepk;
            const R istar_inv =
                R(inv_istar[rows_per_vector ? int64_t(ipv) * npb + pb : int64_t(pb)]);
            const R* lw = ldw + pb * ng;
            const R* dk_ = dTk + pb * ng;
            R acc = R(0);
            R gt[6] = {0, 0, 0, 0, 0, 0};
            R gkt = R(0);
            const double inv_nss = 1.0 / nss;
            for (int s = 0; s < nss; ++s) {
                const double x = (t + ex * ((s + 0.5) * inv_nss - 0.5)) - p.t0;
                const double u = x * p.invP;
                if (!in_phase_window(u, p, 0.0)) continue;
                const double dt = x - p.P * rint(u);
                bool front;
                R dz[6];
                const R z = separation_grad<R>(R(dt), R(x), orb, dv, invP, &front, dz);
                if (!front || !(z < onepk)) continue;
                const R v = z * inv1pk * gscale;
                int m = int(v);
                m = m > ng - 2 ? ng - 2 : m;
                const R al = v - R(m);
                const R ip = (R(1) - al) * lw[m] + al * lw[m + 1];
                R Az, Ak;
                const R A = lens_area_grad<R>(k, z, &Az, &Ak);
                acc += ip * A * istar_inv;
                if (want_grad) {
                    const R slope = (lw[m + 1] - lw[m]) * gscale;
                    const R ddz = (slope * inv1pk * A + ip * Az) * istar_inv;
                    const R ipk = slope * (-z * inv1pk * inv1pk) +
                                  (R(1) - al) * dk_[m] + al * dk_[m + 1];
                    gkt += (ipk * A + ip * Ak) * istar_inv;
#pragma unroll
                    for (int q = 0; q < 6; ++q) gt[q] += ddz * dz[q];
                }
            }
            // residual in FP64: d - F = (d - 1) + mean delta
            const double mean_delta = double(acc) / nss;
            const double r = (double(obs[it]) - 1.0) + mean_delta;
            ll -= 0.5 * r * r * inv_sig2;
            const double wgt = -(r * inv_sig2) / nss;       // dlogL / d delta_s
            if (want_grad) {
#pragma unroll
                for (int q = 0; q < 6; ++q) ga[q] += wgt * double(gt[q]);
#pragma unroll
                for (int q = 0; q < NPBT; ++q) gk[q] += (q == pb) ? wgt * double(gkt) : 0.0;
            }
            if (kProf) {
                // psi-weighted lerp weights of each overlapping subsample
                const double cw = wgt * (wprof ? wprof[ipv] : 1.0);
                for (int s = 0; s < nss; ++s) {
                    const double x = (t + ex * ((s + 0.5) * inv_nss - 0.5)) - p.t0;
                    const double u = x * p.invP;
                    if (!in_phase_window(u, p, 0.0)) continue;
                    const double dt = x - p.P * rint(u);
                    bool front;
                    const R z = separation<R>(R(dt), orb, &front);
                    if (!front || !(z < onepk)) continue;
                    const R v = z * inv1pk * gscale;
                    int m = int(v);
                    m = m > ng - 2 ? ng - 2 : m;
                    const double al = double(v - R(m));
                    const double A = double(lens_area<R>(R(1), k, z)) * double(istar_inv);
                    const double cc = cw * A;
                    atomicAdd(&gw[pb * ng + m], (1.0 - al) * cc);
                    atomicAdd(&gw[pb * ng + m + 1], al * cc);
                    const double ip = (1.0 - al) * double(lw[m]) + al * double(lw[m + 1]);
                    atomicAdd(&gi[pb], -cw * ip * A * double(istar_inv));
                }
            }
        }
    }

    if (kProf) {
        __syncthreads();                 // every wave's LDS additions done
        // the waves' copies added in wave order
        auto wsum = [&](const double* base, int stride, int idx) {
            double v = base[idx];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) v += base[w * stride + idx];
            return v;
        };
        double* out = seg_gw + slot * npb * ng;
        if (seg_flag) {
            if (tid == 0) seg_flag[slot] = ready ? 1 : 0;
            if (ready) {
                for (int idx = tid; idx < npb * ng; idx += kAdjBlock)
                    out[idx] = wsum(gw_all, npb * ng, idx);
                if (tid < npb) seg_gi[slot * npb + tid] = wsum(gi_all, npb, tid);
            }
        } else {
            for (int idx = tid; idx < npb * ng; idx += kAdjBlock)
                out[idx] = ready ? wsum(gw_all, npb * ng, idx) : 0.0;
            if (tid < npb) seg_gi[slot * npb + tid] = ready ? wsum(gi_all, npb, tid) : 0.0;
        }
    }

    // fixed-order reduction of the per-lane sums
    double vals[kNq + NPBT];
    vals[0] = ll;
#pragma unroll
    for (int q = 0; q < 6; ++q) vals[1 + q] = ga[q];
#pragma unroll
    for (int q = 0; q < NPBT; ++q) vals[kNq + q] = gk[q];
#pragma unroll
    for (int q = 0; q < kNq + NPBT; ++q) {
        const double v = wave_sum(vals[q]);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (tid < nq) {
        double sum = 0.0;
        for (int w = 0; w < kAdjBlock / 64; ++w) sum += red[w][tid];
        part[tid] = sum;
    }
}

// d logL / d ldw_row and d logL / d I_star per vector: the flagged parts of
// k_adjoint added in part order.  Thread idx < npv npb ng sums
// one ldw entry, the next npv npb threads one I_star entry each.
__global__ void k_prof_seg_sum(const double* __restrict__ seg_gw,
                               const double* __restrict__ seg_gi,
                               const int32_t* __restrict__ seg_flag, int32_t npv, int32_t nseg,
                               int32_t nw, int32_t npb, double* __restrict__ gldw_pv,
                               double* __restrict__ gist_pv) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n1 = int64_t(npv) * nw;
    if (idx < n1) {
        const int64_t ipv = idx / nw, e = idx - ipv * nw;
        gldw_pv[idx] = flagged_sum(
            nseg, [&](int sg) { return seg_flag[ipv * nseg + sg] != 0; },
            [&](int sg) { return seg_gw[(ipv * nseg + sg) * nw + e]; });
    } else if (idx < n1 + int64_t(npv) * npb) {
        const int64_t j = idx - n1, ipv = j / npb, pb = j - ipv * npb;
        gist_pv[j] = flagged_sum(
            nseg, [&](int sg) { return seg_flag[ipv * nseg + sg] != 0; },
            [&](int sg) { return seg_gi[(ipv * nseg + sg) * npb + pb]; });
    }
}

__global__ void k_fill(double* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// One wave per (row, quantity): lane l sums the partials of tiles l, l + 64,
// ... in order, then a fixed butterfly across the lanes.
__global__ void k_adjoint_reduce(const double* __restrict__ partials, int32_t npv,
                                 int32_t ntiles, int32_t npb, double* __restrict__ logl,
                                 double* __restrict__ grad) {
    const int nq = kNq + npb;
    const int64_t wv = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wv >= int64_t(npv) * nq) return;                 // whole waves leave together
    const int ipv = int(wv / nq), q = int(wv - int64_t(ipv) * nq);
    double s = 0.0;
    for (int tl = lane; tl < ntiles; tl += 64) s += partials[(int64_t(ipv) * ntiles + tl) * nq + q];
    s = wave_sum(s);
    if (lane != 0) return;
    if (q == 0) {
        if (logl) logl[ipv] = s;
    } else if (grad) {
        grad[int64_t(ipv) * (6 + npb) + (q - 1)] = s;
    }
}

// k-row index and lerp weight of every (row, passband) for the table
// gradient: kidx = ik (kNoRow for an invalid row, so that neither ik nor
// ik + 1 matches any k-row), kfrac = ak.
constexpr int kNoRow = -2;
__global__ void k_row_kidx(const double* __restrict__ pv, int32_t npv, int32_t npar,
                           const PvConst* __restrict__ pvc, GridDev g,
                           int32_t* __restrict__ kidx, double* __restrict__ kfrac) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(npv) * g.npb) return;
    const int ipv = int(idx / g.npb), pb = int(idx - int64_t(ipv) * g.npb);
    if (!(pvc[ipv].flags & kValid)) {
        kidx[idx] = kNoRow;
        kfrac[idx] = 0.0;
        return;
    }
    const double u = (pv[int64_t(ipv) * npar + 6 + pb] - g.k0) / g.dk;
    int ik = int(floor(u));
    ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
    kidx[idx] = ik;
    kfrac[idx] = u - ik;
}

// dlogL/dT[pb][i][m] = sum over rows of [(ik == i)(1 - ak) + (ik + 1 == i) ak]
// dlogL/dldw_row[pb][m], in two fixed-order stages.  Workgroup (x, i, c npb +
// pb), x a block of m, sums the rows of chunk c in row order; each wave reads
// the k-rows of 64 rows at a time and visits only those touching k-row i (a
// ballot), with eight loads in flight.  A chunk with no such row writes only
// its flag.  k_table_grad_sum then adds the flagged chunks in order.
__global__ void k_table_grad(const double* __restrict__ gldw_pv,
                             const int32_t* __restrict__ kidx, const double* __restrict__ kfrac,
                             int32_t npv, int32_t rows_per_chunk, GridDev g,
                             double* __restrict__ part, int32_t* __restrict__ flags) {
    const int c = int(blockIdx.z) / g.npb, pb = int(blockIdx.z) - c * g.npb, i = int(blockIdx.y);
    const int m = int(blockIdx.x) * kBlock + int(threadIdx.x);
    const int lane = threadIdx.x & 63;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(npv, r0 + rows_per_chunk);
    double s = 0.0;
    bool touched = false;
    for (int base = r0; base < r1; base += 64) {
        const int r = base + lane;
        const int ik = r < r1 ? kidx[int64_t(r) * g.npb + pb] : kNoRow;
        const double ak = r < r1 ? kfrac[int64_t(r) * g.npb + pb] : 0.0;
        uint64_t hit = __ballot(ik == i || ik + 1 == i);
        touched = touched || hit != 0;
        while (hit) {
            // up to 8 hits at a time: their loads are issued together, the
            // sum still runs in row order
            constexpr int kB = 8;
            int qs[kB];
            int n = 0;
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                qs[b] = hit ? __builtin_ctzll(hit) : 0;
                n += hit ? 1 : 0;
                hit &= hit - 1;
            }
            double wv[kB], gv[kB];
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                const int ikq = __shfl(ik, qs[b]);
                const double akq = __shfl(ak, qs[b]);
                wv[b] = (ikq == i) ? 1.0 - akq : akq;
                gv[b] = (b < n && m < g.ng)
                            ? gldw_pv[(int64_t(base + qs[b]) * g.npb + pb) * g.ng + m] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < kB; ++b)
                if (b < n) s += wv[b] * gv[b];
        }
    }
    const int64_t slot = (int64_t(c) * g.npb + pb) * g.nk + i;
    if (blockIdx.x == 0 && threadIdx.x == 0) flags[slot] = touched ? 1 : 0;
    if (touched && m < g.ng) part[slot * g.ng + m] = s;
}

// GT = the flagged chunk partials in chunk order; rowflag[pb nk + i] = 1 if
// any chunk touched k-row i (k_ldp_grad skips the other rows).
__global__ void k_table_grad_sum(const double* __restrict__ part,
                                 const int32_t* __restrict__ flags, int32_t nchunks, GridDev g,
                                 double* __restrict__ GT, int32_t* __restrict__ rowflag) {
    const int64_t per = int64_t(g.npb) * g.nk * g.ng;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= per) return;
    const int64_t row = idx / g.ng;                       // pb nk + i
    bool any;
    GT[idx] = flagged_sum(
        nchunks, [&](int c) { return flags[int64_t(c) * g.npb * g.nk + row] != 0; },
        [&](int c) { return part[int64_t(c) * per + idx]; }, &any);
    if (idx - row * g.ng == 0) rowflag[row] = any ? 1 : 0;
}

// dlogL/dldp[pb][j] = sum_{i,m} W[i][j][m] dlogL/dT[pb][i][m], in two fixed-
// order stages: workgroup (c, j, pb) sums the k-rows of chunk c with a
// fixed-shape tree, then k_ldp_sum adds the chunks in order.
constexpr int kLdpChunks = 16;
__global__ void k_ldp_grad(const double* __restrict__ W, const double* __restrict__ GT,
                           const int32_t* __restrict__ rowflag, GridDev g,
                           double* __restrict__ part_out) {
    __shared__ double part[kBlock];
    const int c = blockIdx.x;
    const int j = int(blockIdx.y), pb = int(blockIdx.z);
    const int per_chunk = (g.nk + kLdpChunks - 1) / kLdpChunks;
    const int i0 = c * per_chunk, i1 = min(g.nk, i0 + per_chunk);
    const int64_t per = int64_t(g.nk) * g.ng;
    double s = 0.0;
    for (int i = i0; i < i1; ++i) {
        if (!rowflag[pb * g.nk + i]) continue;          // GT row i is zero
        for (int m = threadIdx.x; m < g.ng; m += kBlock)
            s += W[(int64_t(i) * g.nz + j) * g.ng + m] * GT[pb * per + int64_t(i) * g.ng + m];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part_out[(int64_t(pb) * g.nz + j) * kLdpChunks + c] = part[0];
}

__global__ void k_ldp_sum(const double* __restrict__ part, int32_t n, double* __restrict__ gldp) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double s = 0.0;
    for (int c = 0; c < kLdpChunks; ++c) s += part[int64_t(idx) * kLdpChunks + c];
    gldp[idx] = s;
}

// Sum over valid rows of dlogL/dI_star[pb], one workgroup per passband,
// fixed-shape tree.
__global__ void k_gist_sum(const double* __restrict__ gist_pv, int32_t npv,
                           const PvConst* __restrict__ pvc, int32_t npb,
                           double* __restrict__ gist) {
    __shared__ double part[kBlock];
    const int pb = blockIdx.x;
    double s = 0.0;
    for (int ipv = threadIdx.x; ipv < npv; ipv += kBlock)
        if (pvc[ipv].flags & kValid) s += gist_pv[int64_t(ipv) * npb + pb];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gist[pb] = part[0];
}

// Profile gradient: chain dlogL/dldp (profile at the bin means, linear in
// the samples with the weights of the piecewise-linear interpolant) and
// dlogL/dI_star (I_star linear in the samples, Eq. 2 / Eq. 4) back to the
// samples prof[pb][s].  Workgroup (x, pb) handles samples x 256 .. + 255 of
// passband pb.  It walks the bins in chunks of kJChunk: for every bin j of
// the chunk it tabulates in LDS the interpolation segment of mu_j (a binary
// search over the samples, staged in LDS when there are at most kMuLds of
// them) and dlogL/dldp[pb][j]; then each thread adds its sample's weights
// times dlogL/dldp over the chunk's bins in order (only the run of bins that
// interpolate from its sample).
constexpr int kJChunk = 1024;
constexpr int kMuLds = 1024;
__global__ void k_prof_grad(const double* __restrict__ gldp, const double* __restrict__ gist,
                            const double* __restrict__ mu_s, int32_t nmu,
                            const double* __restrict__ zm, int32_t nz, int32_t npb,
                            int32_t istar_fixed, double* __restrict__ out) {
    __shared__ int seg_lo[kJChunk];
    __shared__ double seg_tau[kJChunk];
    __shared__ double gl[kJChunk];
    __shared__ double mu_l[kMuLds];
    const int pb = blockIdx.y;
    const int s = int(blockIdx.x) * kBlock + int(threadIdx.x);
    const bool staged = nmu <= kMuLds;
    if (staged)
        for (int i = threadIdx.x; i < nmu; i += kBlock) mu_l[i] = mu_s[i];
    __syncthreads();
    const double* ms = staged ? mu_l : mu_s;
    double acc = 0.0;
    for (int j0 = 0; j0 < nz; j0 += kJChunk) {
        const int jn = min(kJChunk, nz - j0);
        for (int jj = threadIdx.x; jj < jn; jj += kBlock) {
            const double z = zm[j0 + jj];
            const double mu = sqrt(1.0 - z * z);
            int lo;
            double tau;
            if (mu <= ms[0]) {
                lo = -1; tau = 0.0;                     // weight 1 on sample 0
            } else if (mu >= ms[nmu - 1]) {
                lo = nmu - 1; tau = 1.0;                // weight 1 on sample nmu - 1
            } else {
                int a = 0, b = nmu - 1;
                while (b - a > 1) {
                    const int mid = (a + b) >> 1;
                    if (ms[mid] <= mu) a = mid; else b = mid;
                }
                lo = a;
                tau = (mu - ms[a]) / (ms[a + 1] - ms[a]);
            }
            seg_lo[jj] = lo;
            seg_tau[jj] = tau;
            gl[jj] = gldp[int64_t(pb) * nz + j0 + jj];
        }
        __syncthreads();
        if (s < nmu) {
            // mu_j decreases with j, so seg_lo is non-increasing in j and
            // the bins with a nonzero weight for sample s (seg_lo in
            // {s - 1, s}) are one contiguous run: two binary searches find
            // it, and the run is added in bin order
            int lo_i = 0, hi_i = jn;
            while (lo_i < hi_i) {                       // first bin with seg_lo <= s
                const int mid = (lo_i + hi_i) >> 1;
                if (seg_lo[mid] <= s) hi_i = mid; else lo_i = mid + 1;
            }
            const int ja = lo_i;
            hi_i = jn;
            while (lo_i < hi_i) {                       // first bin with seg_lo < s - 1
                const int mid = (lo_i + hi_i) >> 1;
                if (seg_lo[mid] < s - 1) hi_i = mid; else lo_i = mid + 1;
            }
            for (int jj = ja; jj < lo_i; ++jj) {
                const int lo = seg_lo[jj];
                // lo == s: 1 - tau (1 for the last sample); lo == s - 1: tau
                // (1 for sample 0, whose run holds the bins below mu_s[0])
                const double w = lo == s ? (s == nmu - 1 ? 1.0 : 1.0 - seg_tau[jj])
                                         : (s == 0 ? 1.0 : seg_tau[jj]);
                if (w != 0.0) acc += w * gl[jj];
            }
        }
        __syncthreads();
    }
    if (s >= nmu) return;
    // I_star weight of sample s
    double qs = 0.0;
    if (s < nmu - 1) {
        const double ma = ms[s], mb = ms[s + 1];
        qs += (mb - ma) / 6.0 * (2.0 * ma + mb);
    }
    if (s > 0) {
        const double ma = ms[s - 1], mb = ms[s];
        qs += (mb - ma) / 6.0 * (ma + 2.0 * mb);
    }
    if (s == 0) qs += 0.5 * ms[0] * ms[0];
    if (s == nmu - 1) qs += 0.5 * (1.0 - ms[nmu - 1] * ms[nmu - 1]);
    qs *= 2.0 * Num<double>::pi;
    // a normaliser set by the caller does not depend on the samples
    out[int64_t(pb) * nmu + s] = istar_fixed ? acc : acc + qs * gist[pb];
}

inline unsigned nblocks(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

// Per-vector LD: dlogL/dldp_r[j] = sum_m (W[ik][j][m] (1 - ak) +
// W[ik+1][j][m] ak) dlogL/dldw_r[m] for row r = (vector, passband): the
// transpose of the row's k-interpolated T = W . l.  Workgroup (sorted row,
// 16 bins): each wave takes 4 bins; per bin, lane l sums m = l, l + 64, ...
// in order, then a fixed butterfly across the lanes.  Rows of tiles that go
// to the matrix cores (k_pv_ldp_grad_mfma) are skipped.
constexpr int kLdpBins = 16;
template <typename WT>
__global__ __launch_bounds__(kBlock) void k_pv_ldp_grad(const WT* __restrict__ W,
                                                        const double* __restrict__ gldw,
                                                        const double* __restrict__ pv,
                                                        int32_t npar, const int32_t* __restrict__ ikr,
                                                        const int32_t* __restrict__ perm,
                                                        int64_t nr, int32_t nz, GridDev g,
                                                        double* __restrict__ gldp) {
    const int nchunk = (nz + kLdpBins - 1) / kLdpBins;
    const int64_t b = blockIdx.x;
    const int64_t pos = b / nchunk;
    const int jc = int(b - pos * nchunk);
    if (tile_on_matrix_cores(ikr, perm, nr, pos / 16)) return;     // uniform
    const int64_t r = perm[pos];
    const int64_t ipv = r / g.npb;
    const int pb = int(r - ipv * g.npb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double u = (pv[ipv * npar + 6 + pb] - g.k0) / g.dk;
    double uf = floor(u);
    if (!(uf >= 0.0)) uf = 0.0;                  // invalid rows carry zero gldw
    if (uf > g.nk - 2) uf = g.nk - 2;
    const int ik = int(uf);
    const double ak = u - ik;
    const bool finite_k = ak == ak;
    const double* gr = gldw + r * g.ng;
    constexpr int kPerWave = kLdpBins / (kBlock / 64);
#pragma unroll
    for (int q = 0; q < kPerWave; ++q) {
        const int j = jc * kLdpBins + wave * kPerWave + q;
        if (j >= nz) break;                      // uniform per wave
        const WT* w0 = W + (int64_t(ik) * nz + j) * g.ng;
        const WT* w1 = w0 + int64_t(nz) * g.ng;
        // eight columns' loads in flight, added in column order
        double s = 0.0;
        for (int m0 = lane; m0 < g.ng; m0 += 8 * 64) {
            double x0[8], x1[8], gv[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int m = m0 + 64 * b;
                const bool in = m < g.ng;
                x0[b] = in ? double(w0[m]) : 0.0;
                x1[b] = in ? double(w1[m]) : 0.0;
                gv[b] = in ? gr[m] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) s += ((1.0 - ak) * x0[b] + ak * x1[b]) * gv[b];
        }
        s = wave_sum(finite_k ? s : 0.0);
        if (lane == 0) gldp[r * nz + j] = s;
    }
}

template <typename R, int NPBT, bool kProf>
void launch_adjoint_t(const AdjointArgs& A, size_t lds, hipStream_t s, const KernelEvents& ev) {
    // one part per vector: the profile sums are final and go to gldw_pv
    const bool one = A.nparts == 1;
    launch_timed(k_adjoint<R, NPBT, kProf>, dim3(unsigned(int64_t(A.nparts) * A.npv)),
                 dim3(kAdjBlock), lds, s, ev.before, ev.after, A.times, A.lcids, A.npt, *A.lc,
                 A.pv, A.npar, A.pvc, A.g, static_cast<const R*>(A.T), A.inv_istar,
                 static_cast<const R*>(A.obs), A.inv_sig2, A.ntiles, A.nparts, A.tpp,
                 A.want_grad, A.wprof, A.partials, one ? A.gldw_pv : A.seg_gw,
                 one ? A.gist_pv : A.seg_gi, one ? nullptr : A.seg_flag, A.rows_per_vector);
}

template <typename R>
void launch_adjoint_r(const AdjointArgs& A, size_t lds, hipStream_t s, const KernelEvents& ev) {
    if (A.want_prof) {
        if (A.g.npb <= 1) launch_adjoint_t<R, 1, true>(A, lds, s, ev);
        else if (A.g.npb <= 4) launch_adjoint_t<R, 4, true>(A, lds, s, ev);
        else launch_adjoint_t<R, 16, true>(A, lds, s, ev);
    } else {
        if (A.g.npb <= 1) launch_adjoint_t<R, 1, false>(A, lds, s, ev);
        else if (A.g.npb <= 4) launch_adjoint_t<R, 4, false>(A, lds, s, ev);
        else launch_adjoint_t<R, 16, false>(A, lds, s, ev);
    }
}

}  // namespace

hipError_t launch_fill(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

size_t adjoint_lds_bytes(int32_t precision, int32_t npb, int32_t ng, bool prof) {
    const size_t elt = precision == RR_FP64 ? sizeof(double) : sizeof(float);
    const size_t tables = ((2 * elt * size_t(npb) * ng + 7) / 8) * 8;
    if (!prof) return tables;
    return tables + sizeof(double) * (kAdjBlock / 64) * (size_t(npb) * ng + npb);
}

hipError_t launch_adjoint(const AdjointArgs& A, int32_t precision, hipStream_t s) {
    const size_t lds = adjoint_lds_bytes(precision, A.g.npb, A.g.ng, A.want_prof != 0);
    const KernelEvents ev = kernel_events();
    if (precision == RR_FP64) launch_adjoint_r<double>(A, lds, s, ev);
    else launch_adjoint_r<float>(A, lds, s, ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (A.want_prof && A.nparts > 1) {
        const int32_t nw = A.g.npb * A.g.ng;
        hipLaunchKernelGGL(k_prof_seg_sum, dim3(nblocks(int64_t(A.npv) * (nw + A.g.npb))),
                           dim3(kBlock), 0, s, A.seg_gw, A.seg_gi, A.seg_flag, A.npv, A.nparts,
                           nw, A.g.npb, A.gldw_pv, A.gist_pv);
    }
    hipLaunchKernelGGL(k_adjoint_reduce, dim3(nblocks(int64_t(A.npv) * (kNq + A.g.npb) * 64)),
                       dim3(kBlock), 0, s, A.partials, A.npv, A.nparts, A.g.npb, A.logl,
                       A.grad);
    return hipGetLastError();
}

// The same on the matrix cores for tiles of 16 sorted rows on at most
// kMfmaMaxRuns k-rows: per wave a 16 (bins) x 16 (rows) tile of
// D[j][q] = sum_m W[ik][j][m] (1 - ak_q) g_q[m] + W[ik+1][j][m] ak_q g_q[m]
// (g_q = dlogL/dldw of row q, zero for rows on another k-row), two
// v_mfma_f64_16x16x4f64 chains into one accumulator; lane layout as in
// the matrix-core part of k_pv_tables.  Block = 4 waves = 64 bins x 16 rows.
typedef double v4d __attribute__((ext_vector_type(4)));
template <typename WT>
__global__ __launch_bounds__(kBlock) void k_pv_ldp_grad_mfma(
    const WT* __restrict__ W, const double* __restrict__ gldw,
    const double* __restrict__ pv, int32_t npar, const int32_t* __restrict__ ikr,
    const int32_t* __restrict__ perm, int64_t nr, int32_t nz, GridDev g,
    double* __restrict__ gldp) {
    const int njb = (nz + 63) / 64;
    const int64_t rt = int64_t(blockIdx.x) / njb;
    const int jb = int(int64_t(blockIdx.x) - rt * njb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j0 = jb * 64 + wave * 16;
    const int ka = lane >> 4, col = lane & 15;
    const int64_t pos = rt * 16 + col;
    const int64_t r = pos < nr ? perm[pos] : -1;
    const int ik = r >= 0 ? ikr[r] : 0x7fffffff;
    const int prev_ik = __shfl(ik, (lane & 48) | ((col + 15) & 15), 64);
    const uint64_t starts = __ballot(lane < 16 && r >= 0 && (col == 0 || ik != prev_ik));
    if (__popcll(starts) > kMfmaMaxRuns) return;                  // k_pv_ldp_grad's tile
    double ak = 0.0;
    if (r >= 0) {
        const int64_t ipv = r / g.npb;
        const int pb = int(r - ipv * g.npb);
        ak = (pv[ipv * npar + 6 + pb] - g.k0) / g.dk - ik;
        if (!(ak == ak)) ak = 0.0;                  // non-finite k: zero gldw anyway
    }
    const int jj = j0 + col;                          // A row of this lane
    const bool jin = jj < nz;
    v4d d = {0.0, 0.0, 0.0, 0.0};
    int cur = ik;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cur = min(cur, __shfl_xor(cur, off, 64));
    while (cur != 0x7fffffff) {
        const bool take = ik == cur;
        const WT* w0 = W + (int64_t(cur) * nz + (jin ? jj : 0)) * g.ng;
        const WT* w1 = w0 + int64_t(nz) * g.ng;
        const double* gr = gldw + (take ? r : 0) * g.ng;
        for (int m0 = 0; m0 < g.ng; m0 += 16) {
            double a0[4], a1[4], b0[4], b1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {               // four k-steps' loads in flight
                const int m = m0 + 4 * u + ka;
                const bool min_ = m < g.ng;
                a0[u] = jin && min_ ? double(w0[m]) : 0.0;
                a1[u] = jin && min_ ? double(w1[m]) : 0.0;
                const double gq = take && min_ ? gr[m] : 0.0;
                b0[u] = (1.0 - ak) * gq;
                b1[u] = ak * gq;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], d, 0, 0, 0);
            }
        }
        int nxt = ik > cur ? ik : 0x7fffffff;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nxt = min(nxt, __shfl_xor(nxt, off, 64));
        cur = nxt;
    }
    if (r < 0) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = j0 + 4 * i + ka;
        if (j < nz) gldp[r * nz + j] = d[i];
    }
}

hipError_t launch_pv_prof_grad(const rr_tables* t, const AdjointArgs& A, const int32_t* ikr,
                               const int32_t* perm, double* gldp, double* out, hipStream_t s,
                               bool w32) {
    const GridDev g = A.g;
    const int64_t nr = int64_t(A.npv) * g.npb;
    const int64_t nchunk = (t->nz + kLdpBins - 1) / kLdpBins;
    const dim3 gm(unsigned(((nr + 15) / 16) * ((t->nz + 63) / 64)));
    const dim3 gr(unsigned(nr * nchunk));
    // the transpose of the contraction that built the rows, with its weights
    if (w32) {
        hipLaunchKernelGGL(k_pv_ldp_grad_mfma<float>, gm, dim3(kBlock), 0, s, t->W32, A.gldw_pv,
                           A.pv, A.npar, ikr, perm, nr, t->nz, g, gldp);
        hipLaunchKernelGGL(k_pv_ldp_grad<float>, gr, dim3(kBlock), 0, s, t->W32, A.gldw_pv, A.pv,
                           A.npar, ikr, perm, nr, t->nz, g, gldp);
    } else {
        hipLaunchKernelGGL(k_pv_ldp_grad_mfma<double>, gm, dim3(kBlock), 0, s, t->W, A.gldw_pv,
                           A.pv, A.npar, ikr, perm, nr, t->nz, g, gldp);
        hipLaunchKernelGGL(k_pv_ldp_grad<double>, gr, dim3(kBlock), 0, s, t->W, A.gldw_pv, A.pv,
                           A.npar, ikr, perm, nr, t->nz, g, gldp);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the shared profile's last step with every (vector, passband) as one
    // profile: its own dlogL/dldp and dlogL/dI_star
    for (int64_t r0 = 0; r0 < nr; r0 += 65535) {
        const int32_t n = int32_t(std::min<int64_t>(65535, nr - r0));
        hipLaunchKernelGGL(k_prof_grad, dim3(nblocks(t->nmu), unsigned(n)), dim3(kBlock), 0, s,
                           gldp + r0 * t->nz, A.gist_pv + r0, t->mu_s, t->nmu, t->zm, t->nz, n,
                           0,
                           out + r0 * t->nmu);
    }
    return hipGetLastError();
}

hipError_t launch_profile_grad(const rr_tables* t, const AdjointArgs& A,
                               const ProfGradScratch& w, double* out, hipStream_t s) {
    const GridDev g = A.g;
    const int64_t nrk = int64_t(A.npv) * g.npb;
    hipLaunchKernelGGL(k_row_kidx, dim3(nblocks(nrk)), dim3(kBlock), 0, s, A.pv, A.npv, A.npar,
                       A.pvc, g, w.kidx, w.kfrac);
    const int32_t rpc = (A.npv + w.nchunks - 1) / w.nchunks;
    hipLaunchKernelGGL(k_table_grad,
                       dim3(unsigned((g.ng + kBlock - 1) / kBlock), unsigned(g.nk),
                            unsigned(w.nchunks * g.npb)),
                       dim3(kBlock), 0, s, A.gldw_pv, w.kidx, w.kfrac, A.npv, rpc, g,
                       w.gt_part, w.gt_flags);
    hipLaunchKernelGGL(k_table_grad_sum, dim3(nblocks(int64_t(g.npb) * g.nk * g.ng)),
                       dim3(kBlock), 0, s, w.gt_part, w.gt_flags, w.nchunks, g, w.GT,
                       w.gt_rowflag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ldp_grad, dim3(unsigned(kLdpChunks), unsigned(g.nz), unsigned(g.npb)),
                       dim3(kBlock), 0, s, t->W, w.GT, w.gt_rowflag, g, w.ldp_part);
    hipLaunchKernelGGL(k_ldp_sum, dim3(nblocks(int64_t(g.npb) * g.nz)), dim3(kBlock), 0, s,
                       w.ldp_part, g.npb * g.nz, w.gldp);
    hipLaunchKernelGGL(k_gist_sum, dim3(unsigned(g.npb)), dim3(kBlock), 0, s, A.gist_pv, A.npv,
                       A.pvc, g.npb, w.gist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (w.grad_istar) {
        e = hipMemcpyAsync(w.grad_istar, w.gist, sizeof(double) * g.npb,
                           hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    if (out)
        hipLaunchKernelGGL(k_prof_grad, dim3(nblocks(t->nmu), unsigned(g.npb)), dim3(kBlock), 0,
                           s, w.gldp, w.gist, t->mu_s, t->nmu, t->zm, t->nz, g.npb,
                           w.istar_fixed, out);
    return hipGetLastError();
}

}  // namespace rr
