// rr_prep.hip -- table construction on the device (Sect. 2, Sect. 3.1.1,
// Sect. 3.1.2, Sect. 3.2.2).
//
//   k_zgrid     annulus edges ze[nz+1] and means zm[nz]: constant dz on
//               [0, zcut] and constant dmu on [zcut, 1] (Sect. 3.1.1);
//   k_weights   W[nk][nz][ng]: area of annulus j occluded by a planet of
//               radius k_i at separation c = g_m (1 + k_i), over the total
//               occluded area (Sect. 2); g = 1 gets the zero-overlap limit,
//               all weight in the limb annulus; g runs fastest so that the
//               table contraction below reads W coalesced;
//   k_profile   profile at the bin means, mu_m = sqrt(1 - zm^2): the
//               piecewise-linear interpolant of the samples (Sect. 3.2.2);
//   k_istar     I_star = 2 pi int_0^1 mu I(mu) dmu of that interpolant,
//               exact per segment (Eq. 2, Eq. 4), fixed-order reduction;
//   k_tables    T[pb][i][m] = sum_j W[i][j][m] ldp[pb][j] (Sect. 3.1.2), in
//               FP64 and rounded to FP32 for the mixed path.
#include "rr_device.h"

namespace rr {
namespace {

__global__ void k_zgrid(int32_t nzin, int32_t nzlimb, double zcut,
                        double* __restrict__ ze, double* __restrict__ zm) {
    const int nz = nzin + nzlimb;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > nz) return;
    auto edge = [&](int jj) -> double {
        if (jj < nzin) return jj * (zcut / nzin);
        if (jj == nzin) return zcut;
        if (jj == nz) return 1.0;
        const double mucut = sqrt(1.0 - zcut * zcut);
        const double mu = mucut + (jj - nzin) * ((0.0 - mucut) / nzlimb);
        return sqrt(1.0 - mu * mu);
    };
    const double e0 = edge(j);
    ze[j] = e0;
    if (j < nz) zm[j] = 0.5 * (e0 + edge(j + 1));
}

// Weight of annulus j for radius ratio k with the planet centre at c
// (Sect. 2): occluded area of the annulus over the total occluded area tot;
// at zero overlap its limit, all weight in the limb annulus.
__device__ inline double annulus_weight(const double* __restrict__ ze, int nz, int j,
                                        double k, double c, double tot) {
    if (!(tot > 0.0)) return j == nz - 1 ? 1.0 : 0.0;
    return (lens_area<double>(ze[j + 1], k, c) - lens_area<double>(ze[j], k, c)) / tot;
}

__global__ void k_weights(const double* __restrict__ ze, GridDev g,
                          double* __restrict__ W) {
    const int64_t total = int64_t(g.nk) * g.nz * g.ng;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int m = int(idx % g.ng);
    const int64_t r = idx / g.ng;
    const int j = int(r % g.nz);
    const int i = int(r / g.nz);
    const double k = g.k0 + i * g.dk;
    const double gv = double(m) / double(g.ng - 1);
    const double c = gv * (1.0 + k);
    W[idx] = annulus_weight(ze, g.nz, j, k, c, lens_area<double>(1.0, k, c));
}

// The profile's piecewise-linear interpolant at the mean of bin j.
__device__ inline double profile_at_bin(const double* __restrict__ mu_s,
                                        const double* __restrict__ f, int32_t nmu,
                                        double z) {
    const double mu = sqrt(1.0 - z * z);
    if (mu <= mu_s[0]) return f[0];
    if (mu >= mu_s[nmu - 1]) return f[nmu - 1];
    int lo = 0, hi = nmu - 1;          // mu_s[lo] <= mu < mu_s[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (mu_s[mid] <= mu) lo = mid; else hi = mid;
    }
    const double slope = (f[lo + 1] - f[lo]) / (mu_s[lo + 1] - mu_s[lo]);
    return slope * (mu - mu_s[lo]) + f[lo];
}

__global__ void k_profile(const double* __restrict__ mu_s,
                          const double* __restrict__ prof, int32_t nmu,
                          const double* __restrict__ zm, int32_t nz,
                          int32_t npb, double* __restrict__ ldp) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nz * npb) return;
    const int pb = idx / nz, j = idx - pb * nz;
    ldp[idx] = profile_at_bin(mu_s, prof + int64_t(pb) * nmu, nmu, zm[j]);
}

// I_star of one profile by one workgroup of kBlock threads: per-thread
// partial sums over a fixed stride, then a fixed-shape tree in LDS
// (deterministic).  Thread 0 stores I_star and 1/I_star.
__device__ inline void istar_block(const double* __restrict__ mu_s,
                                   const double* __restrict__ f, int32_t nmu,
                                   double* __restrict__ istar,
                                   double* __restrict__ inv_istar) {
    __shared__ double part[kBlock];
    double acc = 0.0;
    for (int s = threadIdx.x; s < nmu - 1; s += kBlock) {
        const double ma = mu_s[s], mb = mu_s[s + 1];
        acc += (mb - ma) / 6.0 * (f[s] * (2.0 * ma + mb) + f[s + 1] * (ma + 2.0 * mb));
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m0 = mu_s[0], m1 = mu_s[nmu - 1];
        const double tot = part[0] + f[0] * 0.5 * m0 * m0 +
                           f[nmu - 1] * 0.5 * (1.0 - m1 * m1);
        const double is = 2.0 * Num<double>::pi * tot;
        *istar = is;
        *inv_istar = 1.0 / is;
    }
}

// One workgroup (kBlock threads) per passband.
__global__ __launch_bounds__(kBlock) void k_istar(const double* __restrict__ mu_s,
                                                  const double* __restrict__ prof, int32_t nmu,
                                                  double* __restrict__ istar,
                                                  double* __restrict__ inv_istar) {
    const int pb = blockIdx.x;
    istar_block(mu_s, prof + int64_t(pb) * nmu, nmu, istar + pb, inv_istar + pb);
}

__global__ void k_tables(const double* __restrict__ W,
                         const double* __restrict__ ldp, GridDev g,
                         double* __restrict__ T64, float* __restrict__ T32) {
    const int64_t per = int64_t(g.nk) * g.ng;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= per * g.npb) return;
    const int pb = int(idx / per);
    const int64_t r = idx - pb * per;
    const int i = int(r / g.ng), m = int(r - int64_t(i) * g.ng);
    const double* wrow = W + int64_t(i) * g.nz * g.ng + m;
    const double* l = ldp + int64_t(pb) * g.nz;
    double acc = 0.0;
    for (int j = 0; j < g.nz; ++j) acc += wrow[int64_t(j) * g.ng] * l[j];
    T64[idx] = acc;
    T32[idx] = float(acc);
}

inline unsigned nblocks(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

}  // namespace

GridDev grid_dev(const rr_tables* t) {
    GridDev g;
    g.nz = t->nz;
    g.ng = t->grid.ng;
    g.nk = t->grid.nk;
    g.npb = t->npb;
    g.k0 = t->grid.k0;
    g.dk = t->dk;
    g.inv_dk = 1.0 / t->dk;
    g.gscale = double(t->grid.ng - 1);
    return g;
}

// FP32 copy of the weights for the mixed-precision per-vector tables.
__global__ void k_weights_f32(const double* __restrict__ W, int64_t n, float* __restrict__ W32) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) W32[i] = float(W[i]);
}

hipError_t launch_prepare_grid_weights(rr_tables* t, hipStream_t s) {
    const GridDev g = grid_dev(t);
    hipLaunchKernelGGL(k_zgrid, dim3(nblocks(t->nz + 1)), dim3(kBlock), 0, s,
                       t->grid.nzin, t->grid.nzlimb, t->grid.zcut, t->ze, t->zm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nw = int64_t(g.nk) * g.nz * g.ng;
    hipLaunchKernelGGL(k_weights, dim3(nblocks(nw)), dim3(kBlock), 0, s, t->ze, g, t->W);
    hipLaunchKernelGGL(k_weights_f32, dim3(nblocks(nw)), dim3(kBlock), 0, s, t->W, nw, t->W32);
    return hipGetLastError();
}

// Per-vector LD rows.  Row r = (vector, passband) needs the two table rows
// T_r[s][m] = sum_j W[ik_r + s][j][m] ldp[r][j], s = 0, 1, around its k
// (Sect. 3.1.2: T = W . l, then the k-interpolation in the forward kernel).
// k_pv_prep sorts the rows by ik, so that rows with equal ik share the W
// reads of one matrix-core tile (the two parts of k_pv_tables below).
// Stable counting sort of the rows by ik, by one workgroup of kBlock
// threads (thread t owns bins 16 t .. 16 t + 15 of at most 4096): the
// histogram and its scan by all waves, then one wave places the rows in
// row order, 64 at a time -- a lane's rank among the lanes with its key
// comes from a ballot per key bit -- so equal keys keep their row order
// and the tiles (and which kernel takes each) depend on the inputs only.
// The keys of the first kSortLds rows also go to LDS (as 16-bit values,
// nk <= 4096), so that the placing wave's serial loop reads them there
// rather than waiting on a global load in every step.
constexpr int kSortLds = 8192;
__device__ inline void sort_rows(const double* __restrict__ pv, int32_t npv, int32_t npar,
                                 const GridDev& g, int32_t* __restrict__ ikr,
                                 int32_t* __restrict__ perm) {
    constexpr int kPer = 4096 / kBlock;
    __shared__ int cnt[4096];
    __shared__ uint16_t keys[kSortLds];
    __shared__ int wsum[kBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = int64_t(npv) * g.npb;
    for (int b = tid; b < g.nk; b += kBlock) cnt[b] = 0;
    __syncthreads();
    for (int64_t r = tid; r < n; r += kBlock) {
        const int64_t ipv = r / g.npb;
        const int pb = int(r - ipv * g.npb);
        const double u = (pv[ipv * npar + 6 + pb] - g.k0) / g.dk;
        double uf = floor(u);
        if (!(uf >= 0.0)) uf = 0.0;              // also a non-finite k (NaN row anyway)
        if (uf > g.nk - 2) uf = g.nk - 2;
        const int ik = int(uf);
        ikr[r] = ik;
        if (r < kSortLds) keys[r] = uint16_t(ik);
        atomicAdd(&cnt[ik], 1);
    }
    __syncthreads();
    int v[kPer], local = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int b = kPer * tid + q;
        v[q] = b < g.nk ? cnt[b] : 0;
        local += v[q];
    }
    int x = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int excl = x - local;
    for (int w = 0; w < wave; ++w) excl += wsum[w];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int b = kPer * tid + q;
        if (b < g.nk) cnt[b] = excl;
        excl += v[q];
    }
    __syncthreads();
    if (wave != 0) return;
    for (int64_t r0 = 0; r0 < n; r0 += 64) {
        const int64_t r = r0 + lane;
        const bool in = r < n;
        const int key = in ? (r < kSortLds ? int(keys[r]) : ikr[r]) : 0;
        uint64_t same = __ballot(in);            // lanes with this lane's key
#pragma unroll
        for (int b = 0; b < 12; ++b) {           // keys < nk <= 4096
            const bool bit = (key >> b) & 1;
            const uint64_t ones = __ballot(in && bit);
            same &= bit ? ones : ~ones;
        }
        const int base = in ? cnt[key] : 0;
        if (in) perm[base + __popcll(same & __lanemask_lt())] = int32_t(r);
        // every lane has read its key's offset before the first lane of each
        // key group (the only writer of that key) advances it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (in && (same & __lanemask_lt()) == 0) cnt[key] = base + __popcll(same);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// One launch for the per-vector preparation: workgroup 0 sorts the rows by
// ik (the longest serial chain, so it is dispatched first), and workgroup
// r + 1 interpolates row r's profile to the bin means and integrates its
// I_star (the table kernels' arithmetic).
__global__ __launch_bounds__(kBlock) void k_pv_prep(const double* __restrict__ mu_s,
                                                    const double* __restrict__ prof,
                                                    int32_t nmu, const double* __restrict__ zm,
                                                    int32_t nz, const double* __restrict__ pv,
                                                    int32_t npv, int32_t npar, GridDev g,
                                                    double* __restrict__ ldp,
                                                    double* __restrict__ istar,
                                                    double* __restrict__ inv_istar,
                                                    int32_t* __restrict__ ikr,
                                                    int32_t* __restrict__ perm) {
    const int64_t nr = int64_t(npv) * g.npb;
    if (blockIdx.x == 0) {
        sort_rows(pv, npv, npar, g, ikr, perm);
        return;
    }
    const int64_t r = int64_t(blockIdx.x) - 1;
    if (r >= nr) return;
    const double* f = prof + r * nmu;
    for (int j = threadIdx.x; j < nz; j += kBlock) ldp[r * nz + j] = profile_at_bin(mu_s, f, nmu, zm[j]);
    istar_block(mu_s, f, nmu, istar + r, inv_istar + r);
}

// Rows of a sorted 16-row tile with at most two distinct k-rows go to the
// matrix cores (pv_tables_mfma, which then reads each W value once for up
// to 16 rows); the rows of the other tiles (k spread over many k-rows, where
// a tile would need a pass per k-row) to pv_tables_rows, one workgroup per
// (row, 256 m).  Both parts evaluate the same test on the sorted keys, so
// every row is written by exactly one of them.
// pv_tables_rows: rows taken in sorted order, with an XCD-aware block order: blocks go round-robin to the eight XCDs, so block
// p works on sorted item (p mod 8) * (blocks / 8) + p / 8 (rounded for a
// remainder) and each XCD walks a contiguous stretch of the sorted rows,
// whose W rows its L2 then serves to the following rows of equal ik.
// The part is bound by the latency of its W loads: 24 in flight per lane
// measured best of 8 to 48.
constexpr int kXcds = 8;
template <typename R, typename WT>
__device__ inline void pv_tables_rows(const WT* __restrict__ W, const double* __restrict__ ldp,
                                      const int32_t* __restrict__ ikr,
                                      const int32_t* __restrict__ perm, int32_t nz, GridDev g,
                                      R* __restrict__ out, int64_t nb, int64_t p,
                                      double* __restrict__ lp) {
    const int64_t q = nb / kXcds, rem = nb % kXcds;
    const int64_t x = p % kXcds;
    const int64_t L = (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + p / kXcds;
    const int nmb = (g.ng + kBlock - 1) / kBlock;
    const int64_t pos = L / nmb;
    const int mb = int(L - pos * nmb);
    if (tile_on_matrix_cores(ikr, perm, int64_t(nb / nmb), pos / 16)) return;   // uniform
    const int64_t r = perm[pos];
    const int ik = ikr[r];
    for (int j = threadIdx.x; j < nz; j += kBlock) lp[j] = ldp[r * nz + j];
    __syncthreads();
    const int m = mb * kBlock + int(threadIdx.x);
    if (m >= g.ng) return;
    const WT* w0 = W + int64_t(ik) * nz * g.ng + m;
    const WT* w1 = w0 + int64_t(nz) * g.ng;
    double a0 = 0.0, a1 = 0.0;
    int j = 0;
    for (; j + 12 <= nz; j += 12) {               // 24 loads in flight
        WT x0[12], x1[12];
#pragma unroll
        for (int b = 0; b < 12; ++b) {
            x0[b] = w0[int64_t(j + b) * g.ng];
            x1[b] = w1[int64_t(j + b) * g.ng];
        }
#pragma unroll
        for (int b = 0; b < 12; ++b) {
            a0 += double(x0[b]) * lp[j + b];
            a1 += double(x1[b]) * lp[j + b];
        }
    }
    for (; j < nz; ++j) {
        a0 += double(w0[int64_t(j) * g.ng]) * lp[j];
        a1 += double(w1[int64_t(j) * g.ng]) * lp[j];
    }
    R* o = out + r * 2 * g.ng;
    o[m] = R(a0);
    o[g.ng + m] = R(a1);
}

// The per-vector table rows on the matrix cores: per wave a 16 (m) x 16 (sorted
// rows) tile of T_r[s][m] = sum_j W[ik_r + s][j][m] ldp_r[j], s = 0, 1, as
// D = A B with A[m][j] = W[ik + s][j][m] and B[j][q] = ldp of row q when the
// row's k-row is ik, else 0, over the distinct ik of the tile's rows (sorted,
// so usually one or two), with v_mfma_f64_16x16x4f64 (FP64 products and
// sums; only the order of the additions over j differs from k_tables).
// Lane l holds A[l & 15][l >> 4], B[l >> 4][l & 15] and D[4 i + (l >> 4)][l & 15]
// (checked on the device).  Block = 4 waves = 64 m x 16 rows.
typedef double v4d __attribute__((ext_vector_type(4)));
template <typename R, typename WT>
__device__ inline void pv_tables_mfma(const WT* __restrict__ W, const double* __restrict__ ldp,
                                      const int32_t* __restrict__ ikr,
                                      const int32_t* __restrict__ perm, int64_t nr, int32_t nz,
                                      GridDev g, R* __restrict__ out, int64_t bid) {
    const int nmb = (g.ng + 63) / 64;
    const int64_t rt = bid / nmb;                              // row tile
    const int mb = int(bid - rt * nmb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = mb * 64 + wave * 16;
    const int ka = lane >> 4, col = lane & 15;
    const int mm = m0 + col;                                   // A row of this lane
    const int64_t pos = rt * 16 + col;                         // B column of this lane
    const int64_t r = pos < nr ? perm[pos] : -1;
    const int ik = r >= 0 ? ikr[r] : 0x7fffffff;
    const bool mok = mm < g.ng;
    // tiles whose rows span more than kMfmaMaxRuns k-rows are k_pv_tables' work
    const int prev_ik = __shfl(ik, (lane & 48) | ((col + 15) & 15), 64);
    const uint64_t starts = __ballot(lane < 16 && r >= 0 && (col == 0 || ik != prev_ik));
    if (__popcll(starts) > kMfmaMaxRuns) return;                  // uniform per wave
    v4d d0 = {0.0, 0.0, 0.0, 0.0}, d1 = {0.0, 0.0, 0.0, 0.0};
    // distinct k-rows of the tile, smallest first (wave-uniform loop)
    int cur = ik;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cur = min(cur, __shfl_xor(cur, off, 64));
    while (cur != 0x7fffffff) {
        const bool take = ik == cur;
        const WT* w0 = W + int64_t(cur) * nz * g.ng + (mok ? mm : 0);
        const WT* w1 = w0 + int64_t(nz) * g.ng;
        const double* lr = ldp + (take ? r : 0) * nz;
        for (int j0 = 0; j0 < nz; j0 += 16) {
            double a0[4], a1[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {               // four k-steps' loads in flight
                const int j = j0 + 4 * u + ka;
                const bool jin = j < nz;
                a0[u] = jin && mok ? double(w0[int64_t(j) * g.ng]) : 0.0;
                a1[u] = jin && mok ? double(w1[int64_t(j) * g.ng]) : 0.0;
                b[u] = jin && take ? lr[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b[u], d0, 0, 0, 0);
                d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b[u], d1, 0, 0, 0);
            }
        }
        int nxt = ik > cur ? ik : 0x7fffffff;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nxt = min(nxt, __shfl_xor(nxt, off, 64));
        cur = nxt;
    }
    // lane l holds rows m0 + 4 i + ka of column col
    if (r < 0) return;
    R* o = out + r * 2 * g.ng;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + 4 * i + ka;
        if (m < g.ng) {
            o[m] = R(d0[i]);
            o[g.ng + m] = R(d1[i]);
        }
    }
}

// One launch for both: blocks [0, n_mfma) take matrix-core tiles, the
// others the per-row work (n_mfma is a multiple of the XCD count, so the
// per-row blocks keep their XCD-aware order).  Each row is written by
// exactly one of the two, as the same test on the sorted keys decides.
template <typename R, typename WT>
__global__ __launch_bounds__(kBlock) void k_pv_tables(const WT* __restrict__ W,
                                                      const double* __restrict__ ldp,
                                                      const int32_t* __restrict__ ikr,
                                                      const int32_t* __restrict__ perm,
                                                      int64_t nr, int32_t nz, GridDev g,
                                                      int64_t n_mfma, R* __restrict__ out) {
    __shared__ double lp[4096];
    const int64_t b = blockIdx.x;
    if (b < n_mfma) {
        pv_tables_mfma<R, WT>(W, ldp, ikr, perm, nr, nz, g, out, b);
        return;
    }
    pv_tables_rows<R, WT>(W, ldp, ikr, perm, nz, g, out, int64_t(gridDim.x) - n_mfma,
                          b - n_mfma, lp);
}

// Direct model (Sect. 3.1.1): the LD-weighted vector of row r = (vector,
// passband) from weights built for the row's own k -- no k-grid, no
// k-interpolation, any k in (0, 1] -- with the tables' profile at the bin
// means: ldw_r[m] = sum_j w_j(k, g_m) ldp[pb][j], bins in order, FP64 (the
// same weights and order as the table, so a k on a table node gives that
// node's row).  Workgroup (r, 256 m); stored twice ([2][ng]) in the
// evaluation precision for the forward kernel, which reads it with zero
// k-weight.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_direct_rows(const double* __restrict__ ze,
                                                        const double* __restrict__ ldp,
                                                        const double* __restrict__ pv,
                                                        int32_t npar, int32_t nz, GridDev g,
                                                        R* __restrict__ out) {
    __shared__ double lp[4096];
    const int nmb = (g.ng + kBlock - 1) / kBlock;
    const int64_t r = int64_t(blockIdx.x) / nmb;
    const int mb = int(int64_t(blockIdx.x) - r * nmb);
    const int64_t ipv = r / g.npb;
    const int pb = int(r - ipv * g.npb);
    for (int j = threadIdx.x; j < nz; j += kBlock) lp[j] = ldp[int64_t(pb) * nz + j];
    __syncthreads();
    const int m = mb * kBlock + int(threadIdx.x);
    if (m >= g.ng) return;
    const double k = pv[ipv * npar + 6 + pb];
    R* o = out + r * 2 * g.ng;
    if (!(k > 0.0 && k <= 1.0)) {           // invalid row: the forward writes NaN
        o[m] = R(0);
        o[g.ng + m] = R(0);
        return;
    }
    const double c = (double(m) / double(g.ng - 1)) * (1.0 + k);
    const double tot = lens_area<double>(1.0, k, c);
    double acc = 0.0;
    if (tot > 0.0) {
        // each edge's area once: the upper edge of bin j is the lower of j + 1
        // (the same values annulus_weight computes)
        double lo = lens_area<double>(ze[0], k, c);
        for (int j = 0; j < nz; ++j) {
            const double hi = lens_area<double>(ze[j + 1], k, c);
            acc += ((hi - lo) / tot) * lp[j];
            lo = hi;
        }
    } else {
        for (int j = 0; j < nz; ++j) acc += annulus_weight(ze, nz, j, k, c, tot) * lp[j];
    }
    o[m] = R(acc);
    o[g.ng + m] = R(acc);
}

// Small-planet approximation (Sect. 3.4.2) as rows of the per-vector path:
// for a row whose k is below k_small, the LD-weighted mean over the planet's
// disk at each g node is replaced by the profile at the planet's centre,
// c = g_m (1 + k) clamped to the limb (mu = sqrt(1 - c^2) on the tables'
// piecewise-linear profile); any other row gets the shared table's two
// k-rows around its k combined with its k-weight, in the evaluation
// precision and in the order the forward kernel combines them.  Workgroup
// (row, kBlock nodes): a small-planet row stages the mu samples and its
// passband's profile in LDS (when they fit) for the binary searches.
// Stored twice ([2][ng]), read with zero k-weight.
constexpr int kSpLds = 1024;
template <typename R>
__global__ __launch_bounds__(kBlock) void k_small_planet_rows(
    const double* __restrict__ mu_s, const double* __restrict__ prof, int32_t nmu,
    const R* __restrict__ T, const double* __restrict__ pv, int32_t npar, double k_small,
    double k1, GridDev g, R* __restrict__ out) {
    __shared__ double smu[kSpLds], sf[kSpLds];
    const int64_t r = blockIdx.x;
    const int m = int(blockIdx.y) * kBlock + int(threadIdx.x);
    const int64_t ipv = r / g.npb;
    const int pb = int(r - ipv * g.npb);
    const double k = pv[ipv * npar + 6 + pb];          // uniform in the workgroup
    R* o = out + r * 2 * g.ng;
    R v = R(0);                                        // invalid rows: the forward writes NaN
    if (k < k_small) {
        if (k > 0.0) {
            const double* f = prof + int64_t(pb) * nmu;
            const bool staged = nmu <= kSpLds;
            if (staged) {
                for (int j = threadIdx.x; j < nmu; j += kBlock) {
                    smu[j] = mu_s[j];
                    sf[j] = f[j];
                }
                __syncthreads();
            }
            if (m >= g.ng) return;
            double c = (double(m) / double(g.ng - 1)) * (1.0 + k);
            c = c < 1.0 ? c : 1.0;
            v = R(staged ? profile_at_bin(smu, sf, nmu, c) : profile_at_bin(mu_s, f, nmu, c));
        }
    } else if (k >= g.k0 && k <= k1) {
        if (m >= g.ng) return;
        const double u = (k - g.k0) / g.dk;
        int ik = int(floor(u));
        ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
        const R ak = R(u - ik);
        const R* t0r = T + (int64_t(pb) * g.nk + ik) * g.ng;
        v = (R(1) - ak) * t0r[m] + ak * t0r[g.ng + m];
    }
    if (m >= g.ng) return;
    o[m] = v;
    o[g.ng + m] = v;
}

hipError_t launch_direct_rows(const rr_tables* t, const double* pv, int32_t npv, int32_t npar,
                              int32_t precision, void* rows, hipStream_t s) {
    const GridDev g = grid_dev(t);
    const int64_t nr = int64_t(npv) * t->npb;
    const dim3 grid(unsigned(nr * ((g.ng + kBlock - 1) / kBlock)));
    if (precision == RR_FP64)
        hipLaunchKernelGGL(k_direct_rows<double>, grid, dim3(kBlock), 0, s, t->ze, t->ldp, pv,
                           npar, t->nz, g, static_cast<double*>(rows));
    else
        hipLaunchKernelGGL(k_direct_rows<float>, grid, dim3(kBlock), 0, s, t->ze, t->ldp, pv,
                           npar, t->nz, g, static_cast<float*>(rows));
    return hipGetLastError();
}

// The small-planet rows for the log-likelihood's adjoint, which reads a
// row pair (row0, row1) per (vector, passband) with the k-weight ak of the
// row's k on the tables' k-grid: ldw = (1 - ak) row0 + ak row1 and
// dldw/dk = (row1 - row0) / dk.  Below k_small the pair is built so that
// these give the centre values v[m] = I(mu(c_m)), c_m = g_m (1 + k), and
// their k-derivative D[m] = I'(mu) (-c_m / mu) g_m (zero where c_m is
// clamped to the limb or the profile is constant beyond its samples):
// row0 = v - ak dk D, row1 = row0 + dk D.  Other rows copy the shared
// table's two k-rows.  Also writes 1/I_star per row (the tables' value).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_small_planet_adj_rows(
    const double* __restrict__ mu_s, const double* __restrict__ prof, int32_t nmu,
    const R* __restrict__ T, const double* __restrict__ inv_istar, const double* __restrict__ pv,
    int32_t npar, double k_small, GridDev g, R* __restrict__ out,
    double* __restrict__ inv_istar_rows) {
    __shared__ double smu[kSpLds], sf[kSpLds];
    const int64_t r = blockIdx.x;
    const int m = int(blockIdx.y) * kBlock + int(threadIdx.x);
    const int64_t ipv = r / g.npb;
    const int pb = int(r - ipv * g.npb);
    const double k = pv[ipv * npar + 6 + pb];          // uniform in the workgroup
    R* o = out + r * 2 * g.ng;
    const double u = (k - g.k0) / g.dk;
    int ik = int(floor(u));
    ik = ik < 0 ? 0 : (ik > g.nk - 2 ? g.nk - 2 : ik);
    R r0 = R(0), r1 = R(0);                           // invalid rows: NaN from the setup
    if (k < k_small) {
        if (k > 0.0) {
            const double* f = prof + int64_t(pb) * nmu;
            const bool staged = nmu <= kSpLds;
            if (staged) {
                for (int j = threadIdx.x; j < nmu; j += kBlock) {
                    smu[j] = mu_s[j];
                    sf[j] = f[j];
                }
                __syncthreads();
            }
            if (m >= g.ng) return;
            const double* ms = staged ? smu : mu_s;
            const double* fs = staged ? sf : f;
            const double gm = double(m) / double(g.ng - 1);
            const double craw = gm * (1.0 + k);
            const double c = craw < 1.0 ? craw : 1.0;
            const double v = profile_at_bin(ms, fs, nmu, c);
            double D = 0.0;
            const double mu = sqrt(1.0 - c * c);
            if (craw < 1.0 && mu > ms[0] && mu < ms[nmu - 1]) {
                int lo = 0, hi = nmu - 1;                  // ms[lo] <= mu < ms[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (ms[mid] <= mu) lo = mid; else hi = mid;
                }
                const double slope = (fs[lo + 1] - fs[lo]) / (ms[lo + 1] - ms[lo]);
                D = slope * (-c / mu) * gm;
            }
            const double ak = u - ik;
            const double b0 = v - ak * g.dk * D;
            r0 = R(b0);
            r1 = R(b0 + g.dk * D);
        }
    } else {
        if (m >= g.ng) return;
        const R* t0r = T + (int64_t(pb) * g.nk + ik) * g.ng;
        r0 = t0r[m];
        r1 = t0r[g.ng + m];
    }
    if (m >= g.ng) return;
    o[m] = r0;
    o[g.ng + m] = r1;
    if (m == 0) inv_istar_rows[r] = inv_istar[pb];
}

hipError_t launch_small_planet_adj_rows(const rr_tables* t, const double* pv, int32_t npv,
                                        int32_t npar, double k_small, int32_t precision,
                                        void* rows, double* inv_istar_rows, hipStream_t s) {
    const GridDev g = grid_dev(t);
    const int64_t nr = int64_t(npv) * t->npb;
    const dim3 grid(unsigned(nr), unsigned((g.ng + kBlock - 1) / kBlock));
    if (precision == RR_FP64)
        hipLaunchKernelGGL(k_small_planet_adj_rows<double>, grid, dim3(kBlock), 0, s, t->mu_s,
                           t->prof, t->nmu, t->T64, t->inv_istar, pv, npar, k_small, g,
                           static_cast<double*>(rows), inv_istar_rows);
    else
        hipLaunchKernelGGL(k_small_planet_adj_rows<float>, grid, dim3(kBlock), 0, s, t->mu_s,
                           t->prof, t->nmu, t->T32, t->inv_istar, pv, npar, k_small, g,
                           static_cast<float*>(rows), inv_istar_rows);
    return hipGetLastError();
}

hipError_t launch_small_planet_rows(const rr_tables* t, const double* pv, int32_t npv,
                                    int32_t npar, double k_small, int32_t precision,
                                    void* rows, hipStream_t s) {
    const GridDev g = grid_dev(t);
    const int64_t nr = int64_t(npv) * t->npb;
    const dim3 grid(unsigned(nr), unsigned((g.ng + kBlock - 1) / kBlock));
    if (precision == RR_FP64)
        hipLaunchKernelGGL(k_small_planet_rows<double>, grid, dim3(kBlock), 0, s, t->mu_s,
                           t->prof, t->nmu, t->T64, pv, npar, k_small, t->grid.k1, g,
                           static_cast<double*>(rows));
    else
        hipLaunchKernelGGL(k_small_planet_rows<float>, grid, dim3(kBlock), 0, s, t->mu_s,
                           t->prof, t->nmu, t->T32, pv, npar, k_small, t->grid.k1, g,
                           static_cast<float*>(rows));
    return hipGetLastError();
}

hipError_t launch_pv_ld(const rr_tables* t, const double* prof, const double* pv,
                        int32_t npv, int32_t npar, int32_t precision, double* ldp,
                        double* istar, double* inv_istar, int32_t* ikr, int32_t* perm,
                        void* rows, hipStream_t s, bool w32) {
    const GridDev g = grid_dev(t);
    const int64_t nr = int64_t(npv) * t->npb;     // (vector, passband) rows
    hipLaunchKernelGGL(k_pv_prep, dim3(unsigned(nr + 1)), dim3(kBlock), 0, s, t->mu_s, prof,
                       t->nmu, t->zm, t->nz, pv, npv, npar, g, ldp, istar, inv_istar, ikr, perm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // matrix-core tiles rounded up to whole rounds of the XCDs, then the
    // per-row blocks; both parts read the same weights (FP64, or the FP32
    // copy with w32), so a row's values do not depend on which part took it
    const int64_t n_mfma = ((nr + 15) / 16 * ((g.ng + 63) / 64) + kXcds - 1) / kXcds * kXcds;
    const int64_t n_rows = nr * ((g.ng + kBlock - 1) / kBlock);
    if (n_mfma + n_rows >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    const dim3 grid(unsigned(n_mfma + n_rows));
    if (precision == RR_FP64)
        hipLaunchKernelGGL((k_pv_tables<double, double>), grid, dim3(kBlock), 0, s, t->W, ldp,
                           ikr, perm, nr, t->nz, g, n_mfma, static_cast<double*>(rows));
    else if (w32)
        hipLaunchKernelGGL((k_pv_tables<float, float>), grid, dim3(kBlock), 0, s, t->W32, ldp,
                           ikr, perm, nr, t->nz, g, n_mfma, static_cast<float*>(rows));
    else
        hipLaunchKernelGGL((k_pv_tables<float, double>), grid, dim3(kBlock), 0, s, t->W, ldp,
                           ikr, perm, nr, t->nz, g, n_mfma, static_cast<float*>(rows));
    return hipGetLastError();
}

__global__ void k_istar_set(const double* __restrict__ src, int32_t npb,
                            double* __restrict__ user, double* __restrict__ istar,
                            double* __restrict__ inv_istar) {
    const int pb = blockIdx.x * blockDim.x + threadIdx.x;
    if (pb >= npb) return;
    const double v = src[pb];
    if (user) user[pb] = v;
    istar[pb] = v;
    inv_istar[pb] = (v > 0.0 && is_finite(v)) ? 1.0 / v : NAN;
}

hipError_t launch_istar_set(rr_tables* t, const double* src, hipStream_t s) {
    hipLaunchKernelGGL(k_istar_set, dim3(1), dim3(kBlock), 0, s, src, t->npb,
                       src == t->istar_user ? nullptr : t->istar_user, t->istar, t->inv_istar);
    return hipGetLastError();
}

hipError_t launch_istar_from_profile(rr_tables* t, hipStream_t s) {
    hipLaunchKernelGGL(k_istar, dim3(t->npb), dim3(kBlock), 0, s, t->mu_s, t->prof,
                       t->nmu, t->istar, t->inv_istar);
    return hipGetLastError();
}

hipError_t launch_prepare_profile(rr_tables* t, hipStream_t s) {
    const GridDev g = grid_dev(t);
    hipLaunchKernelGGL(k_profile, dim3(nblocks(int64_t(t->nz) * t->npb)), dim3(kBlock), 0, s,
                       t->mu_s, t->prof, t->nmu, t->zm, t->nz, t->npb, t->ldp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the caller's normalisers, if set, stay in force over a new profile
    e = t->istar_fixed ? launch_istar_set(t, t->istar_user, s) : launch_istar_from_profile(t, s);
    if (e != hipSuccess) return e;
    const int64_t nt = int64_t(g.npb) * g.nk * g.ng;
    hipLaunchKernelGGL(k_tables, dim3(nblocks(nt)), dim3(kBlock), 0, s, t->W, t->ldp, g,
                       t->T64, t->T32);
    return hipGetLastError();
}

}  // namespace rr
