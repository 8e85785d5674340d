// MDLG coarse-graining of a stored trajectory for many coarse-graining times
// and lattice drifts at once (Eq.(n_i) evaluated for every snapshot pair).
//
// Snapshots p = 0 .. P-1 of a batch of replicas are stacked as
// pos[P][n_tot][2], img[P][n_tot][2].  A job (l, u) takes every pair
// (p - l, p): the lattice of the pair is translated by o dx at the earlier
// snapshot and by (o + u) dx at the later one (one coarse step of a lattice
// moving u cells per coarse step), with o = offset[p - l] the origin chosen for
// pairs starting at snapshot p - l.  A homogeneous gas has the same statistics
// under every translation of the lattice; origins that vary between pairs
// decorrelate the cell-crossing events of overlapping pairs.
//
// One thread per particle walks the snapshots once.  A ring in LDS keeps what
// it needs of its last lmax snapshots, so every snapshot is read from HBM once
// for all jobs; the block's histograms [jobs][50] sit in LDS (a wave ballot
// for the rest velocity, LDS atomics otherwise) and are flushed with one
// global atomic per non-empty bin.  Box-frame displacement moments are per
// lag (they do not depend on u) and come from a second, lighter pass over the
// snapshots: per-wave LDS sums, per-block partials and a fixed-order final
// sum, bitwise reproducible.  Two passes keep each kernel's LDS small enough
// for several blocks per compute unit.
#include <cmath>
#include <cstring>
#include <vector>

#include "mdlg_internal.h"

namespace mdlg {
namespace {

__constant__ VelLut c_lut_series = kLut;

constexpr int kSeriesBS = 128;      // threads (particles) per block
constexpr int kSeriesMaxLag = 32;   // ring depth
constexpr int kSeriesMaxLags = 32;
constexpr int kSeriesMaxU = 16;
constexpr int kSeriesMaxJobs = 256;

struct SeriesBlock {
    long long start;  // first particle (index into n_tot)
    int count;        // particles in this block (<= kSeriesBS)
    int rep;          // replica
};

struct SeriesArgs {
    const double2* __restrict__ pos;
    const int2* __restrict__ img;
    long long n_tot;
    int n_snap, n_lag, n_u, ring;
    const SeriesBlock* __restrict__ blocks;
    const int* __restrict__ lx;        // [n_rep]
    const double* __restrict__ inv;    // [n_rep] lx / L
    const double* __restrict__ box;    // [n_rep] L
    const double* __restrict__ dxl;    // [n_rep] L / lx
    const double* __restrict__ u;      // [n_u][2] cells per coarse step
    const double* __restrict__ off;    // [n_snap][2] lattice origin per pair start, cells
    const int* __restrict__ lags;      // [n_lag]
    unsigned long long* __restrict__ counts;  // [n_rep][n_lag][n_u][50]
    int* __restrict__ err;                    // set when an unwrapped cell leaves the 32-bit range
    double* __restrict__ mpart;               // [n_blocks][n_lag][4]
};

__device__ __forceinline__ double delta_box(double xc, double xp, int di, double L) {
#pragma clang fp contract(off)
    double d = xc - xp;
    double w = L * (double)di;
    return d + w;
}

// lattice shift arithmetic, each operation rounded once as written
__device__ __forceinline__ double scaled(double o, double dxl) {
#pragma clang fp contract(off)
    return o * dxl;
}
__device__ __forceinline__ double sum(double a, double b) {
#pragma clang fp contract(off)
    return a + b;
}

// Counts.  The ring keeps, per particle and snapshot, the unwrapped cell
// q + lx * img on that snapshot's own translated lattice, as two 32-bit
// integers (8 bytes, so that four blocks fit a compute unit); a cell beyond
// the 32-bit range raises *a.err.  The block's histograms are indexed by the
// raw displacement (vy + 3) * 7 + (vx + 3) (49 = beyond |v_a| <= 3) and mapped
// to the D2Q49 numbering when they are flushed; they hold two 16-bit counters
// per word (a block adds at most kSeriesBS x (n_snap - 1) < 2^16 events to
// one bin).
__global__ __launch_bounds__(kSeriesBS) void k_cg_series_counts(SeriesArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int njobs = a.n_lag * a.n_u;
    constexpr int HW = MDLG_NCOUNTS / 2;                              // words per job
    int2* ring = reinterpret_cast<int2*>(smem);                       // [ring][BS]
    unsigned* hist = reinterpret_cast<unsigned*>(ring + a.ring * kSeriesBS);  // [njobs][25]
    __shared__ signed char lut[MDLG_NQ];
    if (tid < MDLG_NQ) lut[tid] = c_lut_series.idx[tid];
    for (int i = tid; i < njobs * HW; i += kSeriesBS) hist[i] = 0u;
    __syncthreads();

    const SeriesBlock blk = a.blocks[blockIdx.x];
    const bool act = tid < blk.count;
    const long long j = blk.start + (act ? tid : 0);
    const int r = blk.rep;
    const long long lx = a.lx[r];
    const double inv = a.inv[r], dxl = a.dxl[r];

    for (int p = 0; p < a.n_snap; ++p) {
        double2 xc = make_double2(0.0, 0.0);
        int2 ic = make_int2(0, 0);
        if (act) {
            xc = a.pos[(long long)p * a.n_tot + j];
            ic = a.img[(long long)p * a.n_tot + j];
        }
        for (int s = 0; s < a.n_lag; ++s) {
            const int l = a.lags[s];
            if (p < l) continue;  // uniform over the block
            const int2 prev = ring[((p - l) % a.ring) * kSeriesBS + tid];
            const double ox = a.off[2 * (p - l)], oy = a.off[2 * (p - l) + 1];
            const long long bx = lx * (long long)ic.x - prev.x, by = lx * (long long)ic.y - prev.y;
            for (int t = 0; t < a.n_u; ++t) {
                const double sx = scaled(sum(ox, a.u[2 * t]), dxl), sy = scaled(sum(oy, a.u[2 * t + 1]), dxl);
                const long long vx = lattice_q(xc.x, sx, inv) + bx;
                const long long vy = lattice_q(xc.y, sy, inv) + by;
                const int raw = (vx >= -3 && vx <= 3 && vy >= -3 && vy <= 3) ? (int)((vy + 3) * 7 + (vx + 3)) : MDLG_NQ;
                unsigned* h = hist + (s * a.n_u + t) * HW;
                // the rest velocity (raw 24), taken by most particles: one
                // ballot and a single-lane add; the others: per-lane LDS atomics
                const unsigned long long b = __ballot(act && raw == 24);
                if (lane == 0 && b) atomicAdd(&h[12], (unsigned)__popcll(b));
                if (act && raw != 24) atomicAdd(&h[raw >> 1], (raw & 1) ? 65536u : 1u);
            }
        }
        // every lag has read its slot: the ring entry of p - ring may go
        __syncthreads();
        const double ox = a.off[2 * p], oy = a.off[2 * p + 1];
        const long long cx = lattice_q(xc.x, scaled(ox, dxl), inv) + lx * ic.x;
        const long long cy = lattice_q(xc.y, scaled(oy, dxl), inv) + lx * ic.y;
        const long long lim = 0x7fffffffLL;
        if (act && (cx > lim || cx < -lim || cy > lim || cy < -lim)) atomicOr(a.err, 1);
        ring[(p % a.ring) * kSeriesBS + tid] = make_int2((int)cx, (int)cy);
        __syncthreads();
    }
    unsigned long long* cnt = a.counts + (long long)r * njobs * MDLG_NCOUNTS;
    for (int i = tid; i < njobs * HW; i += kSeriesBS) {
        const unsigned w = hist[i];
        const int job = i / HW, raw = 2 * (i % HW);
        const int b0 = lut[raw], b1 = raw + 1 < MDLG_NQ ? lut[raw + 1] : MDLG_NQ;
        if (w & 0xFFFFu) atomicAdd(&cnt[job * MDLG_NCOUNTS + b0], (unsigned long long)(w & 0xFFFFu));
        if (w >> 16) atomicAdd(&cnt[job * MDLG_NCOUNTS + b1], (unsigned long long)(w >> 16));
    }
}

// Box-frame displacement moments per lag: a ring of positions and image
// counts, per-wave sums in LDS, per-block partials.
__global__ __launch_bounds__(kSeriesBS) void k_cg_series_disp(SeriesArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = kSeriesBS / 64;
    double2* rp = reinterpret_cast<double2*>(smem);                 // [ring][BS]
    int2* ri = reinterpret_cast<int2*>(rp + a.ring * kSeriesBS);     // [ring][BS]
    double* wm = reinterpret_cast<double*>(ri + a.ring * kSeriesBS);  // [NW][n_lag][4]
    for (int i = tid; i < NW * a.n_lag * 4; i += kSeriesBS) wm[i] = 0.0;
    __syncthreads();
    const SeriesBlock blk = a.blocks[blockIdx.x];
    const bool act = tid < blk.count;
    const long long j = blk.start + (act ? tid : 0);
    const double L = a.box[blk.rep];
    for (int p = 0; p < a.n_snap; ++p) {
        double2 xc = make_double2(0.0, 0.0);
        int2 ic = make_int2(0, 0);
        if (act) {
            xc = a.pos[(long long)p * a.n_tot + j];
            ic = a.img[(long long)p * a.n_tot + j];
        }
        for (int s = 0; s < a.n_lag; ++s) {
            const int l = a.lags[s];
            if (p < l) continue;
            const int slot = (p - l) % a.ring;
            const double2 xp = rp[slot * kSeriesBS + tid];
            const int2 ip = ri[slot * kSeriesBS + tid];
            double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
            if (act) {
                const double dx = delta_box(xc.x, xp.x, ic.x - ip.x, L);
                const double dy = delta_box(xc.y, xp.y, ic.y - ip.y, L);
                const double dx2 = dx * dx, dy2 = dy * dy;
                m0 = dx2 + dy2;
                m1 = dx2 * dx2 + dy2 * dy2;
                m2 = dx;
                m3 = dy;
            }
            m0 = wave_sum(m0);
            m1 = wave_sum(m1);
            m2 = wave_sum(m2);
            m3 = wave_sum(m3);
            if (lane == 0) {
                double* w = wm + (wave * a.n_lag + s) * 4;
                w[0] += m0;
                w[1] += m1;
                w[2] += m2;
                w[3] += m3;
            }
        }
        __syncthreads();
        rp[(p % a.ring) * kSeriesBS + tid] = xc;
        ri[(p % a.ring) * kSeriesBS + tid] = ic;
        __syncthreads();
    }
    for (int i = tid; i < a.n_lag * 4; i += kSeriesBS) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += wm[w * a.n_lag * 4 + i];
        a.mpart[(long long)blockIdx.x * a.n_lag * 4 + i] = t;
    }
}

// moments[r][s] += (2 n_r (P - l_s), sums over the replica's blocks in order)
__global__ void k_series_moments(const double* __restrict__ mpart, const int* __restrict__ rep_block0,
                                 const long long* __restrict__ rep_n, const int* __restrict__ lags, int n_lag,
                                 int n_snap, double* __restrict__ moments) {
    const int r = blockIdx.x;
    for (int i = threadIdx.x; i < n_lag * 5; i += blockDim.x) {
        const int s = i / 5, c = i % 5;
        if (c == 0) {
            moments[((long long)r * n_lag + s) * 5] += 2.0 * (double)rep_n[r] * (double)(n_snap - lags[s]);
            continue;
        }
        double t = 0.0;
        for (int b = rep_block0[r]; b < rep_block0[r + 1]; ++b) t += mpart[((long long)b * n_lag + s) * 4 + c - 1];
        moments[((long long)r * n_lag + s) * 5 + c] += t;
    }
}

}  // namespace
}  // namespace mdlg

using namespace mdlg;

extern "C" mdlg_status mdlg_coarse_grain_series(int32_t n_rep, const int64_t* offsets, const double* box_l,
                                                const int32_t* lx, int32_t n_snap, const double* pos,
                                                const int32_t* img, int32_t n_lag, const int32_t* lags, int32_t n_u,
                                                const double* u, const double* offset, int64_t* counts,
                                                double* moments, void* stream) {
    const char* who = "mdlg_coarse_grain_series: ";
    if (n_rep < 1 || !offsets || !box_l || !lx || !lags || !u || !counts || !pos || !img)
        return fail(MDLG_EINVAL, std::string(who) + "NULL argument or n_rep < 1");
    if (n_lag < 1 || n_lag > kSeriesMaxLags) return fail(MDLG_EINVAL, std::string(who) + "n_lag must be in [1, 32]");
    if (n_u < 1 || n_u > kSeriesMaxU) return fail(MDLG_EINVAL, std::string(who) + "n_u must be in [1, 16]");
    if (n_lag * n_u > kSeriesMaxJobs) return fail(MDLG_EINVAL, std::string(who) + "n_lag * n_u must be <= 256");
    if (n_snap < 2 || n_snap > 512) return fail(MDLG_EINVAL, std::string(who) + "n_snap must be in [2, 512]");
    int lmax = 0;
    for (int s = 0; s < n_lag; ++s) {
        if (lags[s] < 1 || lags[s] > kSeriesMaxLag || lags[s] >= n_snap)
            return fail(MDLG_EINVAL, std::string(who) + "lags must be in [1, min(32, n_snap - 1)]");
        lmax = lags[s] > lmax ? lags[s] : lmax;
    }
    for (int t = 0; t < 2 * n_u; ++t)
        if (!(std::fabs(u[t]) <= 1e6)) return fail(MDLG_EINVAL, std::string(who) + "u must be finite, |u| <= 1e6");
    std::vector<double> off(2 * (size_t)n_snap, 0.0);
    if (offset)
        for (int t = 0; t < 2 * n_snap; ++t) {
            if (!(std::fabs(offset[t]) <= 1e6))
                return fail(MDLG_EINVAL, std::string(who) + "lattice offsets must be finite, |offset| <= 1e6 cells");
            off[t] = offset[t];
        }
    if (offsets[0] != 0) return fail(MDLG_EINVAL, std::string(who) + "offsets[0] must be 0");
    std::vector<SeriesBlock> blocks;
    std::vector<int> rep_block0(n_rep + 1, 0);
    std::vector<long long> rep_n(n_rep);
    std::vector<double> inv(n_rep), dxl(n_rep);
    for (int r = 0; r < n_rep; ++r) {
        const long long n = offsets[r + 1] - offsets[r];
        if (n < 0) return fail(MDLG_EINVAL, std::string(who) + "offsets must be non-decreasing");
        if (lx[r] < 1 || lx[r] > 46340) return fail(MDLG_EINVAL, std::string(who) + "lx must be in [1, 46340]");
        if (!(box_l[r] > 0.0) || !std::isfinite(box_l[r])) return fail(MDLG_EINVAL, std::string(who) + "box_l must be > 0");
        rep_n[r] = n;
        inv[r] = (double)lx[r] / box_l[r];
        dxl[r] = box_l[r] / (double)lx[r];
        rep_block0[r] = (int)blocks.size();
        for (long long s0 = 0; s0 < n; s0 += kSeriesBS)
            blocks.push_back({offsets[r] + s0, (int)(n - s0 < kSeriesBS ? n - s0 : kSeriesBS), r});
    }
    rep_block0[n_rep] = (int)blocks.size();
    const long long n_tot = offsets[n_rep];
    hipStream_t st = (hipStream_t)stream;
    if (blocks.empty()) {
        // no particles: only the sample counts (zero) would change
        return MDLG_OK;
    }
    const int ring = lmax;
    const int nw = kSeriesBS / 64;
    const size_t lds_counts = (size_t)ring * kSeriesBS * sizeof(int2) + (size_t)n_lag * n_u * (MDLG_NCOUNTS / 2) * 4;
    const size_t lds_disp = (size_t)ring * kSeriesBS * (sizeof(double2) + sizeof(int2)) + (size_t)nw * n_lag * 4 * 8;
    if (lds_counts > 150 * 1024 || lds_disp > 150 * 1024)
        return fail(MDLG_EINVAL, std::string(who) + "lags and drifts exceed the LDS budget");
    // one device staging area for the small tables
    const size_t nb = blocks.size();
    const size_t bytes_blocks = sizeof(SeriesBlock) * nb;
    const size_t off_lx = (bytes_blocks + 255) / 256 * 256;
    const size_t off_inv = off_lx + ((sizeof(int) * n_rep + 255) / 256 * 256);
    const size_t off_box = off_inv + sizeof(double) * n_rep;
    const size_t off_dxl = off_box + sizeof(double) * n_rep;
    const size_t off_u = off_dxl + sizeof(double) * n_rep;
    const size_t off_off = off_u + sizeof(double) * 2 * n_u;
    const size_t off_lags = off_off + sizeof(double) * off.size();
    const size_t off_b0 = off_lags + sizeof(int) * kSeriesMaxLags;
    const size_t off_rn = (off_b0 + sizeof(int) * (n_rep + 1) + 7) / 8 * 8;
    const size_t off_err = off_rn + sizeof(long long) * n_rep;
    const size_t off_mp = (off_err + sizeof(int) + 255) / 256 * 256;
    const size_t total = off_mp + sizeof(double) * nb * n_lag * 4;
    std::vector<unsigned char> host(off_mp, 0);
    std::memcpy(host.data(), blocks.data(), bytes_blocks);
    std::memcpy(host.data() + off_lx, lx, sizeof(int) * n_rep);
    std::memcpy(host.data() + off_inv, inv.data(), sizeof(double) * n_rep);
    std::memcpy(host.data() + off_box, box_l, sizeof(double) * n_rep);
    std::memcpy(host.data() + off_dxl, dxl.data(), sizeof(double) * n_rep);
    std::memcpy(host.data() + off_u, u, sizeof(double) * 2 * n_u);
    std::memcpy(host.data() + off_off, off.data(), sizeof(double) * off.size());
    std::memcpy(host.data() + off_lags, lags, sizeof(int) * n_lag);
    std::memcpy(host.data() + off_b0, rep_block0.data(), sizeof(int) * (n_rep + 1));
    std::memcpy(host.data() + off_rn, rep_n.data(), sizeof(long long) * n_rep);
    unsigned char* dev = nullptr;
    MDLG_HIP(hipMallocAsync((void**)&dev, total, st));
    hipError_t e = hipMemcpyAsync(dev, host.data(), off_mp, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host table is freed on return
    SeriesArgs a{};
    a.pos = (const double2*)pos;
    a.img = (const int2*)img;
    a.n_tot = n_tot;
    a.n_snap = n_snap;
    a.n_lag = n_lag;
    a.n_u = n_u;
    a.ring = ring;
    a.blocks = (const SeriesBlock*)dev;
    a.lx = (const int*)(dev + off_lx);
    a.inv = (const double*)(dev + off_inv);
    a.box = (const double*)(dev + off_box);
    a.dxl = (const double*)(dev + off_dxl);
    a.u = (const double*)(dev + off_u);
    a.off = (const double*)(dev + off_off);
    a.lags = (const int*)(dev + off_lags);
    a.counts = (unsigned long long*)counts;
    a.mpart = (double*)(dev + off_mp);
    a.err = (int*)(dev + off_err);
    if (e == hipSuccess && lds_counts > 64 * 1024)
        e = hipFuncSetAttribute((const void*)k_cg_series_counts, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_counts);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_cg_series_counts, dim3((unsigned)nb), dim3(kSeriesBS), lds_counts, st, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess && moments && lds_disp > 64 * 1024)
        e = hipFuncSetAttribute((const void*)k_cg_series_disp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_disp);
    if (e == hipSuccess && moments) {
        hipLaunchKernelGGL(k_cg_series_disp, dim3((unsigned)nb), dim3(kSeriesBS), lds_disp, st, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess && moments) {
        hipLaunchKernelGGL(k_series_moments, dim3((unsigned)n_rep), dim3(64), 0, st, (const double*)a.mpart,
                           (const int*)(dev + off_b0), (const long long*)(dev + off_rn), a.lags, n_lag, n_snap,
                           moments);
        e = hipGetLastError();
    }
    int err = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&err, a.err, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipError_t e2 = hipFreeAsync(dev, st);
    MDLG_HIP(e);
    MDLG_HIP(e2);
    if (err)
        return fail(MDLG_EINVAL, std::string(who) + "an unwrapped cell q + lx * img exceeds 32 bits (counts unspecified)");
    return MDLG_OK;
}
