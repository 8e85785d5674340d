// Histograms of the one-particle displacements of a stored trajectory (the
// binned displacement PDF P^MD(X_i) that Fig. 2 sets beside the single
// Gaussian Eq.(gaussian_df) and the Poisson WSG Eq.(poisson_v2)).
//
// Snapshots p = 0 .. P-1 of a batch of replicas are stacked as
// pos[P][n_tot][2], img[P][n_tot][2] (the layout of the trajectory
// coarse-graining).  For lag l every pair (p - l, p) contributes the
// box-frame displacement delta = (x_p - x_{p-l}) + L (img_p - img_{p-l}) of
// every particle, per axis, to the bins X_k = [(k - n_bin/2) h, (k + 1 -
// n_bin/2) h), k = floor(delta * (1/h) + n_bin/2) rounded once per operation.
//
// The work is HBM-bound: 48 bytes of snapshot data per particle pair and two
// LDS counter increments.  A block owns 256 particles of one replica, one lag
// and one chunk of snapshot pairs; its two per-axis histograms sit in LDS
// (32-bit, at most 256 x 2^24 counts a bin) and are added to the int64 output
// with one global atomic per non-empty bin.
#include <cmath>
#include <cstring>
#include <vector>

#include "mdlg_internal.h"

namespace mdlg {
namespace {

constexpr int kHistBS = 256;
constexpr int kHistMaxLags = 64;
constexpr int kHistMaxSnap = 1 << 24;
constexpr int kHistTargetBlocks = 4096;  // enough waves in flight to cover HBM latency

struct HistBlock {
    long long start;  // first particle (index into n_tot)
    int count;        // particles in this block (<= kHistBS)
    int rep;          // replica
};

struct HistArgs {
    const double2* __restrict__ pos;
    const int2* __restrict__ img;
    long long n_tot;
    int n_snap, n_bin, n_lag, n_chunk;
    double half;                               // n_bin / 2
    const HistBlock* __restrict__ blocks;
    const double* __restrict__ box;            // [n_rep]
    const int* __restrict__ lags;              // [n_lag]
    const double* __restrict__ inv_h;          // [n_lag] 1 / h
    unsigned long long* __restrict__ hist;     // [n_rep][n_lag][2][n_bin + 2]
};

__device__ __forceinline__ double box_delta(double xc, double xp, int di, double L) {
#pragma clang fp contract(off)
    const double d = xc - xp;
    const double w = L * (double)di;
    return d + w;
}

__device__ __forceinline__ int disp_bin(double d, double inv_h, double half, int n_bin) {
#pragma clang fp contract(off)
    const double s = d * inv_h;
    const double t = s + half;
    if (t >= 0.0 && t < (double)n_bin) return (int)floor(t);
    return t < 0.0 ? n_bin : n_bin + 1;
}

__global__ __launch_bounds__(kHistBS) void k_disp_hist(HistArgs a) {
    extern __shared__ unsigned hl[];  // [2][n_bin + 2]
    const int tid = threadIdx.x;
    const int nb2 = 2 * (a.n_bin + 2);
    for (int i = tid; i < nb2; i += kHistBS) hl[i] = 0u;
    __syncthreads();
    const HistBlock blk = a.blocks[blockIdx.x];
    const int s = blockIdx.y;
    const int l = a.lags[s];
    // this block's share of the pairs p = l .. n_snap - 1
    const int npair = a.n_snap - l;
    const int span = (npair + a.n_chunk - 1) / a.n_chunk;
    const int p0 = l + (int)blockIdx.z * span;
    const int p1 = min(a.n_snap, p0 + span);
    if (tid < blk.count && p0 < p1) {
        const double L = a.box[blk.rep];
        const double inv = a.inv_h[s];
        const long long j = blk.start + tid;
        unsigned* hx = hl;
        unsigned* hy = hl + a.n_bin + 2;
#pragma unroll 4
        for (int p = p0; p < p1; ++p) {
            const double2 xc = a.pos[(long long)p * a.n_tot + j];
            const double2 xp = a.pos[(long long)(p - l) * a.n_tot + j];
            const int2 ic = a.img[(long long)p * a.n_tot + j];
            const int2 ip = a.img[(long long)(p - l) * a.n_tot + j];
            const int bx = disp_bin(box_delta(xc.x, xp.x, ic.x - ip.x, L), inv, a.half, a.n_bin);
            const int by = disp_bin(box_delta(xc.y, xp.y, ic.y - ip.y, L), inv, a.half, a.n_bin);
            atomicAdd(hx + bx, 1u);
            atomicAdd(hy + by, 1u);
        }
    }
    __syncthreads();
    unsigned long long* out = a.hist + ((long long)blk.rep * a.n_lag + s) * nb2;
    for (int i = tid; i < nb2; i += kHistBS) {
        const unsigned c = hl[i];
        if (c) atomicAdd(out + i, (unsigned long long)c);
    }
}

}  // namespace
}  // namespace mdlg

using namespace mdlg;

extern "C" mdlg_status mdlg_displacement_hist(int32_t n_rep, const int64_t* offsets, const double* box_l,
                                              int32_t n_snap, const double* pos, const int32_t* img,
                                              int32_t n_lag, const int32_t* lags, const double* bin_width,
                                              int32_t n_bin, int64_t* hist, void* stream) {
    const char* who = "mdlg_displacement_hist: ";
    if (n_rep < 1 || !offsets || !box_l || !lags || !bin_width || !hist || !pos || !img)
        return fail(MDLG_EINVAL, std::string(who) + "NULL argument or n_rep < 1");
    if (n_lag < 1 || n_lag > kHistMaxLags) return fail(MDLG_EINVAL, std::string(who) + "n_lag must be in [1, 64]");
    if (n_snap < 2 || n_snap > kHistMaxSnap)
        return fail(MDLG_EINVAL, std::string(who) + "n_snap must be in [2, 2^24]");
    if (n_bin < 1 || n_bin > MDLG_HIST_MAX_BINS)
        return fail(MDLG_EINVAL, std::string(who) + "n_bin must be in [1, MDLG_HIST_MAX_BINS]");
    std::vector<double> inv_h(n_lag);
    int lmin = n_snap;
    for (int s = 0; s < n_lag; ++s) {
        if (lags[s] < 1 || lags[s] >= n_snap) return fail(MDLG_EINVAL, std::string(who) + "lags must be in [1, n_snap - 1]");
        if (!(bin_width[s] > 0.0) || !std::isfinite(bin_width[s]))
            return fail(MDLG_EINVAL, std::string(who) + "bin widths must be finite and > 0");
        inv_h[s] = 1.0 / bin_width[s];
        if (!std::isfinite(inv_h[s])) return fail(MDLG_EINVAL, std::string(who) + "bin width too small");
        lmin = lags[s] < lmin ? lags[s] : lmin;
    }
    if (offsets[0] != 0) return fail(MDLG_EINVAL, std::string(who) + "offsets[0] must be 0");
    std::vector<HistBlock> blocks;
    for (int r = 0; r < n_rep; ++r) {
        const long long n = offsets[r + 1] - offsets[r];
        if (n < 0) return fail(MDLG_EINVAL, std::string(who) + "offsets must be non-decreasing");
        if (!(box_l[r] > 0.0) || !std::isfinite(box_l[r])) return fail(MDLG_EINVAL, std::string(who) + "box_l must be > 0");
        for (long long s0 = 0; s0 < n; s0 += kHistBS)
            blocks.push_back({offsets[r] + s0, (int)(n - s0 < kHistBS ? n - s0 : kHistBS), r});
    }
    if (blocks.empty()) return MDLG_OK;  // no particles, nothing to add
    const long long nb = (long long)blocks.size();
    if (nb >= (1LL << 24)) return fail(MDLG_EINVAL, std::string(who) + "too many particles (grid limit)");
    // split the snapshot pairs so that the grid holds enough blocks
    long long want = (kHistTargetBlocks + nb * n_lag - 1) / (nb * n_lag);
    const int n_chunk = (int)std::max(1LL, std::min<long long>({want, (long long)(n_snap - lmin), 65535LL}));
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes_blocks = sizeof(HistBlock) * blocks.size();
    const size_t off_box = (bytes_blocks + 255) / 256 * 256;
    const size_t off_inv = off_box + sizeof(double) * n_rep;
    const size_t off_lags = off_inv + sizeof(double) * n_lag;
    const size_t total = off_lags + sizeof(int) * n_lag;
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data(), blocks.data(), bytes_blocks);
    std::memcpy(host.data() + off_box, box_l, sizeof(double) * n_rep);
    std::memcpy(host.data() + off_inv, inv_h.data(), sizeof(double) * n_lag);
    std::memcpy(host.data() + off_lags, lags, sizeof(int) * n_lag);
    unsigned char* dev = nullptr;
    MDLG_HIP(hipMallocAsync((void**)&dev, total, st));
    hipError_t e = hipMemcpyAsync(dev, host.data(), total, hipMemcpyHostToDevice, st);
    const bool copied = e == hipSuccess;
    HistArgs a{};
    a.pos = (const double2*)pos;
    a.img = (const int2*)img;
    a.n_tot = offsets[n_rep];
    a.n_snap = n_snap;
    a.n_bin = n_bin;
    a.n_lag = n_lag;
    a.n_chunk = n_chunk;
    a.half = 0.5 * (double)n_bin;
    a.blocks = (const HistBlock*)dev;
    a.box = (const double*)(dev + off_box);
    a.inv_h = (const double*)(dev + off_inv);
    a.lags = (const int*)(dev + off_lags);
    a.hist = (unsigned long long*)hist;
    const size_t lds = sizeof(unsigned) * 2 * ((size_t)n_bin + 2);
    if (e == hipSuccess && lds > 64 * 1024)
        e = hipFuncSetAttribute((const void*)k_disp_hist, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_disp_hist, dim3((unsigned)nb, (unsigned)n_lag, (unsigned)n_chunk), dim3(kHistBS), lds,
                           st, a);
        e = hipGetLastError();
    }
    // the host table must outlive the copy: wait before it goes out of scope
    if (copied) {
        const hipError_t es = hipStreamSynchronize(st);
        if (e == hipSuccess) e = es;
    }
    hipError_t e2 = hipFreeAsync(dev, st);
    MDLG_HIP(e);
    MDLG_HIP(e2);
    return MDLG_OK;
}
