// Velocity autocorrelation of stored velocity snapshots, and the average
// number of collisions per coarse step read from it (the alternative to the
// moment matching of Eq.(lambda_eq) that the WSG section names).
//
// k_vacf: one thread per particle and lag walks the origins p and sums
// v(p) . v(p + lag) in FP64; waves reduce by shuffles, the block's waves are
// added in a fixed order into one partial per (block, lag), and k_vacf_final
// adds the partials of each replica in block order: the result is bitwise
// reproducible.  Each (particle, origin, lag) reads two 16-byte velocities.
#include <cmath>
#include <cstring>
#include <vector>

#include "mdlg_internal.h"

namespace mdlg {
namespace {

constexpr int kVacfBS = 256;
constexpr int kVacfMaxLags = 1024;

struct VacfBlock {
    long long start;
    int count;
    int rep;
};

__global__ __launch_bounds__(kVacfBS) void k_vacf(const double2* __restrict__ vel, long long n_tot, int n_snap,
                                                  const VacfBlock* __restrict__ blocks, const int* __restrict__ lags,
                                                  int n_lag, double* __restrict__ part) {
    __shared__ double ws[kVacfBS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const VacfBlock blk = blocks[blockIdx.x];
    const int s = blockIdx.y;
    const int l = lags[s];
    double acc = 0.0;
    if (tid < blk.count) {
        const long long j = blk.start + tid;
        for (int p = 0; p + l < n_snap; ++p) {
            const double2 a = vel[(long long)p * n_tot + j];
            const double2 b = vel[(long long)(p + l) * n_tot + j];
            acc += a.x * b.x + a.y * b.y;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) ws[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kVacfBS / 64; ++w) t += ws[w];
        part[(long long)blockIdx.x * n_lag + s] = t;
    }
}

// c[r][s] += sum over the replica's blocks, in block order
__global__ void k_vacf_final(const double* __restrict__ part, const int* __restrict__ rep_block0, int n_lag,
                             double* __restrict__ c) {
    const int r = blockIdx.x;
    for (int s = threadIdx.x; s < n_lag; s += blockDim.x) {
        double t = 0.0;
        for (int b = rep_block0[r]; b < rep_block0[r + 1]; ++b) t += part[(long long)b * n_lag + s];
        c[(long long)r * n_lag + s] += t;
    }
}

}  // namespace
}  // namespace mdlg

using namespace mdlg;

extern "C" mdlg_status mdlg_vacf(int32_t n_rep, const int64_t* offsets, int32_t n_snap, const double* vel,
                                 int32_t n_lag, const int32_t* lags, double* c_sum, void* stream) {
    const char* who = "mdlg_vacf: ";
    if (n_rep < 1 || !offsets || !vel || !lags || !c_sum)
        return fail(MDLG_EINVAL, std::string(who) + "NULL argument or n_rep < 1");
    if (n_snap < 1) return fail(MDLG_EINVAL, std::string(who) + "n_snap must be >= 1");
    if (n_lag < 1 || n_lag > kVacfMaxLags) return fail(MDLG_EINVAL, std::string(who) + "n_lag must be in [1, 1024]");
    for (int s = 0; s < n_lag; ++s)
        if (lags[s] < 0 || lags[s] >= n_snap) return fail(MDLG_EINVAL, std::string(who) + "lags must be in [0, n_snap - 1]");
    if (offsets[0] != 0) return fail(MDLG_EINVAL, std::string(who) + "offsets[0] must be 0");
    std::vector<VacfBlock> blocks;
    std::vector<int> rep_block0(n_rep + 1, 0);
    for (int r = 0; r < n_rep; ++r) {
        const long long n = offsets[r + 1] - offsets[r];
        if (n < 0) return fail(MDLG_EINVAL, std::string(who) + "offsets must be non-decreasing");
        rep_block0[r] = (int)blocks.size();
        for (long long s0 = 0; s0 < n; s0 += kVacfBS)
            blocks.push_back({offsets[r] + s0, (int)(n - s0 < kVacfBS ? n - s0 : kVacfBS), r});
        if (blocks.size() >= (1u << 24)) return fail(MDLG_EINVAL, std::string(who) + "too many particles (grid limit)");
    }
    rep_block0[n_rep] = (int)blocks.size();
    if (blocks.empty()) return MDLG_OK;
    hipStream_t st = (hipStream_t)stream;
    const size_t nb = blocks.size();
    const size_t off_b0 = (sizeof(VacfBlock) * nb + 255) / 256 * 256;
    const size_t off_lags = off_b0 + (sizeof(int) * (n_rep + 1) + 255) / 256 * 256;
    const size_t off_part = off_lags + (sizeof(int) * n_lag + 255) / 256 * 256;
    const size_t total = off_part + sizeof(double) * nb * n_lag;
    std::vector<unsigned char> host(off_part, 0);
    std::memcpy(host.data(), blocks.data(), sizeof(VacfBlock) * nb);
    std::memcpy(host.data() + off_b0, rep_block0.data(), sizeof(int) * (n_rep + 1));
    std::memcpy(host.data() + off_lags, lags, sizeof(int) * n_lag);
    unsigned char* dev = nullptr;
    MDLG_HIP(hipMallocAsync((void**)&dev, total, st));
    hipError_t e = hipMemcpyAsync(dev, host.data(), off_part, hipMemcpyHostToDevice, st);
    const bool copied = e == hipSuccess;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_vacf, dim3((unsigned)nb, (unsigned)n_lag), dim3(kVacfBS), 0, st, (const double2*)vel,
                           (long long)offsets[n_rep], n_snap, (const VacfBlock*)dev, (const int*)(dev + off_lags), n_lag,
                           (double*)(dev + off_part));
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_vacf_final, dim3((unsigned)n_rep), dim3(64), 0, st, (const double*)(dev + off_part),
                           (const int*)(dev + off_b0), n_lag, c_sum);
        e = hipGetLastError();
    }
    // the host table must outlive the copy
    if (copied) {
        const hipError_t es = hipStreamSynchronize(st);
        if (e == hipSuccess) e = es;
    }
    const hipError_t e2 = hipFreeAsync(dev, st);
    MDLG_HIP(e);
    MDLG_HIP(e2);
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_lambda_vacf(int32_t n, const double* t, const double* c, double dt_cg, double cut,
                                        double* tau, double* lambda) {
    const char* who = "mdlg_lambda_vacf: ";
    if (!t || !c || n < 2) return fail(MDLG_EINVAL, std::string(who) + "need t, c and n >= 2");
    if (!(c[0] > 0.0) || !std::isfinite(c[0])) return fail(MDLG_EINVAL, std::string(who) + "C(0) must be finite and > 0");
    if (!(dt_cg > 0.0) || !std::isfinite(dt_cg) || !(cut >= 0.0) || !(cut < 1.0))
        return fail(MDLG_EINVAL, std::string(who) + "need dt_cg > 0 and 0 <= cut < 1");
    if (t[0] != 0.0) return fail(MDLG_EINVAL, std::string(who) + "t[0] must be 0");
    double acc = 0.0;
    for (int k = 1; k < n; ++k) {
        if (!(t[k] > t[k - 1]) || !std::isfinite(c[k]))
            return fail(MDLG_EINVAL, std::string(who) + "t must increase and C be finite");
        acc += (t[k] - t[k - 1]) * (c[k] + c[k - 1]) / (2.0 * c[0]);
        if (c[k] <= cut * c[0]) break;
    }
    if (!(acc > 0.0)) return fail(MDLG_EINVAL, std::string(who) + "the integral of C is not positive");
    if (tau) *tau = acc;
    if (lambda) *lambda = dt_cg / acc;
    return MDLG_OK;
}
