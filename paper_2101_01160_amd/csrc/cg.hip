// MDLG coarse-graining of one pair of snapshots (Eq.(n_i)) on gfx950.
//
// One thread per particle: lattice coordinates q = floor((x + u dx k) lx / L)
// at both coarse steps, unwrapped cells C = q + lx * img, lattice velocity
// v = C(k_cur) - C(k_prev), D2Q49 index by table (overflow bin 49 outside
// |v_a| <= 3).  The block histogram is aggregated in LDS, with one wave ballot
// for the rest velocity that most particles take, then one global atomic per
// non-empty bin.  Displacement moments go through per-block partials and a
// fixed-order final sum, so they are bitwise reproducible.
#include <cmath>
#include <mutex>
#include <string>

#include "mdlg_internal.h"

namespace mdlg {

__constant__ VelLut c_lut = kLut;

struct CgArgs {
    const double2* __restrict__ xp;
    const int2* __restrict__ ip;
    const double2* __restrict__ xc;
    const int2* __restrict__ ic;
    long long n;
    int lx;
    double L, inv_lat, sxp, syp, sxc, syc;
    unsigned long long* __restrict__ counts;
    int* __restrict__ n_event;
    int* __restrict__ cell_acc;
    double* __restrict__ mpart;
};

// Box-frame displacement over the coarse step, rounded as written.
__device__ __forceinline__ double unwrapped_delta(double xc, double xp, int di, double L) {
#pragma clang fp contract(off)
    double d = xc - xp;
    double w = L * (double)di;
    return d + w;
}

template <int BS>
__global__ __launch_bounds__(BS) void k_coarse_grain(CgArgs a) {
    __shared__ int hist[MDLG_NCOUNTS];
    __shared__ double red[BS / 64][4];
    const int tid = threadIdx.x;
    if (tid < MDLG_NCOUNTS) hist[tid] = 0;
    __syncthreads();
    const long long j = (long long)blockIdx.x * BS + tid;
    const bool act = j < a.n;
    int idx = MDLG_NQ;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (act) {
        const double2 p0 = a.xp[j], p1 = a.xc[j];
        const int2 i0 = a.ip ? a.ip[j] : make_int2(0, 0);
        const int2 i1 = a.ic ? a.ic[j] : make_int2(0, 0);
        const long long lx = a.lx;
        const long long qx0 = lattice_q(p0.x, a.sxp, a.inv_lat), qy0 = lattice_q(p0.y, a.syp, a.inv_lat);
        const long long qx1 = lattice_q(p1.x, a.sxc, a.inv_lat), qy1 = lattice_q(p1.y, a.syc, a.inv_lat);
        const long long vx = (qx1 + lx * i1.x) - (qx0 + lx * i0.x);
        const long long vy = (qy1 + lx * i1.y) - (qy0 + lx * i0.y);
        if (vx >= -3 && vx <= 3 && vy >= -3 && vy <= 3) idx = c_lut.idx[(vy + 3) * 7 + (vx + 3)];
        if (idx < MDLG_NQ && (a.n_event || a.cell_acc)) {
            long long cx = qx1 % lx, cy = qy1 % lx;
            if (cx < 0) cx += lx;
            if (cy < 0) cy += lx;
            const long long off = ((long long)idx * lx + cy) * lx + cx;
            if (a.n_event) atomicAdd(&a.n_event[off], 1);
            if (a.cell_acc) atomicAdd(&a.cell_acc[off], 1);
        }
        const double dx = unwrapped_delta(p1.x, p0.x, i1.x - i0.x, a.L);
        const double dy = unwrapped_delta(p1.y, p0.y, i1.y - i0.y, a.L);
        const double dx2 = dx * dx, dy2 = dy * dy;
        m0 = dx2 + dy2;
        m1 = dx2 * dx2 + dy2 * dy2;
        m2 = dx;
        m3 = dy;
    }
    const unsigned long long rest = __ballot(act && idx == 0);
    if ((tid & 63) == 0 && rest) atomicAdd(&hist[0], (int)__popcll(rest));
    if (act && idx != 0) atomicAdd(&hist[idx], 1);
    m0 = wave_sum(m0);
    m1 = wave_sum(m1);
    m2 = wave_sum(m2);
    m3 = wave_sum(m3);
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = m0;
        red[tid >> 6][1] = m1;
        red[tid >> 6][2] = m2;
        red[tid >> 6][3] = m3;
    }
    __syncthreads();
    if (tid < MDLG_NCOUNTS && hist[tid]) atomicAdd(&a.counts[tid], (unsigned long long)hist[tid]);
    if (tid < 4) {
        double t = 0.0;
        for (int w = 0; w < BS / 64; ++w) t += red[w][tid];
        a.mpart[(long long)blockIdx.x * 5 + 1 + tid] = t;
    }
    if (tid == 0) {
        long long nact = a.n - (long long)blockIdx.x * BS;
        nact = nact > BS ? BS : nact;
        a.mpart[(long long)blockIdx.x * 5] = 2.0 * (double)nact;
    }
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, long long nb, double* out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    for (int c = 0; c < 5; ++c) {
        double t = 0.0;
        for (long long b = tid; b < nb; b += 256) t += part[b * 5 + c];
        red[tid] = t;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        if (tid == 0) out[c] += red[0];
        __syncthreads();
    }
}

__global__ void k_zero_i32(int* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace mdlg

using namespace mdlg;

// Scratch of mdlg_coarse_grain_noalloc: the per-block moment partials (5
// doubles per block of 256 particles) of up to kNoAllocMaxN particles.  Each
// GPU the library runs on holds its own copy until the process ends.  In host
// code this name stands for the device array but is not its address: kernels
// get the address that hipGetSymbolAddress returned for the current device.
constexpr long long kNoAllocMaxN = 1LL << 25;
constexpr int kCgBS = 256;
static __device__ __align__(256) double scratch[5 * (kNoAllocMaxN / kCgBS)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per device.
mdlg_status scratch_of_current_device(double** out) {
    int dev = -1;
    MDLG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MDLG_EINVAL, "mdlg_coarse_grain_noalloc: device index beyond " + std::to_string(kMaxDevices));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MDLG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MDLG_OK;
}

mdlg_status check_cg_args(const char* who, const mdlg_lattice* lat, double box_l, int64_t n, const double* pos_prev,
                          const double* pos_cur, const int64_t* counts) {
    const std::string w(who);
    if (!lat || !counts) return fail(MDLG_EINVAL, w + ": lat and counts are required");
    if (n < 0) return fail(MDLG_EINVAL, w + ": n must be >= 0");
    if (n > 0 && (!pos_prev || !pos_cur)) return fail(MDLG_EINVAL, w + ": positions are required");
    if (lat->lx < 1 || lat->lx > 46340) return fail(MDLG_EINVAL, w + ": lx must be in [1, 46340]");
    if (!(box_l > 0.0) || !std::isfinite(box_l)) return fail(MDLG_EINVAL, w + ": box_l must be > 0");
    if (!std::isfinite(lat->u[0]) || !std::isfinite(lat->u[1])) return fail(MDLG_EINVAL, w + ": u must be finite");
    return MDLG_OK;
}

// The event itself, with the moment partials in `mpart` (5 doubles per block).
hipError_t coarse_grain_launch(const mdlg_lattice* lat, double box_l, int64_t n, const double* pos_prev,
                               const int32_t* img_prev, int64_t k_prev, const double* pos_cur,
                               const int32_t* img_cur, int64_t k_cur, int64_t* counts, double* moments,
                               int32_t* n_event, int32_t* cell_acc, double* mpart, hipStream_t st) {
    const long long lx = lat->lx;
    const long long field = (long long)MDLG_NQ * lx * lx;
    if (n_event) {
        hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((field + 255) / 256)), dim3(256), 0, st, n_event, field);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n == 0) return hipSuccess;
    const long long nb = (n + kCgBS - 1) / kCgBS;
    CgArgs a{};
    a.xp = (const double2*)pos_prev;
    a.ip = (const int2*)img_prev;
    a.xc = (const double2*)pos_cur;
    a.ic = (const int2*)img_cur;
    a.n = n;
    a.lx = lat->lx;
    a.L = box_l;
    a.inv_lat = (double)lat->lx / box_l;
    const double dxl = box_l / (double)lat->lx;
    a.sxp = (lat->u[0] * dxl) * (double)k_prev;
    a.syp = (lat->u[1] * dxl) * (double)k_prev;
    a.sxc = (lat->u[0] * dxl) * (double)k_cur;
    a.syc = (lat->u[1] * dxl) * (double)k_cur;
    a.counts = (unsigned long long*)counts;
    a.n_event = n_event;
    a.cell_acc = cell_acc;
    a.mpart = mpart;
    hipLaunchKernelGGL(k_coarse_grain<kCgBS>, dim3((unsigned)nb), dim3(kCgBS), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && moments) {
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double*)mpart, nb, moments);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

extern "C" mdlg_status mdlg_coarse_grain(const mdlg_lattice* lat, double box_l, int64_t n, const double* pos_prev,
                                         const int32_t* img_prev, int64_t k_prev, const double* pos_cur,
                                         const int32_t* img_cur, int64_t k_cur, int64_t* counts, double* moments,
                                         int32_t* n_event, int32_t* cell_acc, void* stream) {
    mdlg_status s = check_cg_args("mdlg_coarse_grain", lat, box_l, n, pos_prev, pos_cur, counts);
    if (s != MDLG_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    double* mpart = nullptr;
    if (n > 0) MDLG_HIP(hipMallocAsync((void**)&mpart, sizeof(double) * 5 * ((n + kCgBS - 1) / kCgBS), st));
    hipError_t e = coarse_grain_launch(lat, box_l, n, pos_prev, img_prev, k_prev, pos_cur, img_cur, k_cur, counts,
                                       moments, n_event, cell_acc, mpart, st);
    hipError_t e2 = mpart ? hipFreeAsync(mpart, st) : hipSuccess;
    MDLG_HIP(e);
    MDLG_HIP(e2);
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_coarse_grain_noalloc(const mdlg_lattice* lat, double box_l, int64_t n,
                                                 const double* pos_prev, const int32_t* img_prev, int64_t k_prev,
                                                 const double* pos_cur, const int32_t* img_cur, int64_t k_cur,
                                                 int64_t* counts, double* moments, int32_t* n_event,
                                                 int32_t* cell_acc, void* stream) {
    mdlg_status s = check_cg_args("mdlg_coarse_grain_noalloc", lat, box_l, n, pos_prev, pos_cur, counts);
    if (s != MDLG_OK) return s;
    if (n > kNoAllocMaxN)
        return fail(MDLG_EINVAL, "mdlg_coarse_grain_noalloc: n = " + std::to_string(n) + " exceeds the limit of " +
                                     std::to_string(kNoAllocMaxN) + " particles of its fixed scratch");
    double* mpart = nullptr;
    s = scratch_of_current_device(&mpart);
    if (s != MDLG_OK) return s;
    MDLG_HIP(coarse_grain_launch(lat, box_l, n, pos_prev, img_prev, k_prev, pos_cur, img_cur, k_cur, counts, moments,
                                 n_event, cell_acc, mpart, (hipStream_t)stream));
    return MDLG_OK;
}
