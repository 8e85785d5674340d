// Non-equilibrium MDLG of a replica ensemble: ensemble sums of the occupation
// numbers n_i(x, t) (Eq.(n_i)) at every coarse step of stored trajectories,
// and of the lattice gas collision operator of Eq.(mdlg_evolution),
// Xi_i(x, t) = n_i(x + v_i, t + dt) - n_i(x, t).  Divided by the ensemble size
// they are the MDLB distribution f_i = <n_i> and collision operator
// Omega_i = <Xi_i> ("Molecular dynamics lattice gas method" section).
//
// Since Xi is linear in n, the ensemble sum of Xi is the shifted difference
// of the ensemble sums of n: the replicas never need dense fields of their
// own.  Two kernels:
//   k_neq_scatter  one thread per particle walks its snapshots once, keeps the
//                  previous unwrapped cell in registers, and adds 1 to the
//                  destination cell of its lattice velocity (global atomics:
//                  the counters of one coarse step, 196 lx^2 bytes, stay in
//                  L2/MALL); displacements outside D2Q49 are counted per
//                  wave by a ballot and added with one atomic per wave;
//   k_neq_xi       Xi sums as f[k+1](x + v_i) - f[k](x) over the periodic
//                  lattice, one thread per output element (HBM-bound stencil).
#include <cmath>

#include "mdlg_internal.h"

namespace mdlg {
namespace {

__constant__ VelLut c_lut_neq = kLut;
__constant__ VelTable c_vel_neq = kVel;

constexpr int kNeqBS = 256;
constexpr int kNeqTargetBlocks = 2048;

__global__ void k_fill_i32(int* __restrict__ p, long long n) {
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        p[k] = 0;
}

__global__ void k_fill_i64(long long* __restrict__ p, long long n) {
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        p[k] = 0;
}

__device__ __forceinline__ long long cell_of(double x, double inv) {
#pragma clang fp contract(off)
    return (long long)floor(x * inv);
}

// Events p = p0 .. p1-1 (1 <= p0) of particle j: f_sum[p-1][i][cell] += 1.
__global__ __launch_bounds__(kNeqBS) void k_neq_scatter(const double2* __restrict__ pos, const int2* __restrict__ img,
                                                        long long n_tot, int n_snap, int n_chunk, int lx, double inv,
                                                        unsigned* __restrict__ f_sum,
                                                        unsigned long long* __restrict__ ovf) {
    const int tid = threadIdx.x, lane = tid & 63;
    const long long j = (long long)blockIdx.x * kNeqBS + tid;
    const bool act = j < n_tot;
    const int nev = n_snap - 1;
    const int span = (nev + n_chunk - 1) / n_chunk;
    const int p0 = 1 + (int)blockIdx.y * span;
    const int p1 = min(n_snap, p0 + span);
    if (p0 >= p1) return;  // uniform over the block
    const long long lxl = lx, lx2 = lxl * lxl;
    long long cx = 0, cy = 0;
    if (act) {
        const double2 x = pos[(long long)(p0 - 1) * n_tot + j];
        const int2 m = img[(long long)(p0 - 1) * n_tot + j];
        cx = cell_of(x.x, inv) + lxl * m.x;
        cy = cell_of(x.y, inv) + lxl * m.y;
    }
    for (int p = p0; p < p1; ++p) {
        bool out = false;
        if (act) {
            const double2 x = pos[(long long)p * n_tot + j];
            const int2 m = img[(long long)p * n_tot + j];
            const long long qx = cell_of(x.x, inv), qy = cell_of(x.y, inv);
            const long long nx = qx + lxl * m.x, ny = qy + lxl * m.y;
            const long long vx = nx - cx, vy = ny - cy;
            cx = nx;
            cy = ny;
            if (vx >= -3 && vx <= 3 && vy >= -3 && vy <= 3) {
                const int i = c_lut_neq.idx[(vy + 3) * 7 + (vx + 3)];
                long long ux = qx % lxl, uy = qy % lxl;  // q may reach lx (or -1) by rounding
                ux += ux < 0 ? lxl : 0;
                uy += uy < 0 ? lxl : 0;
                atomicAdd(f_sum + ((long long)(p - 1) * MDLG_NQ + i) * lx2 + uy * lxl + ux, 1u);
            } else {
                out = true;
            }
        }
        // displacements beyond D2Q49 are rare: one global atomic per wave that has any
        const unsigned long long b = __ballot(out);
        if (b && lane == 0) atomicAdd(ovf + (p - 1), (unsigned long long)__popcll(b));
    }
}

// xi[k][i][y][x] = f[k+1][i][(y + v_iy) mod lx][(x + v_ix) mod lx] - f[k][i][y][x]
__global__ void k_neq_xi(const int* __restrict__ f, int* __restrict__ xi, int n_k, int lx) {
    const long long lxl = lx, lx2 = lxl * lxl;
    const long long total = (long long)n_k * MDLG_NQ * lx2;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long x = e % lxl;
        const long long y = (e / lxl) % lxl;
        const long long ki = e / lx2;  // k * 49 + i
        const int i = (int)(ki % MDLG_NQ);
        long long xs = x + c_vel_neq.v[i][0], ys = y + c_vel_neq.v[i][1];
        xs += xs < 0 ? lxl : (xs >= lxl ? -lxl : 0);
        ys += ys < 0 ? lxl : (ys >= lxl ? -lxl : 0);
        xi[e] = f[(ki + MDLG_NQ) * lx2 + ys * lxl + xs] - f[e];
    }
}

}  // namespace
}  // namespace mdlg

using namespace mdlg;

extern "C" mdlg_status mdlg_neq_mdlg(int64_t n_total, double box_l, int32_t lx, int32_t n_snap, const double* pos,
                                     const int32_t* img, int32_t* f_sum, int64_t* overflow, int32_t* xi_sum,
                                     void* stream) {
    const char* who = "mdlg_neq_mdlg: ";
    if (!pos || !img || !f_sum || !overflow) return fail(MDLG_EINVAL, std::string(who) + "NULL argument");
    if (n_total < 0 || n_total > 0x7fffffffLL) return fail(MDLG_EINVAL, std::string(who) + "n_total must be in [0, 2^31)");
    if (n_snap < 2) return fail(MDLG_EINVAL, std::string(who) + "n_snap must be >= 2");
    if (lx < 7 || lx > 46340) return fail(MDLG_EINVAL, std::string(who) + "lx must be in [7, 46340]");
    if (!(box_l > 0.0) || !std::isfinite(box_l)) return fail(MDLG_EINVAL, std::string(who) + "box_l must be finite and > 0");
    hipStream_t st = (hipStream_t)stream;
    const long long per = (long long)MDLG_NQ * lx * lx;
    const long long nf = (long long)(n_snap - 1) * per;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<long long>((nf + 255) / 256, 65536)), dim3(256), 0, st,
                       f_sum, nf);
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)std::min<long long>((n_snap - 1 + 255) / 256, 65536)), dim3(256), 0,
                       st, (long long*)overflow, (long long)(n_snap - 1));
    MDLG_HIP(hipGetLastError());
    if (n_total > 0) {
        const long long nb = (n_total + kNeqBS - 1) / kNeqBS;
        const long long want = (kNeqTargetBlocks + nb - 1) / nb;
        const int n_chunk = (int)std::max(1LL, std::min<long long>({want, (long long)(n_snap - 1), 65535LL}));
        hipLaunchKernelGGL(k_neq_scatter, dim3((unsigned)nb, (unsigned)n_chunk), dim3(kNeqBS), 0, st,
                           (const double2*)pos, (const int2*)img, (long long)n_total, n_snap, n_chunk, lx,
                           (double)lx / box_l, (unsigned*)f_sum, (unsigned long long*)overflow);
        MDLG_HIP(hipGetLastError());
    }
    if (xi_sum && n_snap > 2) {
        const long long nx = (long long)(n_snap - 2) * per;
        hipLaunchKernelGGL(k_neq_xi, dim3((unsigned)std::min<long long>((nx + 255) / 256, 1 << 20)), dim3(256), 0, st,
                           (const int*)f_sum, xi_sum, n_snap - 2, lx);
        MDLG_HIP(hipGetLastError());
    }
    return MDLG_OK;
}
