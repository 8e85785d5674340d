// Internal helpers shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "mdlg.h"

namespace mdlg {

// ----------------------------------------------------------- error state ---
void set_error(const std::string& msg);
mdlg_status fail(mdlg_status code, const std::string& msg);

#define MDLG_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::mdlg::fail(MDLG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------- D2Q49 velocity set ---
// Numbering: ascending |v|^2, then counter-clockwise from +x.
struct VelTable {
    int8_t v[MDLG_NQ][2];
};
struct VelLut {
    int8_t idx[MDLG_NQ];  // [(vy + 3) * 7 + (vx + 3)] -> velocity index
};

constexpr VelTable kVel = {{{0, 0},
                            {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                            {1, 1}, {-1, 1}, {-1, -1}, {1, -1},
                            {2, 0}, {0, 2}, {-2, 0}, {0, -2},
                            {2, 1}, {1, 2}, {-1, 2}, {-2, 1}, {-2, -1}, {-1, -2}, {1, -2}, {2, -1},
                            {2, 2}, {-2, 2}, {-2, -2}, {2, -2},
                            {3, 0}, {0, 3}, {-3, 0}, {0, -3},
                            {3, 1}, {1, 3}, {-1, 3}, {-3, 1}, {-3, -1}, {-1, -3}, {1, -3}, {3, -1},
                            {3, 2}, {2, 3}, {-2, 3}, {-3, 2}, {-3, -2}, {-2, -3}, {2, -3}, {3, -2},
                            {3, 3}, {-3, 3}, {-3, -3}, {3, -3}}};

constexpr VelLut make_lut() {
    VelLut l{};
    for (int i = 0; i < MDLG_NQ; ++i) l.idx[(kVel.v[i][1] + 3) * 7 + (kVel.v[i][0] + 3)] = (int8_t)i;
    return l;
}
constexpr VelLut kLut = make_lut();

// ------------------------------------------------------- launch helpers ---
constexpr int kNumXcd = 8;

// Map the hardware block index to a logical tile so that each XCD (blocks are
// dealt to the 8 XCDs round-robin) works on one contiguous band of tiles and
// its L2 holds that band and its neighbours.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    int q = nb / kNumXcd, r = nb % kNumXcd;
    int x = b % kNumXcd, k = b / kNumXcd;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Lattice coordinate floor((x + shift) * inv), every operation rounded once,
// exactly as written (no fused multiply-add), so that host and device agree
// on the cell of a position bit for bit.
__device__ __forceinline__ double lattice_qf(double x, double shift, double inv) {
#pragma clang fp contract(off)
    double t = x + shift;
    double u = t * inv;
    return floor(u);
}

__device__ __forceinline__ long long lattice_q(double x, double shift, double inv) {
    return (long long)lattice_qf(x, shift, inv);
}

__device__ __forceinline__ double frame_shift(double per_step, long long k) {
#pragma clang fp contract(off)
    return per_step * (double)k;
}

}  // namespace mdlg
