// 2D Lennard-Jones velocity-Verlet MD with a cell list, fused with MDLG
// coarse-graining, for gfx950 (MI355X).
//
// Physics ("Simulations setup" section of the paper): 6-12 LJ pairs with
// sigma = m = 1, cut at rc (energy optionally shifted), velocity Verlet NVE in
// a periodic square box.  Coarse-graining: Eq.(n_i), evaluated every s_cg MD
// steps inside the step kernel.
//
// Layout (per replica, replicas back to back, each padded to a multiple of
// kPad slots):
//   pos[2]  double2 ping-pong   positions, sorted by cell-list cell
//   vel     double2             half-step velocity (full-step right after init)
//   img     int2                periodic image counts
//   id      int                 caller index of the particle (-1: pad slot)
//   snap    double2             position at the previous coarse step
// Cells of width w >= rc + skin, cell_start[] by counting sort, particles
// within a cell ordered by id (deterministic).  Rebuilt every K steps.
//
// One MD step is one kernel: each thread takes one slot, gathers the 3 x 3
// block of cells around its particle's current cell (coalesced: neighbouring
// threads hold neighbouring cells), sums the pair forces, completes the
// previous half kick, kicks, drifts and wraps.  On coarse-graining steps the
// same kernel maps the particle's lattice displacement to a D2Q49 index,
// aggregates the histogram in LDS with a wave ballot for the dominant v = 0,
// and writes fixed-order moment partials.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "mdlg_internal.h"

namespace mdlg {

__constant__ VelLut d_lut = kLut;

constexpr int kPad = 512;  // slot padding of each replica (largest block size)

enum : int { ERR_NONFINITE = 1, ERR_SKIN = 2 };

struct RepDev {
    double L, halfL, inv_w, w, skin_half;
    double rc2, eps24, eps4, vshift;
    float rc2f, eps24f;
    int nc, cell0;  // cells per side; first cell (sentinel of the pad slots at cell0 + nc*nc)
    int slot0, n;   // first slot, real particles
    int tile0, ntile;  // tiles (blocks) of this replica, in units of the block size
    // coarse-graining lattice
    int lx, pad_;
    double inv_lat, sx, sy;  // lx / L; frame drift per coarse step (u * dx)
    long long cacc0;         // offset of this replica in cell_acc
};

struct StepArgs {
    const double2* __restrict__ pin;
    double2* __restrict__ pout;
    double2* __restrict__ vel;
    int2* __restrict__ img;
    const int* __restrict__ cs;
    const RepDev* __restrict__ reps;
    const int* __restrict__ tile_rep;
    double dt, hdt;
    int* err;
    // coarse-graining
    double2* __restrict__ snap;
    unsigned long long* __restrict__ counts;
    double* __restrict__ mpart;
    int* __restrict__ cell_acc;
    const long long* __restrict__ event_k;
    // observation
    const int* __restrict__ id;
    double2* opos;
    double2* ovel;
    int2* oimg;
    double2* ofrc;
    double* epart;
};

__device__ __forceinline__ int cell_coord(double x, double inv_w, int nc) {
    double t = x * inv_w;
    if (!(t >= 0.0)) t = 0.0;  // also catches NaN
    int c = (int)fmin(t, (double)(nc - 1));
    return c;
}

__device__ __forceinline__ double min_image(double d, double L, double halfL) {
    return d > halfL ? d - L : (d < -halfL ? d + L : d);
}

// Sum of LJ pair forces (and, if PE, half the shifted pair energies) on the
// particle in slot s at (px, py) from the 3 x 3 cells around its current cell.
template <bool F32, bool PE>
__device__ __forceinline__ void pair_forces(const double2* __restrict__ pin, const int* __restrict__ cs,
                                            const RepDev& R, int s, double px, double py, double& fx,
                                            double& fy, double& pe) {
    const int nc = R.nc;
    const int cx = cell_coord(px, R.inv_w, nc);
    const int cy = cell_coord(py, R.inv_w, nc);
    double ax = 0.0, ay = 0.0, ae = 0.0;
    float bx = 0.0f, by = 0.0f;
    for (int oy = -1; oy <= 1; ++oy) {
        int row = cy + oy;
        row = row < 0 ? row + nc : (row >= nc ? row - nc : row);
        const int base = R.cell0 + row * nc;
        int a0, a1, b0 = 0, b1 = 0;
        if (cx > 0 && cx < nc - 1) {
            a0 = cs[base + cx - 1];
            a1 = cs[base + cx + 2];
        } else if (cx == 0) {
            a0 = cs[base];
            a1 = cs[base + 2];
            b0 = cs[base + nc - 1];
            b1 = cs[base + nc];
        } else {
            a0 = cs[base + nc - 2];
            a1 = cs[base + nc];
            b0 = cs[base];
            b1 = cs[base + 1];
        }
        const int na = a1 - a0;
        const int tot = na + (b1 - b0);
        for (int t = 0; t < tot; ++t) {
            const int k = t < na ? a0 + t : b0 + (t - na);
            if (k == s) continue;
            const double2 q = pin[k];
            const double dx = min_image(px - q.x, R.L, R.halfL);
            const double dy = min_image(py - q.y, R.L, R.halfL);
            if (F32) {
                const float fdx = (float)dx, fdy = (float)dy;
                const float r2 = fdx * fdx + fdy * fdy;
                if (r2 < R.rc2f) {
                    const float ir2 = 1.0f / r2;
                    const float ir6 = ir2 * ir2 * ir2;
                    const float fr = R.eps24f * ir6 * (2.0f * ir6 - 1.0f) * ir2;
                    bx += fr * fdx;
                    by += fr * fdy;
                    if (PE) ae += 0.5 * (R.eps4 * (double)ir6 * ((double)ir6 - 1.0) - R.vshift);
                }
            } else {
                const double r2 = dx * dx + dy * dy;
                if (r2 < R.rc2) {
                    const double ir2 = 1.0 / r2;
                    const double ir6 = ir2 * ir2 * ir2;
                    const double fr = R.eps24 * ir6 * (2.0 * ir6 - 1.0) * ir2;
                    ax += fr * dx;
                    ay += fr * dy;
                    if (PE) ae += 0.5 * (R.eps4 * ir6 * (ir6 - 1.0) - R.vshift);
                }
            }
        }
    }
    if (F32) {
        fx = (double)bx;
        fy = (double)by;
    } else {
        fx = ax;
        fy = ay;
    }
    pe = ae;
}

// Coarse-graining epilogue of one step kernel block (all threads take part).
template <int BS>
__device__ __forceinline__ void cg_epilogue(const StepArgs& a, const RepDev& R, int r, int tile, int s,
                                            bool act, double2 p) {
    __shared__ int hist[MDLG_NCOUNTS];
    __shared__ double red[BS / 64][4];
    const int tid = threadIdx.x;
    if (tid < MDLG_NCOUNTS) hist[tid] = 0;
    __syncthreads();
    int idx = MDLG_NQ;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (act) {
        const long long k = *a.event_k;
        const double2 sp = a.snap[s];
        const int lx = R.lx;
        const long long qxc = lattice_q(p.x, frame_shift(R.sx, k), R.inv_lat);
        const long long qyc = lattice_q(p.y, frame_shift(R.sy, k), R.inv_lat);
        const long long qxp = lattice_q(sp.x, frame_shift(R.sx, k - 1), R.inv_lat);
        const long long qyp = lattice_q(sp.y, frame_shift(R.sy, k - 1), R.inv_lat);
        long long vx = qxc - qxp, vy = qyc - qyp;
        // lattice minimum image: a particle that crossed the box edge
        if (2 * vx > lx) vx -= lx; else if (2 * vx < -lx) vx += lx;
        if (2 * vy > lx) vy -= lx; else if (2 * vy < -lx) vy += lx;
        if (vx >= -3 && vx <= 3 && vy >= -3 && vy <= 3) idx = d_lut.idx[(vy + 3) * 7 + (vx + 3)];
        if (idx < MDLG_NQ && a.cell_acc) {
            long long cxm = qxc, cym = qyc;
            if (cxm < 0 || cxm >= lx) { cxm %= lx; if (cxm < 0) cxm += lx; }
            if (cym < 0 || cym >= lx) { cym %= lx; if (cym < 0) cym += lx; }
            atomicAdd(&a.cell_acc[R.cacc0 + ((long long)idx * lx + cym) * lx + cxm], 1);
        }
        const double dx = min_image(p.x - sp.x, R.L, R.halfL);
        const double dy = min_image(p.y - sp.y, R.L, R.halfL);
        const double dx2 = dx * dx, dy2 = dy * dy;
        m0 = dx2 + dy2;
        m1 = dx2 * dx2 + dy2 * dy2;
        m2 = dx;
        m3 = dy;
        a.snap[s] = p;
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
    if (tid < MDLG_NCOUNTS && hist[tid])
        atomicAdd(&a.counts[(long long)r * MDLG_NCOUNTS + tid], (unsigned long long)hist[tid]);
    if (tid < 4) {
        double t = 0.0;
        for (int w = 0; w < BS / 64; ++w) t += red[w][tid];
        a.mpart[(long long)tile * MDLG_NMOMENTS + 1 + tid] = t;
    }
    if (tid == 0) {
        int nact = R.n - (tile * BS - R.slot0);
        nact = nact < 0 ? 0 : (nact > BS ? BS : nact);
        a.mpart[(long long)tile * MDLG_NMOMENTS] = 2.0 * (double)nact;
    }
}

// One velocity-Verlet step (FIRST: the stored velocity is a full-step one).
template <int BS, bool F32, bool FIRST, bool CG>
__global__ __launch_bounds__(BS) void k_step(StepArgs a) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int r = a.tile_rep[tile];
    const RepDev& R = a.reps[r];
    const int s = tile * BS + threadIdx.x;
    const bool act = s - R.slot0 < R.n;
    double2 pn = make_double2(0.0, 0.0);
    if (act) {
        const double2 p = a.pin[s];
        double fx, fy, pe;
        pair_forces<F32, false>(a.pin, a.cs, R, s, p.x, p.y, fx, fy, pe);
        double2 v = a.vel[s];
        if (!FIRST) {
            v.x = v.x + a.hdt * fx;
            v.y = v.y + a.hdt * fy;
        }
        v.x = v.x + a.hdt * fx;
        v.y = v.y + a.hdt * fy;
        pn.x = p.x + a.dt * v.x;
        pn.y = p.y + a.dt * v.y;
        int wx = 0, wy = 0;
        if (pn.x >= R.L) { pn.x -= R.L; wx = 1; }
        else if (pn.x < 0.0) { pn.x += R.L; wx = -1; if (pn.x >= R.L) { pn.x = 0.0; wx = 0; } }
        if (pn.y >= R.L) { pn.y -= R.L; wy = 1; }
        else if (pn.y < 0.0) { pn.y += R.L; wy = -1; if (pn.y >= R.L) { pn.y = 0.0; wy = 0; } }
        if (wx | wy) {
            int2 im = a.img[s];
            im.x += wx;
            im.y += wy;
            a.img[s] = im;
        }
        if (!isfinite(pn.x) || !isfinite(pn.y) || !isfinite(v.x) || !isfinite(v.y)) atomicOr(a.err, ERR_NONFINITE);
        a.pout[s] = pn;
        a.vel[s] = v;
    }
    if (CG) cg_epilogue<BS>(a, R, r, tile, s, act, pn);
}

// Observation at the current positions: forces, full-step velocities, state
// copied out in caller order, and per-tile partials of {KE, PE, Px, Py}.
template <int BS, bool F32, bool HALF>
__global__ __launch_bounds__(BS) void k_observe(StepArgs a) {
    __shared__ double red[BS / 64][4];
    const int tile = blockIdx.x;
    const int r = a.tile_rep[tile];
    const RepDev& R = a.reps[r];
    const int s = tile * BS + threadIdx.x;
    const bool act = s - R.slot0 < R.n;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0, e3 = 0.0;
    if (act) {
        const double2 p = a.pin[s];
        double fx, fy, pe;
        pair_forces<F32, true>(a.pin, a.cs, R, s, p.x, p.y, fx, fy, pe);
        double2 v = a.vel[s];
        if (HALF) {
            v.x = v.x + a.hdt * fx;
            v.y = v.y + a.hdt * fy;
        }
        const int j = a.id[s];
        if (a.opos) a.opos[j] = p;
        if (a.ovel) a.ovel[j] = v;
        if (a.oimg) a.oimg[j] = a.img[s];
        if (a.ofrc) a.ofrc[j] = make_double2(fx, fy);
        e0 = 0.5 * (v.x * v.x + v.y * v.y);
        e1 = pe;
        e2 = v.x;
        e3 = v.y;
    }
    if (a.epart) {
        e0 = wave_sum(e0);
        e1 = wave_sum(e1);
        e2 = wave_sum(e2);
        e3 = wave_sum(e3);
        const int tid = threadIdx.x;
        if ((tid & 63) == 0) {
            red[tid >> 6][0] = e0;
            red[tid >> 6][1] = e1;
            red[tid >> 6][2] = e2;
            red[tid >> 6][3] = e3;
        }
        __syncthreads();
        if (tid < 4) {
            double t = 0.0;
            for (int w = 0; w < BS / 64; ++w) t += red[w][tid];
            a.epart[(long long)tile * 4 + tid] = t;
        }
    }
}

// Per-replica fixed-order sum of per-tile partials: out[r][j] (+)= sum over the
// replica's tiles of part[tile][j].  Optionally advances the coarse-step index.
__global__ __launch_bounds__(256) void k_reduce_rep(const double* __restrict__ part, int ncomp,
                                                    const RepDev* __restrict__ reps, double* out,
                                                    int accumulate, long long* event_k) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    const RepDev& R = reps[r];
    const int tid = threadIdx.x;
    for (int j = 0; j < ncomp; ++j) {
        double t = 0.0;
        for (int b = R.tile0 + tid; b < R.tile0 + R.ntile; b += 256) t += part[(long long)b * ncomp + j];
        red[tid] = t;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        if (tid == 0) out[(long long)r * ncomp + j] = accumulate ? out[(long long)r * ncomp + j] + red[0] : red[0];
        __syncthreads();
    }
    if (event_k && r == 0 && tid == 0) *event_k += 1;
}

// ------------------------------------------------------------ rebuild ---

template <int BS>
__global__ __launch_bounds__(BS) void k_bin(const double2* __restrict__ pos, const RepDev* __restrict__ reps,
                                            const int* __restrict__ tile_rep, int* __restrict__ cnt,
                                            int* __restrict__ key, int* __restrict__ rank,
                                            const int* __restrict__ cellof, int check, int* err) {
    const int tile = blockIdx.x;
    const RepDev& R = reps[tile_rep[tile]];
    const int s = tile * BS + threadIdx.x;
    int c;
    if (s - R.slot0 < R.n) {
        const double2 p = pos[s];
        const int cx = cell_coord(p.x, R.inv_w, R.nc);
        const int cy = cell_coord(p.y, R.inv_w, R.nc);
        c = R.cell0 + cy * R.nc + cx;
        if (check) {
            // drift check: the particle must still lie within the skin around
            // the cell it was sorted into at the previous rebuild (checked here
            // against half the skin, a factor-2 margin)
            const int co = cellof[s] - R.cell0;
            const int ox = co % R.nc, oy = co / R.nc;
            const double ex = fabs(min_image(p.x - (ox + 0.5) * R.w, R.L, R.halfL)) - 0.5 * R.w;
            const double ey = fabs(min_image(p.y - (oy + 0.5) * R.w, R.L, R.halfL)) - 0.5 * R.w;
            if (ex > R.skin_half || ey > R.skin_half) atomicOr(err, ERR_SKIN);
            if (!isfinite(p.x) || !isfinite(p.y)) atomicOr(err, ERR_NONFINITE);
        }
    } else {
        c = R.cell0 + R.nc * R.nc;  // pad slots go to the replica's sentinel cell
    }
    key[s] = c;
    rank[s] = atomicAdd(&cnt[c], 1);
}

__global__ void k_fill_i32(int* p, long long n, int v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* p, long long n, double v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_set_i64(long long* p, long long v) { *p = v; }

// Exclusive scan of n ints (cnt) into out[0..n] (out[n] = total), three passes
// over tiles of 4096 elements (1024 threads x 4).
constexpr int kScanTile = 4096;

__device__ __forceinline__ int block_excl_scan_1024(int v, int* lds, int& total) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int w = lane < 16 ? lds[lane] : 0;
        for (int o = 1; o < 16; o <<= 1) {
            int y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < 16) lds[16 + lane] = w;
    }
    __syncthreads();
    total = lds[31];
    const int wave_off = wid > 0 ? lds[16 + wid - 1] : 0;
    const int res = wave_off + x - v;
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(1024) void k_scan_reduce(const int* __restrict__ in, long long n, int* __restrict__ bsum) {
    __shared__ int lds[32];
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * 4;
    int s = 0;
    for (int j = 0; j < 4; ++j)
        if (base + j < n) s += in[base + j];
    int total;
    block_excl_scan_1024(s, lds, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int* bsum, int nb) {
    __shared__ int lds[32];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int total;
        const int ex = block_excl_scan_1024(v, lds, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(1024) void k_scan_final(const int* __restrict__ in, long long n,
                                                     const int* __restrict__ boff, int* __restrict__ out) {
    __shared__ int lds[32];
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * 4;
    int v[4];
    int s = 0;
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += v[j];
    }
    int total;
    int ex = block_excl_scan_1024(s, lds, total) + boff[blockIdx.x];
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
    if (base <= n - 1 && n - 1 < base + 4) out[n] = ex;  // thread holding the last element
}

__global__ void k_scatter(const int* __restrict__ key, const int* __restrict__ rank, const int* __restrict__ cs,
                          int* __restrict__ perm, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) perm[cs[key[s]] + rank[s]] = s;
}

struct Bufs {
    const double2* pos_o;
    double2* pos_n;
    const double2* vel_o;
    double2* vel_n;
    const int2* img_o;
    int2* img_n;
    const int* id_o;
    int* id_n;
    const double2* snap_o;
    double2* snap_n;
};

// One thread per cell: order the cell's particles by caller index, then move
// their state into the new slot order.
__global__ void k_sort_gather(const int* __restrict__ cs, int* __restrict__ perm, int C, Bufs b,
                              int* __restrict__ cellof) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int lo = cs[c], hi = cs[c + 1];
    for (int i = lo + 1; i < hi; ++i) {
        const int x = perm[i];
        const int kx = b.id_o[x];
        int j = i - 1;
        while (j >= lo && b.id_o[perm[j]] > kx) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = x;
    }
    for (int d = lo; d < hi; ++d) {
        const int src = perm[d];
        b.pos_n[d] = b.pos_o[src];
        b.vel_n[d] = b.vel_o[src];
        b.img_n[d] = b.img_o[src];
        b.id_n[d] = b.id_o[src];
        b.snap_n[d] = b.snap_o[src];
        cellof[d] = c;
    }
}

// Initial placement: slot slot0_r + j of replica r holds particle off_r + j.
__global__ void k_init_slots(const double* __restrict__ pos0, const double* __restrict__ vel0,
                             const RepDev* __restrict__ reps, const int* __restrict__ tile_rep,
                             const long long* __restrict__ poff, int BS, double2* pos, double2* vel,
                             int2* img, int* id, double2* snap) {
    const int tile = blockIdx.x;
    const int r = tile_rep[tile];
    const RepDev& R = reps[r];
    const int s = tile * BS + threadIdx.x;
    const int j = s - R.slot0;
    if (j < R.n) {
        const long long g = poff[r] + j;
        pos[s] = make_double2(pos0[2 * g], pos0[2 * g + 1]);
        vel[s] = make_double2(vel0[2 * g], vel0[2 * g + 1]);
        id[s] = (int)g;
    } else {
        pos[s] = make_double2(0.0, 0.0);
        vel[s] = make_double2(0.0, 0.0);
        id[s] = -1;
    }
    img[s] = make_int2(0, 0);
    snap[s] = pos[s];
}

__global__ void k_vmax(const double2* __restrict__ vel, const int* __restrict__ id, int S,
                       unsigned long long* out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double v2 = 0.0;
    if (s < S && id[s] >= 0) {
        const double2 v = vel[s];
        v2 = v.x * v.x + v.y * v.y;
        if (!isfinite(v2)) v2 = 1e300;
    }
    for (int o = 32; o > 0; o >>= 1) v2 = fmax(v2, __shfl_xor(v2, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v2));
}

__global__ void k_copy_d2(const double2* __restrict__ src, double2* __restrict__ dst, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) dst[s] = src[s];
}

__global__ void k_finite_check(const double* __restrict__ a, long long n, int* err) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicOr(err, ERR_NONFINITE);
}

}  // namespace mdlg

// ====================================================================== host

using namespace mdlg;

namespace {

struct RepHost {
    RepDev d;
    long long poff;  // first caller index
    int nslots;
};

struct GraphKey {
    int K, phase, ppar, opar;
    bool operator<(const GraphKey& o) const {
        return std::tie(K, phase, ppar, opar) < std::tie(o.K, o.phase, o.ppar, o.opar);
    }
};

struct GraphVal {
    hipGraphExec_t exec;
    int ppar_after, opar_after;
    int events;
};

template <typename T>
hipError_t dalloc(T** p, size_t n) {
    return hipMalloc((void**)p, sizeof(T) * (n > 0 ? n : 1));
}

}  // namespace

struct lj_md {
    int R = 0;
    int S = 0;   // total slots
    int C = 0;   // total cells including one sentinel per replica
    int BS = 256;
    int ntile = 0;
    bool f32 = false;
    double dt = 0.0;
    std::vector<RepHost> reps;
    long long n_total = 0;
    RepDev* d_reps = nullptr;
    int* d_tile_rep = nullptr;
    double2* pos[2] = {nullptr, nullptr};
    double2* vel[2] = {nullptr, nullptr};
    int2* img[2] = {nullptr, nullptr};
    int* id[2] = {nullptr, nullptr};
    double2* snap[2] = {nullptr, nullptr};
    int *key = nullptr, *rank = nullptr, *perm = nullptr, *cellof = nullptr;
    int *cnt = nullptr, *cs = nullptr, *bsum = nullptr;
    int nscan = 0;
    int ppar = 0, opar = 0;  // current buffer of pos / of the other per-particle arrays
    bool vel_full = true;
    bool have_cellof = false;
    bool broken = false;
    int K = 50;
    bool K_auto = true;
    int K_base = 50;
    long long steps_done = 0;
    int since_rebuild = 0;
    int* d_err = nullptr;
    double* d_epart = nullptr;
    double* d_eout = nullptr;
    unsigned long long* d_vmax = nullptr;
    // coarse-graining
    bool cg_on = false;
    int s_cg = 0;
    long long cg_t = 0;
    long long events = 0;
    unsigned long long* counts = nullptr;
    double* moments = nullptr;
    int* cell_acc = nullptr;
    double* d_mpart = nullptr;
    long long* d_event_k = nullptr;
    hipStream_t cap = nullptr;
    std::map<GraphKey, GraphVal> graphs;
    bool use_graphs = true;
};

namespace {

void clear_graphs(lj_md* md) {
    for (auto& kv : md->graphs) (void)hipGraphExecDestroy(kv.second.exec);
    md->graphs.clear();
}

StepArgs make_args(lj_md* md) {
    StepArgs a{};
    a.pin = md->pos[md->ppar];
    a.pout = md->pos[md->ppar ^ 1];
    a.vel = md->vel[md->opar];
    a.img = md->img[md->opar];
    a.cs = md->cs;
    a.reps = md->d_reps;
    a.tile_rep = md->d_tile_rep;
    a.dt = md->dt;
    a.hdt = 0.5 * md->dt;
    a.err = md->d_err;
    a.snap = md->snap[md->opar];
    a.counts = md->counts;
    a.mpart = md->d_mpart;
    a.cell_acc = md->cell_acc;
    a.event_k = md->d_event_k;
    a.id = md->id[md->opar];
    return a;
}

#define LAUNCH_BS(BSV, KERNEL, ...)                                                             \
    switch (BSV) {                                                                              \
        case 64: hipLaunchKernelGGL((KERNEL<64, __VA_ARGS__>), dim3(grid), dim3(64), 0, st, a); break;   \
        case 128: hipLaunchKernelGGL((KERNEL<128, __VA_ARGS__>), dim3(grid), dim3(128), 0, st, a); break; \
        case 256: hipLaunchKernelGGL((KERNEL<256, __VA_ARGS__>), dim3(grid), dim3(256), 0, st, a); break; \
        default: hipLaunchKernelGGL((KERNEL<512, __VA_ARGS__>), dim3(grid), dim3(512), 0, st, a); break;  \
    }

hipError_t launch_step(lj_md* md, hipStream_t st, bool first, bool cg) {
    StepArgs a = make_args(md);
    const int grid = md->ntile;
    if (md->f32) {
        if (first) {
            if (cg) { LAUNCH_BS(md->BS, k_step, true, true, true) } else { LAUNCH_BS(md->BS, k_step, true, true, false) }
        } else {
            if (cg) { LAUNCH_BS(md->BS, k_step, true, false, true) } else { LAUNCH_BS(md->BS, k_step, true, false, false) }
        }
    } else {
        if (first) {
            if (cg) { LAUNCH_BS(md->BS, k_step, false, true, true) } else { LAUNCH_BS(md->BS, k_step, false, true, false) }
        } else {
            if (cg) { LAUNCH_BS(md->BS, k_step, false, false, true) } else { LAUNCH_BS(md->BS, k_step, false, false, false) }
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (cg) {
        hipLaunchKernelGGL(k_reduce_rep, dim3(md->R), dim3(256), 0, st, (const double*)md->d_mpart, MDLG_NMOMENTS,
                           (const RepDev*)md->d_reps, md->moments, 1, md->d_event_k);
        e = hipGetLastError();
    }
    md->ppar ^= 1;
    return e;
}

hipError_t launch_observe(lj_md* md, hipStream_t st, double2* opos, double2* ovel, int2* oimg, double2* ofrc,
                          bool energy) {
    StepArgs a = make_args(md);
    a.opos = opos;
    a.ovel = ovel;
    a.oimg = oimg;
    a.ofrc = ofrc;
    a.epart = energy ? md->d_epart : nullptr;
    const int grid = md->ntile;
    const bool half = !md->vel_full;
    if (md->f32) {
        if (half) { LAUNCH_BS(md->BS, k_observe, true, true) } else { LAUNCH_BS(md->BS, k_observe, true, false) }
    } else {
        if (half) { LAUNCH_BS(md->BS, k_observe, false, true) } else { LAUNCH_BS(md->BS, k_observe, false, false) }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !energy) return e;
    hipLaunchKernelGGL(k_reduce_rep, dim3(md->R), dim3(256), 0, st, (const double*)md->d_epart, 4,
                       (const RepDev*)md->d_reps, md->d_eout, 0, (long long*)nullptr);
    return hipGetLastError();
}

hipError_t launch_rebuild(lj_md* md, hipStream_t st) {
    const int S = md->S, C = md->C;
    hipLaunchKernelGGL(k_fill_i32, dim3((C + 255) / 256), dim3(256), 0, st, md->cnt, (long long)C, 0);
    const int o = md->opar;
    const int grid = md->ntile;
    const int check = md->have_cellof ? 1 : 0;
    switch (md->BS) {
        case 64: hipLaunchKernelGGL(k_bin<64>, dim3(grid), dim3(64), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err); break;
        case 128: hipLaunchKernelGGL(k_bin<128>, dim3(grid), dim3(128), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err); break;
        case 256: hipLaunchKernelGGL(k_bin<256>, dim3(grid), dim3(256), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err); break;
        default: hipLaunchKernelGGL(k_bin<512>, dim3(grid), dim3(512), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err); break;
    }
    const int nb = (C + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(1024), 0, st, (const int*)md->cnt, (long long)C, md->bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, md->bsum, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(1024), 0, st, (const int*)md->cnt, (long long)C,
                       (const int*)md->bsum, md->cs);
    hipLaunchKernelGGL(k_scatter, dim3((S + 255) / 256), dim3(256), 0, st, (const int*)md->key,
                       (const int*)md->rank, (const int*)md->cs, md->perm, S);
    Bufs b;
    b.pos_o = md->pos[md->ppar];
    b.pos_n = md->pos[md->ppar ^ 1];
    b.vel_o = md->vel[o];
    b.vel_n = md->vel[o ^ 1];
    b.img_o = md->img[o];
    b.img_n = md->img[o ^ 1];
    b.id_o = md->id[o];
    b.id_n = md->id[o ^ 1];
    b.snap_o = md->snap[o];
    b.snap_n = md->snap[o ^ 1];
    hipLaunchKernelGGL(k_sort_gather, dim3((C + 255) / 256), dim3(256), 0, st, (const int*)md->cs, md->perm, C, b,
                       md->cellof);
    md->ppar ^= 1;
    md->opar ^= 1;
    md->have_cellof = true;
    md->since_rebuild = 0;
    return hipGetLastError();
}

bool event_due(lj_md* md, long long t_after) { return md->cg_on && (t_after % md->s_cg) == 0; }

// One MD step launched eagerly (rebuild first if due).
hipError_t eager_step(lj_md* md, hipStream_t st) {
    hipError_t e;
    if (md->since_rebuild >= md->K) {
        e = launch_rebuild(md, st);
        if (e != hipSuccess) return e;
    }
    const bool ev = event_due(md, md->cg_t + 1);
    e = launch_step(md, st, md->vel_full, ev);
    if (e != hipSuccess) return e;
    md->vel_full = false;
    md->steps_done += 1;
    md->since_rebuild += 1;
    if (md->cg_on) {
        md->cg_t += 1;
        if (ev) md->events += 1;
    }
    return hipSuccess;
}

// rebuild + K steps, replayed from a captured graph.
mdlg_status graph_unit(lj_md* md, hipStream_t st) {
    GraphKey key{md->K, md->cg_on ? (int)(md->cg_t % md->s_cg) : -1, md->ppar, md->opar};
    auto it = md->graphs.find(key);
    if (it == md->graphs.end()) {
        const long long steps0 = md->steps_done, cg_t0 = md->cg_t, ev0 = md->events;
        MDLG_HIP(hipStreamBeginCapture(md->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_rebuild(md, md->cap);
        for (int j = 0; j < md->K && e == hipSuccess; ++j) {
            const bool ev = event_due(md, md->cg_t + 1);
            e = launch_step(md, md->cap, false, ev);
            md->since_rebuild += 1;
            if (md->cg_on) {
                md->cg_t += 1;
                if (ev) md->events += 1;
            }
        }
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(md->cap, &g);
        if (e != hipSuccess) return fail(MDLG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        MDLG_HIP(e2);
        hipGraphExec_t ex = nullptr;
        MDLG_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        GraphVal val{ex, md->ppar, md->opar, (int)(md->events - ev0)};
        md->graphs[key] = val;
        // the capture only recorded work: restore the counters, then replay
        md->ppar = key.ppar;
        md->opar = key.opar;
        md->steps_done = steps0;
        md->cg_t = cg_t0;
        md->events = ev0;
        it = md->graphs.find(key);
    }
    MDLG_HIP(hipGraphLaunch(it->second.exec, st));
    md->ppar = it->second.ppar_after;
    md->opar = it->second.opar_after;
    md->steps_done += md->K;
    md->since_rebuild = md->K;
    md->have_cellof = true;
    if (md->cg_on) {
        md->cg_t += md->K;
        md->events += it->second.events;
    }
    return MDLG_OK;
}

mdlg_status check_params(const lj_params& p, int r) {
    auto bad = [&](const char* what) {
        return fail(MDLG_EINVAL, "lj_md_init: replica " + std::to_string(r) + ": " + what);
    };
    if (p.n < 2 || p.n > (1LL << 30)) return bad("n must be in [2, 2^30]");
    if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return bad("dt must be > 0");
    if (!(p.rc > 0.0) || !std::isfinite(p.rc)) return bad("rc must be > 0");
    if (!(p.eps >= 0.0) || !std::isfinite(p.eps)) return bad("eps must be >= 0");
    if (!(p.skin >= 0.0) || !std::isfinite(p.skin)) return bad("skin must be >= 0");
    const double skin = p.skin > 0.0 ? p.skin : 0.5;
    if (!(p.box_l >= 3.0 * (p.rc + skin)) || !std::isfinite(p.box_l)) return bad("box_l must be >= 3 (rc + skin)");
    if (p.force_bits != 64 && p.force_bits != 32) return bad("force_bits must be 64 or 32");
    if (p.block_size != 0 && p.block_size != 64 && p.block_size != 128 && p.block_size != 256 && p.block_size != 512)
        return bad("block_size must be 0, 64, 128, 256 or 512");
    if (p.rebuild_every < 0) return bad("rebuild_every must be >= 0");
    return MDLG_OK;
}

mdlg_status sync_check(lj_md* md, hipStream_t st) {
    MDLG_HIP(hipStreamSynchronize(st));
    int err = 0;
    MDLG_HIP(hipMemcpy(&err, md->d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) {
        md->broken = true;
        if (err & ERR_NONFINITE) return fail(MDLG_ENONFINITE, "non-finite position or velocity on the device");
        return fail(MDLG_ESKIN, "a particle drifted beyond the cell-list skin between rebuilds; lower rebuild_every or raise skin");
    }
    return MDLG_OK;
}

int aligned_K(int K, int s_cg) {
    if (s_cg <= 0) return K;
    if (K >= s_cg) return s_cg * (K / s_cg);
    for (int d = K; d >= 1; --d)
        if (s_cg % d == 0) return d;
    return 1;
}

mdlg_status destroy_on_fail(lj_md* md, mdlg_status st) {
    lj_md_destroy(md);
    return st;
}

}  // namespace

extern "C" mdlg_status lj_md_init(lj_md** out, const lj_params* p, const double* pos0, const double* vel0,
                                  void* stream) {
    return lj_md_init_batch(out, 1, p, pos0, vel0, stream);
}

extern "C" mdlg_status lj_md_init_batch(lj_md** out, int32_t n_rep, const lj_params* p, const double* pos0,
                                        const double* vel0, void* stream) {
    if (!out || !p || !pos0 || !vel0) return fail(MDLG_EINVAL, "lj_md_init: NULL argument");
    *out = nullptr;
    if (n_rep < 1) return fail(MDLG_EINVAL, "lj_md_init: n_rep must be >= 1");
    for (int r = 0; r < n_rep; ++r) {
        mdlg_status s = check_params(p[r], r);
        if (s != MDLG_OK) return s;
    }
    hipStream_t st = (hipStream_t)stream;
    lj_md* md = new lj_md();
    md->R = n_rep;
    md->BS = p[0].block_size ? p[0].block_size : 256;
    md->f32 = p[0].force_bits == 32;
    md->dt = p[0].dt;
    long long slots = 0, cells = 0, poff = 0;
    double skin_half_min = 1e300;
    for (int r = 0; r < n_rep; ++r) {
        const lj_params& q = p[r];
        RepHost h{};
        const double skin = q.skin > 0.0 ? q.skin : 0.5;
        const int nc = (int)std::floor(q.box_l / (q.rc + skin));
        RepDev& d = h.d;
        d.L = q.box_l;
        d.halfL = 0.5 * q.box_l;
        d.nc = nc;
        d.w = q.box_l / nc;
        d.inv_w = (double)nc / q.box_l;
        d.skin_half = 0.5 * (d.w - q.rc);
        d.rc2 = q.rc * q.rc;
        d.rc2f = (float)d.rc2;
        d.eps24 = 24.0 * q.eps;
        d.eps24f = (float)d.eps24;
        d.eps4 = 4.0 * q.eps;
        const double irc6 = 1.0 / (q.rc * q.rc * q.rc * q.rc * q.rc * q.rc);
        d.vshift = q.energy_shift ? 4.0 * q.eps * irc6 * (irc6 - 1.0) : 0.0;
        d.cell0 = (int)cells;
        d.slot0 = (int)slots;
        d.n = (int)q.n;
        h.nslots = (int)(((q.n + kPad - 1) / kPad) * kPad);
        d.tile0 = (int)(slots / md->BS);
        d.ntile = h.nslots / md->BS;
        d.lx = 0;
        h.poff = poff;
        cells += (long long)nc * nc + 1;
        slots += h.nslots;
        poff += q.n;
        skin_half_min = std::min(skin_half_min, d.skin_half);
        md->reps.push_back(h);
    }
    if (slots >= (1LL << 31) || cells >= (1LL << 31)) {
        delete md;
        return fail(MDLG_EINVAL, "lj_md_init: too many particles or cells for 32-bit slot indices");
    }
    md->S = (int)slots;
    md->C = (int)cells;
    md->n_total = poff;
    md->ntile = md->S / md->BS;
    md->nscan = (md->C + kScanTile - 1) / kScanTile;

    auto A = [&](hipError_t e) { return e == hipSuccess; };
    bool ok = A(dalloc(&md->d_reps, n_rep)) && A(dalloc(&md->d_tile_rep, md->ntile));
    for (int b = 0; b < 2 && ok; ++b)
        ok = A(dalloc(&md->pos[b], md->S)) && A(dalloc(&md->vel[b], md->S)) && A(dalloc(&md->img[b], md->S)) &&
             A(dalloc(&md->id[b], md->S)) && A(dalloc(&md->snap[b], md->S));
    ok = ok && A(dalloc(&md->key, md->S)) && A(dalloc(&md->rank, md->S)) && A(dalloc(&md->perm, md->S)) &&
         A(dalloc(&md->cellof, md->S)) && A(dalloc(&md->cnt, md->C)) && A(dalloc(&md->cs, (size_t)md->C + 1)) &&
         A(dalloc(&md->bsum, md->nscan)) && A(dalloc(&md->d_err, 1)) && A(dalloc(&md->d_epart, (size_t)md->ntile * 4)) &&
         A(dalloc(&md->d_eout, (size_t)n_rep * 4)) && A(dalloc(&md->d_vmax, 1)) &&
         A(dalloc(&md->d_mpart, (size_t)md->ntile * MDLG_NMOMENTS)) && A(dalloc(&md->d_event_k, 1)) &&
         A(hipStreamCreateWithFlags(&md->cap, hipStreamNonBlocking));
    if (!ok) return destroy_on_fail(md, fail(MDLG_ENOMEM, "lj_md_init: device allocation failed"));

    std::vector<RepDev> hd(n_rep);
    std::vector<int> trep(md->ntile);
    std::vector<long long> hpoff(n_rep);
    for (int r = 0; r < n_rep; ++r) {
        hd[r] = md->reps[r].d;
        hpoff[r] = md->reps[r].poff;
        for (int t = 0; t < hd[r].ntile; ++t) trep[hd[r].tile0 + t] = r;
    }
    long long* d_poff = nullptr;
    if (hipMalloc((void**)&d_poff, sizeof(long long) * n_rep) != hipSuccess)
        return destroy_on_fail(md, fail(MDLG_ENOMEM, "lj_md_init: device allocation failed"));
    hipError_t e = hipMemcpy(md->d_reps, hd.data(), sizeof(RepDev) * n_rep, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(md->d_tile_rep, trep.data(), sizeof(int) * md->ntile, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_poff, hpoff.data(), sizeof(long long) * n_rep, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(md->d_err, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(md->d_vmax, 0, sizeof(unsigned long long), st);
    // reject non-finite inputs before they reach the cell index arithmetic
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_finite_check, dim3((unsigned)((2 * md->n_total + 255) / 256)), dim3(256), 0, st, pos0,
                           2 * md->n_total, md->d_err);
        hipLaunchKernelGGL(k_finite_check, dim3((unsigned)((2 * md->n_total + 255) / 256)), dim3(256), 0, st, vel0,
                           2 * md->n_total, md->d_err);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_init_slots, dim3(md->ntile), dim3(md->BS), 0, st, pos0, vel0, (const RepDev*)md->d_reps,
                           (const int*)md->d_tile_rep, (const long long*)d_poff, md->BS, md->pos[0], md->vel[0],
                           md->img[0], md->id[0], md->snap[0]);
        hipLaunchKernelGGL(k_vmax, dim3((md->S + 255) / 256), dim3(256), 0, st, (const double2*)md->vel[0],
                           (const int*)md->id[0], md->S, md->d_vmax);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_poff);
    if (e != hipSuccess) return destroy_on_fail(md, fail(MDLG_EHIP, std::string("lj_md_init: ") + hipGetErrorString(e)));
    int err = 0;
    unsigned long long vbits = 0;
    if (hipMemcpy(&err, md->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&vbits, md->d_vmax, sizeof(vbits), hipMemcpyDeviceToHost) != hipSuccess)
        return destroy_on_fail(md, fail(MDLG_EHIP, "lj_md_init: copy failed"));
    if (err) return destroy_on_fail(md, fail(MDLG_EINVAL, "lj_md_init: non-finite position or velocity"));
    // positions must be wrapped into the box (checked on the host side copy for
    // clarity of the error; cheap relative to the allocation above)
    {
        std::vector<double> hp(2 * md->n_total);
        if (hipMemcpy(hp.data(), pos0, sizeof(double) * hp.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return destroy_on_fail(md, fail(MDLG_EHIP, "lj_md_init: copy failed"));
        for (int r = 0; r < n_rep; ++r) {
            const double L = md->reps[r].d.L;
            for (long long j = md->reps[r].poff; j < md->reps[r].poff + md->reps[r].d.n; ++j)
                if (!(hp[2 * j] >= 0.0 && hp[2 * j] < L && hp[2 * j + 1] >= 0.0 && hp[2 * j + 1] < L))
                    return destroy_on_fail(md, fail(MDLG_EINVAL, "lj_md_init: position outside [0, L) for particle " +
                                                                     std::to_string(j)));
        }
    }
    double vmax = std::sqrt(std::max(0.0, (double)__builtin_bit_cast(double, vbits)));
    if (p[0].rebuild_every > 0) {
        md->K_auto = false;
        md->K = p[0].rebuild_every;
    } else {
        // half the skin may be crossed at twice the fastest initial speed
        double k = vmax > 0.0 ? skin_half_min / (2.0 * vmax * md->dt) : 1000.0;
        md->K = (int)std::max(1.0, std::min(1000.0, std::floor(k)));
    }
    md->K_base = md->K;
    // first rebuild (no drift check)
    if (launch_rebuild(md, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return destroy_on_fail(md, fail(MDLG_EHIP, "lj_md_init: initial cell sort failed"));
    md->vel_full = true;
    *out = md;
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_cg_attach(lj_md* md, int32_t s_cg, const mdlg_lattice* lat, int64_t* counts,
                                       double* moments, int32_t* cell_acc, void* stream) {
    if (!md || !lat || !counts || !moments) return fail(MDLG_EINVAL, "lj_md_cg_attach: NULL argument");
    if (md->broken) return fail(MDLG_EINVAL, "lj_md_cg_attach: handle is unusable after a device fault");
    if (s_cg < 1) return fail(MDLG_EINVAL, "lj_md_cg_attach: s_cg must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    long long cacc = 0;
    std::vector<RepDev> hd(md->R);
    for (int r = 0; r < md->R; ++r) {
        const mdlg_lattice& l = lat[r];
        if (l.lx < 7) return fail(MDLG_EINVAL, "lj_md_cg_attach: lx must be >= 7");
        if (!std::isfinite(l.u[0]) || !std::isfinite(l.u[1])) return fail(MDLG_EINVAL, "lj_md_cg_attach: u not finite");
        RepDev& d = md->reps[r].d;
        d.lx = l.lx;
        d.inv_lat = (double)l.lx / d.L;
        const double dxl = d.L / (double)l.lx;
        d.sx = l.u[0] * dxl;
        d.sy = l.u[1] * dxl;
        d.cacc0 = cacc;
        cacc += (long long)MDLG_NQ * l.lx * l.lx;
        hd[r] = d;
    }
    MDLG_HIP(hipStreamSynchronize(st));
    MDLG_HIP(hipMemcpy(md->d_reps, hd.data(), sizeof(RepDev) * md->R, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_copy_d2, dim3((md->S + 255) / 256), dim3(256), 0, st, (const double2*)md->pos[md->ppar],
                       md->snap[md->opar], md->S);
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, md->d_event_k, 1LL);
    MDLG_HIP(hipGetLastError());
    clear_graphs(md);
    md->cg_on = true;
    md->s_cg = s_cg;
    md->cg_t = 0;
    md->events = 0;
    md->counts = (unsigned long long*)counts;
    md->moments = moments;
    md->cell_acc = cell_acc;
    if (md->K_auto) md->K = aligned_K(md->K_base, s_cg);
    md->since_rebuild = md->K;  // start the next chunk with a rebuild
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_cg_detach(lj_md* md) {
    if (!md) return fail(MDLG_EINVAL, "lj_md_cg_detach: NULL handle");
    clear_graphs(md);
    md->cg_on = false;
    md->counts = nullptr;
    md->moments = nullptr;
    md->cell_acc = nullptr;
    if (md->K_auto) md->K = md->K_base;
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_step(lj_md* md, int64_t nsteps, void* stream) {
    if (!md) return fail(MDLG_EINVAL, "lj_md_step: NULL handle");
    if (md->broken) return fail(MDLG_EINVAL, "lj_md_step: handle is unusable after a device fault");
    if (nsteps < 0) return fail(MDLG_EINVAL, "lj_md_step: nsteps must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    while (nsteps > 0) {
        if (!md->vel_full && md->use_graphs && nsteps >= md->K) {
            mdlg_status s = graph_unit(md, st);
            if (s != MDLG_OK) return s;
            nsteps -= md->K;
            continue;
        }
        hipError_t e = eager_step(md, st);
        if (e != hipSuccess) return fail(MDLG_EHIP, std::string("lj_md_step: ") + hipGetErrorString(e));
        nsteps -= 1;
    }
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_step_timed(lj_md* md, int64_t nsteps, double* ms_out, int32_t* n_out,
                                        void* stream) {
    if (!md || !ms_out) return fail(MDLG_EINVAL, "lj_md_step_timed: NULL argument");
    if (md->broken) return fail(MDLG_EINVAL, "lj_md_step_timed: handle is unusable after a device fault");
    if (nsteps < 0 || nsteps > 100000) return fail(MDLG_EINVAL, "lj_md_step_timed: nsteps must be in [0, 1e5]");
    hipStream_t st = (hipStream_t)stream;
    struct Rec {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Rec> recs;
    auto rec_begin = [&](int kind) -> hipError_t {
        Rec r{nullptr, nullptr, kind};
        hipError_t e = hipEventCreate(&r.a);
        if (e == hipSuccess) e = hipEventCreate(&r.b);
        if (e == hipSuccess) e = hipEventRecord(r.a, st);
        recs.push_back(r);
        return e;
    };
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < nsteps && e == hipSuccess; ++i) {
        if (md->since_rebuild >= md->K) {
            e = rec_begin(2);
            if (e == hipSuccess) e = launch_rebuild(md, st);
            if (e == hipSuccess) e = hipEventRecord(recs.back().b, st);
        }
        const bool ev = event_due(md, md->cg_t + 1);
        if (e == hipSuccess) e = rec_begin(ev ? 1 : 0);
        if (e == hipSuccess) e = launch_step(md, st, md->vel_full, ev);
        if (e == hipSuccess) e = hipEventRecord(recs.back().b, st);
        if (e != hipSuccess) break;
        md->vel_full = false;
        md->steps_done += 1;
        md->since_rebuild += 1;
        if (md->cg_on) {
            md->cg_t += 1;
            if (ev) md->events += 1;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    double sum[3] = {0, 0, 0};
    int cnt[3] = {0, 0, 0};
    for (auto& r : recs) {
        float ms = 0.0f;
        if (e == hipSuccess && r.a && r.b) e = hipEventElapsedTime(&ms, r.a, r.b);
        sum[r.kind] += ms;
        cnt[r.kind] += 1;
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    if (e != hipSuccess) return fail(MDLG_EHIP, std::string("lj_md_step_timed: ") + hipGetErrorString(e));
    for (int k = 0; k < 3; ++k) {
        ms_out[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
        if (n_out) n_out[k] = cnt[k];
    }
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_get_state(lj_md* md, double* pos, double* vel, int32_t* img, void* stream) {
    if (!md) return fail(MDLG_EINVAL, "lj_md_get_state: NULL handle");
    hipError_t e = launch_observe(md, (hipStream_t)stream, (double2*)pos, (double2*)vel, (int2*)img, nullptr, false);
    if (e != hipSuccess) return fail(MDLG_EHIP, std::string("lj_md_get_state: ") + hipGetErrorString(e));
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_forces(lj_md* md, double* force, void* stream) {
    if (!md || !force) return fail(MDLG_EINVAL, "lj_md_forces: NULL argument");
    hipError_t e = launch_observe(md, (hipStream_t)stream, nullptr, nullptr, nullptr, (double2*)force, false);
    if (e != hipSuccess) return fail(MDLG_EHIP, std::string("lj_md_forces: ") + hipGetErrorString(e));
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_energy(lj_md* md, double* out, void* stream) {
    if (!md || !out) return fail(MDLG_EINVAL, "lj_md_energy: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_observe(md, st, nullptr, nullptr, nullptr, nullptr, true);
    if (e != hipSuccess) return fail(MDLG_EHIP, std::string("lj_md_energy: ") + hipGetErrorString(e));
    mdlg_status s = sync_check(md, st);
    if (s != MDLG_OK) return s;
    MDLG_HIP(hipMemcpy(out, md->d_eout, sizeof(double) * 4 * md->R, hipMemcpyDeviceToHost));
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_check(lj_md* md, void* stream) {
    if (!md) return fail(MDLG_EINVAL, "lj_md_check: NULL handle");
    return sync_check(md, (hipStream_t)stream);
}

extern "C" mdlg_status lj_md_info(const lj_md* md, lj_md_info_t* info) {
    if (!md || !info) return fail(MDLG_EINVAL, "lj_md_info: NULL argument");
    info->n_rep = md->R;
    info->rebuild_every = md->K;
    info->n_total = md->n_total;
    info->steps_done = md->steps_done;
    info->events_done = md->events;
    info->cells_per_side = md->reps[0].d.nc;
    info->block_size = md->BS;
    info->cell_width = md->reps[0].d.w;
    return MDLG_OK;
}

extern "C" void lj_md_destroy(lj_md* md) {
    if (!md) return;
    clear_graphs(md);
    if (md->cap) (void)hipStreamDestroy(md->cap);
    void* ptrs[] = {md->d_reps, md->d_tile_rep, md->pos[0], md->pos[1], md->vel[0], md->vel[1], md->img[0],
                    md->img[1], md->id[0], md->id[1], md->snap[0], md->snap[1], md->key, md->rank, md->perm,
                    md->cellof, md->cnt, md->cs, md->bsum, md->d_err, md->d_epart, md->d_eout, md->d_vmax,
                    md->d_mpart, md->d_event_k};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete md;
}
