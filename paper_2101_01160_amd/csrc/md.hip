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
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <tuple>
#include <vector>

#include <hip/hip_ext.h>

#include "mdlg_internal.h"

namespace mdlg {

__constant__ VelLut d_lut = kLut;

constexpr int kPad = 512;  // slot padding of each replica (largest block size)

enum : int { ERR_NONFINITE = 1, ERR_SKIN = 2, ERR_NLIST = 4, ERR_TILE = 8 };

struct RepDev {
    double L, halfL, inv_w, w, skin_half;
    double rc2, eps24, eps4, vshift;
    float rc2f, eps24f;
    int nc, cell0;  // cells per side; first cell (sentinel of the pad slots at cell0 + nc*nc)
    int slot0, n;   // first slot, real particles
    int tile0, ntile;  // slot tiles (blocks of the block size) of this replica
    int ttile0, nttile;  // cell tiles of the step kernel: nc rows x tpr tiles of tw cells
    int tw, tpr;
    // fused tiles (two or three steps per launch): pT x pT cells, pts per side, the first global index pt0
    int pt0, pT, pts, pnt;
    // coarse-graining lattice
    int lx, npad;  // lattice cells per side; pad slots after the replica's particles
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
    int* __restrict__ hpart;                 // [component][pstride]: histogram partials per tile
    int pstride;                             // tiles per component row of hpart / mpart
    const int* __restrict__ ttile_rep;
    const int* __restrict__ tinfo;
    int nrep;
    int nslots;     // total slots: loads of the prologue are clamped below it
    int stage_max;  // tile kernel: largest staged particle count (<= its LDS capacity)
    const short* __restrict__ nbl;          // neighbour lists [maxnb][S]: slot offsets
    const unsigned char* __restrict__ nbc;  // neighbour counts [S]
    // two- and three-step launches
    double2* __restrict__ vout;                 // velocities written by the fused kernels
    const int* __restrict__ plist;              // [tiles][kPairCap]: staged slots, owned then ring by ring
    const int4* __restrict__ pcnt;              // [tiles]: staged counts up to the owned, ring 1, ring 2, all
    const unsigned short* __restrict__ tlist;   // [tiles][maxnb][kPairCap]: neighbours as staged indices
    const unsigned char* __restrict__ tcnt;     // [tiles][kPairCap]: neighbour counts of all rings but the last
    int maxnb;
    int rings;                                  // cell rings staged around a fused tile
    const int* __restrict__ ptile_rep;          // [tiles] replica
    int* __restrict__ cell_acc;
    const long long* __restrict__ event_k;
    // the previous event's finish, done by blocks [0, fin_n) of a later launch
    // (0: none; see cg_finish_one)
    int fin_n;
    double* __restrict__ moments;
    long long* __restrict__ event_kw;
    // cell binning on the last launch before a rebuild (counting sort input)
    int* __restrict__ cnt;
    int* __restrict__ key;
    int* __restrict__ rank;
    const double2* __restrict__ pref;
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

// Lattice velocity index (D2Q49, 49 = overflow) and destination cell of one
// particle between its snapshot sp (coarse step k-1) and position p (step k).
__device__ __forceinline__ int cg_index(const RepDev& R, long long k, double2 p, double2 sp, long long& cell) {
    const double fxc = lattice_qf(p.x, frame_shift(R.sx, k), R.inv_lat);
    const double fyc = lattice_qf(p.y, frame_shift(R.sy, k), R.inv_lat);
    const double fxp = lattice_qf(sp.x, frame_shift(R.sx, k - 1), R.inv_lat);
    const double fyp = lattice_qf(sp.y, frame_shift(R.sy, k - 1), R.inv_lat);
    // lattice coordinates below 2^29 in magnitude (every run short of ~2^29
    // cells of frame drift) take 32-bit integers, exactly as the 64-bit path
    if (fmax(fmax(fabs(fxc), fabs(fyc)), fmax(fabs(fxp), fabs(fyp))) < 536870912.0) {
        const int lx = R.lx;
        const int qxc = (int)fxc, qyc = (int)fyc;
        int vx = qxc - (int)fxp, vy = qyc - (int)fyp;
        if (2 * vx > lx) vx -= lx; else if (2 * vx < -lx) vx += lx;
        if (2 * vy > lx) vy -= lx; else if (2 * vy < -lx) vy += lx;
        int idx = MDLG_NQ;
        if (vx >= -3 && vx <= 3 && vy >= -3 && vy <= 3) idx = d_lut.idx[(vy + 3) * 7 + (vx + 3)];
        int cxm = qxc, cym = qyc;
        if (cxm < 0 || cxm >= lx) { cxm %= lx; if (cxm < 0) cxm += lx; }
        if (cym < 0 || cym >= lx) { cym %= lx; if (cym < 0) cym += lx; }
        cell = (long long)cym * lx + cxm;
        return idx;
    }
    const long long lx = R.lx;
    const long long qxc = (long long)fxc, qyc = (long long)fyc;
    long long vx = qxc - (long long)fxp, vy = qyc - (long long)fyp;
    // lattice minimum image: a particle that crossed the box edge
    if (2 * vx > lx) vx -= lx; else if (2 * vx < -lx) vx += lx;
    if (2 * vy > lx) vy -= lx; else if (2 * vy < -lx) vy += lx;
    int idx = MDLG_NQ;
    if (vx >= -3 && vx <= 3 && vy >= -3 && vy <= 3) idx = d_lut.idx[(vy + 3) * 7 + (vx + 3)];
    long long cxm = qxc, cym = qyc;
    if (cxm < 0 || cxm >= lx) { cxm %= lx; if (cxm < 0) cxm += lx; }
    if (cym < 0 || cym >= lx) { cym %= lx; if (cym < 0) cym += lx; }
    cell = cym * lx + cxm;
    return idx;
}

// Per-tile table of the step kernel's LDS staging, rebuilt with the cell
// list: for each of the three staged rows (row-1, row, row+1) the global slot
// start and count of its three pieces: the left halo cell, the tile's own
// cells x0..x1-1, and the right halo cell.
constexpr int kTileInfo = 18;

__global__ void k_tile_info(const int* __restrict__ cs, const RepDev* __restrict__ reps,
                            const int* __restrict__ ttile_rep, int TT, int* __restrict__ tinfo) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= TT) return;
    const RepDev& R = reps[ttile_rep[t]];
    const int nc = R.nc;
    const int lt = t - R.ttile0;
    const int row = lt / R.tpr;
    const int x0 = (lt % R.tpr) * R.tw;
    const int x1 = min(nc, x0 + R.tw);
    const int xa = x0 > 0 ? x0 - 1 : nc - 1;
    const int xc = x1 < nc ? x1 : 0;
    for (int rr = 0; rr < 3; ++rr) {
        int rw = row + rr - 1;
        rw = rw < 0 ? rw + nc : (rw >= nc ? rw - nc : rw);
        const int base = R.cell0 + rw * nc;
        int* o = tinfo + (long long)t * kTileInfo + rr * 6;
        o[0] = cs[base + xa];
        o[1] = cs[base + xa + 1] - o[0];
        o[2] = cs[base + x0];
        o[3] = cs[base + x1] - o[2];
        o[4] = cs[base + xc];
        o[5] = cs[base + xc + 1] - o[4];
    }
}

// One velocity-Verlet step over one tile of cells (FIRST: the stored velocity
// is a full-step one; CG: this step ends a coarse step).
//
// A tile is `tw` consecutive cells of one cell row.  The block stages the
// particles of the three rows around it (cells x0-1 .. x1 of rows row-1 ..
// row+1, periodic) into LDS with coalesced loads, shifting halo copies that
// lie across the box edge by -L or +L so that plain differences are minimum-
// image separations.  Each thread then takes one particle of the tile's own
// cells and sums its pair forces over the 3 x 3 cells around the cell it was
// sorted into.  LDS layout per staged row: left halo cell, the tile's cells,
// right halo cell; lcs[row][c] is the LDS offset of cell c of that row (c = 0:
// left halo).  All global loads of the prologue are issued before the first
// LDS write.  A tile whose rows do not fit in LDS reads them from global
// memory instead (same loop, minimum image applied).
template <int BS, bool F32, bool FIRST, bool CG>
__global__ __launch_bounds__(BS) void k_step_tile(StepArgs a) {
    constexpr int MAXP = 4 * BS;
    constexpr int MAXTW = 2 * BS;
    constexpr int NLCS = (3 * (MAXTW + 1) + BS - 1) / BS;
    __shared__ double2 lp[MAXP];
    __shared__ int lcs[3][MAXTW + 3];
    __shared__ int hist[MDLG_NCOUNTS];
    __shared__ double red[BS / 64][4];

    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int r = a.nrep == 1 ? 0 : __builtin_amdgcn_readfirstlane(a.ttile_rep[t]);
    const RepDev& R = a.reps[r];
    const int nc = R.nc;
    const double L = R.L, halfL = R.halfL, rc2 = R.rc2, eps24 = R.eps24;
    const float rc2f = R.rc2f, eps24f = R.eps24f;
    const int lt = t - R.ttile0;
    const int row = lt / R.tpr;
    const int x0 = (lt % R.tpr) * R.tw;
    const int x1 = min(nc, x0 + R.tw);
    const int tw = x1 - x0;
    const int tid = threadIdx.x;
    const int* ti = a.tinfo + (long long)t * kTileInfo;
    int gA[3], nA[3], gB[3], nB[3], gC[3], nC[3], off[4];
    off[0] = 0;
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
        gA[rr] = ti[rr * 6 + 0];
        nA[rr] = ti[rr * 6 + 1];
        gB[rr] = ti[rr * 6 + 2];
        nB[rr] = ti[rr * 6 + 3];
        gC[rr] = ti[rr * 6 + 4];
        nC[rr] = ti[rr * 6 + 5];
        off[rr + 1] = off[rr] + nA[rr] + nB[rr] + nC[rr];
    }
    const int total = off[3];
    const bool staged = total <= MAXP && total <= a.stage_max;
    const int nown = nB[1];
    const int lown = off[1] + nA[1];
    // periodic shifts of the halo copies
    const double sxa = x0 == 0 ? -L : 0.0, sxc = x1 == nc ? L : 0.0;
    const double sy0 = row == 0 ? -L : 0.0, sy2 = row == nc - 1 ? L : 0.0;

    // ---- prologue: every global load first ----
    const int nl = 3 * (tw + 1);
    int cv[NLCS];
#pragma unroll
    for (int u = 0; u < NLCS; ++u) {
        const int i = tid + u * BS;
        const int ii = i < nl ? i : 0;
        const int rr = ii / (tw + 1), j = ii - rr * (tw + 1);
        int rw = row + rr - 1;
        rw = rw < 0 ? rw + nc : (rw >= nc ? rw - nc : rw);
        cv[u] = a.cs[R.cell0 + rw * nc + x0 + j];
    }
    double2 sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = tid + u * BS;
        int g = min(gB[1], a.nslots - 1);
        if (staged && i < total) {
            const int rr = i < off[1] ? 0 : (i < off[2] ? 1 : 2);
            const int q = i - (rr == 0 ? off[0] : (rr == 1 ? off[1] : off[2]));
            const int na = rr == 0 ? nA[0] : (rr == 1 ? nA[1] : nA[2]);
            const int nb = rr == 0 ? nB[0] : (rr == 1 ? nB[1] : nB[2]);
            const int ga = rr == 0 ? gA[0] : (rr == 1 ? gA[1] : gA[2]);
            const int gb = rr == 0 ? gB[0] : (rr == 1 ? gB[1] : gB[2]);
            const int gc = rr == 0 ? gC[0] : (rr == 1 ? gC[1] : gC[2]);
            g = q < na ? ga + q : (q < na + nb ? gb + q - na : gc + q - na - nb);
        }
        sv[u] = a.pin[g];
    }
    const int s0 = min(gB[1] + (tid < nown ? tid : 0), a.nslots - 1);
    double2 v0 = a.vel[s0];
    double2 sp0 = make_double2(0.0, 0.0);
    if (CG) sp0 = a.snap[s0];

    // ---- LDS writes ----
#pragma unroll
    for (int u = 0; u < NLCS; ++u) {
        const int i = tid + u * BS;
        if (i < nl) {
            const int rr = i / (tw + 1), j = i - rr * (tw + 1);
            const int o = rr == 0 ? off[0] : (rr == 1 ? off[1] : off[2]);
            const int na = rr == 0 ? nA[0] : (rr == 1 ? nA[1] : nA[2]);
            const int gb = rr == 0 ? gB[0] : (rr == 1 ? gB[1] : gB[2]);
            lcs[rr][1 + j] = o + na + (cv[u] - gb);
        }
    }
    if (tid < 3) {
        lcs[tid][0] = tid == 0 ? off[0] : (tid == 1 ? off[1] : off[2]);
        lcs[tid][tw + 2] = tid == 0 ? off[1] : (tid == 1 ? off[2] : off[3]);
    }
    if (staged) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = tid + u * BS;
            if (i < total) {
                const int rr = i < off[1] ? 0 : (i < off[2] ? 1 : 2);
                const int q = i - (rr == 0 ? off[0] : (rr == 1 ? off[1] : off[2]));
                const int na = rr == 0 ? nA[0] : (rr == 1 ? nA[1] : nA[2]);
                const int nb = rr == 0 ? nB[0] : (rr == 1 ? nB[1] : nB[2]);
                double2 w = sv[u];
                w.x += q < na ? sxa : (q < na + nb ? 0.0 : sxc);
                w.y += rr == 0 ? sy0 : (rr == 2 ? sy2 : 0.0);
                lp[i] = w;
            }
        }
    }
    if (CG && tid < MDLG_NCOUNTS) hist[tid] = 0;
    __syncthreads();

    long long kcg = 0;
    if (CG) kcg = *a.event_k;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    for (int i0 = 0; i0 < nown; i0 += BS) {
        const int i = i0 + tid;
        const bool act = i < nown;
        const int l = lown + i;
        const int s = gB[1] + i;
        int idx = MDLG_NQ;
        if (act) {
            const double2 p = staged ? lp[l] : a.pin[s];
            // the cell this particle was sorted into: largest j with lcs[1][1 + j] <= l
            int lo = 0, hi = tw;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (lcs[1][1 + mid] <= l) lo = mid; else hi = mid;
            }
            const int j = lo;
            double ax = 0.0, ay = 0.0;
            float bx = 0.0f, by = 0.0f;
#pragma unroll
            for (int rr = 0; rr < 3; ++rr) {
                const int k0 = lcs[rr][j], k1 = lcs[rr][j + 3];
                for (int k = k0; k < k1; ++k) {
                    if (rr == 1 && k == l) continue;
                    double dx, dy;
                    if (staged) {
                        const double2 q = lp[k];
                        dx = p.x - q.x;
                        dy = p.y - q.y;
                    } else {
                        const int o = rr == 0 ? off[0] : (rr == 1 ? off[1] : off[2]);
                        const int na = rr == 0 ? nA[0] : (rr == 1 ? nA[1] : nA[2]);
                        const int nb = rr == 0 ? nB[0] : (rr == 1 ? nB[1] : nB[2]);
                        const int ga = rr == 0 ? gA[0] : (rr == 1 ? gA[1] : gA[2]);
                        const int gb = rr == 0 ? gB[0] : (rr == 1 ? gB[1] : gB[2]);
                        const int gc = rr == 0 ? gC[0] : (rr == 1 ? gC[1] : gC[2]);
                        const int qq = k - o;
                        const int g = qq < na ? ga + qq : (qq < na + nb ? gb + qq - na : gc + qq - na - nb);
                        const double2 q = a.pin[g];
                        dx = min_image(p.x - q.x, L, halfL);
                        dy = min_image(p.y - q.y, L, halfL);
                    }
                    if (F32) {
                        const float fdx = (float)dx, fdy = (float)dy;
                        const float r2 = fdx * fdx + fdy * fdy;
                        if (r2 < rc2f) {
                            const float ir2 = 1.0f / r2;
                            const float ir6 = ir2 * ir2 * ir2;
                            const float fr = eps24f * ir6 * (2.0f * ir6 - 1.0f) * ir2;
                            bx += fr * fdx;
                            by += fr * fdy;
                        }
                    } else {
                        const double r2 = dx * dx + dy * dy;
                        if (r2 < rc2) {
                            const double ir2 = 1.0 / r2;
                            const double ir6 = ir2 * ir2 * ir2;
                            const double fr = eps24 * ir6 * (2.0 * ir6 - 1.0) * ir2;
                            ax += fr * dx;
                            ay += fr * dy;
                        }
                    }
                }
            }
            const double fx = F32 ? (double)bx : ax;
            const double fy = F32 ? (double)by : ay;
            double2 v = i0 == 0 ? v0 : a.vel[s];
            if (!FIRST) {
                v.x = v.x + a.hdt * fx;
                v.y = v.y + a.hdt * fy;
            }
            v.x = v.x + a.hdt * fx;
            v.y = v.y + a.hdt * fy;
            double2 pn;
            pn.x = p.x + a.dt * v.x;
            pn.y = p.y + a.dt * v.y;
            int wx = 0, wy = 0;
            if (pn.x >= L) { pn.x -= L; wx = 1; }
            else if (pn.x < 0.0) { pn.x += L; wx = -1; if (pn.x >= L) { pn.x = 0.0; wx = 0; } }
            if (pn.y >= L) { pn.y -= L; wy = 1; }
            else if (pn.y < 0.0) { pn.y += L; wy = -1; if (pn.y >= L) { pn.y = 0.0; wy = 0; } }
            if (wx | wy) {
                int2 im = a.img[s];
                im.x += wx;
                im.y += wy;
                a.img[s] = im;
            }
            if (!isfinite(pn.x) || !isfinite(pn.y) || !isfinite(v.x) || !isfinite(v.y)) atomicOr(a.err, ERR_NONFINITE);
            a.pout[s] = pn;
            a.vel[s] = v;
            if (CG) {
                const double2 sp = i0 == 0 ? sp0 : a.snap[s];
                long long cell;
                idx = cg_index(R, kcg, pn, sp, cell);
                if (idx < MDLG_NQ && a.cell_acc)
                    atomicAdd(&a.cell_acc[R.cacc0 + (long long)idx * R.lx * R.lx + cell], 1);
                const double dx = min_image(pn.x - sp.x, L, halfL);
                const double dy = min_image(pn.y - sp.y, L, halfL);
                const double dx2 = dx * dx, dy2 = dy * dy;
                m0 += dx2 + dy2;
                m1 += dx2 * dx2 + dy2 * dy2;
                m2 += dx;
                m3 += dy;
                a.snap[s] = pn;
            }
        }
        if (CG) {
            // most particles keep their cell over a coarse step: count v = 0 with one ballot per wave
            const unsigned long long rest = __ballot(act && idx == 0);
            if ((tid & 63) == 0 && rest) atomicAdd(&hist[0], (int)__popcll(rest));
            if (act && idx != 0) atomicAdd(&hist[idx], 1);
        }
    }
    if (CG) {
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
        if (tid < MDLG_NCOUNTS) a.hpart[(long long)tid * a.pstride + t] = hist[tid];
        if (tid < 4) {
            double sum = 0.0;
            for (int w = 0; w < BS / 64; ++w) sum += red[w][tid];
            a.mpart[(long long)(1 + tid) * a.pstride + t] = sum;
        }
        if (tid == 0) a.mpart[t] = 2.0 * (double)nown;
    }
}

// One velocity-Verlet step, one thread per slot, neighbours gathered from
// global memory (FIRST: the stored velocity is a full-step one; CG: this step
// ends a coarse step).
//
// Latency, not bandwidth, bounds this kernel at low density, so every wave
// keeps its chain of dependent memory round trips short: position and
// velocity are loaded together; the nine cell bounds of the 3 x 3 stencil
// (three contiguous row ranges, split at the periodic edge) together; then
// the candidate neighbours in batches of U independent loads.
template <int BS, bool F32, bool FIRST, bool CG, int U>
__global__ __launch_bounds__(BS) void k_step_gather(StepArgs a) {
    __shared__ int hist[MDLG_NCOUNTS];
    __shared__ double red[BS / 64][4];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int r = __builtin_amdgcn_readfirstlane(a.tile_rep[tile]);
    const RepDev& R = a.reps[r];
    const double L = R.L, halfL = R.halfL, rc2 = R.rc2, eps24 = R.eps24, inv_w = R.inv_w;
    const float rc2f = R.rc2f, eps24f = R.eps24f;
    const int nc = R.nc, cell0 = R.cell0;
    const int tid = threadIdx.x;
    const int s = tile * BS + tid;
    const int nact_blk = min(BS, max(0, R.n - (tile * BS - R.slot0)));
    const bool act = tid < nact_blk;
    if (CG && tid < MDLG_NCOUNTS) hist[tid] = 0;

    const int sl = act ? s : tile * BS;  // a valid slot for the inactive lanes' loads
    const double2 p = a.pin[sl];
    double2 v = a.vel[sl];
    const int cx = cell_coord(p.x, inv_w, nc);
    const int cy = cell_coord(p.y, inv_w, nc);
    // stencil ranges: per row either one range (cells cx-1..cx+1) or two at the edge
    int ra[3], rb[3], na[3], nb[3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
        int rw = cy + rr - 1;
        rw = rw < 0 ? rw + nc : (rw >= nc ? rw - nc : rw);
        const int base = cell0 + rw * nc;
        const int xl = cx > 0 ? cx - 1 : 0;
        const int xr = cx < nc - 1 ? cx + 2 : nc;
        const int c0 = a.cs[base + xl], c1 = a.cs[base + xr];
        // the wrapped cell (if any): nc - 1 when cx == 0, 0 when cx == nc - 1
        const int xw = cx == 0 ? nc - 1 : 0;
        const bool wrap = (cx == 0) || (cx == nc - 1);
        const int w0 = wrap ? a.cs[base + xw] : 0, w1 = wrap ? a.cs[base + xw + 1] : 0;
        ra[rr] = c0;
        na[rr] = c1 - c0;
        rb[rr] = w0;
        nb[rr] = w1 - w0;
    }
    const int e0 = na[0], e1 = e0 + nb[0], e2 = e1 + na[1], e3 = e2 + nb[1], e4 = e3 + na[2], e5 = e4 + nb[2];
    const int tot = act ? e5 : 0;
    double ax = 0.0, ay = 0.0;
    float bx = 0.0f, by = 0.0f;
    for (int t0 = 0; t0 < tot; t0 += U) {
        double2 q[U];
        int kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u;
            int k = t < e0 ? ra[0] + t
                  : t < e1 ? rb[0] + (t - e0)
                  : t < e2 ? ra[1] + (t - e1)
                  : t < e3 ? rb[1] + (t - e2)
                  : t < e4 ? ra[2] + (t - e3)
                           : rb[2] + (t - e4);
            k = t < tot ? k : sl;
            kk[u] = t < tot ? k : -1;
            q[u] = a.pin[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (kk[u] < 0 || kk[u] == s) continue;
            const double dx = min_image(p.x - q[u].x, L, halfL);
            const double dy = min_image(p.y - q[u].y, L, halfL);
            if (F32) {
                const float fdx = (float)dx, fdy = (float)dy;
                const float r2 = fdx * fdx + fdy * fdy;
                if (r2 < rc2f) {
                    const float ir2 = 1.0f / r2;
                    const float ir6 = ir2 * ir2 * ir2;
                    const float fr = eps24f * ir6 * (2.0f * ir6 - 1.0f) * ir2;
                    bx += fr * fdx;
                    by += fr * fdy;
                }
            } else {
                const double r2 = dx * dx + dy * dy;
                if (r2 < rc2) {
                    const double ir2 = 1.0 / r2;
                    const double ir6 = ir2 * ir2 * ir2;
                    const double fr = eps24 * ir6 * (2.0 * ir6 - 1.0) * ir2;
                    ax += fr * dx;
                    ay += fr * dy;
                }
            }
        }
    }
    int idx = MDLG_NQ;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (act) {
        const double fx = F32 ? (double)bx : ax;
        const double fy = F32 ? (double)by : ay;
        if (!FIRST) {
            v.x = v.x + a.hdt * fx;
            v.y = v.y + a.hdt * fy;
        }
        v.x = v.x + a.hdt * fx;
        v.y = v.y + a.hdt * fy;
        double2 pn;
        pn.x = p.x + a.dt * v.x;
        pn.y = p.y + a.dt * v.y;
        int wx = 0, wy = 0;
        if (pn.x >= L) { pn.x -= L; wx = 1; }
        else if (pn.x < 0.0) { pn.x += L; wx = -1; if (pn.x >= L) { pn.x = 0.0; wx = 0; } }
        if (pn.y >= L) { pn.y -= L; wy = 1; }
        else if (pn.y < 0.0) { pn.y += L; wy = -1; if (pn.y >= L) { pn.y = 0.0; wy = 0; } }
        if (wx | wy) {
            int2 im = a.img[s];
            im.x += wx;
            im.y += wy;
            a.img[s] = im;
        }
        if (!isfinite(pn.x) || !isfinite(pn.y) || !isfinite(v.x) || !isfinite(v.y)) atomicOr(a.err, ERR_NONFINITE);
        a.pout[s] = pn;
        a.vel[s] = v;
        if (CG) {
            const double2 sp = a.snap[s];
            long long cell;
            idx = cg_index(R, *a.event_k, pn, sp, cell);
            if (idx < MDLG_NQ && a.cell_acc) atomicAdd(&a.cell_acc[R.cacc0 + (long long)idx * R.lx * R.lx + cell], 1);
            const double dx = min_image(pn.x - sp.x, L, halfL);
            const double dy = min_image(pn.y - sp.y, L, halfL);
            const double dx2 = dx * dx, dy2 = dy * dy;
            m0 = dx2 + dy2;
            m1 = dx2 * dx2 + dy2 * dy2;
            m2 = dx;
            m3 = dy;
            a.snap[s] = pn;
        }
    }
    if (CG) {
        __syncthreads();  // hist cleared
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
        if (tid < MDLG_NCOUNTS) a.hpart[(long long)tid * a.pstride + tile] = hist[tid];
        if (tid < 4) {
            double sum = 0.0;
            for (int w = 0; w < BS / 64; ++w) sum += red[w][tid];
            a.mpart[(long long)(1 + tid) * a.pstride + tile] = sum;
        }
        if (tid == 0) a.mpart[tile] = 2.0 * (double)nact_blk;
    }
}

// Minimum-image separation through the nearest whole number of boxes:
// d - L rint(d / L), rounded once; equal to the compare-and-select form for
// |d| < L.
__device__ __forceinline__ double min_image_rint(double d, double L, double invL) {
    return fma(-L, rint(d * invL), d);
}

// 1/x for x > 0 from the hardware reciprocal r and one third-order step,
// r (1 + e + e^2) with e = 1 - x r (the error of r is cubed, as two Newton
// steps would square it twice).  On gfx950 this equalled the correctly rounded
// quotient for 2^20 random x in [0.5, 10], as two Newton steps did, with one
// fused multiply-add fewer; one Newton step left up to 11 units in the last
// place.
__device__ __forceinline__ double recip(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(fma(e, e, e), r, r);
}

// Squared separation tested against the neighbour-list range, rounded as
// written (the same expression wherever lists are built).
__device__ __forceinline__ bool within_list_range(double dx, double dy, double rl2) {
#pragma clang fp contract(off)
    const double r2 = dx * dx + dy * dy;
    return r2 < rl2;
}

// Neighbour lists: for every slot, the slots within rc + skin (the cell width)
// of it, found through the 3 x 3 cells right after the cell-list rebuild.
// Layout nbl[j * S + s] (consecutive slots consecutive in memory for each j).
// An entry is the neighbour's slot relative to the particle's own slot,
// reduced modulo the replica's particle count into [-n/2, n/2): in cell order
// a neighbour lies within about three cell rows (also across the periodic
// edge, after the reduction), which fits 16 bits; counts fit 8 bits.  With
// CELL (for the tile list builder) an entry is instead the neighbour's cell
// relative to the particle's, (oy + 1) 3 + (ox + 1) in bits 12-15, and its
// index within that cell in bits 0-11, and ncol[s] holds the particle's cell
// column.  Also records the positions of the build for the next drift check.
template <bool CELL>
__global__ __launch_bounds__(256) void k_nlist_build(const double2* __restrict__ pos, const int* __restrict__ cs,
                                                     const RepDev* __restrict__ reps, const int* __restrict__ tile_rep,
                                                     int BSt, int S, int maxnb, short* __restrict__ nbl,
                                                     unsigned char* __restrict__ nbc, unsigned short* __restrict__ ncol,
                                                     double2* __restrict__ pref, int* err) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const RepDev& R = reps[tile_rep[min(s, S - 1) / BSt]];
    const bool act = s < S && s - R.slot0 < R.n;
    const double2 p = pos[act ? s : 0];
    const int nc = R.nc;
    const int cx = cell_coord(p.x, R.inv_w, nc);
    const int cy = cell_coord(p.y, R.inv_w, nc);
    // a wave whose particles all lie in cells 1 .. nc - 2 has no candidate
    // across the periodic edge (candidates within one cell: separations below
    // 2 w <= L / 2 for nc >= 4): the minimum image would leave them unchanged,
    // bit for bit
    const bool inner = nc >= 4 && cx >= 1 && cx < nc - 1 && cy >= 1 && cy < nc - 1;
    const bool interior = __ballot(act && !inner) == 0ull;
    if (s >= S) return;
    if (!act) {
        nbc[s] = 0;
        return;
    }
    pref[s] = p;
    const double invL = 1.0 / R.L;
    const double rl2 = R.w * R.w;
    if (CELL) ncol[s] = (unsigned short)cx;
    int cnt = 0;
    for (int oy = -1; oy <= 1; ++oy) {
        int rw = cy + oy;
        rw = rw < 0 ? rw + nc : (rw >= nc ? rw - nc : rw);
        const int base = R.cell0 + rw * nc;
        // cells cx-1 .. cx+1 as one range, or two at the periodic edge
        const int xl = cx > 0 ? cx - 1 : 0;
        const int xr = cx < nc - 1 ? cx + 2 : nc;
        const bool wrap = (cx == 0) || (cx == nc - 1);
        const int xw = cx == 0 ? nc - 1 : 0;
        const int a0 = cs[base + xl], a1 = cs[base + xr];
        const int b0 = wrap ? cs[base + xw] : 0, b1 = wrap ? cs[base + xw + 1] : 0;
        // with CELL, the first slots of the range's second and third cells
        const int m1 = CELL && xr - xl >= 2 ? cs[base + xl + 1] : a1;
        const int m2 = CELL && xr - xl >= 3 ? cs[base + xl + 2] : a1;
        const int na = a1 - a0, tot = na + (b1 - b0);
        for (int t = 0; t < tot; ++t) {
            const int k = t < na ? a0 + t : b0 + (t - na);
            if (k == s) continue;
            const double2 q = pos[k];
            double dx = p.x - q.x, dy = p.y - q.y;
            if (!interior) {
                dx = min_image_rint(dx, R.L, invL);
                dy = min_image_rint(dy, R.L, invL);
            }
            if (within_list_range(dx, dy, rl2)) {
                int e;
                if (CELL) {
                    int ox, first;
                    if (t < na) {
                        const int j = (k >= m1 ? 1 : 0) + (k >= m2 ? 1 : 0);
                        ox = xl + j - cx;
                        first = j == 0 ? a0 : (j == 1 ? m1 : m2);
                    } else {
                        ox = cx == 0 ? -1 : 1;
                        first = b0;
                    }
                    const int idx = k - first;
                    if (idx > 4095) atomicOr(err, ERR_NLIST);
                    e = (((oy + 1) * 3 + (ox + 1)) << 12) | (idx & 4095);
                } else {
                    e = k - s;
                    if (2 * e >= R.n) e -= R.n;
                    else if (2 * e < -R.n) e += R.n;
                    if (e < -32768 || e > 32767) atomicOr(err, ERR_NLIST);
                }
                if (cnt < maxnb) nbl[(long long)cnt * S + s] = (short)e;
                ++cnt;
            }
        }
    }
    if (cnt > maxnb) {
        atomicOr(err, ERR_NLIST);
        cnt = maxnb;
    }
    nbc[s] = (unsigned char)cnt;
}

// Pair force on a particle at p from the nn entries of its neighbour list
// (entry j at list[off + j * stride]); fetch(entry) returns the neighbour's
// position.  kListU entries per pass: their index loads, then their
// position loads, then the arithmetic (entries past the list are masked).
// Two per pass leave fewer masked slots than four: the lanes of a wave run as
// many passes as the longest list among them.
// Without `interior` every separation goes through the minimum image, which
// leaves separations below L/2 unchanged bit for bit.
// Neighbour-list entries are read U rows at a time.  The list has maxnb rows,
// a multiple of U, so rows j0 .. j0 + U - 1 exist whenever j0 < nn: they are
// loaded without waiting for the count nn, and entries past nn are replaced
// by 0 (a valid index) before they are used as one.
constexpr int kListU = 2;              // fused kernels (lists ordered by length within a tile)
constexpr int kListUOne = 4;           // one-step kernel (slot order: fewer, longer passes keep more loads in flight)
constexpr int kListPre = 4 * kListU;  // rows loaded ahead for a thread's first particle (maxnb >= 16)
constexpr int kListPreEvent = 2 * kListU;  // the same in the event and binning launches
static_assert(kListPre % kListU == 0, "whole passes of the fused kernels' rows loaded ahead");

template <int N, typename Entry>
__device__ __forceinline__ void list_rows(const Entry* __restrict__ list, unsigned int off, unsigned int stride,
                                          int (&kk)[N]) {
#pragma unroll
    for (int u = 0; u < N; ++u) kk[u] = list[off + u * stride];
}

// With use_first, the rows of the passes that lie within the first P come
// from `first`.
template <bool F32, int U, int P, typename Entry, typename Fetch>
__device__ __forceinline__ void nlist_force(double2 p, int nn, const Entry* __restrict__ list, unsigned int off,
                                            unsigned int stride, Fetch fetch, bool interior, double L, double invL,
                                            double rc2, double eps24, float rc2f, float eps24f, double& fx,
                                            double& fy, const int (&first)[P], bool use_first) {
    double ax = 0.0, ay = 0.0;
    float bx = 0.0f, by = 0.0f;
    for (int j0 = 0; j0 < nn; j0 += U, off += U * stride) {
        int kk[U];
        if (use_first && j0 + U <= P) {
#pragma unroll
            for (int b = 0; b < P / U; ++b)
                if (j0 == b * U) {
#pragma unroll
                    for (int u = 0; u < U; ++u) kk[u] = first[b * U + u];
                }
        } else {
            list_rows(list, off, stride, kk);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) kk[u] = j0 + u < nn ? kk[u] : 0;
        double2 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = fetch(kk[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool valid = j0 + u < nn;
            double dx = p.x - q[u].x, dy = p.y - q[u].y;
            if (!interior) {
                dx = min_image_rint(dx, L, invL);
                dy = min_image_rint(dy, L, invL);
            }
            // entries past the list (index 0: any staged particle, or the particle
            // itself) are computed and then dropped with the cutoff test; a zero
            // separation gives a NaN there, which the select discards
            if (F32) {
                const float fdx = (float)dx, fdy = (float)dy;
                const float r2 = fdx * fdx + fdy * fdy;
                const float ir2 = __builtin_amdgcn_rcpf(r2);
                const float ir2n = ir2 * (2.0f - r2 * ir2);
                const float ir6 = ir2n * ir2n * ir2n;
                float fr = eps24f * ir6 * (2.0f * ir6 - 1.0f) * ir2n;
                fr = (valid && r2 < rc2f) ? fr : 0.0f;
                bx += fr * fdx;
                by += fr * fdy;
            } else {
                const double r2 = dx * dx + dy * dy;
                const double ir2 = recip(r2);
                const double ir6 = ir2 * ir2 * ir2;
                double fr = eps24 * ir6 * (2.0 * ir6 - 1.0) * ir2;
                fr = (valid && r2 < rc2) ? fr : 0.0;
                ax += fr * dx;
                ay += fr * dy;
            }
        }
    }
    fx = F32 ? (double)bx : ax;
    fy = F32 ? (double)by : ay;
}

template <bool F32, int U, typename Entry, typename Fetch>
__device__ __forceinline__ void nlist_force(double2 p, int nn, const Entry* __restrict__ list, unsigned int off,
                                            unsigned int stride, Fetch fetch, bool interior, double L, double invL,
                                            double rc2, double eps24, float rc2f, float eps24f, double& fx,
                                            double& fy) {
    const int none[1] = {};
    nlist_force<F32, U, 1>(p, nn, list, off, stride, fetch, interior, L, invL, rc2, eps24, rc2f, eps24f, fx, fy,
                           none, false);
}

// Velocity-Verlet update with the force at the current position: complete
// the half-step velocity (not on the first step, whose velocity is a full-step
// one), kick, drift, wrap into [0, L) with the image change in (wx, wy).
template <bool FIRST, bool WRAP = true>
__device__ __forceinline__ double2 vv_update(double2 p, double2& v, double fx, double fy, double dt, double hdt,
                                             double L, int& wx, int& wy) {
    if (!FIRST) {
        v.x = v.x + hdt * fx;
        v.y = v.y + hdt * fy;
    }
    v.x = v.x + hdt * fx;
    v.y = v.y + hdt * fy;
    double2 pn;
    pn.x = p.x + dt * v.x;
    pn.y = p.y + dt * v.y;
    wx = 0;
    wy = 0;
    if (!WRAP) return pn;  // the caller knows that no particle reaches the box edge
    if (pn.x >= L) { pn.x -= L; wx = 1; }
    else if (pn.x < 0.0) { pn.x += L; wx = -1; if (pn.x >= L) { pn.x = 0.0; wx = 0; } }
    if (pn.y >= L) { pn.y -= L; wy = 1; }
    else if (pn.y < 0.0) { pn.y += L; wy = -1; if (pn.y >= L) { pn.y = 0.0; wy = 0; } }
    return pn;
}

// One velocity-Verlet step, one thread per slot, pair forces over the slot's
// neighbour list (FIRST: the stored velocity is a full-step one; CG: this step
// ends a coarse step).  Per neighbour: one coalesced index load, one position
// gather, the minimum image through rint, and the pair force with the
// reciprocal from the hardware estimate refined by Newton steps.
template <int BS, bool F32, bool FIRST, bool CG>
__global__ __launch_bounds__(BS) void k_step_nlist(StepArgs a) {
    __shared__ int hist[MDLG_NCOUNTS];
    __shared__ double red[BS / 64][4];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int r = a.nrep == 1 ? 0 : __builtin_amdgcn_readfirstlane(a.tile_rep[tile]);
    const RepDev& R = a.reps[r];
    const double L = R.L, halfL = R.halfL;
    const double invL = 1.0 / L;
    const int tid = threadIdx.x;
    const int s = tile * BS + tid;
    const int nact_blk = min(BS, max(0, R.n - (tile * BS - R.slot0)));
    const bool act = tid < nact_blk;
    if (CG && tid < MDLG_NCOUNTS) hist[tid] = 0;

    const double2 p = a.pin[s];
    double2 v = a.vel[s];
    const int nn = act ? a.nbc[s] : 0;
    // A wave whose particles all lie two cell widths or more inside the box has
    // no neighbour across the periodic edge: its separations need no image.
    const double edge = 2.0 * R.w;
    const bool near_edge = act && (p.x < edge || p.x > L - edge || p.y < edge || p.y > L - edge);
    const bool interior = __ballot(near_edge) == 0ull;
    const int srel = s - R.slot0, nr = R.n, slot0 = R.slot0;
    const double2* __restrict__ pin = a.pin;
    auto fetch = [&](int k) {
        int kr = srel + k;
        kr = kr < 0 ? kr + nr : (kr >= nr ? kr - nr : kr);
        return pin[slot0 + kr];
    };
    double fx, fy;
    nlist_force<F32, kListUOne>(p, nn, a.nbl, (unsigned int)s, (unsigned int)a.nslots, fetch, interior, L, invL, R.rc2, R.eps24,
                     R.rc2f, R.eps24f, fx, fy);
    int idx = MDLG_NQ;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (act) {
        int wx, wy;
        const double2 pn = vv_update<FIRST>(p, v, fx, fy, a.dt, a.hdt, L, wx, wy);
        if (wx | wy) {
            int2 im = a.img[s];
            im.x += wx;
            im.y += wy;
            a.img[s] = im;
        }
        if (!isfinite(pn.x) || !isfinite(pn.y) || !isfinite(v.x) || !isfinite(v.y)) atomicOr(a.err, ERR_NONFINITE);
        a.pout[s] = pn;
        a.vel[s] = v;
        if (CG) {
            const double2 sp = a.snap[s];
            long long cell;
            idx = cg_index(R, *a.event_k, pn, sp, cell);
            if (idx < MDLG_NQ && a.cell_acc) atomicAdd(&a.cell_acc[R.cacc0 + (long long)idx * R.lx * R.lx + cell], 1);
            const double dx = min_image(pn.x - sp.x, L, halfL);
            const double dy = min_image(pn.y - sp.y, L, halfL);
            const double dx2 = dx * dx, dy2 = dy * dy;
            m0 = dx2 + dy2;
            m1 = dx2 * dx2 + dy2 * dy2;
            m2 = dx;
            m3 = dy;
            a.snap[s] = pn;
        }
    }
    if (CG) {
        __syncthreads();  // hist cleared
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
        if (tid < MDLG_NCOUNTS) a.hpart[(long long)tid * a.pstride + tile] = hist[tid];
        if (tid < 4) {
            double sum = 0.0;
            for (int w = 0; w < BS / 64; ++w) sum += red[w][tid];
            a.mpart[(long long)(1 + tid) * a.pstride + tile] = sum;
        }
        if (tid == 0) a.mpart[tile] = 2.0 * (double)nact_blk;
    }
}

// Fused tiles: several consecutive ordinary steps per launch.  The box is cut
// into square tiles of pT x pT cells; a block owns the particles of one tile.
// Its staged set is those particles (owned), then the particles of the ring of
// cells around the tile (ring 1), then those of the next rings (`rings` in
// all, two or three).  Neighbour lists reach one cell width, so ring k + 1
// holds every neighbour of a ring-k particle.  A launch of NS <= rings steps
// loads the positions of the owned particles and rings 1 .. NS (and the
// velocities of owned and rings 1 .. NS - 1) into LDS once; step j advances
// the owned particles and rings 1 .. NS - j from the previous step's positions
// in LDS (ring particles are advanced by their own tiles too: the halo work is
// repeated, not shared), through per-tile neighbour lists of staged indices
// built at the rebuild.  Every step runs the same force and update code as the
// one-step kernel, in the same neighbour order, so NS steps per launch equal NS
// one-step launches bit for bit.  Velocities go to a second buffer: other
// tiles still read the old ones.
constexpr int kPairCap = 768;      // staged particles of one tile (owned + its rings)
constexpr int kStep2BS = 512;      // threads of the fused step kernels and of the tile builder
constexpr int kPairAutoT = 16;     // smallest tile side (cells) of the default fused choice
constexpr int kPairTarget = 520;   // staged particles aimed at when choosing the tile side, two rings
constexpr int kPairTarget3 = 580;  // the same with three rings
constexpr int kPairSeg = 248;      // row segments of one tile: 7 pT + 24 <= 248 for pT <= 32, three rings
constexpr int kPairBuildBS = 256;  // threads of the tile list builder
constexpr int kPairPre = 4;        // list rows it reads ahead per particle (maxnb >= 16)

// End of a coarse step: per replica and component, the fixed-order sum over
// the replica's tiles of the histogram and moment partials is added to the
// caller's accumulators.  Block (r, c): c < 50 counts, c >= 50 moments.  Tiles
// of the step kernel that wrote the partials: mode 0 slot tiles, 1 cell tiles,
// 2 fused tiles.  Partials are stored component-major, so a block reads one
// contiguous row; each thread issues its loads (up to kFinishU per chunk of
// 256 kFinishU tiles) together and sums them in order, then a wave tree and
// the waves in order finish the block.  Block 0 advances the coarse-step
// index (no kernel of this launch reads it).  The same code runs as a kernel
// of its own or in the first blocks of the fused launch after the event (the
// same sums in the same order either way).
constexpr int kFinishU = 16;
constexpr int kFinishBS = 256;  // threads that load and sum (a block may be wider; the rest join the barrier)

__device__ __forceinline__ void cg_finish_one(const int* __restrict__ hpart, const double* __restrict__ mpart,
                                              int pstride, const RepDev* __restrict__ reps,
                                              unsigned long long* counts, double* moments, long long* event_k,
                                              int mode, int blk) {
    __shared__ double red[4];
    __shared__ long long redi[4];
    const int r = blk / (MDLG_NCOUNTS + MDLG_NMOMENTS);
    const int c = blk % (MDLG_NCOUNTS + MDLG_NMOMENTS);
    const RepDev& R = reps[r];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool act = tid < kFinishBS;
    const int b0 = mode == 2 ? R.pt0 : (mode == 1 ? R.ttile0 : R.tile0);
    const int nb = mode == 2 ? R.pnt : (mode == 1 ? R.nttile : R.ntile);
    if (c < MDLG_NCOUNTS) {
        const int* __restrict__ row = hpart + (long long)c * pstride + b0;
        long long sum = 0;
        if (act) {
            for (int base = 0; base < nb; base += kFinishBS * kFinishU) {
                int v[kFinishU];
#pragma unroll
                for (int u = 0; u < kFinishU; ++u) {
                    const int b = base + tid + u * kFinishBS;
                    v[u] = b < nb ? row[b] : 0;
                }
#pragma unroll
                for (int u = 0; u < kFinishU; ++u) sum += v[u];
            }
        }
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (act && lane == 0) redi[wv] = sum;
        __syncthreads();
        if (tid == 0) {
            const long long tot = redi[0] + redi[1] + redi[2] + redi[3];
            if (tot) counts[(long long)r * MDLG_NCOUNTS + c] += (unsigned long long)tot;
        }
    } else {
        const int j = c - MDLG_NCOUNTS;
        const double* __restrict__ row = mpart + (long long)j * pstride + b0;
        double sum = 0.0;
        if (act) {
            for (int base = 0; base < nb; base += kFinishBS * kFinishU) {
                double v[kFinishU];
#pragma unroll
                for (int u = 0; u < kFinishU; ++u) {
                    const int b = base + tid + u * kFinishBS;
                    v[u] = b < nb ? row[b] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kFinishU; ++u) sum += v[u];
            }
        }
        sum = wave_sum(sum);
        if (act && lane == 0) red[wv] = sum;
        __syncthreads();
        if (tid == 0) moments[(long long)r * MDLG_NMOMENTS + j] += ((red[0] + red[1]) + red[2]) + red[3];
    }
    if (blk == 0 && tid == 0) *event_k += 1;
}

// NS ordinary steps of one tile (FIRST: the stored velocity is a full-step one,
// only as a launch of one step; CG: the last step ends a coarse step, and the
// owned particles also evaluate the event of Eq.(n_i): lattice index and
// destination cell, the block's histogram in LDS with one count per wave for
// the rest velocity, moment partials of the tile in a fixed order; BIN: the
// launch is the last before a cell-list rebuild, and the owned particles are
// also binned for its counting sort at their final positions: cell key, rank
// within the cell by an atomic count, and the drift check against the
// positions of the list build, the work of k_bin without its pass over the
// positions).  A launch without an event may also carry the finish of the
// previous one in its first a.fin_n blocks, after their tile.
template <int BS, bool F32, int NS, bool FIRST, bool CG, bool BIN>
__global__ __launch_bounds__(BS, 8) void k_step_fused(StepArgs a) {
    static_assert(NS >= 1 && NS <= 3 && (!FIRST || NS == 1), "one to three steps; a first step alone");
    static_assert(BS <= kPairCap && kPairCap <= 2 * BS, "two staged particles per thread at most");
    constexpr int NB = NS >= 2 ? kPairCap : 1;
    __shared__ double2 xa[kPairCap];  // staged positions at time t; after step 2 of three
    __shared__ double2 xb[NB];        // positions after step 1
    __shared__ double2 vs[kPairCap];  // velocities of the particles advanced in step 1
    __shared__ char2 wr[NB];          // image changes of owned particles before the last step
    __shared__ int hist[CG ? MDLG_NCOUNTS : 1];
    __shared__ double red[CG ? BS / 64 : 1][4];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    // a thread stages q = tid and tid + BS: their slots, and for the first its
    // neighbour count and first list rows, all read before the tile's counts
    // and replica arrive (every tile has kPairCap slot and count entries and
    // maxnb rows; those past the counts are not used)
    const int* __restrict__ list = a.plist + (long long)t * kPairCap;
    const unsigned short* __restrict__ tl = a.tlist + (long long)t * a.maxnb * kPairCap;
    const unsigned char* __restrict__ tc = a.tcnt + (long long)t * kPairCap;
    const unsigned int SL = (unsigned int)kPairCap;
    const int qf = threadIdx.x;
    // the block's histogram starts from zero (ordered before its first use by
    // the staging barrier; cleared first so that no address stays live)
    if (CG && qf < MDLG_NCOUNTS) hist[qf] = 0;
    const int s_first = list[qf];
    const int s_second = qf + BS < kPairCap ? list[qf + BS] : 0;
    const int nn_first = tc[qf];
    // the event and binning launches, short of registers, load fewer rows ahead
    constexpr int PRE = (CG || BIN) ? kListPreEvent : kListPre;
    int pre[PRE];
    list_rows(tl, (unsigned int)qf, SL, pre);
    const int4 c = a.pcnt[t];
    const int own = c.x;
    const int nst = NS == 1 ? c.y : (NS == 2 ? c.z : c.w);   // staged positions: owned and rings 1 .. NS
    const int nvel = NS == 1 ? c.x : (NS == 2 ? c.y : c.z);  // advanced in step 1
    const int r = a.nrep == 1 ? 0 : __builtin_amdgcn_readfirstlane(a.ptile_rep[t]);
    const RepDev& R = a.reps[r];
    const double L = R.L;
    const double invL = 1.0 / L;
    const double2* __restrict__ pin = a.pin;
    // the four state loads in flight together (slot 0 stands in for unused ones)
    const bool h0 = qf < nst, h1 = qf + BS < nst;
    const double2 p0 = pin[h0 ? s_first : 0];
    const double2 v0 = a.vel[qf < nvel ? s_first : 0];
    const double2 p1 = pin[h1 ? s_second : 0];
    const double2 v1 = a.vel[qf + BS < nvel ? s_second : 0];
    long long ek = 0;
    if (CG) ek = *a.event_k;
    double2 q0 = make_double2(0.0, 0.0), q1 = q0;  // positions of the list build (drift check)
    if (BIN) {
        q0 = a.pref[qf < c.x ? s_first : 0];
        q1 = a.pref[qf + BS < c.x ? s_second : 0];
    }
    // A tile rings + 1 cells or more from every box edge stages particles of
    // cells 1 .. nc - 2 only; they move less than a cell between rebuilds, so
    // none crosses the periodic boundary: separations need no image, positions
    // no wrap and images no update.
    const int nc = R.nc, T = R.pT, lt = t - R.pt0;
    const int c0 = (lt % R.pts) * T, r0 = (lt / R.pts) * T;
    const int c1 = min(c0 + T, nc), r1 = min(r0 + T, nc);
    const int edge = a.rings + 1;
    const bool interior = c0 >= edge && r0 >= edge && c1 <= nc - edge && r1 <= nc - edge;
    if (h0) xa[qf] = p0;
    if (qf < nvel) vs[qf] = v0;
    if (h1) xa[qf + BS] = p1;
    if (qf + BS < nvel) vs[qf + BS] = v1;
    __syncthreads();
    // an intermediate step: particles [0, count) from src into dst (LDS); the
    // image changes of owned particles are kept (set on the first step, added
    // on the second)
    auto middle = [&](int count, const double2* src, double2* dst, bool first_step) {
        for (int q = threadIdx.x; q < count; q += BS) {
            const bool firstq = q == qf;
            const double2 p = src[q];
            double2 v = vs[q];
            const int nn = firstq ? nn_first : tc[q];
            auto fetch = [&](int k) { return src[k]; };
            double fx, fy;
            nlist_force<F32, kListU, PRE>(p, nn, tl, (unsigned int)q, SL, fetch, interior, L, invL, R.rc2, R.eps24,
                                     R.rc2f, R.eps24f, fx, fy, pre, firstq);
            int wx, wy;
            const double2 pn = interior ? vv_update<false, false>(p, v, fx, fy, a.dt, a.hdt, L, wx, wy)
                                        : vv_update<false, true>(p, v, fx, fy, a.dt, a.hdt, L, wx, wy);
            dst[q] = pn;
            vs[q] = v;
            if (q < own && !interior) {
                if (first_step) {
                    wr[q] = make_char2((signed char)wx, (signed char)wy);
                } else {
                    const char2 w = wr[q];
                    wr[q] = make_char2((signed char)(w.x + wx), (signed char)(w.y + wy));
                }
            }
        }
    };
    const double2* last = xa;
    if constexpr (NS == 2) {
        middle(c.y, xa, xb, true);
        __syncthreads();
        last = xb;
    } else if constexpr (NS == 3) {
        middle(c.z, xa, xb, true);
        __syncthreads();
        middle(c.y, xb, xa, false);  // every read of xa is done
        __syncthreads();
    }
    // the last step: owned particles, to global memory
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    int rest = 0;
    for (int q = threadIdx.x; q < own; q += BS) {
        const bool firstq = q == qf;
        const int s = firstq ? s_first : s_second;
        const double2 p = last[q];
        double2 v = vs[q];
        const int nn = firstq ? nn_first : tc[q];
        auto fetch = [&](int k) { return last[k]; };
        double fx, fy;
        nlist_force<F32, kListU, PRE>(p, nn, tl, (unsigned int)q, SL, fetch, interior, L, invL, R.rc2, R.eps24, R.rc2f,
                                 R.eps24f, fx, fy, pre, firstq);
        int wx, wy;
        const double2 pn = interior ? vv_update<FIRST, false>(p, v, fx, fy, a.dt, a.hdt, L, wx, wy)
                                    : vv_update<FIRST, true>(p, v, fx, fy, a.dt, a.hdt, L, wx, wy);
        if (NS >= 2 && !interior) {
            const char2 w1 = wr[q];
            wx += w1.x;
            wy += w1.y;
        }
        if (wx | wy) {
            int2 im = a.img[s];
            im.x += wx;
            im.y += wy;
            a.img[s] = im;
        }
        if (!isfinite(pn.x) || !isfinite(pn.y) || !isfinite(v.x) || !isfinite(v.y)) atomicOr(a.err, ERR_NONFINITE);
        a.pout[s] = pn;
        a.vout[s] = v;
        if (BIN) {
            const int k = R.cell0 + cell_coord(pn.y, R.inv_w, nc) * nc + cell_coord(pn.x, R.inv_w, nc);
            const double2 q = firstq ? q0 : q1;
            const double ex = fabs(min_image(pn.x - q.x, L, R.halfL));
            const double ey = fabs(min_image(pn.y - q.y, L, R.halfL));
            if (!(ex * ex + ey * ey <= R.skin_half * R.skin_half)) atomicOr(a.err, ERR_SKIN);
            a.key[s] = k;
            a.rank[s] = atomicAdd(&a.cnt[k], 1);
        }
        if (CG) {
            const double2 sp = a.snap[s];
            long long cell;
            const int idx = cg_index(R, ek, pn, sp, cell);
            if (idx < MDLG_NQ && a.cell_acc) atomicAdd(&a.cell_acc[R.cacc0 + (long long)idx * R.lx * R.lx + cell], 1);
            if (idx == 0) ++rest;
            else atomicAdd(&hist[idx], 1);
            const double dx = min_image(pn.x - sp.x, L, R.halfL);
            const double dy = min_image(pn.y - sp.y, L, R.halfL);
            const double dx2 = dx * dx, dy2 = dy * dy;
            m0 += dx2 + dy2;
            m1 += dx2 * dx2 + dy2 * dy2;
            m2 += dx;
            m3 += dy;
            a.snap[s] = pn;
        }
    }
    if (BIN && t == R.pt0 && threadIdx.x == 0) a.cnt[R.cell0 + nc * nc] = R.npad;
    if (CG) {
        // rest velocities: one LDS add per wave; then the tile's partials
        for (int o = 32; o > 0; o >>= 1) rest += __shfl_xor(rest, o, 64);
        const int tid = threadIdx.x;
        if ((tid & 63) == 0 && rest) atomicAdd(&hist[0], rest);
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
        if (tid < MDLG_NCOUNTS) a.hpart[(long long)tid * a.pstride + t] = hist[tid];
        if (tid < 4) {
            double sum = 0.0;
            for (int w = 0; w < BS / 64; ++w) sum += red[w][tid];
            a.mpart[(long long)(1 + tid) * a.pstride + t] = sum;
        }
        if (tid == 0) a.mpart[t] = 2.0 * (double)own;
    }
    if constexpr (!CG) {
        // the previous event's finish rides on the first blocks of this launch
        if (a.fin_n > 0 && (int)blockIdx.x < a.fin_n)
            cg_finish_one(a.hpart, a.mpart, a.pstride, a.reps, a.counts, a.moments, a.event_kw, 2, blockIdx.x);
    }
}

// Per tile, after the neighbour lists (entries by cell and index within the
// cell): the staged slots, as contiguous slot ranges of the row-major cell
// order (owned rows; then ring 1: the rows above and below and the cells left
// and right of each owned row; then ring 2 and, with three rings, ring 3
// likewise one cell further out each), the counts (owned, up to ring 1, up to
// ring 2, all), and for the particles of every ring but the last their
// neighbour counts and lists as staged indices, [tile][row j][staged index q].
// Neighbour lists reach one cell, so the neighbours of a ring-k particle lie
// within ring k + 1.  A tile that stages more than kPairCap particles raises
// ERR_TILE, a neighbour outside that bound ERR_NLIST.
template <int BS>
__global__ __launch_bounds__(BS) void k_pair_build(const int* __restrict__ cs, const RepDev* __restrict__ reps,
                                                    const int* __restrict__ ptrep, const short* __restrict__ nbl,
                                                    const unsigned char* __restrict__ nbc,
                                                    const unsigned short* __restrict__ ncol, int S, int maxnb, int rings,
                                                    int* __restrict__ plist, int4* __restrict__ pcnt,
                                                    unsigned short* __restrict__ tlist,
                                                    unsigned char* __restrict__ tcnt, int* err) {
    static_assert(kPairSeg <= 256 && BS % 256 == 0, "one segment per thread of each 256 threads");
    __shared__ int sa[kPairSeg], sn[kPairSeg], so[kPairSeg + 1];
    const int t = blockIdx.x;
    const RepDev& R = reps[ptrep[t]];
    const int nc = R.nc, T = R.pT;
    const int lt = t - R.pt0, ty = lt / R.pts, tx = lt % R.pts;
    const int c0 = tx * T, c1 = min(c0 + T, nc), r0 = ty * T, r1 = min(r0 + T, nc);
    const int nr = r1 - r0;
    // Segments: owned rows [0, nr); ring k (1 <= k <= rings) from
    // first(k) = nr + (k - 1) 2 nr + 2 k (k - 1): the rows r0 - k and r1 + k - 1 over
    // columns [c0 - k, c1 + k) as two pieces each (inside the box, wrapped
    // across it), then the cells c0 - k and c1 + k - 1 of the rows
    // r0 - k + 1 .. r1 + k - 2.  nc >= pT + 2 rings keeps every cell distinct.
    auto first = [&](int k) { return nr + (k - 1) * 2 * nr + 2 * k * (k - 1); };
    const int ns = first(rings + 1);
    for (int q = threadIdx.x; q < ns; q += blockDim.x) {
        int row, a, b, piece = -1;  // columns [a, b) before wrapping; piece >= 0: a row range
        if (q < nr) {
            row = r0 + q;
            a = c0;
            b = c1;
        } else {
            int k = 1;
            while (q >= first(k + 1)) ++k;
            const int e = q - first(k);
            if (e < 4) {
                row = (e >> 1) ? r1 + k - 1 : r0 - k;
                a = c0 - k;
                b = c1 + k;
                piece = e & 1;
            } else {
                const int f = e - 4;
                row = r0 - k + 1 + (f >> 1);
                a = (f & 1) ? c1 + k - 1 : c0 - k;
                b = a + 1;
            }
        }
        row = row < 0 ? row + nc : (row >= nc ? row - nc : row);
        int ca, cb;
        if (piece < 0) {
            ca = a < 0 ? a + nc : (a >= nc ? a - nc : a);  // one cell, or an owned row inside the box
            cb = ca + (b - a);
        } else if (piece == 0) {
            ca = max(a, 0);
            cb = min(b, nc);
        } else if (a < 0) {
            ca = a + nc;
            cb = nc;
        } else if (b > nc) {
            ca = 0;
            cb = b - nc;
        } else {
            ca = 0;
            cb = 0;
        }
        const int base = R.cell0 + row * nc;
        const int a0 = cs[base + ca], n0 = cs[base + cb] - a0;
        sa[q] = a0;
        sn[q] = n0;
    }
    __syncthreads();
    // first staged index of each segment: exclusive prefix sums of the lengths
    {
        __shared__ int wsum[BS / 64];
        const int q = threadIdx.x, lane = q & 63, wv = q >> 6;
        const int v = q < ns ? sn[q] : 0;
        int x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wv; ++w) off += wsum[w];
        if (q < ns) so[q] = off + x - v;
        if (q == BS - 1) so[ns] = off + x;  // the total (entries past ns are 0)
    }
    __syncthreads();
    // staged counts up to each ring: n[0] owned, n[k] owned and rings 1 .. k
    int n[4];
    for (int k = 0; k < 4; ++k) n[k] = min(so[first(min(k, rings) + 1)], kPairCap);
    const int own = n[0];
    int tot = so[ns];
    if (tot > kPairCap) {
        if (threadIdx.x == 0) atomicOr(err, ERR_TILE);
        tot = kPairCap;
    }
    if (threadIdx.x == 0) pcnt[t] = make_int4(own, n[1], n[2], tot);
    // Staged slots: segment order, then within each ring that has lists (all
    // but the last) reordered by the particle's number of list-row groups
    // (kListU rows each), most first, so that the lanes of a wave mostly run
    // the same number of passes over their lists.  Within a group the order is
    // the segment order (a stable counting sort), so every per-tile sum over
    // the staged particles rounds the same way in every run.
    // List entries name a neighbour by its cell relative to the particle's and
    // its index in that cell; a map of the tile's cells (owned and rings, local
    // coordinates relative to column c0 - rings and row r0 - rings, modulo nc)
    // gives each cell's first staged index (segment order).  A cell's particles
    // are consecutive there (one segment holds the cell, in slot order), so the
    // first of each run of equal cells writes the map.
    constexpr int kMapSide = 32 + 6;  // pT <= 32, rings <= 3
    __shared__ unsigned short mst[kMapSide * kMapSide];
    __shared__ unsigned short ckey[kPairCap];  // local cell, segment order
    __shared__ unsigned short lcell[kPairCap];  // local cell, final order
    __shared__ unsigned short qn_of[kPairCap];  // final index of each segment index
    __shared__ int lq[kPairCap];   // slot of each staged index
    __shared__ int lq0[kPairCap];  // slots in segment order
    __shared__ unsigned char gq[kPairCap];
    __shared__ unsigned char cntq[kPairCap];  // list lengths, segment order
    __shared__ unsigned char lcnt[kPairCap];  // list lengths, final order
    constexpr int kGroups = 128;  // list-row groups 0 .. maxnb / kListU (maxnb <= 248)
    __shared__ int gcnt[3][kGroups];
    const int ng = maxnb / kListU + 1;
    const int sx = (c1 - c0) + 2 * rings, sy = nr + 2 * rings, cl0 = c0 - rings, rl0 = r0 - rings;
    auto wrap = [&](int x) { return x < 0 ? x + nc : (x >= nc ? x - nc : x); };
    for (int e = threadIdx.x; e < 3 * kGroups; e += BS) gcnt[e / kGroups][e % kGroups] = 0;
    for (int g = threadIdx.x; g < ns; g += BS) {
        const int q0 = so[g], a0 = sa[g];
        const int m = min(sn[g], kPairCap - q0);
        // the segment's row, local (the same for all its particles)
        int row;
        if (g < nr) {
            row = r0 + g;
        } else {
            int k = 1;
            while (g >= first(k + 1)) ++k;
            const int e = g - first(k);
            row = e < 4 ? ((e >> 1) ? r1 + k - 1 : r0 - k) : r0 - k + 1 + ((e - 4) >> 1);
        }
        const int ly = wrap(wrap(row) - rl0);
        for (int i = 0; i < m; ++i) {
            lq0[q0 + i] = a0 + i;
            ckey[q0 + i] = (unsigned short)ly;
        }
    }
    __syncthreads();
    const int listed = n[rings - 1];
    auto ring_of = [&](int q) {
        int r = 0;
        while (q >= n[r]) ++r;
        return r;
    };
    // local cells of all staged particles; list lengths, group counts per ring,
    // and per 64-particle chunk one ballot of each bit of the group number
    // (every wave's lanes cover one chunk at a time)
    static_assert(kGroups == 128, "group numbers have 7 bits");
    const int nbits = ng > 1 ? 32 - __clz(ng - 1) : 0;
    __shared__ unsigned long long gbit[kPairCap / 64][7];
    constexpr unsigned short kOutside = 0xffff;
    for (int base = threadIdx.x & ~63; base < tot; base += BS) {
        const int q = base + (threadIdx.x & 63);
        int g = 0;
        if (q < tot) {
            const int slot = lq0[q];
            const int lx = wrap(ncol[slot] - cl0), ly = ckey[q];
            ckey[q] = lx < sx && ly < sy ? (unsigned short)(ly * kMapSide + lx) : kOutside;
            if (q < listed) {
                const int nn = nbc[slot];
                g = (nn + kListU - 1) / kListU;
                cntq[q] = (unsigned char)nn;
                gq[q] = (unsigned char)g;
                atomicAdd(&gcnt[ring_of(q)][g], 1);
            }
        }
        if (base < listed) {
            for (int b = 0; b < nbits; ++b) {
                const unsigned long long m = __ballot((g >> b) & 1);
                if ((threadIdx.x & 63) == 0) gbit[base >> 6][b] = m;
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < tot; q += BS) {
        const unsigned short k = ckey[q];
        if (k == kOutside) atomicOr(err, ERR_NLIST);
        else if (q == 0 || ckey[q - 1] != k) mst[k] = (unsigned short)q;
    }
    if (threadIdx.x < rings) {  // first staged index of each (ring, group), most groups first
        const int r = threadIdx.x;
        int acc = r == 0 ? 0 : n[r - 1];
        for (int g = ng - 1; g >= 0; --g) {
            const int c = gcnt[r][g];
            gcnt[r][g] = acc;
            acc += c;
        }
    }
    __syncthreads();
    // A listed particle's place: its group's first index plus the number of
    // earlier particles of the same ring and group in segment order, counted
    // chunk by chunk from the group-bit ballots over the ring's range, so that
    // the staged order does not depend on the timing of atomics.
    int* list = plist + (long long)t * kPairCap;
    auto below = [](int e) { return e >= 64 ? ~0ull : (1ull << e) - 1ull; };
    for (int q = threadIdx.x; q < tot; q += BS) {
        int qn = q;
        if (q < listed) {
            const int r = ring_of(q), g = gq[q];
            const int lo = r == 0 ? 0 : n[r - 1], hi = n[r], c = q >> 6;
            int rank = gcnt[r][g];
            for (int cc = lo >> 6; cc <= c; ++cc) {
                const int a = min(max(lo - cc * 64, 0), 64);
                const int e = cc == c ? (q & 63) : min(max(hi - cc * 64, 0), 64);
                unsigned long long m = below(e) & ~below(a);
                for (int b = 0; b < nbits; ++b) m &= ((g >> b) & 1) ? gbit[cc][b] : ~gbit[cc][b];
                rank += __popcll(m);
            }
            qn = rank;
            qn_of[q] = (unsigned short)qn;
            lcnt[qn] = cntq[q];
            lcell[qn] = ckey[q];
        }
        const int slot = lq0[q];
        lq[qn] = slot;
        list[qn] = slot;
    }
    __syncthreads();
    // particles of every ring but the last: neighbour counts and lists as staged
    // indices.  The first kPairPre list rows of a particle are read together
    // (they always exist, see list_rows), further ones kListU at a time.
    unsigned short* tl = tlist + (long long)t * maxnb * kPairCap;
    for (int q = threadIdx.x; q < listed; q += blockDim.x) {
        const int s = lq[q];
        const int nn = lcnt[q];
        const int own_cell = lcell[q];
        int first_rows[kPairPre];
        list_rows(nbl, (unsigned int)s, (unsigned int)S, first_rows);
        tcnt[(long long)t * kPairCap + q] = (unsigned char)nn;
        const int ring = ring_of(q);
        const int lim = ring + 1 < rings ? n[ring + 1] : tot;
        const int lx = own_cell % kMapSide, ly = own_cell / kMapSide;
        auto map_entry = [&](int e, int j) {
            const unsigned int u = (unsigned int)(unsigned short)e;
            const int code = (int)(u >> 12), idx = (int)(u & 4095u);
            const int xx = lx + code % 3 - 1, yy = ly + code / 3 - 1;
            int loc = -1;
            if (own_cell != kOutside && code < 9 && xx >= 0 && xx < sx && yy >= 0 && yy < sy) {
                const int k = (int)mst[yy * kMapSide + xx] + idx;
                loc = k < listed ? (int)qn_of[k] : k;
            }
            if (loc < 0 || loc >= lim) {
                atomicOr(err, ERR_NLIST);
                loc = 0;
            }
            tl[(long long)j * kPairCap + q] = (unsigned short)loc;
        };
#pragma unroll
        for (int j = 0; j < kPairPre; ++j)
            if (j < nn) map_entry(first_rows[j], j);
        for (int j0 = kPairPre; j0 < nn; j0 += kListU) {
            int rows[kListU];
            list_rows(nbl, (unsigned int)s + (unsigned int)j0 * (unsigned int)S, (unsigned int)S, rows);
#pragma unroll
            for (int u = 0; u < kListU; ++u)
                if (j0 + u < nn) map_entry(rows[u], j0 + u);
        }
    }
}

// The finish as a kernel of its own (one block per replica and component).
__global__ __launch_bounds__(kFinishBS) void k_cg_finish(const int* __restrict__ hpart, const double* __restrict__ mpart,
                                                         int pstride, const RepDev* __restrict__ reps,
                                                         unsigned long long* counts, double* moments,
                                                         long long* event_k, int mode) {
    cg_finish_one(hpart, mpart, pstride, reps, counts, moments, event_k, mode, blockIdx.x);
}

// Observation at the current positions: forces, full-step velocities, state
// copied out in caller order, and per-tile partials of {KE, PE, Px, Py}.
template <int BS, bool F32, bool HALF>
__global__ __launch_bounds__(BS) void k_observe(StepArgs a) {
    __shared__ double red[BS / 64][4];
    const int tile = blockIdx.x;
    const int r = __builtin_amdgcn_readfirstlane(a.tile_rep[tile]);
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
                                            const int* __restrict__ cellof, int check, int* err,
                                            const double2* __restrict__ pref) {
    const int tile = blockIdx.x;
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(tile_rep[tile])];
    const int s = tile * BS + threadIdx.x;
    int c;
    if (s - R.slot0 < R.n) {
        const double2 p = pos[s];
        const int cx = cell_coord(p.x, R.inv_w, R.nc);
        const int cy = cell_coord(p.y, R.inv_w, R.nc);
        c = R.cell0 + cy * R.nc + cx;
        if (check && pref) {
            // neighbour lists hold every pair within rc + skin at the list build,
            // which covers all pairs within rc while no particle has moved more
            // than half the skin since then
            const double2 q = pref[s];
            const double ex = fabs(min_image(p.x - q.x, R.L, R.halfL));
            const double ey = fabs(min_image(p.y - q.y, R.L, R.halfL));
            if (!(ex * ex + ey * ey <= R.skin_half * R.skin_half)) atomicOr(err, ERR_SKIN);
        } else if (check) {
            // the cell-stencil kernels centre the stencil on the cell a particle
            // was sorted into, which finds every pair within rc as long as no
            // particle has left that cell's box by more than half the skin
            const int co = cellof[s] - R.cell0;
            const int ox = co % R.nc, oy = co / R.nc;
            const double ex = fabs(min_image(p.x - (ox + 0.5) * R.w, R.L, R.halfL)) - 0.5 * R.w;
            const double ey = fabs(min_image(p.y - (oy + 0.5) * R.w, R.L, R.halfL)) - 0.5 * R.w;
            if (ex > R.skin_half || ey > R.skin_half) atomicOr(err, ERR_SKIN);
        }
        if (check && (!isfinite(p.x) || !isfinite(p.y))) atomicOr(err, ERR_NONFINITE);
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

// Image counts given in caller order moved to the slots (pad slots keep theirs).
__global__ void k_put_img(const int2* __restrict__ img_in, const int* __restrict__ id, int S, int2* __restrict__ img) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S && id[s] >= 0) img[s] = img_in[id[s]];
}

// Exclusive scan of n ints (cnt) into out[0..n] (out[n] = total), in tiles of
// kScanTile elements (kScanBS threads x 4): per-tile totals, then each tile's
// offset and its elements (above kScanDirect tiles, a pass over the totals
// in between).
constexpr int kScanBS = 256;
constexpr int kScanTile = 4 * kScanBS;
constexpr int kScanDirect = 2048;  // up to this many tiles, two kernels (each tile sums the totals before it)

// Exclusive scan over the block of NT threads; lds holds 2 NT / 64 ints.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* lds, int& total) {
    static_assert(NT % 64 == 0 && NT <= 1024, "whole waves, at most 16");
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int w = lane < NW ? lds[lane] : 0;
        for (int o = 1; o < NW; o <<= 1) {
            int y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < NW) lds[NW + lane] = w;
    }
    __syncthreads();
    total = lds[2 * NW - 1];
    const int wave_off = wid > 0 ? lds[NW + wid - 1] : 0;
    const int res = wave_off + x - v;
    __syncthreads();
    return res;
}

// A thread's four elements from base: one 16-byte load when all lie below n
// (base is a multiple of 4 and the arrays are 16-byte aligned), else one by one.
__device__ __forceinline__ void load4(const int* __restrict__ in, long long base, long long n, int (&v)[4]) {
    if (base + 3 < n) {
        const int4 q = *reinterpret_cast<const int4*>(in + base);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
        for (int j = 0; j < 4; ++j) v[j] = base + j < n ? in[base + j] : 0;
    }
}

__global__ __launch_bounds__(kScanBS) void k_scan_reduce(const int* __restrict__ in, long long n,
                                                         int* __restrict__ bsum) {
    __shared__ int lds[2 * kScanBS / 64];
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * 4;
    int v[4];
    load4(in, base, n, v);
    int total;
    block_excl_scan<kScanBS>(v[0] + v[1] + v[2] + v[3], lds, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int* bsum, int nb) {
    __shared__ int lds[32];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int total;
        const int ex = block_excl_scan<1024>(v, lds, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
}

// With `sums`, boff holds the tile totals and each block adds up those of the
// tiles before it (short scans, see kScanDirect); else boff holds the tile
// offsets from k_scan_top.  The counts are cleared for the next rebuild.
__global__ __launch_bounds__(kScanBS) void k_scan_final(int* __restrict__ in, long long n,
                                                        const int* __restrict__ boff, int* __restrict__ out,
                                                        int sums) {
    __shared__ int lds[2 * kScanBS / 64];
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * 4;
    int v[4];
    load4(in, base, n, v);
    int tile_off;
    if (sums) {
        int part = 0;
        for (int b = threadIdx.x; b < (int)blockIdx.x; b += kScanBS) part += boff[b];
        block_excl_scan<kScanBS>(part, lds, tile_off);
    } else {
        tile_off = boff[blockIdx.x];
    }
    int total;
    int ex = block_excl_scan<kScanBS>(v[0] + v[1] + v[2] + v[3], lds, total) + tile_off;
    int o[4];
    for (int j = 0; j < 4; ++j) {
        o[j] = ex;
        ex += v[j];
    }
    if (base + 3 < n) {
        *reinterpret_cast<int4*>(in + base) = make_int4(0, 0, 0, 0);
        *reinterpret_cast<int4*>(out + base) = make_int4(o[0], o[1], o[2], o[3]);
    } else {
        for (int j = 0; j < 4; ++j)
            if (base + j < n) {
                in[base + j] = 0;
                out[base + j] = o[j];
            }
    }
    if (base <= n - 1 && n - 1 < base + 4) out[n] = ex;  // thread holding the last element
}

__global__ void k_scatter(const int* __restrict__ key, const int* __restrict__ rank, const int* __restrict__ cs,
                          const int* __restrict__ id, int* __restrict__ perm, int* __restrict__ permid, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) {
        const int d = cs[key[s]] + rank[s];
        perm[d] = s;
        permid[d] = id[s];
    }
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

// One thread per slot of the scattered order: the particle's final slot is
// its cell's first slot plus the number of particles of that cell with a
// smaller caller index (pad slots, id -1, keep their scattered order), so the
// order within a cell does not depend on the atomics of the binning; then its
// state moves there.
__global__ void k_place(const int* __restrict__ cs, const int* __restrict__ key, const int* __restrict__ perm,
                        const int* __restrict__ permid, int S, Bufs b, int* __restrict__ cellof) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= S) return;
    const int src = perm[d];
    const int myid = permid[d];
    const int c = key[src];
    int dst = d;
    if (myid >= 0) {
        const int lo = cs[c], hi = cs[c + 1];
        dst = lo;
        for (int e = lo; e < hi; ++e) dst += permid[e] < myid ? 1 : 0;
    }
    b.pos_n[dst] = b.pos_o[src];
    b.vel_n[dst] = b.vel_o[src];
    b.img_n[dst] = b.img_o[src];
    b.id_n[dst] = myid;
    b.snap_n[dst] = b.snap_o[src];
    if (cellof) cellof[dst] = c;  // the drift check of the cell-stencil kernels (lists keep positions instead)
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

// Largest squared speed, as the bits of a non-negative double (ordered as
// integers): a wave maximum, the block's in LDS, and one atomic per block
// only where it raises the value already there (one address takes every
// block's update, so most blocks skip it).
__global__ __launch_bounds__(256) void k_vmax(const double2* __restrict__ vel, const int* __restrict__ id, int S,
                                              unsigned long long* out) {
    __shared__ double wmax[4];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double v2 = 0.0;
    if (s < S && id[s] >= 0) {
        const double2 v = vel[s];
        v2 = v.x * v.x + v.y * v.y;
        if (!isfinite(v2)) v2 = 1e300;
    }
    for (int o = 32; o > 0; o >>= 1) v2 = fmax(v2, __shfl_xor(v2, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v2;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double b = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        const unsigned long long bits = (unsigned long long)__double_as_longlong(b);
        if (bits > __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(out, bits);
    }
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

// Cell-list intervals captured into one graph by lj_md_step when at least
// that many remain.
constexpr int kGraphUnits = 8;

struct GraphKey {
    int K, phase, ppar, opar, vpar, binned, units;
    bool operator<(const GraphKey& o) const {
        return std::tie(K, phase, ppar, opar, vpar, binned, units) <
               std::tie(o.K, o.phase, o.ppar, o.opar, o.vpar, o.binned, o.units);
    }
};

struct GraphVal {
    hipGraphExec_t exec;
    int ppar_after, opar_after, vpar_after;
    int events;
    bool binned_after;
};

template <typename T>
hipError_t dalloc(T** p, size_t n) {
    return hipMalloc((void**)p, sizeof(T) * (n > 0 ? n : 1));
}

}  // namespace

struct lj_md {
    std::vector<lj_params> params;  // as given at init (saved by lj_md_save)
    int R = 0;
    int S = 0;   // total slots
    int C = 0;   // total cells including one sentinel per replica
    int BS = 256;
    int ntile = 0;
    int TT = 0;  // cell tiles of the step kernel
    int variant = 3;  // step kernel: 1 gather, 2 LDS tile, 3 neighbour list
    int ubatch = 8;   // gather kernel: candidate loads in flight per batch
    int stage_max = 1 << 30;  // tile kernel staging limit (MDLG_TILE_STAGE_MAX lowers it, for tests)
    bool f32 = false;
    double dt = 0.0;
    std::vector<RepHost> reps;
    long long n_total = 0;
    RepDev* d_reps = nullptr;
    int* d_tile_rep = nullptr;
    int* d_ttile_rep = nullptr;
    int* d_tinfo = nullptr;
    short* nbl = nullptr;     // neighbour lists (step kernel 3)
    unsigned char* nbc = nullptr;
    unsigned short* ncol = nullptr;  // cell column of each slot (tile list builder)
    // two ordinary steps per launch (step kernel 3)
    bool two_step = false;
    bool three_step = false;          // also three ordinary steps per launch (implies two_step)
    int rings = 2;                    // cell rings staged per fused tile
    int npt = 0;                      // fused tiles
    int* d_ptrep = nullptr;           // [npt] replica
    int* plist = nullptr;             // [npt][kPairCap]
    int4* pcnt = nullptr;             // [npt]
    unsigned short* tlist = nullptr;  // [npt][maxnb][kPairCap]
    unsigned char* tcnt = nullptr;    // [npt][kPairCap]
    double2* pref = nullptr;  // positions at the list build
    int maxnb = 0;
    int* d_hpart = nullptr;
    int pstride = 0;  // tiles per component row of the partials (the most of any kind of tile)
    double2* pos[2] = {nullptr, nullptr};
    double2* vel[2] = {nullptr, nullptr};
    int2* img[2] = {nullptr, nullptr};
    int* id[2] = {nullptr, nullptr};
    double2* snap[2] = {nullptr, nullptr};
    int *key = nullptr, *rank = nullptr, *perm = nullptr, *permid = nullptr, *cellof = nullptr;
    int *cnt = nullptr, *cs = nullptr, *bsum = nullptr;
    int nscan = 0;
    int ppar = 0, opar = 0, vpar = 0;  // current buffer of pos / of img, id, snap / of vel
    bool vel_full = true;
    bool have_cellof = false;
    bool binned = false;  // key and cnt hold the current positions' binning (done by the last step launch)
    bool fin_pending = false;  // the last event's partials await their finish (see launch_fused)
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
    // graphs of lj_md_step_timed: rebuild | ordinary steps | rest of a unit
    struct TimedGraphs {
        std::array<hipGraphExec_t, 3> g;
        int M, tail_events;
        int ppar_after, opar_after, vpar_after;
        bool binned_after;
    };
    std::map<std::tuple<int, int, int, int, int, int>, TimedGraphs> tgraphs;
    bool use_graphs = true;
};

namespace {

void clear_graphs(lj_md* md) {
    for (auto& kv : md->graphs) (void)hipGraphExecDestroy(kv.second.exec);
    md->graphs.clear();
    for (auto& kv : md->tgraphs)
        for (auto x : kv.second.g)
            if (x) (void)hipGraphExecDestroy(x);
    md->tgraphs.clear();
}

#define EXT_LAUNCH(KERNEL, BSV, GRIDV) \
    hipExtLaunchKernelGGL(KERNEL, dim3(GRIDV), dim3(BSV), 0, st, ev0, ev1, 0, a)

template <int BS, bool F32, bool FIRST, bool CG>
void launch_step_bs(const lj_md* md, hipStream_t st, const StepArgs& a, hipEvent_t ev0, hipEvent_t ev1) {
    if (md->variant == 2) {
        EXT_LAUNCH((k_step_tile<BS, F32, FIRST, CG>), BS, md->TT);
    } else if (md->variant == 3) {
        EXT_LAUNCH((k_step_nlist<BS, F32, FIRST, CG>), BS, md->ntile);
    } else if (md->ubatch <= 4) {
        EXT_LAUNCH((k_step_gather<BS, F32, FIRST, CG, 4>), BS, md->ntile);
    } else if (md->ubatch <= 8) {
        EXT_LAUNCH((k_step_gather<BS, F32, FIRST, CG, 8>), BS, md->ntile);
    } else {
        EXT_LAUNCH((k_step_gather<BS, F32, FIRST, CG, 16>), BS, md->ntile);
    }
}

StepArgs make_args(lj_md* md) {
    StepArgs a{};
    a.pin = md->pos[md->ppar];
    a.pout = md->pos[md->ppar ^ 1];
    a.vel = md->vel[md->vpar];
    a.vout = md->vel[md->vpar ^ 1];
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
    a.hpart = md->d_hpart;
    a.pstride = md->pstride;
    a.ttile_rep = md->d_ttile_rep;
    a.tinfo = md->d_tinfo;
    a.nrep = md->R;
    a.nslots = md->S;
    a.stage_max = md->stage_max;
    a.nbl = md->nbl;
    a.nbc = md->nbc;
    a.plist = md->plist;
    a.pcnt = md->pcnt;
    a.tlist = md->tlist;
    a.tcnt = md->tcnt;
    a.maxnb = md->maxnb;
    a.rings = md->rings;
    a.ptile_rep = md->d_ptrep;
    a.cell_acc = md->cell_acc;
    a.event_k = md->d_event_k;
    a.id = md->id[md->opar];
    a.cnt = md->cnt;
    a.key = md->key;
    a.rank = md->rank;
    a.pref = md->pref;
    return a;
}

#define LAUNCH_BS(BSV, KERNEL, ...)                                                             \
    switch (BSV) {                                                                              \
        case 64: hipLaunchKernelGGL((KERNEL<64, __VA_ARGS__>), dim3(grid), dim3(64), 0, st, a); break;   \
        case 128: hipLaunchKernelGGL((KERNEL<128, __VA_ARGS__>), dim3(grid), dim3(128), 0, st, a); break; \
        case 256: hipLaunchKernelGGL((KERNEL<256, __VA_ARGS__>), dim3(grid), dim3(256), 0, st, a); break; \
        default: hipLaunchKernelGGL((KERNEL<512, __VA_ARGS__>), dim3(grid), dim3(512), 0, st, a); break;  \
    }

// Step kernel launch; with ev0/ev1 the events are stamped at the kernel's own
// start and end (hipExtLaunchKernelGGL), which times the kernel alone.

template <int BS, bool F32, bool FIRST, bool CG>
void launch_step_bs(const lj_md* md, hipStream_t st, const StepArgs& a, hipEvent_t ev0, hipEvent_t ev1);

template <bool F32, bool FIRST, bool CG>
void launch_step_kernel(const lj_md* md, hipStream_t st, const StepArgs& a, hipEvent_t ev0, hipEvent_t ev1) {
    switch (md->BS) {
        case 64: launch_step_bs<64, F32, FIRST, CG>(md, st, a, ev0, ev1); break;
        case 128: launch_step_bs<128, F32, FIRST, CG>(md, st, a, ev0, ev1); break;
        case 256: launch_step_bs<256, F32, FIRST, CG>(md, st, a, ev0, ev1); break;
        default: launch_step_bs<512, F32, FIRST, CG>(md, st, a, ev0, ev1); break;
    }
}

// The finish of an event whose partials are still pending, as a kernel of
// its own: before anything reads the accumulators or the event counter, and
// at the end of every run of launches (so that no pending finish outlives a
// captured graph or a call).
hipError_t flush_finish(lj_md* md, hipStream_t st) {
    if (!md->fin_pending) return hipSuccess;
    hipLaunchKernelGGL(k_cg_finish, dim3(md->R * (MDLG_NCOUNTS + MDLG_NMOMENTS)), dim3(kFinishBS), 0, st,
                       (const int*)md->d_hpart, (const double*)md->d_mpart, md->pstride, (const RepDev*)md->d_reps,
                       md->counts, md->moments, md->d_event_k, 2);
    md->fin_pending = false;
    return hipGetLastError();
}

hipError_t launch_step(lj_md* md, hipStream_t st, bool first, bool cg, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr) {
    hipError_t fe = flush_finish(md, st);
    if (fe != hipSuccess) return fe;
    StepArgs a = make_args(md);
    if (md->f32) {
        if (first) {
            if (cg) launch_step_kernel<true, true, true>(md, st, a, ev0, ev1);
            else launch_step_kernel<true, true, false>(md, st, a, ev0, ev1);
        } else {
            if (cg) launch_step_kernel<true, false, true>(md, st, a, ev0, ev1);
            else launch_step_kernel<true, false, false>(md, st, a, ev0, ev1);
        }
    } else {
        if (first) {
            if (cg) launch_step_kernel<false, true, true>(md, st, a, ev0, ev1);
            else launch_step_kernel<false, true, false>(md, st, a, ev0, ev1);
        } else {
            if (cg) launch_step_kernel<false, false, true>(md, st, a, ev0, ev1);
            else launch_step_kernel<false, false, false>(md, st, a, ev0, ev1);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (cg) {
        hipLaunchKernelGGL(k_cg_finish, dim3(md->R * (MDLG_NCOUNTS + MDLG_NMOMENTS)), dim3(256), 0, st,
                           (const int*)md->d_hpart, (const double*)md->d_mpart, md->pstride, (const RepDev*)md->d_reps,
                           md->counts, md->moments, md->d_event_k, md->variant == 2 ? 1 : 0);
        e = hipGetLastError();
    }
    md->ppar ^= 1;
    return e;
}

template <bool F32, int NS, bool FIRST, bool CG, bool BIN>
void launch_fused_t(hipStream_t st, int grid, const StepArgs& a) {
    hipLaunchKernelGGL((k_step_fused<kStep2BS, F32, NS, FIRST, CG, BIN>), dim3(grid), dim3(kStep2BS), 0, st, a);
}

template <bool F32, int NS, bool FIRST>
void launch_fused_cb(hipStream_t st, int grid, const StepArgs& a, bool cg, bool bin) {
    if (cg) {
        if (bin) launch_fused_t<F32, NS, FIRST, true, true>(st, grid, a);
        else launch_fused_t<F32, NS, FIRST, true, false>(st, grid, a);
    } else {
        if (bin) launch_fused_t<F32, NS, FIRST, false, true>(st, grid, a);
        else launch_fused_t<F32, NS, FIRST, false, false>(st, grid, a);
    }
}

template <bool F32>
void launch_fused_f(hipStream_t st, int grid, const StepArgs& a, int ns, bool first, bool cg, bool bin) {
    if (ns == 3) launch_fused_cb<F32, 3, false>(st, grid, a, cg, bin);
    else if (ns == 2) launch_fused_cb<F32, 2, false>(st, grid, a, cg, bin);
    else if (first) launch_fused_cb<F32, 1, true>(st, grid, a, cg, bin);
    else launch_fused_cb<F32, 1, false>(st, grid, a, cg, bin);
}

// `ns` ordinary steps (ns <= rings) in one launch on the fused tiles (see
// k_step_fused), the last one with the coarse-graining event and its
// reduction when `cg`, binning the particles for the next rebuild when `bin`.
hipError_t launch_fused(lj_md* md, hipStream_t st, int ns, bool first, bool cg, bool bin) {
    StepArgs a = make_args(md);
    // a pending finish goes with this launch unless it is an event itself
    // (whose partials would overwrite the pending ones) or has fewer blocks
    // than the finish
    const int fin_n = md->R * (MDLG_NCOUNTS + MDLG_NMOMENTS);
    hipError_t e = hipSuccess;
    if (md->fin_pending && (cg || fin_n > md->npt)) e = flush_finish(md, st);
    if (e != hipSuccess) return e;
    if (md->fin_pending) {
        a.fin_n = fin_n;
        a.moments = md->moments;
        a.event_kw = md->d_event_k;
    }
    if (md->f32) launch_fused_f<true>(st, md->npt, a, ns, first, cg, bin);
    else launch_fused_f<false>(st, md->npt, a, ns, first, cg, bin);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.fin_n) md->fin_pending = false;
    // this event's finish rides on the next launch, or flush_finish issues it
    if (cg) md->fin_pending = true;
    md->ppar ^= 1;
    md->vpar ^= 1;
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
    const int o = md->opar;
    const int grid = md->ntile;
    const int check = md->have_cellof ? 1 : 0;
    // the binning of the counting sort, unless the last step launch did it
    if (!md->binned) {
        switch (md->BS) {
            case 64: hipLaunchKernelGGL(k_bin<64>, dim3(grid), dim3(64), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err, (const double2*)(md->variant == 3 ? md->pref : nullptr)); break;
            case 128: hipLaunchKernelGGL(k_bin<128>, dim3(grid), dim3(128), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err, (const double2*)(md->variant == 3 ? md->pref : nullptr)); break;
            case 256: hipLaunchKernelGGL(k_bin<256>, dim3(grid), dim3(256), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err, (const double2*)(md->variant == 3 ? md->pref : nullptr)); break;
            default: hipLaunchKernelGGL(k_bin<512>, dim3(grid), dim3(512), 0, st, (const double2*)md->pos[md->ppar], (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->cnt, md->key, md->rank, (const int*)md->cellof, check, md->d_err, (const double2*)(md->variant == 3 ? md->pref : nullptr)); break;
        }
    }
    const int nb = (C + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBS), 0, st, (const int*)md->cnt, (long long)C, md->bsum);
    const int direct = nb <= kScanDirect ? 1 : 0;
    if (!direct) hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, md->bsum, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanBS), 0, st, md->cnt, (long long)C, (const int*)md->bsum,
                       md->cs, direct);
    if (md->variant == 2)
        hipLaunchKernelGGL(k_tile_info, dim3((md->TT + 255) / 256), dim3(256), 0, st, (const int*)md->cs,
                           (const RepDev*)md->d_reps, (const int*)md->d_ttile_rep, md->TT, md->d_tinfo);
    hipLaunchKernelGGL(k_scatter, dim3((S + 255) / 256), dim3(256), 0, st, (const int*)md->key,
                       (const int*)md->rank, (const int*)md->cs, (const int*)md->id[o], md->perm, md->permid, S);
    Bufs b;
    b.pos_o = md->pos[md->ppar];
    b.pos_n = md->pos[md->ppar ^ 1];
    b.vel_o = md->vel[md->vpar];
    b.vel_n = md->vel[md->vpar ^ 1];
    b.img_o = md->img[o];
    b.img_n = md->img[o ^ 1];
    b.id_o = md->id[o];
    b.id_n = md->id[o ^ 1];
    b.snap_o = md->snap[o];
    b.snap_n = md->snap[o ^ 1];
    hipLaunchKernelGGL(k_place, dim3((S + 255) / 256), dim3(256), 0, st, (const int*)md->cs, (const int*)md->key,
                       (const int*)md->perm, (const int*)md->permid, S, b, md->variant == 3 ? nullptr : md->cellof);
    // the tile lists take entries by cell and index within the cell; the
    // one-step kernel takes slot offsets
    if (md->variant == 3 && md->two_step)
        hipLaunchKernelGGL(k_nlist_build<true>, dim3((S + 255) / 256), dim3(256), 0, st, (const double2*)b.pos_n,
                           (const int*)md->cs, (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->BS, S,
                           md->maxnb, md->nbl, md->nbc, md->ncol, md->pref, md->d_err);
    else if (md->variant == 3)
        hipLaunchKernelGGL(k_nlist_build<false>, dim3((S + 255) / 256), dim3(256), 0, st, (const double2*)b.pos_n,
                           (const int*)md->cs, (const RepDev*)md->d_reps, (const int*)md->d_tile_rep, md->BS, S,
                           md->maxnb, md->nbl, md->nbc, (unsigned short*)nullptr, md->pref, md->d_err);
    if (md->two_step)
        hipLaunchKernelGGL(k_pair_build<kPairBuildBS>, dim3(md->npt), dim3(kPairBuildBS), 0, st, (const int*)md->cs,
                           (const RepDev*)md->d_reps, (const int*)md->d_ptrep, (const short*)md->nbl,
                           (const unsigned char*)md->nbc, (const unsigned short*)md->ncol, S, md->maxnb, md->rings,
                           md->plist, md->pcnt, md->tlist, md->tcnt, md->d_err);
    md->ppar ^= 1;
    md->opar ^= 1;
    md->vpar ^= 1;
    md->have_cellof = true;
    md->binned = false;
    md->since_rebuild = 0;
    return hipGetLastError();
}

// One launch of a planned run: n steps, the last one ending a coarse step
// (cg), the first step after initialisation (first: its velocity is a
// full-step one).
struct LaunchPlan {
    int n;
    bool cg, first;
};

// The next launch for `avail` steps without a rebuild, from coarse step
// counter cg_t: a first step goes alone; otherwise the steps up to the next
// coarse-graining event (or all of them) are split into launches of up to mx
// steps with the event on the last step of the last one, which takes mx steps
// where the split allows it (m = mx k, or a shorter launch or two before it).
LaunchPlan plan_next(const lj_md* md, long long cg_t, bool vel_full, int avail) {
    const int mx = md->three_step ? 3 : (md->two_step ? 2 : 1);
    auto ev_at = [&](int k) { return md->cg_on && (cg_t + k) % md->s_cg == 0; };
    if (vel_full || mx == 1) return {1, ev_at(1), vel_full};
    int m = 1;
    while (m < avail && !ev_at(m)) ++m;
    int n;
    if (mx == 2) n = (m % 2 == 1) ? 1 : 2;
    else if (m % 3 == 0) n = 3;
    else if (m % 3 == 2) n = m >= 8 ? 3 : 2;
    else n = m == 1 ? 1 : (m >= 10 ? 3 : 2);
    return {n, ev_at(m) && n == m, false};
}

// The launches of `count` steps without a rebuild from the current state.
std::vector<LaunchPlan> plan_steps(const lj_md* md, int count) {
    std::vector<LaunchPlan> out;
    long long cg_t = md->cg_t;
    bool vel_full = md->vel_full;
    while (count > 0) {
        const LaunchPlan p = plan_next(md, cg_t, vel_full, count);
        out.push_back(p);
        if (md->cg_on) cg_t += p.n;
        vel_full = false;
        count -= p.n;
    }
    return out;
}

// Enqueue one planned launch and advance the host counters.
hipError_t issue(lj_md* md, hipStream_t st, const LaunchPlan& p) {
    // the launch that completes the cell-list interval bins for the rebuild
    const bool bin = md->two_step && md->since_rebuild + p.n == md->K;
    hipError_t e = md->two_step ? launch_fused(md, st, p.n, p.first, p.cg, bin) : launch_step(md, st, p.first, p.cg);
    if (e != hipSuccess) return e;
    md->binned = bin;
    md->vel_full = false;
    md->steps_done += p.n;
    md->since_rebuild += p.n;
    if (md->cg_on) {
        md->cg_t += p.n;
        if (p.cg) md->events += 1;
    }
    return hipSuccess;
}

// `count` MD steps from the current state: a rebuild whenever the cell lists
// are K steps old, planned launches in between.
hipError_t run_steps(lj_md* md, hipStream_t st, long long count) {
    hipError_t e = hipSuccess;
    while (count > 0 && e == hipSuccess) {
        if (md->since_rebuild >= md->K) {
            e = launch_rebuild(md, st);
            if (e != hipSuccess) break;
        }
        const int avail = (int)std::min<long long>(count, md->K - md->since_rebuild);
        const LaunchPlan p = plan_next(md, md->cg_t, md->vel_full, avail);
        e = issue(md, st, p);
        count -= p.n;
    }
    if (e == hipSuccess) e = flush_finish(md, st);
    return e;
}

// Steps until whole cell-list intervals (rebuild + K steps) hold their
// coarse-graining events at fixed offsets that end launches: with K a multiple
// of s_cg the coarse step counter is brought to a fixed residue modulo s_cg,
// with s_cg a multiple of K modulo K; otherwise events fall at varying offsets
// of the intervals and no alignment helps (0).  On fused tiles the residue is
// 2, so that an interval's last event ends the launch before its last one (a
// launch of two steps): the event and the binning for the rebuild (which the
// last launch does) then never share a launch, whose registers would not hold
// both.
int steps_to_alignment(const lj_md* md) {
    if (!md->cg_on) return 0;
    int period = 1;
    if (md->s_cg <= md->K) period = md->K % md->s_cg == 0 ? md->s_cg : 1;
    else period = md->s_cg % md->K == 0 ? md->K : 1;
    const long long residue = (md->two_step && period >= 3) ? 2 : 0;
    const long long r = ((md->cg_t - residue) % period + period) % period;
    return r == 0 ? 0 : (int)(period - r);
}

// What distinguishes the kernel sequence of a unit (rebuild + K steps) starting
// now: the offsets of its coarse-graining events.  With s_cg <= K they follow
// from cg_t mod s_cg; with s_cg > K a unit holds at most one event, after
// to_event steps (1 .. K), or none (0).  -1 without coarse-graining.
int unit_phase(const lj_md* md) {
    if (!md->cg_on) return -1;
    const long long r = md->cg_t % md->s_cg;
    if (md->s_cg <= md->K) return (int)r;
    const long long to_event = md->s_cg - r;
    return to_event <= md->K ? (int)to_event : 0;
}

// Whether several units may share a graph: the launches of later units follow
// from the first unit's exact coarse-step residue, and the residues repeat
// with a short period only when one of K and s_cg divides the other.
bool multi_unit_ok(const lj_md* md) {
    if (!md->cg_on) return true;
    return md->s_cg <= md->K ? md->K % md->s_cg == 0 : md->s_cg % md->K == 0;
}

// `units` x (rebuild + K steps), replayed from a captured graph.  One unit is
// keyed by unit_phase (units without an event share a graph); several units
// by the exact coarse-step residue, which fixes every later unit's events.
mdlg_status graph_unit(lj_md* md, hipStream_t st, int units = 1) {
    const int phase = units > 1 && md->cg_on ? (int)(md->cg_t % md->s_cg) : unit_phase(md);
    GraphKey key{md->K, phase, md->ppar, md->opar, md->vpar, md->binned ? 1 : 0, units};
    auto it = md->graphs.find(key);
    if (it == md->graphs.end()) {
        const long long steps0 = md->steps_done, cg_t0 = md->cg_t, ev0 = md->events;
        MDLG_HIP(hipStreamBeginCapture(md->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int u = 0; u < units && e == hipSuccess; ++u) {
            e = launch_rebuild(md, md->cap);
            if (e == hipSuccess) e = run_steps(md, md->cap, md->K);
        }
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(md->cap, &g);
        if (e != hipSuccess) return fail(MDLG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        MDLG_HIP(e2);
        hipGraphExec_t ex = nullptr;
        MDLG_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        GraphVal val{ex, md->ppar, md->opar, md->vpar, (int)(md->events - ev0), md->binned};
        md->graphs[key] = val;
        // the capture only recorded work: restore the counters, then replay
        md->ppar = key.ppar;
        md->opar = key.opar;
        md->vpar = key.vpar;
        md->binned = key.binned != 0;
        md->steps_done = steps0;
        md->cg_t = cg_t0;
        md->events = ev0;
        it = md->graphs.find(key);
    }
    MDLG_HIP(hipGraphLaunch(it->second.exec, st));
    md->ppar = it->second.ppar_after;
    md->opar = it->second.opar_after;
    md->vpar = it->second.vpar_after;
    md->binned = it->second.binned_after;
    md->steps_done += (long long)units * md->K;
    md->since_rebuild = md->K;
    md->have_cellof = true;
    if (md->cg_on) {
        md->cg_t += (long long)units * md->K;
        md->events += it->second.events;
    }
    return MDLG_OK;
}

// The length of the next run of steps launched directly (not from a graph):
// a first step alone, the steps up to the alignment of the intervals, or all
// that remain when fewer than a whole interval do.  0: a graph unit is next.
long long eager_len(const lj_md* md, long long nsteps) {
    if (md->vel_full) return 1;
    const int align = steps_to_alignment(md);
    if (align > 0) return std::min<long long>(align, nsteps);
    if (md->use_graphs && nsteps >= md->K) return 0;
    return nsteps;
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
    if (p.step_kernel < 0 || p.step_kernel > 3) return bad("step_kernel must be 0, 1, 2 or 3");
    if (p.gather_batch != 0 && p.gather_batch != 4 && p.gather_batch != 8 && p.gather_batch != 16)
        return bad("gather_batch must be 0, 4, 8 or 16");
    if (p.fuse_steps < 0 || p.fuse_steps > 3) return bad("fuse_steps must be 0, 1, 2 or 3");
    return MDLG_OK;
}

mdlg_status sync_check(lj_md* md, hipStream_t st) {
    MDLG_HIP(hipStreamSynchronize(st));
    int err = 0;
    MDLG_HIP(hipMemcpy(&err, md->d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) {
        md->broken = true;
        // capacity first: an overflow leaves forces incomplete, which can end in non-finite values
        if (err & ERR_TILE)
            return fail(MDLG_ECAPACITY, "a fused-step tile staged more than 768 particles (the particles clustered "
                                        "since the tiles were sized); use fuse_steps 1");
        if (err & ERR_NLIST) return fail(MDLG_ECAPACITY, "a neighbour list overflowed its capacity");
        if (err & ERR_NONFINITE) return fail(MDLG_ENONFINITE, "non-finite position or velocity on the device");
        return fail(MDLG_ESKIN, "a particle drifted beyond the cell-list skin between rebuilds; lower rebuild_every or raise skin");
    }
    return MDLG_OK;
}

// Rebuild interval with coarse-graining attached: a multiple of s_cg when K >= s_cg
// (every unit then holds the same events), else the largest divisor of s_cg in
// [K/2, K] (a unit then ends with an event or holds none), else K itself: a unit holds at
// most one event, at an offset that varies from unit to unit (see unit_phase).
int aligned_K(int K, int s_cg) {
    if (s_cg <= 0) return K;
    if (K >= s_cg) return s_cg * (K / s_cg);
    for (int d = K; d >= (K + 1) / 2; --d)
        if (s_cg % d == 0) return d;
    return K;
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
    md->variant = p[0].step_kernel ? p[0].step_kernel : 3;
    md->ubatch = p[0].gather_batch ? p[0].gather_batch : 8;
    if (const char* e = std::getenv("MDLG_TILE_STAGE_MAX")) md->stage_max = std::max(0, std::atoi(e));
    md->dt = p[0].dt;
    md->params.assign(p, p + n_rep);
    long long slots = 0, cells = 0, poff = 0, ttiles = 0;
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
        {
            // cell tiles: about 0.7 * block size particles per tile on average
            const double occ = (double)q.n / ((double)nc * nc);
            int twt = (int)std::floor(0.7 * md->BS / std::max(occ, 1e-9));
            twt = std::max(1, std::min(std::min(twt, 2 * md->BS), nc));
            d.tpr = (nc + twt - 1) / twt;
            d.tw = (nc + d.tpr - 1) / d.tpr;
            d.ttile0 = (int)ttiles;
            d.nttile = nc * d.tpr;
            ttiles += d.nttile;
        }
        d.lx = 0;
        d.npad = h.nslots - (int)q.n;
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
    if (ttiles >= (1LL << 31)) {
        delete md;
        return fail(MDLG_EINVAL, "lj_md_init: too many cell tiles");
    }
    md->TT = (int)ttiles;
    md->nscan = (md->C + kScanTile - 1) / kScanTile;
    // fused tiles: about kPairTarget3 staged particles on average with three
    // rings (kPairTarget with two), so that one block of kStep2BS threads
    // advances a tile in about one pass per step; k rings of distinct cells
    // need nc >= pT + 2 k.  fuse_steps 0: three steps per launch where such
    // tiles are at least kPairAutoT cells wide, else two where the two-ring
    // tiles are (the rings then add at most ~45% and ~20% to the first step);
    // 2: two steps wherever the geometry allows; 3: three wherever it allows,
    // else two.
    md->two_step = md->variant == 3 && p[0].fuse_steps != 1;
    {
        const int fs = p[0].fuse_steps;
        const int tmin = fs >= 2 ? 2 : kPairAutoT;
        auto tiles = [&](int rings, int target) {
            long long pt = 0;
            for (int r = 0; r < n_rep; ++r) {
                RepDev& d = md->reps[r].d;
                const double ppc = std::max((double)d.n / ((double)d.nc * d.nc), 1e-9);
                int T = (int)std::floor(std::sqrt((double)target / ppc)) - 2 * rings;
                T = std::min(std::min(T, 32), d.nc - 2 * rings);
                if (T < tmin || d.nc > 65535) return false;  // cell columns are 16-bit in the tile lists
                d.pT = T;
                d.pts = (d.nc + T - 1) / T;
                d.pnt = d.pts * d.pts;
                d.pt0 = (int)pt;
                pt += d.pnt;
            }
            if (pt >= (1LL << 31) / kPairCap) return false;
            md->npt = (int)pt;
            md->rings = rings;
            return true;
        };
        if (md->two_step) {
            if (fs != 2 && tiles(3, kPairTarget3)) md->three_step = true;
            else if (!tiles(2, kPairTarget)) md->two_step = false;
        }
        if (!md->two_step) md->npt = 0;
    }

    auto A = [&](hipError_t e) { return e == hipSuccess; };
    md->pstride = std::max(std::max(md->TT, md->ntile), md->npt);  // partials of every kind of tile
    const size_t part_tiles = (size_t)md->pstride;
    bool ok = A(dalloc(&md->d_reps, n_rep)) && A(dalloc(&md->d_tile_rep, md->ntile)) &&
              A(dalloc(&md->d_ttile_rep, md->TT)) && A(dalloc(&md->d_hpart, part_tiles * MDLG_NCOUNTS)) &&
              A(dalloc(&md->d_tinfo, (size_t)md->TT * kTileInfo));
    for (int b = 0; b < 2 && ok; ++b)
        ok = A(dalloc(&md->pos[b], md->S)) && A(dalloc(&md->vel[b], md->S)) && A(dalloc(&md->img[b], md->S)) &&
             A(dalloc(&md->id[b], md->S)) && A(dalloc(&md->snap[b], md->S));
    ok = ok && A(dalloc(&md->key, md->S)) && A(dalloc(&md->rank, md->S)) && A(dalloc(&md->perm, md->S)) && A(dalloc(&md->permid, md->S)) &&
         A(dalloc(&md->cellof, md->S)) && A(dalloc(&md->cnt, md->C)) && A(dalloc(&md->cs, (size_t)md->C + 1)) &&
         A(dalloc(&md->bsum, md->nscan)) && A(dalloc(&md->d_err, 1)) && A(dalloc(&md->d_epart, (size_t)md->ntile * 4)) &&
         A(dalloc(&md->d_eout, (size_t)n_rep * 4)) && A(dalloc(&md->d_vmax, 1)) &&
         A(dalloc(&md->d_mpart, part_tiles * MDLG_NMOMENTS)) && A(dalloc(&md->d_event_k, 1)) &&
         A(hipStreamCreateWithFlags(&md->cap, hipStreamNonBlocking));
    if (ok && md->variant == 3) {
        // list capacity: twice the mean neighbour count of the densest replica plus 16
        double mean_max = 0.0;
        for (int r = 0; r < n_rep; ++r) {
            const RepDev& d = md->reps[r].d;
            mean_max = std::max(mean_max, 3.14159265358979 * d.w * d.w * (double)d.n / (d.L * d.L));
        }
        md->maxnb = std::min(248, ((int)std::ceil(2.0 * mean_max + 16.0) + 7) / 8 * 8);
        static_assert(248 % kListU == 0 && 248 % kListUOne == 0 && kListPre <= 16, "list rows are read in whole passes");
        for (int r = 0; r < n_rep; ++r) {
            // list entries are 16-bit slot offsets: a neighbour lies within about
            // three cell rows of a particle in cell order
            const RepDev& d = md->reps[r].d;
            if (4.0 * d.n / d.nc >= 32767.0)
                return destroy_on_fail(md, fail(MDLG_EINVAL, "lj_md_init: replica " + std::to_string(r) +
                                                                 " has too many particles per cell row for 16-bit "
                                                                 "neighbour offsets; use step_kernel 1"));
        }
        if ((double)md->maxnb * md->S >= 1073741824.0)
            return destroy_on_fail(md, fail(MDLG_EINVAL, "lj_md_init: neighbour lists of this size exceed 2^30 "
                                                         "entries; use step_kernel 1"));
        ok = A(dalloc(&md->nbl, (size_t)md->maxnb * md->S)) && A(dalloc(&md->nbc, md->S)) && A(dalloc(&md->pref, md->S));
        if (ok && md->two_step)
            ok = A(dalloc(&md->d_ptrep, md->npt)) && A(dalloc(&md->plist, (size_t)md->npt * kPairCap)) &&
                 A(dalloc(&md->pcnt, md->npt)) && A(dalloc(&md->tlist, (size_t)md->npt * md->maxnb * kPairCap)) &&
                 A(dalloc(&md->tcnt, (size_t)md->npt * kPairCap)) && A(dalloc(&md->ncol, md->S));
    }
    if (!ok) return destroy_on_fail(md, fail(MDLG_ENOMEM, "lj_md_init: device allocation failed"));

    std::vector<RepDev> hd(n_rep);
    std::vector<int> trep(md->ntile), ttrep(md->TT), ptrep(md->npt);
    std::vector<long long> hpoff(n_rep);
    for (int r = 0; r < n_rep; ++r) {
        hd[r] = md->reps[r].d;
        hpoff[r] = md->reps[r].poff;
        for (int t = 0; t < hd[r].ntile; ++t) trep[hd[r].tile0 + t] = r;
        for (int t = 0; t < hd[r].nttile; ++t) ttrep[hd[r].ttile0 + t] = r;
        if (md->two_step)
            for (int t = 0; t < hd[r].pnt; ++t) ptrep[hd[r].pt0 + t] = r;
    }
    long long* d_poff = nullptr;
    if (hipMalloc((void**)&d_poff, sizeof(long long) * n_rep) != hipSuccess)
        return destroy_on_fail(md, fail(MDLG_ENOMEM, "lj_md_init: device allocation failed"));
    hipError_t e = hipMemcpy(md->d_reps, hd.data(), sizeof(RepDev) * n_rep, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(md->d_tile_rep, trep.data(), sizeof(int) * md->ntile, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_poff, hpoff.data(), sizeof(long long) * n_rep, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(md->d_ttile_rep, ttrep.data(), sizeof(int) * md->TT, hipMemcpyHostToDevice);
    if (e == hipSuccess && md->two_step)
        e = hipMemcpy(md->d_ptrep, ptrep.data(), sizeof(int) * md->npt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(md->d_err, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(md->cnt, 0, sizeof(int) * md->C, st);
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
        const long long n = eager_len(md, nsteps);
        if (n == 0) {
            // whole intervals, kGraphUnits to a graph where they fill one (each
            // graph boundary costs the device ~15 us)
            const int units = nsteps >= (long long)kGraphUnits * md->K && multi_unit_ok(md) ? kGraphUnits : 1;
            mdlg_status s = graph_unit(md, st, units);
            if (s != MDLG_OK) return s;
            nsteps -= (long long)units * md->K;
            continue;
        }
        hipError_t e = run_steps(md, st, n);
        if (e != hipSuccess) return fail(MDLG_EHIP, std::string("lj_md_step: ") + hipGetErrorString(e));
        nsteps -= n;
    }
    return MDLG_OK;
}

namespace {

// Capture `fn` (which enqueues work on the capture stream and updates the host
// state) into an executable graph.
template <typename F>
mdlg_status capture(lj_md* md, F fn, hipGraphExec_t* out) {
    MDLG_HIP(hipStreamBeginCapture(md->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = fn(md->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(md->cap, &g);
    if (e != hipSuccess) return fail(MDLG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    MDLG_HIP(e2);
    hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    MDLG_HIP(e3);
    return MDLG_OK;
}

}  // namespace

extern "C" mdlg_status lj_md_step_timed(lj_md* md, int64_t nunits, int32_t sample_every, double* ms_out,
                                        int32_t* n_out, void* stream) {
    if (!md || !ms_out) return fail(MDLG_EINVAL, "lj_md_step_timed: NULL argument");
    if (md->broken) return fail(MDLG_EINVAL, "lj_md_step_timed: handle is unusable after a device fault");
    if (nunits < 3 || nunits > 10000) return fail(MDLG_EINVAL, "lj_md_step_timed: nunits must be in [3, 1e4]");
    if (sample_every < 1 || sample_every > nunits / 3)
        return fail(MDLG_EINVAL, "lj_md_step_timed: sample_every must be in [1, nunits / 3]");
    if (!md->use_graphs && sample_every > 1)
        return fail(MDLG_EINVAL, "lj_md_step_timed: sample_every > 1 needs graph replay");
    hipStream_t st = (hipStream_t)stream;
    // direct launches up to the first interval aligned with the coarse steps
    while (md->vel_full || steps_to_alignment(md) > 0) {
        const long long n = md->vel_full ? 1 : steps_to_alignment(md);
        hipError_t e = run_steps(md, st, n);
        if (e != hipSuccess) return fail(MDLG_EHIP, std::string("lj_md_step_timed: ") + hipGetErrorString(e));
    }
    const int K = md->K;
    const int mx = md->three_step ? 3 : (md->two_step ? 2 : 1);
    struct UnitRec {
        std::array<int, 4> ev;
        int M, tail_events;
    };
    using Graphs = lj_md::TimedGraphs;
    auto& cache = md->tgraphs;
    int last_capture = -1;  // index of the last unit whose graphs were captured in this call
    std::vector<hipEvent_t> evs;
    std::vector<UnitRec> order;
    mdlg_status status = MDLG_OK;
    for (int64_t u = 0; u < nunits && status == MDLG_OK; ++u) {
        if (u % sample_every != 0) {
            // the units up to the next sampled one (or the end): one graph
            // (rebuilds + their K steps each), as lj_md_step runs them
            const int run = multi_unit_ok(md) ? (int)std::min<int64_t>(sample_every - u % sample_every, nunits - u) : 1;
            const size_t cached = md->graphs.size();
            status = graph_unit(md, st, run);
            if (md->graphs.size() != cached) last_capture = (int)order.size() - 1;
            u += run - 1;
            continue;
        }
        const int phase = unit_phase(md);
        const auto key = std::make_tuple(K, md->ppar, md->opar, md->vpar, phase, md->binned ? 1 : 0);
        auto it = cache.find(key);
        const long long steps0 = md->steps_done, cg_t0 = md->cg_t, ev0 = md->events;
        Graphs G{{nullptr, nullptr, nullptr}, 0, 0, 0, 0, 0, false};
        if (it == cache.end()) {
            // the unit's launches: the leading full-length ones without an
            // event, then the rest (shorter launches and the events)
            const std::vector<LaunchPlan> plan = plan_steps(md, K);
            size_t lead = 0;
            while (lead < plan.size() && plan[lead].n == mx && !plan[lead].cg) {
                G.M += plan[lead].n;
                ++lead;
            }
            status = capture(md, [&](hipStream_t cs) { return launch_rebuild(md, cs); }, &G.g[0]);
            if (status == MDLG_OK && lead > 0)
                status = capture(md, [&](hipStream_t cs) {
                    hipError_t e = hipSuccess;
                    for (size_t i = 0; i < lead && e == hipSuccess; ++i) e = issue(md, cs, plan[i]);
                    if (e == hipSuccess) e = flush_finish(md, cs);
                    return e;
                }, &G.g[1]);
            if (status == MDLG_OK && lead < plan.size())
                status = capture(md, [&](hipStream_t cs) {
                    hipError_t e = hipSuccess;
                    for (size_t i = lead; i < plan.size() && e == hipSuccess; ++i) e = issue(md, cs, plan[i]);
                    if (e == hipSuccess) e = flush_finish(md, cs);
                    return e;
                }, &G.g[2]);
            G.tail_events = (int)(md->events - ev0);
            G.ppar_after = md->ppar;
            G.opar_after = md->opar;
            G.vpar_after = md->vpar;
            G.binned_after = md->binned;
            if (status != MDLG_OK) {
                for (auto x : G.g)
                    if (x) (void)hipGraphExecDestroy(x);
                break;
            }
            cache[key] = G;
            last_capture = (int)order.size();  // this unit's record
            // captures only recorded work: restore the step counters
            md->ppar = std::get<1>(key);
            md->opar = std::get<2>(key);
            md->vpar = std::get<3>(key);
            md->binned = std::get<5>(key) != 0;
            md->steps_done = steps0;
            md->cg_t = cg_t0;
            md->events = ev0;
        } else {
            G = it->second;
        }
        UnitRec rec{{}, G.M, G.tail_events};
        for (int q = 0; q < 4; ++q) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) {
                status = fail(MDLG_EHIP, "lj_md_step_timed: event creation failed");
                break;
            }
            rec.ev[q] = (int)evs.size();
            evs.push_back(e);
        }
        if (status != MDLG_OK) break;
        hipError_t e = hipEventRecord(evs[rec.ev[0]], st);
        for (int q = 0; q < 3 && e == hipSuccess; ++q) {
            if (G.g[q]) e = hipGraphLaunch(G.g[q], st);
            if (e == hipSuccess) e = hipEventRecord(evs[rec.ev[q + 1]], st);
        }
        if (e != hipSuccess) {
            status = fail(MDLG_EHIP, std::string("lj_md_step_timed: ") + hipGetErrorString(e));
            break;
        }
        order.push_back(rec);
        // host state after the unit: the capture's effect, replayed
        md->ppar = G.ppar_after;
        md->opar = G.opar_after;
        md->vpar = G.vpar_after;
        md->binned = G.binned_after;
        md->steps_done += K;
        md->since_rebuild = K;
        md->have_cellof = true;
        if (md->cg_on) {
            md->cg_t += K;
            md->events += G.tail_events;
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (status == MDLG_OK && e != hipSuccess) status = fail(MDLG_EHIP, std::string("lj_md_step_timed: ") + hipGetErrorString(e));
    if (status == MDLG_OK) {
        // units up to the last capture of this call ran while the host captured
        // graphs (the GPU idled meanwhile): they warm up and are not counted.
        double sum_lead = 0.0, sum_rest = 0.0, sum_rebuild = 0.0;
        long long n_lead = 0, n_events = 0, n_rebuild = 0;
        size_t first = last_capture >= 0 ? (size_t)last_capture + 1 : 0;
        if (first >= order.size()) first = order.size() - 1;
        for (size_t ui = first; ui < order.size(); ++ui) {
            const UnitRec& rec = order[ui];
            float t[3] = {0, 0, 0};
            for (int q = 0; q < 3; ++q) (void)hipEventElapsedTime(&t[q], evs[rec.ev[q]], evs[rec.ev[q + 1]]);
            sum_rebuild += t[0];
            n_rebuild += 1;
            sum_lead += t[1];
            n_lead += rec.M;
            if (rec.tail_events > 0) {
                sum_rest += t[2];
                n_events += rec.tail_events;
            }
        }
        ms_out[0] = n_lead ? sum_lead / (double)n_lead : 0.0;
        ms_out[1] = n_events ? sum_rest / (double)n_events : 0.0;
        ms_out[2] = n_rebuild ? sum_rebuild / (double)n_rebuild : 0.0;
        if (n_out) {
            n_out[0] = (int32_t)n_lead;
            n_out[1] = (int32_t)n_events;
            n_out[2] = (int32_t)n_rebuild;
        }
    }
    for (auto x : evs) (void)hipEventDestroy(x);
    return status;
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

namespace {

// File layout of lj_md_save (little-endian, as the host stores it)
struct SaveHeader {
    char magic[8];            // "MDLGLJMD"
    uint32_t version;         // 1
    uint32_t params_bytes;    // sizeof(lj_params)
    int32_t n_rep;
    int32_t reserved;
    int64_t n_total;
    int64_t steps_done;
};
constexpr char kSaveMagic[8] = {'M', 'D', 'L', 'G', 'L', 'J', 'M', 'D'};

struct FileCloser {
    FILE* f;
    ~FileCloser() {
        if (f) std::fclose(f);
    }
};

}  // namespace

extern "C" mdlg_status lj_md_save(lj_md* md, const char* path, void* stream) {
    if (!md || !path) return fail(MDLG_EINVAL, "lj_md_save: NULL argument");
    if (md->broken) return fail(MDLG_EINVAL, "lj_md_save: handle is unusable after a device fault");
    hipStream_t st = (hipStream_t)stream;
    const long long n = md->n_total;
    std::vector<double> pos(2 * (size_t)n), vel(2 * (size_t)n);
    std::vector<int32_t> img(2 * (size_t)n);
    if (n > 0) {
        unsigned char* dev = nullptr;
        const size_t bp = sizeof(double) * 2 * (size_t)n, bi = sizeof(int32_t) * 2 * (size_t)n;
        MDLG_HIP(hipMallocAsync((void**)&dev, 2 * bp + bi, st));
        hipError_t e = launch_observe(md, st, (double2*)dev, (double2*)(dev + bp), (int2*)(dev + 2 * bp), nullptr, false);
        if (e == hipSuccess) e = hipMemcpyAsync(pos.data(), dev, bp, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(vel.data(), dev + bp, bp, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(img.data(), dev + 2 * bp, bi, hipMemcpyDeviceToHost, st);
        const hipError_t e2 = hipFreeAsync(dev, st);
        const hipError_t e3 = hipStreamSynchronize(st);
        MDLG_HIP(e);
        MDLG_HIP(e2);
        MDLG_HIP(e3);
    }
    mdlg_status s = sync_check(md, st);  // never save a faulted state
    if (s != MDLG_OK) return s;
    FileCloser fc{std::fopen(path, "wb")};
    if (!fc.f) return fail(MDLG_EINVAL, std::string("lj_md_save: cannot open ") + path);
    SaveHeader h{};
    std::memcpy(h.magic, kSaveMagic, 8);
    h.version = 1;
    h.params_bytes = (uint32_t)sizeof(lj_params);
    h.n_rep = md->R;
    h.n_total = n;
    h.steps_done = md->steps_done;
    bool ok = std::fwrite(&h, sizeof(h), 1, fc.f) == 1 &&
              std::fwrite(md->params.data(), sizeof(lj_params), md->params.size(), fc.f) == md->params.size();
    if (ok && n > 0)
        ok = std::fwrite(pos.data(), sizeof(double), pos.size(), fc.f) == pos.size() &&
             std::fwrite(vel.data(), sizeof(double), vel.size(), fc.f) == vel.size() &&
             std::fwrite(img.data(), sizeof(int32_t), img.size(), fc.f) == img.size();
    if (ok) ok = std::fflush(fc.f) == 0;
    if (!ok) return fail(MDLG_EINVAL, std::string("lj_md_save: write failed for ") + path);
    return MDLG_OK;
}

extern "C" mdlg_status lj_md_load(lj_md** out, const char* path, void* stream) {
    if (!out || !path) return fail(MDLG_EINVAL, "lj_md_load: NULL argument");
    *out = nullptr;
    FileCloser fc{std::fopen(path, "rb")};
    if (!fc.f) return fail(MDLG_EINVAL, std::string("lj_md_load: cannot open ") + path);
    SaveHeader h{};
    if (std::fread(&h, sizeof(h), 1, fc.f) != 1 || std::memcmp(h.magic, kSaveMagic, 8) != 0 || h.version != 1 ||
        h.params_bytes != sizeof(lj_params) || h.n_rep < 1 || h.n_rep > (1 << 20) || h.n_total < 1)
        return fail(MDLG_EINVAL, std::string("lj_md_load: not a state file of this library: ") + path);
    std::vector<lj_params> params((size_t)h.n_rep);
    if (std::fread(params.data(), sizeof(lj_params), params.size(), fc.f) != params.size())
        return fail(MDLG_EINVAL, "lj_md_load: truncated file");
    long long sum = 0;
    for (const auto& q : params) sum += q.n;
    if (sum != h.n_total) return fail(MDLG_EINVAL, "lj_md_load: particle counts disagree");
    const size_t n = (size_t)h.n_total;
    std::vector<double> pos(2 * n), vel(2 * n);
    std::vector<int32_t> img(2 * n);
    if (std::fread(pos.data(), sizeof(double), pos.size(), fc.f) != pos.size() ||
        std::fread(vel.data(), sizeof(double), vel.size(), fc.f) != vel.size() ||
        std::fread(img.data(), sizeof(int32_t), img.size(), fc.f) != img.size())
        return fail(MDLG_EINVAL, "lj_md_load: truncated file");
    hipStream_t st = (hipStream_t)stream;
    const size_t bp = sizeof(double) * 2 * n, bi = sizeof(int32_t) * 2 * n;
    unsigned char* dev = nullptr;
    MDLG_HIP(hipMalloc((void**)&dev, 2 * bp + bi));
    hipError_t e = hipMemcpy(dev, pos.data(), bp, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dev + bp, vel.data(), bp, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dev + 2 * bp, img.data(), bi, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return fail(MDLG_EHIP, std::string("lj_md_load: ") + hipGetErrorString(e));
    }
    lj_md* md = nullptr;
    mdlg_status s = lj_md_init_batch(&md, h.n_rep, params.data(), (const double*)dev, (const double*)(dev + bp), stream);
    if (s == MDLG_OK) {
        hipLaunchKernelGGL(k_put_img, dim3((md->S + 255) / 256), dim3(256), 0, st, (const int2*)(dev + 2 * bp),
                           (const int*)md->id[md->opar], md->S, md->img[md->opar]);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) s = fail(MDLG_EHIP, std::string("lj_md_load: ") + hipGetErrorString(e));
    }
    (void)hipFree(dev);
    if (s != MDLG_OK) {
        lj_md_destroy(md);
        return s;
    }
    md->steps_done = h.steps_done;
    *out = md;
    return MDLG_OK;
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
    info->steps_per_launch = md->three_step ? 3 : (md->two_step ? 2 : 1);
    info->reserved = 0;
    return MDLG_OK;
}

extern "C" void lj_md_destroy(lj_md* md) {
    if (!md) return;
    clear_graphs(md);
    if (md->cap) (void)hipStreamDestroy(md->cap);
    void* ptrs[] = {md->d_reps, md->d_tile_rep, md->d_ttile_rep, md->d_tinfo, md->nbl, md->nbc, md->ncol, md->pref, md->d_hpart, md->pos[0], md->pos[1], md->vel[0], md->vel[1], md->img[0],
                    md->img[1], md->id[0], md->id[1], md->snap[0], md->snap[1], md->key, md->rank, md->perm, md->permid,
                    md->cellof, md->cnt, md->cs, md->bsum, md->d_err, md->d_epart, md->d_eout, md->d_vmax,
                    md->d_mpart, md->d_event_k, md->d_ptrep, md->plist, md->pcnt, md->tlist, md->tcnt};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete md;
}
