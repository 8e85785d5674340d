/*
 * CPU oracle: 2D Lennard-Jones velocity-Verlet molecular dynamics and the
 * MDLG coarse-graining (occupation numbers n_i(x,t)).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source with
 * the GPU library and must never be called by the product path.
 *
 * Plain, single-threaded FP64, written for reading rather than speed.  Build
 * with -O2 -ffp-contract=off -fno-fast-math so that every product and sum is
 * rounded exactly once, in the order written.
 *
 * What it follows:
 *  - Pair potential: the 6-12 Lennard-Jones potential of the "Simulations
 *    setup" section, V(r) = 4 eps [(1/r)^12 - (1/r)^6] with sigma = m = 1.
 *    The paper states no cutoff; this oracle truncates at rc (2.5) and
 *    optionally shifts the energy by -V(rc) (force unshifted).
 *  - Integrator: velocity Verlet, NVE (same section), periodic square box.
 *  - Coarse-graining: the occupation number definition Eq.(n_i) of the
 *    "Molecular dynamics lattice gas method" section: particle j adds one to
 *    n_i(x, t) when it sits in lattice cell x at time t and sat in cell x - v_i
 *    at time t - dt_cg.
 *  - Non-equilibrium MDLG: the lattice gas evolution Eq.(mdlg_evolution)
 *    defines the collision operator Xi_i = n_i(x + v_i, t + dt) - n_i(x, t);
 *    the MDLB quantities f_i = <n_i> and Omega_i = <Xi_i> are averages over
 *    an ensemble of trajectories ("Molecular dynamics lattice gas method").
 *  - Displacement histogram: the binned one-particle displacement PDF
 *    P^MD(X_i) that the displacement-PDF figure (Fig. 2) sets beside the
 *    single-Gaussian Eq.(gaussian_df) and the Poisson WSG Eq.(poisson_v2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 49 /* D2Q49: |v_x|, |v_y| <= 3 */

/* ---------------------------------------------------------------- sums --- */

/* Neumaier-compensated running sum, so that the oracle's reductions carry
 * less rounding error than any GPU tree reduction compared against them. */
typedef struct {
    double s, c;
} nsum;

static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum* a) { return a->s + a->c; }

/* -------------------------------------------------------------- forces --- */

/* Minimum-image separation along one axis of a periodic box of side L. */
static double min_image(double d, double L) { return d - L * rint(d / L); }

/* Lennard-Jones pair at squared distance r2 (< rc^2):
 *   fr = |F| / r = 24 eps (2 r^-12 - r^-6) / r^2, so that F_j = fr * (r_j - r_k)
 *   e  = 4 eps (r^-12 - r^-6)                     (unshifted energy)       */
static void lj_pair(double r2, double eps, double* fr, double* e) {
    double ir2 = 1.0 / r2;
    double ir6 = ir2 * ir2 * ir2;
    *fr = 24.0 * eps * ir6 * (2.0 * ir6 - 1.0) * ir2;
    *e = 4.0 * eps * ir6 * (ir6 - 1.0);
}

static double lj_energy_at(double r, double eps) {
    double ir6 = 1.0 / (r * r * r * r * r * r);
    return 4.0 * eps * ir6 * (ir6 - 1.0);
}

/* All-pairs O(N^2) forces.  Each ordered pair (j, k != j) adds to j only, and
 * half its (shifted) pair energy to the total. */
void orc_forces_brute(int64_t n, double L, double rc, double eps, int32_t shift,
                      const double* pos, double* f, double* pe_out) {
    double rc2 = rc * rc;
    double vshift = shift ? lj_energy_at(rc, eps) : 0.0;
    nsum pe = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        double fx = 0.0, fy = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            if (k == j) continue;
            double dx = min_image(pos[2 * j] - pos[2 * k], L);
            double dy = min_image(pos[2 * j + 1] - pos[2 * k + 1], L);
            double r2 = dx * dx + dy * dy;
            if (r2 < rc2) {
                double fr, e;
                lj_pair(r2, eps, &fr, &e);
                fx += fr * dx;
                fy += fr * dy;
                nsum_add(&pe, 0.5 * (e - vshift));
            }
        }
        f[2 * j] = fx;
        f[2 * j + 1] = fy;
    }
    if (pe_out) *pe_out = nsum_get(&pe);
}

/* Linked-cell forces: cells of side w = L / nc >= rc, each particle visits the
 * 3 x 3 block of cells around its own (periodic).  Falls back to the all-pairs
 * loop when fewer than 3 cells fit per side. */
void orc_forces_cells(int64_t n, double L, double rc, double eps, int32_t shift,
                      const double* pos, double* f, double* pe_out) {
    int64_t nc = (int64_t)floor(L / rc);
    if (nc < 3) {
        orc_forces_brute(n, L, rc, eps, shift, pos, f, pe_out);
        return;
    }
    double rc2 = rc * rc;
    double vshift = shift ? lj_energy_at(rc, eps) : 0.0;
    double w = L / (double)nc;
    int64_t* head = (int64_t*)malloc(sizeof(int64_t) * nc * nc);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t* cx = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t* cy = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t c = 0; c < nc * nc; ++c) head[c] = -1;
    for (int64_t j = 0; j < n; ++j) {
        int64_t a = (int64_t)floor(pos[2 * j] / w);
        int64_t b = (int64_t)floor(pos[2 * j + 1] / w);
        if (a >= nc) a = nc - 1;
        if (b >= nc) b = nc - 1;
        if (a < 0) a = 0;
        if (b < 0) b = 0;
        cx[j] = a;
        cy[j] = b;
        next[j] = head[b * nc + a];
        head[b * nc + a] = j;
    }
    nsum pe = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        double fx = 0.0, fy = 0.0;
        for (int64_t oy = -1; oy <= 1; ++oy) {
            for (int64_t ox = -1; ox <= 1; ++ox) {
                int64_t a = (cx[j] + ox + nc) % nc;
                int64_t b = (cy[j] + oy + nc) % nc;
                for (int64_t k = head[b * nc + a]; k >= 0; k = next[k]) {
                    if (k == j) continue;
                    double dx = min_image(pos[2 * j] - pos[2 * k], L);
                    double dy = min_image(pos[2 * j + 1] - pos[2 * k + 1], L);
                    double r2 = dx * dx + dy * dy;
                    if (r2 < rc2) {
                        double fr, e;
                        lj_pair(r2, eps, &fr, &e);
                        fx += fr * dx;
                        fy += fr * dy;
                        nsum_add(&pe, 0.5 * (e - vshift));
                    }
                }
            }
        }
        f[2 * j] = fx;
        f[2 * j + 1] = fy;
    }
    if (pe_out) *pe_out = nsum_get(&pe);
    free(head);
    free(next);
    free(cx);
    free(cy);
}

static void forces(int32_t use_cells, int64_t n, double L, double rc, double eps, int32_t shift,
                   const double* pos, double* f, double* pe) {
    if (use_cells)
        orc_forces_cells(n, L, rc, eps, shift, pos, f, pe);
    else
        orc_forces_brute(n, L, rc, eps, shift, pos, f, pe);
}

/* Kinetic energy, potential energy and total momentum: out = {KE, PE, Px, Py}. */
void orc_energy(int64_t n, double L, double rc, double eps, int32_t shift, int32_t use_cells,
                const double* pos, const double* vel, double* out) {
    double* f = (double*)malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double pe = 0.0;
    forces(use_cells, n, L, rc, eps, shift, pos, f, &pe);
    nsum ke = {0, 0}, px = {0, 0}, py = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        nsum_add(&ke, 0.5 * (vel[2 * j] * vel[2 * j] + vel[2 * j + 1] * vel[2 * j + 1]));
        nsum_add(&px, vel[2 * j]);
        nsum_add(&py, vel[2 * j + 1]);
    }
    out[0] = nsum_get(&ke);
    out[1] = pe;
    out[2] = nsum_get(&px);
    out[3] = nsum_get(&py);
    free(f);
}

/* ----------------------------------------------------- coarse-graining --- */

typedef struct {
    int32_t lx;          /* lattice cells per side                                */
    int32_t s_cg;        /* MD steps per coarse time step (0: no coarse-graining) */
    double ux, uy;       /* frame drift in lattice cells per coarse step          */
    int64_t k0;          /* coarse-step index of the starting snapshot            */
    const int32_t* vtab; /* [49][2] lattice velocities, the oracle's numbering    */
    int64_t* counts;     /* [50] += : n_i summed over cells, index 49 = overflow  */
    int32_t* cell_acc;   /* [49][lx][lx] += or NULL                               */
    double* moments;     /* [5] += : samples, sum d^2, sum d^4 (pooled over axes), sum dx, sum dy,
                          * d = displacement over the coarse step in the box frame */
} orc_cg;

static int32_t find_velocity(const int32_t* vtab, int64_t vx, int64_t vy) {
    for (int32_t i = 0; i < NQ; ++i)
        if (vtab[2 * i] == vx && vtab[2 * i + 1] == vy) return i;
    return NQ; /* |v_x| or |v_y| > 3: overflow bin */
}

static int64_t pmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/* Lattice coordinate along one axis: q = floor((x + s) * (lx / L)), where s is
 * the frame shift of the coarse step.  The cell on the periodic lattice is q
 * mod lx; the unwrapped cell adds lx times the periodic image count. */
static int64_t lattice_q(double x, double s, double inv) { return (int64_t)floor((x + s) * inv); }

/* One coarse-graining event between two snapshots (binned form), on a lattice
 * translated by (sxp, syp) at the earlier snapshot and by (sxc, syc) at the
 * later one (lengths).  A lattice moving u cells per coarse step has shifts
 * u dx k; a common translation of both is another origin of the same lattice,
 * which leaves the statistics of a homogeneous gas unchanged.
 * pos_*: [n][2] wrapped positions; img_*: [n][2] image counts (NULL = zero).
 * n_event: dense n_i(x, t) [49][lx][lx], overwritten (NULL to skip). */
void orc_coarse_grain_shift(int32_t lx, double L, double sxp, double syp, double sxc, double syc,
                            const int32_t* vtab, int64_t n,
                            const double* pos_prev, const int64_t* img_prev,
                            const double* pos_cur, const int64_t* img_cur,
                            int64_t* counts, int32_t* n_event, int32_t* cell_acc, double* moments) {
    double inv = (double)lx / L;
    int64_t lx2 = (int64_t)lx * lx;
    if (n_event) memset(n_event, 0, sizeof(int32_t) * NQ * lx2);
    nsum m2 = {0, 0}, m4 = {0, 0}, mx = {0, 0}, my = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        int64_t ixp = img_prev ? img_prev[2 * j] : 0, iyp = img_prev ? img_prev[2 * j + 1] : 0;
        int64_t ixc = img_cur ? img_cur[2 * j] : 0, iyc = img_cur ? img_cur[2 * j + 1] : 0;
        int64_t qxp = lattice_q(pos_prev[2 * j], sxp, inv);
        int64_t qyp = lattice_q(pos_prev[2 * j + 1], syp, inv);
        int64_t qxc = lattice_q(pos_cur[2 * j], sxc, inv);
        int64_t qyc = lattice_q(pos_cur[2 * j + 1], syc, inv);
        int64_t vx = (qxc + lx * ixc) - (qxp + lx * ixp);
        int64_t vy = (qyc + lx * iyc) - (qyp + lx * iyp);
        int32_t i = find_velocity(vtab, vx, vy);
        counts[i] += 1;
        if (i < NQ) {
            int64_t cell = pmod(qyc, lx) * lx + pmod(qxc, lx);
            if (n_event) n_event[i * lx2 + cell] += 1;
            if (cell_acc) cell_acc[i * lx2 + cell] += 1;
        }
        if (moments) {
            /* displacement in the rest frame of the box: the frame drift is a
             * Galilean boost, so the moments about the drift are these */
            double dx = (pos_cur[2 * j] - pos_prev[2 * j]) + L * (double)(ixc - ixp);
            double dy = (pos_cur[2 * j + 1] - pos_prev[2 * j + 1]) + L * (double)(iyc - iyp);
            double dx2 = dx * dx, dy2 = dy * dy;
            nsum_add(&m2, dx2);
            nsum_add(&m2, dy2);
            nsum_add(&m4, dx2 * dx2);
            nsum_add(&m4, dy2 * dy2);
            nsum_add(&mx, dx);
            nsum_add(&my, dy);
        }
    }
    if (moments) {
        moments[0] += 2.0 * (double)n;
        moments[1] += nsum_get(&m2);
        moments[2] += nsum_get(&m4);
        moments[3] += nsum_get(&mx);
        moments[4] += nsum_get(&my);
    }
}

/* The event at coarse steps k_prev, k_cur of a lattice moving u cells per step. */
void orc_coarse_grain(int32_t lx, double L, double ux, double uy, const int32_t* vtab, int64_t n,
                      const double* pos_prev, const int64_t* img_prev, int64_t k_prev,
                      const double* pos_cur, const int64_t* img_cur, int64_t k_cur,
                      int64_t* counts, int32_t* n_event, int32_t* cell_acc, double* moments) {
    double dxl = L / (double)lx;
    double sxp = (ux * dxl) * (double)k_prev, syp = (uy * dxl) * (double)k_prev;
    double sxc = (ux * dxl) * (double)k_cur, syc = (uy * dxl) * (double)k_cur;
    orc_coarse_grain_shift(lx, L, sxp, syp, sxc, syc, vtab, n, pos_prev, img_prev, pos_cur, img_cur,
                           counts, n_event, cell_acc, moments);
}

/* The same event evaluated literally from Eq.(n_i): for every lattice cell x
 * and velocity v_i, count the particles j with x_j(t) in cell x and
 * x_j(t - dt_cg) in cell x - v_i, on the periodic lattice from wrapped
 * positions alone.  O(lx^2 * 49 * n): tiny inputs only.  Agrees with the
 * binned form whenever lx >= 7 and every true displacement is below lx/2. */
void orc_coarse_grain_literal(int32_t lx, double L, double ux, double uy, const int32_t* vtab,
                              int64_t n, const double* pos_prev, int64_t k_prev,
                              const double* pos_cur, int64_t k_cur, int64_t* counts,
                              int32_t* n_event) {
    double dxl = L / (double)lx;
    double inv = (double)lx / L;
    double sxp = (ux * dxl) * (double)k_prev, syp = (uy * dxl) * (double)k_prev;
    double sxc = (ux * dxl) * (double)k_cur, syc = (uy * dxl) * (double)k_cur;
    int64_t lx2 = (int64_t)lx * lx;
    int64_t total = 0;
    for (int64_t cy = 0; cy < lx; ++cy) {
        for (int64_t cx = 0; cx < lx; ++cx) {
            for (int32_t i = 0; i < NQ; ++i) {
                int64_t px = pmod(cx - vtab[2 * i], lx);
                int64_t py = pmod(cy - vtab[2 * i + 1], lx);
                int32_t cnt = 0;
                for (int64_t j = 0; j < n; ++j) {
                    int now = pmod(lattice_q(pos_cur[2 * j], sxc, inv), lx) == cx &&
                              pmod(lattice_q(pos_cur[2 * j + 1], syc, inv), lx) == cy;
                    int before = pmod(lattice_q(pos_prev[2 * j], sxp, inv), lx) == px &&
                                 pmod(lattice_q(pos_prev[2 * j + 1], syp, inv), lx) == py;
                    cnt += (now && before);
                }
                if (n_event) n_event[i * lx2 + cy * lx + cx] = cnt;
                counts[i] += cnt;
                total += cnt;
            }
        }
    }
    counts[NQ] += n - total;
}

/* --------------------------------------------- non-equilibrium MDLG --- */

/* Ensemble sums of the occupation numbers and of the lattice gas collision
 * operator over n_rep replica trajectories.  Replica r owns particles
 * offsets[r] .. offsets[r+1]-1 of the stacked snapshots pos [n_snap][n_tot][2]
 * and img [n_snap][n_tot][2]; every replica has box side L and an lx x lx
 * lattice at rest.  Event p (1 <= p < n_snap) is the coarse step from
 * snapshot p-1 to p.  Outputs (overwritten):
 *   f_sum [n_snap-1][49][lx][lx]: sum over r of n_i^r(x, t_p)
 *   ovf   [n_snap-1]:            particles of event p whose lattice
 *                                displacement is outside D2Q49
 *   xi_sum [n_snap-2][49][lx][lx] (NULL to skip): sum over r of
 *         Xi_i^r(x, t_p) = n_i^r(x + v_i, t_{p+1}) - n_i^r(x, t_p), x + v_i
 *         taken on the periodic lattice, for 1 <= p < n_snap - 1.
 * Each replica's n_i comes from the binned coarse-graining above and its
 * Xi_i from the definition, before anything is summed over replicas. */
int orc_neq_mdlg(int32_t lx, double L, const int32_t* vtab, int32_t n_rep, const int64_t* offsets,
                 int32_t n_snap, int64_t n_tot, const double* pos, const int64_t* img, int32_t* f_sum,
                 int64_t* ovf, int32_t* xi_sum) {
    int64_t lx2 = (int64_t)lx * lx;
    int64_t per = NQ * lx2;
    int32_t* prev = (int32_t*)calloc((size_t)per, sizeof(int32_t));
    int32_t* cur = (int32_t*)calloc((size_t)per, sizeof(int32_t));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return -1;
    }
    memset(f_sum, 0, sizeof(int32_t) * (size_t)(n_snap - 1) * (size_t)per);
    memset(ovf, 0, sizeof(int64_t) * (size_t)(n_snap - 1));
    if (xi_sum && n_snap > 2) memset(xi_sum, 0, sizeof(int32_t) * (size_t)(n_snap - 2) * (size_t)per);
    for (int32_t r = 0; r < n_rep; ++r) {
        int64_t a = offsets[r], n = offsets[r + 1] - offsets[r];
        if (n == 0) continue;
        for (int32_t p = 1; p < n_snap; ++p) {
            int64_t counts[NQ + 1];
            memset(counts, 0, sizeof(counts));
            const double* xp = pos + 2 * ((int64_t)(p - 1) * n_tot + a);
            const double* xc = pos + 2 * ((int64_t)p * n_tot + a);
            const int64_t* ip = img + 2 * ((int64_t)(p - 1) * n_tot + a);
            const int64_t* ic = img + 2 * ((int64_t)p * n_tot + a);
            orc_coarse_grain_shift(lx, L, 0.0, 0.0, 0.0, 0.0, vtab, n, xp, ip, xc, ic, counts, cur, NULL, NULL);
            ovf[p - 1] += counts[NQ];
            int32_t* f = f_sum + (int64_t)(p - 1) * per;
            for (int64_t k = 0; k < per; ++k) f[k] += cur[k];
            if (xi_sum && p >= 2) {
                /* event p-1 is t, event p is t + dt */
                int32_t* xi = xi_sum + (int64_t)(p - 2) * per;
                for (int32_t i = 0; i < NQ; ++i)
                    for (int64_t y = 0; y < lx; ++y)
                        for (int64_t x = 0; x < lx; ++x) {
                            int64_t xs = pmod(x + vtab[2 * i], lx), ys = pmod(y + vtab[2 * i + 1], lx);
                            xi[i * lx2 + y * lx + x] += cur[i * lx2 + ys * lx + xs] - prev[i * lx2 + y * lx + x];
                        }
            }
            int32_t* t = prev;
            prev = cur;
            cur = t;
        }
    }
    free(prev);
    free(cur);
    return 0;
}

/* ------------------------------------------------ displacement PDF --- */

/* Histogram of the box-frame displacements of one snapshot pair, per axis.
 * delta = (x_cur - x_prev) + L (img_cur - img_prev).  The n_bin intervals
 * X_k = [(k - n_bin/2) h, (k + 1 - n_bin/2) h), k = 0 .. n_bin - 1, tile
 * [-n_bin h / 2, n_bin h / 2); a displacement falls in X_k with
 * k = floor(delta * (1 / h) + n_bin / 2), evaluated in that order in FP64.
 * hist [2][n_bin + 2] (axis x, then y) is added to: index k for X_k, n_bin
 * below the range, n_bin + 1 at or above it (and for a non-number). */
void orc_displacement_hist(int64_t n, double L, double h, int32_t n_bin, const double* pos_prev,
                           const int64_t* img_prev, const double* pos_cur, const int64_t* img_cur,
                           int64_t* hist) {
    double inv_h = 1.0 / h;
    double half = 0.5 * (double)n_bin;
    for (int64_t j = 0; j < n; ++j) {
        for (int a = 0; a < 2; ++a) {
            int64_t ip = img_prev ? img_prev[2 * j + a] : 0;
            int64_t ic = img_cur ? img_cur[2 * j + a] : 0;
            double delta = (pos_cur[2 * j + a] - pos_prev[2 * j + a]) + L * (double)(ic - ip);
            double t = delta * inv_h + half;
            int64_t k;
            if (t >= 0.0 && t < (double)n_bin)
                k = (int64_t)floor(t);
            else if (t < 0.0)
                k = n_bin;
            else
                k = (int64_t)n_bin + 1;
            hist[(int64_t)a * (n_bin + 2) + k] += 1;
        }
    }
}

/* -------------------------------------------------------- integration --- */

/* Periodic wrap of one coordinate after a drift, with image bookkeeping.  A
 * negative coordinate whose sum with L rounds up to L is mapped to 0. */
static void wrap(double* x, int64_t* img, double L) {
    if (*x >= L) {
        *x -= L;
        *img += 1;
    } else if (*x < 0.0) {
        *x += L;
        *img -= 1;
        if (*x >= L) {
            *x = 0.0;
            *img += 1;
        }
    }
}

/* Velocity-Verlet NVE run of nsteps steps of size dt, in place.
 *   F = F(x); per step: v += dt/2 F; x += dt v; wrap; F = F(x); v += dt/2 F.
 * With cg != NULL and cg->s_cg > 0, a coarse-graining event is evaluated after
 * every s_cg-th step between the snapshot of the previous event (the start
 * state for the first one) and the current state; events are numbered from
 * cg->k0 + 1.  energy (optional, [nsteps / energy_every + 1][4]) records
 * {KE, PE, Px, Py} at step 0 and every energy_every steps.
 * Returns the number of coarse-graining events evaluated. */
int64_t orc_md_run(int64_t n, double L, double dt, double rc, double eps, int32_t shift,
                   int32_t use_cells, int64_t nsteps, double* pos, double* vel, int64_t* img,
                   const orc_cg* cg, double* energy, int64_t energy_every) {
    size_t n2 = (size_t)2 * (n > 0 ? n : 1);
    double* f = (double*)malloc(sizeof(double) * n2);
    double* snap = NULL;
    int64_t* snap_img = NULL;
    int use_cg = cg && cg->s_cg > 0;
    int64_t events = 0;
    if (use_cg) {
        snap = (double*)malloc(sizeof(double) * n2);
        snap_img = (int64_t*)malloc(sizeof(int64_t) * n2);
        memcpy(snap, pos, sizeof(double) * 2 * n);
        memcpy(snap_img, img, sizeof(int64_t) * 2 * n);
    }
    double pe = 0.0;
    forces(use_cells, n, L, rc, eps, shift, pos, f, &pe);
    int64_t rec = 0;
    if (energy && energy_every > 0) {
        orc_energy(n, L, rc, eps, shift, use_cells, pos, vel, energy);
        rec = 1;
    }
    double hdt = 0.5 * dt;
    for (int64_t step = 1; step <= nsteps; ++step) {
        for (int64_t j = 0; j < 2 * n; ++j) vel[j] = vel[j] + hdt * f[j];
        for (int64_t j = 0; j < 2 * n; ++j) {
            pos[j] = pos[j] + dt * vel[j];
            wrap(&pos[j], &img[j], L);
        }
        forces(use_cells, n, L, rc, eps, shift, pos, f, &pe);
        for (int64_t j = 0; j < 2 * n; ++j) vel[j] = vel[j] + hdt * f[j];
        if (use_cg && step % cg->s_cg == 0) {
            int64_t kp = cg->k0 + events;
            orc_coarse_grain(cg->lx, L, cg->ux, cg->uy, cg->vtab, n, snap, snap_img, kp, pos, img,
                             kp + 1, cg->counts, NULL, cg->cell_acc, cg->moments);
            memcpy(snap, pos, sizeof(double) * 2 * n);
            memcpy(snap_img, img, sizeof(int64_t) * 2 * n);
            ++events;
        }
        if (energy && energy_every > 0 && step % energy_every == 0) {
            orc_energy(n, L, rc, eps, shift, use_cells, pos, vel, energy + 4 * rec);
            ++rec;
        }
    }
    free(f);
    free(snap);
    free(snap_img);
    return events;
}
