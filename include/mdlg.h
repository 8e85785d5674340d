/*
 * mdlg.h -- C ABI of libmdlg.so, the MI355X (gfx950) hot path of the
 * molecular dynamics lattice gas (MDLG) method for 2D Lennard-Jones particles
 * (Pachalieva & Wagner, "Molecular dynamics lattice gas equilibrium
 * distribution function for Lennard-Jones particles").
 *
 * The library runs 2D Lennard-Jones velocity-Verlet molecular dynamics (the
 * "Simulations setup" section), coarse-grains the trajectory onto a lattice
 * into the occupation numbers n_i(x,t) of Eq.(n_i), averages them into the
 * measured equilibrium distribution of Eq.(theory_feq), and evaluates the
 * single-Gaussian (Eq.(feq_gaussian)) and Poisson weighted-sum-of-Gaussians
 * (Eq.(f_eq_wsg)) equilibria with lambda from Eq.(lambda_eq).
 *
 * Conventions shared by every entry point
 *  - Units: sigma = epsilon(=1 unless set) = m = k_B = 1 (LJ units).
 *  - Pointers marked "device" are HIP device pointers (for example the
 *    data_ptr() of a torch tensor on the GPU); "host" pointers are ordinary
 *    memory.  The caller owns every array it passes; handles own their
 *    internals.  Device pointers must be 8-byte aligned.
 *  - Positions, velocities and forces are [n][2] row-major float64 (x, y per
 *    particle); image counts are [n][2] int32.  Positions are wrapped into
 *    [0, L); the unwrapped position is pos + L * img.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Functions that
 *    take a stream only enqueue work on it unless they say "synchronises".
 *  - Every function returns an mdlg_status.  Invalid arguments are rejected
 *    on the host before anything is launched.  Faults found on the device
 *    (non-finite state, a particle beyond the cell-list skin) are recorded in
 *    the handle and reported by the next synchronising call; the handle is
 *    unusable afterwards.  mdlg_last_error() gives a message for the last
 *    failure on the calling thread.
 *  - Handles are not thread-safe: use one handle from one thread and stream.
 */
#ifndef MDLG_H
#define MDLG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mdlg_status;
#define MDLG_OK 0
#define MDLG_EINVAL (-1)      /* invalid argument                                */
#define MDLG_ENOMEM (-2)      /* device or host allocation failed                */
#define MDLG_EHIP (-3)        /* a HIP runtime call failed                       */
#define MDLG_ENONFINITE (-4)  /* non-finite position or velocity on the device   */
#define MDLG_ESKIN (-5)       /* a particle drifted past the cell-list skin      */
#define MDLG_ENOTIMPL (-6)    /* feature not available in this library           */
#define MDLG_ECAPACITY (-7)   /* a neighbour list or a fused-step tile overflowed its capacity */
#define MDLG_ERANGE (-8)      /* a parameter point outside the range a fitted table covers */

#define MDLG_NQ 49            /* D2Q49 lattice velocities, |v_x|, |v_y| <= 3     */
#define MDLG_HIST_MAX_BINS 4094 /* displacement-histogram bins (2 more count the tails) */
#define MDLG_NCOUNTS 50       /* 49 velocities + 1 overflow bin (|v_a| > 3)      */
#define MDLG_NMOMENTS 5       /* samples, sum d^2, sum d^4, sum d_x, sum d_y     */

/* Message of the last failure on this thread (static storage, valid until the
 * next failing call on this thread). */
const char* mdlg_last_error(void);
/* Library version string. */
const char* mdlg_version(void);

/* D2Q49 lattice velocities in this library's numbering (figure 1b of the paper
 * shows a numbering but is not reproduced; this one sorts by |v|^2 and then
 * by angle counter-clockwise from +x, which gives the six D2Q25 sets the
 * Results section lists: 0 | 1-4 | 5-8 | 9-12 | 13-20 | 21-24).
 * out: host [49][2] int32. */
mdlg_status mdlg_velocity_table(int32_t* out);

/* ------------------------------------------------------------------------ */
/* Molecular dynamics (2D LJ, velocity Verlet, NVE; "Simulations setup")      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;              /* particles (>= 2)                                  */
    double box_l;           /* periodic square box side L (> 3 * (rc + skin))    */
    double dt;              /* MD time step (> 0), 1e-4 in the paper             */
    double rc;              /* cutoff radius (> 0), 2.5                          */
    double eps;             /* well depth epsilon (>= 0); 0 = free particles     */
    int32_t energy_shift;   /* 1: pair energy V(r) - V(rc) inside rc             */
    int32_t force_bits;     /* 64: FP64 pair arithmetic; 32: FP32 pair arithmetic
                               (separation formed in FP64, then rounded)          */
    double skin;            /* cell-list skin: cells are >= rc + skin wide.
                               0 = default 0.5                                    */
    int32_t rebuild_every;  /* MD steps between cell-list rebuilds; 0 = chosen
                               from the fastest initial speed (see lj_md_info)    */
    int32_t block_size;     /* threads per block of the step kernel: 0 = 256;
                               64, 128, 256 or 512                                */
    int32_t step_kernel;    /* 0 = default (3); 1 = one thread per particle with
                               neighbours gathered from global memory; 2 = tiles
                               of cells with the neighbour rows staged in LDS;
                               3 = one thread per particle over a neighbour list
                               of the pairs within rc + skin, rebuilt with the
                               cells                                              */
    int32_t gather_batch;   /* kernel 1: neighbour loads issued per batch, 0 = 8;
                               4, 8 or 16                                         */
    int32_t fuse_steps;     /* kernel 3: consecutive ordinary steps per launch
                               (square tiles of cells staged in LDS with one
                               ring of halo cells per step; the intermediate
                               positions stay in LDS): 0 = three where such
                               tiles are at least 16 cells wide, else two where
                               the two-step tiles are (dilute systems, where
                               the halo is cheap), else one; 1 = one; 2 = two
                               wherever the geometry allows; 3 = three wherever
                               it allows, else two.  Results are the same bit
                               for bit.                                        */
} lj_params;

typedef struct lj_md lj_md; /* opaque handle; owns all device state */

/* Create a handle for one system.  pos0, vel0: device [n][2] float64 (copied;
 * positions must lie in [0, L)).  Velocities are full-step velocities at
 * time 0.  Synchronises `stream`. */
mdlg_status lj_md_init(lj_md** out, const lj_params* p, const double* pos0, const double* vel0,
                       void* stream);

/* Create a handle for n_rep independent systems stepped together (one launch
 * per MD step covers every replica).  p: host [n_rep]; all replicas share dt,
 * force_bits and block_size (the values of p[0]).  pos0, vel0: device,
 * replicas back to back ([sum n_r][2] float64).  Synchronises `stream`. */
mdlg_status lj_md_init_batch(lj_md** out, int32_t n_rep, const lj_params* p, const double* pos0,
                             const double* vel0, void* stream);

/* Lattice of the MDLG coarse-graining ("Molecular dynamics lattice gas
 * method" section): lx x lx cells of side dx = L / lx over the periodic box.
 * Cell of a coordinate x at coarse step k: floor((x + u dx k) * (lx / L))
 * modulo lx, where u is a frame drift in cells per coarse step (a Galilean
 * boost of the lattice frame; u = 0 for the rest frame). */
typedef struct {
    int32_t lx;             /* cells per side (>= 7)                             */
    int32_t reserved;
    double u[2];            /* frame drift, cells per coarse step                */
} mdlg_lattice;

/* Attach fused coarse-graining to a handle: takes the current positions as the
 * snapshot of coarse step 0; from then on, after every s_cg-th MD step, the
 * step kernel evaluates one coarse-graining event (Eq.(n_i)) between the
 * previous snapshot and the new positions and accumulates (+=):
 *   counts   device int64 [n_rep][50]: n_i summed over cells, [49] = overflow
 *   moments  device double [n_rep][5]: samples (2 per particle-event), sum of
 *            d^2 and d^4 pooled over both axes, sum d_x, sum d_y, where d is
 *            the displacement over the coarse step in the box frame
 *   cell_acc device int32 or NULL: per replica [49][lx][lx] (replicas back to
 *            back), n_i(x, t) summed over coarse steps
 * lat: host [n_rep].  The lattice displacement of a particle is taken by the
 * lattice minimum image (exact while a particle moves less than L/2 per
 * coarse step).  The caller zeroes the accumulators.  Replaces any previous
 * attachment. */
mdlg_status lj_md_cg_attach(lj_md* md, int32_t s_cg, const mdlg_lattice* lat, int64_t* counts,
                            double* moments, int32_t* cell_acc, void* stream);
/* Stop coarse-graining. */
mdlg_status lj_md_cg_detach(lj_md* md);

/* Advance every replica by nsteps MD steps (velocity Verlet):
 *   v += dt/2 F(x); x += dt v; wrap; v += dt/2 F(x)
 * The library keeps the half-step velocity between steps and completes it at
 * the start of the next step, which is the same sequence of operations.
 * Repeated chunks are replayed from captured HIP graphs. */
mdlg_status lj_md_step(lj_md* md, int64_t nsteps, void* stream);

/* Advance the replicas by nunits x rebuild_every MD steps like lj_md_step,
 * timing the kernels as the captured graphs run them: every sample_every-th
 * unit (one cell-list interval; the first of the call included) is replayed
 * as three graphs with HIP events on `stream` between them: the cell
 * rebuild, the ordinary steps before the unit's first coarse-graining step,
 * and the remaining steps; the other units run as one graph each, as
 * lj_md_step runs them (a graph boundary costs the device ~15 us, so
 * sampling keeps the timing's own cost small).  ms_out (host [3]) receives
 * the device time per launch of [0] an ordinary step kernel (the ordinary
 * steps' graph time over their number), [1] a coarse-graining step with
 * the launches after it in its unit (the last graph's time less its
 * ordinary steps, per event) and [2] a cell rebuild, each averaged over the
 * counted sampled units; n_out (host [3], may be NULL) the number of kernels
 * or graphs behind each.  The graphs stay in the handle for later calls;
 * sampled units up to the last capture of this call warm up (capture
 * leaves the GPU idle) and are not counted.  nunits >= 3, sample_every in
 * [1, nunits / 3] (above 1 only with graph replay).  Synchronises `stream`. */
mdlg_status lj_md_step_timed(lj_md* md, int64_t nunits, int32_t sample_every, double* ms_out, int32_t* n_out,
                             void* stream);

/* Copy the state out in the caller's particle order (index = position in
 * pos0).  Any output may be NULL.  pos, vel: device [n_total][2] float64
 * (full-step velocities); img: device [n_total][2] int32. */
mdlg_status lj_md_get_state(lj_md* md, double* pos, double* vel, int32_t* img, void* stream);

/* Forces on every particle at the current positions, caller order.
 * force: device [n_total][2] float64. */
mdlg_status lj_md_forces(lj_md* md, double* force, void* stream);

/* Kinetic energy, potential energy and total momentum per replica.
 * out: host [n_rep][4] = {KE, PE, Px, Py}.  Fixed-order reductions
 * (bitwise reproducible).  Synchronises `stream`; reports device faults. */
mdlg_status lj_md_energy(lj_md* md, double* out, void* stream);

/* Synchronise `stream` and report any device fault recorded so far. */
mdlg_status lj_md_check(lj_md* md, void* stream);

typedef struct {
    int32_t n_rep;
    int32_t rebuild_every;  /* MD steps between cell-list rebuilds              */
    int64_t n_total;        /* particles over all replicas                      */
    int64_t steps_done;     /* MD steps taken since init                        */
    int64_t events_done;    /* coarse-graining events since the last attach     */
    int32_t cells_per_side; /* cell-list cells per side of replica 0            */
    int32_t block_size;
    double cell_width;      /* of replica 0                                     */
    int32_t steps_per_launch; /* ordinary MD steps per step-kernel launch: 1, 2 or 3 */
    int32_t reserved;
} lj_md_info_t;
mdlg_status lj_md_info(const lj_md* md, lj_md_info_t* info);

/* Checkpoint: write the handle's replicas to the file `path` (binary, the
 * host's byte order): the lj_params given at init, the MD steps done, and per
 * particle in caller order the wrapped position, the full-step velocity and
 * the image counts (as lj_md_get_state returns them).  Coarse-graining
 * attachments and their accumulators are not saved.  Synchronises `stream`;
 * refuses a handle with a recorded device fault.  EINVAL when the file cannot
 * be written. */
mdlg_status lj_md_save(lj_md* md, const char* path, void* stream);

/* Resume: a new handle from a file written by lj_md_save, with the same
 * replicas, parameters and caller order, the saved positions, velocities and
 * image counts, and steps_done as saved.  The cell lists are built afresh,
 * so the continuation equals the uninterrupted run up to the summation order
 * of the pair forces.  EINVAL for a missing, foreign or truncated file.
 * Synchronises `stream`. */
mdlg_status lj_md_load(lj_md** out, const char* path, void* stream);

/* Free the handle and its device memory (NULL-safe). */
void lj_md_destroy(lj_md* md);

/* Autotuner of the MD step launch for a batch (or one system): times candidate
 * configurations on the given initial state (each runs a few cell-list
 * intervals on a handle of its own; pos0/vel0 are not modified) and writes the
 * fastest into p_out (host [n_rep]): stage 1 picks step_kernel and
 * block_size, stage 2 one skin for all replicas, stage 3 the skin per replica
 * size class (factor-4 bins of N x bins of 0.05 in number density).  With a
 * lattice (lat host [n_rep], s_cg >= 1) the coarse-graining is attached while
 * timing.  Results are cached in $MDLG_AUTOTUNE_CACHE (default
 * ~/.cache/mdlg_autotune.txt) by a signature of the batch; flags bit 0 skips
 * the cache.  us_per_step (may be NULL): the best measured time per MD step, or
 * -1 when taken from the cache.  Synchronises `stream`. */
mdlg_status lj_md_autotune(int32_t n_rep, const lj_params* p_in, const double* pos0, const double* vel0,
                           int32_t s_cg, const mdlg_lattice* lat, int32_t flags, lj_params* p_out,
                           double* us_per_step, void* stream);

/* ------------------------------------------------------------------------ */
/* Coarse-graining of one pair of snapshots (Eq.(n_i))                        */
/* ------------------------------------------------------------------------ */

/* One coarse-graining event between two snapshots of n particles in a box of
 * side box_l.  pos_prev/pos_cur: device [n][2] float64 wrapped positions at
 * coarse steps k_prev and k_cur; img_prev/img_cur: device [n][2] int32 image
 * counts (either may be NULL for zero).  The lattice velocity of particle j is
 * C_j(k_cur) - C_j(k_prev) with the unwrapped cell C = floor((x + u dx k) *
 * lx / L) + lx * img; n_i counts it at its destination cell at k_cur.
 * Outputs (device, any may be NULL except counts):
 *   counts  int64 [50]   += n_i summed over cells ([49]: overflow)
 *   moments double [5]   += as in lj_md_cg_attach, d from pos + L * img
 *   n_event int32 [49][lx][lx] overwritten with n_i(x, t)
 *   cell_acc int32 [49][lx][lx] += n_i(x, t)
 * Bitwise equal to the definition for identical inputs (integer counts);
 * moments use a fixed-order reduction. */
mdlg_status mdlg_coarse_grain(const mdlg_lattice* lat, double box_l, int64_t n,
                              const double* pos_prev, const int32_t* img_prev, int64_t k_prev,
                              const double* pos_cur, const int32_t* img_cur, int64_t k_cur,
                              int64_t* counts, double* moments, int32_t* n_event, int32_t* cell_acc,
                              void* stream);

/* mdlg_coarse_grain for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (counts and moments bitwise
 * equal to mdlg_coarse_grain's); it calls no allocating routine.  Its moment
 * partials live in a fixed device array of the library (5.2 MB, one copy per
 * GPU, held until the process ends), which limits n to 2^25 = 33,554,432
 * particles: larger n is rejected with MDLG_EINVAL before anything is
 * launched.  The stream must belong to the current device.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from several threads) race and give wrong moments; calls on one
 * stream are ordered and safe. */
mdlg_status mdlg_coarse_grain_noalloc(const mdlg_lattice* lat, double box_l, int64_t n,
                                      const double* pos_prev, const int32_t* img_prev, int64_t k_prev,
                                      const double* pos_cur, const int32_t* img_cur, int64_t k_cur,
                                      int64_t* counts, double* moments, int32_t* n_event,
                                      int32_t* cell_acc, void* stream);

/* Coarse-graining of a stored trajectory for many coarse-graining times and
 * lattice drifts in one pass (Eq.(n_i) for every snapshot pair).  The batch
 * holds n_rep replicas; replica r owns particles offsets[r] .. offsets[r+1]-1
 * (host [n_rep + 1], offsets[0] = 0) in a box of side box_l[r] (host) with an
 * lx[r] x lx[r] lattice (host).  pos (device [n_snap][n_tot][2] float64) and
 * img (device [n_snap][n_tot][2] int32) stack 2 <= n_snap <= 512 snapshots at
 * a fixed stride.  For each lag lags[s] (host [n_lag], 1 .. min(32,
 * n_snap - 1), in snapshots) and drift u[t] (host [n_u][2], cells per coarse
 * step), every pair (p - lag, p) is one event on a lattice translated by
 * o dx at snapshot p - lag and by (o + u) dx at snapshot p (one coarse step
 * of a lattice moving u cells per step), o = offset[p - lag] (host
 * [n_snap][2], cells, |o| <= 1e6; NULL = all zero, which makes each pair
 * the event of mdlg_coarse_grain with k_prev = 0, k_cur = 1; |u| <= 1e6).
 * A homogeneous gas has the
 * same statistics on every translated lattice; origins that vary between
 * pairs decorrelate overlapping pairs.  Adds to counts (device int64
 * [n_rep][n_lag][n_u][50]) and, if not NULL, to moments (device float64
 * [n_rep][n_lag][5], box-frame displacement sums as in mdlg_coarse_grain,
 * the same for every drift).  n_lag <= 32, n_u <= 16, n_lag * n_u <= 256.
 * Synchronises the stream.  Counts are bitwise those of the per-pair calls;
 * moments use a fixed-order reduction.  EINVAL (counts unspecified) when an
 * unwrapped cell q + lx * img leaves the 32-bit range. */
mdlg_status mdlg_coarse_grain_series(int32_t n_rep, const int64_t* offsets, const double* box_l,
                                     const int32_t* lx, int32_t n_snap, const double* pos,
                                     const int32_t* img, int32_t n_lag, const int32_t* lags,
                                     int32_t n_u, const double* u, const double* offset,
                                     int64_t* counts, double* moments, void* stream);

/* ------------------------------------------------------------------------ */
/* Equilibria (host, FP64)                                                    */
/* ------------------------------------------------------------------------ */

/* Measured equilibrium (Eq.(theory_feq)): g_i = f_i^eq / rho with
 * rho = N / lx^2, i.e. g_i = counts[i] / (n_particles * n_events).
 * symmetrize = 1 averages g over each |v|^2 shell (the Results section's
 * symmetrised D2Q25 sets; meaningful for zero mean velocity).
 * counts: host [50]; g_out: host [49]; overflow_frac: host, may be NULL. */
mdlg_status mdlg_feq_measured(const int64_t* counts, int64_t n_particles, int64_t n_events,
                              int32_t symmetrize, double* g_out, double* overflow_frac);

/* Displacement moments from accumulated sums: mu2 = <d^2>, mu4 = <d^4>
 * (pooled over both axes) and a^2 = mu2 / dx^2 (Eq.(a2_n_ua)).
 * moments: host [5]; any output may be NULL. */
mdlg_status mdlg_moments(const double* moments, double dx, double* mu2, double* mu4, double* a2);

/* Average number of collisions lambda of the Poisson-WSG model from the
 * second and fourth displacement moments (Eq.(lambda_eq)).  With
 * r = mu4 / (3 mu2^2) the roots are lambda and 1/lambda; branch 2 returns the
 * larger root (the printed lambda_2, which the paper uses), branch 1 the
 * smaller.  r <= 1 gives lambda = 0 (single Gaussian); r >= 5/4, beyond the
 * model's range, gives lambda = 1.  r may be NULL. */
mdlg_status mdlg_lambda_from_moments(double mu2, double mu4, int32_t branch, double* lambda,
                                     double* r);

/* Single-Gaussian equilibrium g^G_i = f^eq,G_i / rho (Eq.(feq_prod) and
 * Eq.(feq_gaussian)); a2 >= 0 in lattice units^2, u host [2] mean
 * displacement in cells per coarse step (NULL = 0).  g_out host [49]. */
mdlg_status mdlg_feq_gauss(double a2, const double* u, double* g_out);

/* Poisson-WSG equilibrium (Eq.(f_eq_wsg)): sum over collision counts c of
 * e^-lambda lambda^c / c! times the product over axes of the Gaussian form
 * with variance a2 (c+1)/(lambda+1).  The sum is truncated where the
 * remaining Poisson weight is below 1e-20.  lambda = 0 gives mdlg_feq_gauss. */
mdlg_status mdlg_feq_wsg(double a2, double lambda, const double* u, double* g_out);

/* ------------------------------------------------------------------------ */
/* Non-equilibrium MDLG of a replica ensemble                                */
/* ------------------------------------------------------------------------ */

/* Ensemble sums of the occupation numbers (Eq.(n_i)) at every coarse step of
 * stored trajectories and of the lattice gas collision operator defined with
 * Eq.(mdlg_evolution), Xi_i(x, t) = n_i(x + v_i, t + dt) - n_i(x, t).  Divided
 * by the ensemble size they are the MDLB distribution f_i = <n_i>_neq and
 * collision operator Omega_i = <Xi_i>_neq of the "Molecular dynamics lattice
 * gas method" section.  The ensemble is n_total particles over any number of
 * replicas of one system (box side box_l, an lx x lx lattice at rest,
 * 7 <= lx <= 46340): the sums do not depend on which particle belongs to
 * which replica.  pos (device [n_snap][n_total][2] float64, wrapped into
 * [0, box_l)) and img (device [n_snap][n_total][2] int32 image counts) stack
 * n_snap >= 2 snapshots one coarse step apart; event p (1 <= p < n_snap) is
 * the step from snapshot p-1 to p, with the lattice velocity of a particle
 * C(p) - C(p-1) of its unwrapped cells C = floor(x lx / box_l) + lx img.
 * Outputs (device, overwritten):
 *   f_sum    int32 [n_snap-1][49][lx][lx]: sum of n_i(x, t_p), cell (x, y) at
 *            [i][y][x], the destination cell taken modulo lx
 *   overflow int64 [n_snap-1]: particles of event p whose lattice
 *            displacement is outside D2Q49 (not counted in f_sum)
 *   xi_sum   int32 [n_snap-2][49][lx][lx] or NULL: sum of Xi_i(x, t_p) for
 *            1 <= p < n_snap - 1, x + v_i on the periodic lattice
 * Integer results, exact and independent of the launch.  Asynchronous on
 * `stream`; allocates nothing. */
mdlg_status mdlg_neq_mdlg(int64_t n_total, double box_l, int32_t lx, int32_t n_snap, const double* pos,
                          const int32_t* img, int32_t* f_sum, int64_t* overflow, int32_t* xi_sum,
                          void* stream);

/* ------------------------------------------------------------------------ */
/* Velocity autocorrelation and lambda from it                               */
/* ------------------------------------------------------------------------ */

/* Velocity autocorrelation sums of stored velocity snapshots, for estimating
 * the average number of collisions lambda of the Poisson-WSG model from the
 * velocity autocorrelation function (the alternative to moment matching
 * named in the section on the Poisson weighted sum of Gaussians).  Replica r
 * owns particles offsets[r] .. offsets[r+1]-1 (host [n_rep + 1], offsets[0]
 * = 0); vel (device [n_snap][n_tot][2] float64) stacks n_snap >= 1 snapshots
 * at a fixed stride.  For each lag lags[s] (host [n_lag], 0 .. n_snap - 1,
 * n_lag <= 1024) adds to c_sum (device float64 [n_rep][n_lag]) the sum over
 * the replica's particles j and origins p = 0 .. n_snap-1-lag of
 * v_j(p) . v_j(p + lag); the caller divides by n_r (n_snap - lag).  FP64,
 * fixed-order reductions (bitwise reproducible).  Synchronises the stream. */
mdlg_status mdlg_vacf(int32_t n_rep, const int64_t* offsets, int32_t n_snap, const double* vel,
                      int32_t n_lag, const int32_t* lags, double* c_sum, void* stream);

/* lambda = dt_cg / tau, the expected number of collisions in a coarse step if
 * collisions arrive as a Poisson process of rate 1/tau that each forget the
 * velocity (then C(t) = C(0) exp(-t / tau)).  tau is the trapezoid integral
 * of C(t) / C(0) over the samples (t host [n] increasing, t[0] = 0; c host
 * [n], C(0) > 0) up to and including the first one with C <= cut C(0), or
 * over all of them.  Outputs (host, may be NULL): tau, lambda. */
mdlg_status mdlg_lambda_vacf(int32_t n, const double* t, const double* c, double dt_cg, double cut,
                             double* tau, double* lambda);

/* ------------------------------------------------------------------------ */
/* Displacement PDFs and the KL divergence (Fig. 2)                          */
/* ------------------------------------------------------------------------ */

/* Histograms of the one-particle box-frame displacements of a stored
 * trajectory: the binned displacement PDF P^MD(X_k) compared with the single
 * Gaussian (Eq.(gaussian_df)) and the Poisson WSG (Eq.(poisson_v2)).
 * Replica r owns particles offsets[r] .. offsets[r+1]-1 (host [n_rep + 1],
 * offsets[0] = 0) in a box of side box_l[r] (host).  pos (device
 * [n_snap][n_tot][2] float64, wrapped) and img (device [n_snap][n_tot][2]
 * int32 image counts) stack 2 <= n_snap <= 2^24 snapshots.  For lag
 * lags[s] (host [n_lag], 1 .. n_snap - 1, n_lag <= 64) and every pair
 * (p - lag, p), each particle's displacement per axis
 *   delta = (x_p - x_{p-lag}) + L (img_p - img_{p-lag})
 * falls in bin k = floor(delta * (1 / h) + n_bin / 2) (FP64, each operation
 * rounded once), h = bin_width[s] (host [n_lag], > 0): the intervals
 * X_k = [(k - n_bin/2) h, (k + 1 - n_bin/2) h), k < n_bin, tile
 * [-n_bin h / 2, n_bin h / 2).  Adds to hist (device int64
 * [n_rep][n_lag][2][n_bin + 2], axis x then y): [k] for X_k, [n_bin] below
 * the range, [n_bin + 1] at or above it.  1 <= n_bin <= MDLG_HIST_MAX_BINS.
 * Counts are exact integers, independent of the launch.  Synchronises the
 * stream. */
mdlg_status mdlg_displacement_hist(int32_t n_rep, const int64_t* offsets, const double* box_l,
                                   int32_t n_snap, const double* pos, const int32_t* img,
                                   int32_t n_lag, const int32_t* lags, const double* bin_width,
                                   int32_t n_bin, int64_t* hist, void* stream);

/* Probability of each histogram bin under the one-axis single Gaussian
 * P^G (Eq.(gaussian_df), variance msd) and the Poisson WSG P^WSG
 * (Eq.(poisson_v2) with P^c of Eq.(p_wsg_one), variance msd (c + 1) /
 * (lambda + 1)), both centred on `mean` (the mean displacement u dt, in the
 * units of h).  msd is the second moment about the mean, > 0.  The bins are
 * those of mdlg_displacement_hist (n_bin, width h); [n_bin] and [n_bin + 1]
 * receive the masses below and above the range.  The Poisson sum uses the
 * window of mdlg_feq_wsg; lambda = 0 gives P^WSG = P^G.  Outputs host
 * [n_bin + 2]; either may be NULL. */
mdlg_status mdlg_pdf_bins(double msd, double lambda, double mean, double h, int32_t n_bin,
                          double* p_gauss, double* p_wsg);

/* P^MD(X_k): n_hist histograms of n counts each (host [n_hist][n], e.g. the
 * two axes of one lag) summed bin by bin and divided by their total.
 * p_out host [n].  EINVAL for negative counts or an empty total. */
mdlg_status mdlg_pdf_measured(const int64_t* hist, int32_t n_hist, int32_t n, double* p_out);

/* Element-wise Kullback-Leibler divergence K(X_i) = R_i log(R_i / Q_i)
 * (Eq.(k_Xi)) into k_out (host [n], may be NULL) and its sum D_KL(R || Q)
 * (Eq.(kullback_leibler), compensated, index order) into d_kl (may be NULL).
 * A term with R_i = 0 is 0; R_i > 0 with Q_i = 0 is +inf (and so is D_KL).
 * r, q host [n], finite and >= 0; they are not renormalised. */
mdlg_status mdlg_kl_divergence(const double* r, const double* q, int32_t n, double* k_out,
                               double* d_kl);

/* ------------------------------------------------------------------------ */
/* Surrogate network for f_eq (device, BF16 matrix cores)                    */
/* ------------------------------------------------------------------------ */

/* A small multilayer perceptron maps the six inputs
 *   x = (phi, kT, dt_cg / dx, |u|, cos theta_u, sin theta_u)
 * of an equilibrium LJ gas and its lattice (area fraction, temperature,
 * coarse-graining time over lattice spacing in tau/sigma, the mean
 * displacement in cells per coarse step and its direction) to the 49 values
 * g_i = f_i^eq / rho of the D2Q49 equilibrium (Eq.(theory_feq)):
 *   h1 = silu(x' W1 + b1), h2 = silu(h1 W2 + b2), h3 = silu(h2 W3 + b3),
 *   g = softmax(h3 W4 + b4),  widths 6 -> 256 -> 256 -> 256 -> 49,
 * with the fixed input map x' = (phi / 0.4, ln kT / ln 20, (ln(dt_cg/dx) + 6) / 1.5,
 * 5 |u| cos, 5 |u| sin, 5 |u|) (fp32; logarithms of the two scales, whose
 * product kT (dt_cg/dx)^2 is a^2 in the ballistic limit; the drift as a
 * vector, so that the lattice's reflection symmetries are linear in it).
 * It is trained on measured f_eq with the Kullback-Leibler divergence of
 * Eq.(kullback_leibler), sum_i R_i log(R_i / g_i) averaged over the batch,
 * as the loss, by Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 *
 * Parameters are one flat float32 vector of MDLG_MLP_NPARAMS values:
 * W1 [6][256] (input-major), b1 [256], W2 [256][256], b2, W3 [256][256], b3,
 * W4 [256][49], b4 [49].  The handle keeps float32 master weights and Adam
 * state; the matrix products read bfloat16 copies (round to nearest even) of
 * the weights and of the layer inputs and accumulate in float32; biases,
 * pre-activations, softmax and loss stay float32.  Arrays [B][6] and
 * [B][49] are row-major float32. */
#define MDLG_MLP_NPARAMS 145969
typedef struct mdlg_mlp mdlg_mlp; /* opaque handle; owns all device state */

/* Create a network with the given initial parameters (host [NPARAMS], all
 * finite) and room for batches of up to max_batch (1 .. 2^20) samples.
 * Synchronises the stream.  Errors: EINVAL, ENOMEM, EHIP. */
mdlg_status mdlg_mlp_create(mdlg_mlp** out, const float* params, int32_t max_batch, void* stream);
/* Copy the float32 master parameters to host [NPARAMS].  Synchronises. */
mdlg_status mdlg_mlp_params(const mdlg_mlp* mlp, float* host_out, void* stream);
/* Inference: g_out device [B][49] = network(x device [B][6]), 1 <= B <= max_batch. */
mdlg_status mdlg_mlp_forward(mdlg_mlp* mlp, const float* x, int32_t B, float* g_out, void* stream);
/* Loss and its gradient at the current parameters, without an update:
 * target device [B][49] (rows summing to one), loss device [1] and grad
 * device [NPARAMS] (either may be NULL). */
mdlg_status mdlg_mlp_gradient(mdlg_mlp* mlp, const float* x, const float* target, int32_t B,
                              float* loss, float* grad, void* stream);
/* One training step: forward, loss, backward and an Adam update with
 * learning rate lr > 0.  loss device [1] (may be NULL) receives the loss
 * before the update. */
mdlg_status mdlg_mlp_train_step(mdlg_mlp* mlp, const float* x, const float* target, int32_t B,
                                float lr, float* loss, void* stream);
/* Surrogate f_eq with a closed-form guard: evaluates the network at host
 * x[6], compares it with the Poisson-WSG equilibrium (Eq.(f_eq_wsg)) of the
 * given a2 and lambda at the drift u = |u| (cos, sin), and returns the
 * network's values when max_i |g_net - g_wsg| <= tol, else the WSG values
 * with *used_fallback = 1.  g_out host [49]; err host (may be NULL) gets the
 * max difference.  Synchronises.  Errors: EINVAL, EHIP. */
mdlg_status mdlg_feq_surrogate(mdlg_mlp* mlp, const double* x, double a2, double lambda, double tol,
                               double* g_out, int32_t* used_fallback, double* err, void* stream);
/* Release the handle and its device memory (NULL is ignored). */
void mdlg_mlp_destroy(mdlg_mlp* mlp);

/* Displacement moments without a trajectory: the Poisson-WSG guard above
 * needs a^2 (Eq.(theory_a)) and lambda (Eq.(lambda_eq)), which the method
 * measures.  A moment table fits them over the training runs' parameter
 * points so that the guard needs no molecular dynamics.  Fields ln a^2 and
 * r = mu4 / (3 mu2^2) are fitted on a regular grid of dims[0] x dims[1] x
 * dims[2] nodes spanning the samples' range of the coordinates
 * (phi, ln kT, ln(dt_cg/dx)) by least squares with multilinear hat functions
 * plus smooth * n / P times the sum of squared second differences along each
 * axis (node units; zero for any multilinear function, which the fit thus
 * reproduces exactly); evaluation interpolates multilinearly and takes
 * lambda from r on the given root branch (as mdlg_lambda_from_moments).
 * Host-only, FP64; the handle owns host memory only. */
typedef struct mdlg_moment_table mdlg_moment_table;

/* samples host [n][5] = (phi, kT, dt_cg/dx, a2, r) with kT, dt_cg/dx, a2 > 0;
 * dims host [3], each in [1, 64], product <= 2048 (an axis whose samples do
 * not spread needs dims 1); lo, hi host [3] = (phi, kT, dt_cg/dx): the box
 * the grid spans (both NULL: the samples' bounding box; given, it must hold
 * every sample, and the penalty extends the fit linearly to its edges);
 * smooth >= 0 (0 only when samples reach every node); branch 1 or 2.
 * Errors: EINVAL (arguments, or a singular fit). */
mdlg_status mdlg_moment_table_create(mdlg_moment_table** out, const double* samples, int64_t n,
                                     const int32_t* dims, const double* lo, const double* hi,
                                     double smooth, int32_t branch);
/* x host [3] = (phi, kT, dt_cg/dx) -> a2, lambda and r (each may be NULL).
 * ERANGE when x lies outside the grid's box. */
mdlg_status mdlg_moment_table_eval(const mdlg_moment_table* table, const double* x, double* a2,
                                   double* lambda, double* r);
/* The grid: dims [3], coordinate bounds lo/hi [3] (phi, ln kT, ln(dt_cg/dx))
 * and node values nodes [P][2] = (ln a2, r); any pointer may be NULL. */
mdlg_status mdlg_moment_table_info(const mdlg_moment_table* table, int32_t* dims, double* lo, double* hi,
                                   double* nodes);
/* Release the table (NULL is ignored). */
void mdlg_moment_table_destroy(mdlg_moment_table* table);

/* mdlg_feq_surrogate with a2 and lambda from the table at (x[0], x[1], x[2])
 * (the network's phi, kT and dt_cg/dx), so that neither the network nor its
 * guard needs a trajectory.  a2_out and lambda_out (host, may be NULL)
 * receive the interpolated moments.  ERANGE outside the table's range (the
 * caller then measures); otherwise as mdlg_feq_surrogate. */
mdlg_status mdlg_feq_surrogate_table(mdlg_mlp* mlp, const mdlg_moment_table* table, const double* x,
                                     double tol, double* g_out, int32_t* used_fallback, double* err,
                                     double* a2_out, double* lambda_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MDLG_H */
