/*
 * fte.h - C ABI of the MI355X focused-transport pseudo-particle library.
 *
 * The library integrates independent energetic test particles through the
 * focused transport equation (FTE) written as Ito stochastic differential
 * equations: streaming along the mean magnetic field plus solar-wind
 * advection, magnetic focusing, adiabatic deceleration, pitch-angle
 * scattering and optional cross-field diffusion (arXiv:2404.12164, section
 * 2.1, Eqs. 1-5).  The solar-wind velocity V and field B come from snapshots
 * on a stretched, block-AMR spherical grid (section 2.4); observer intensities
 * j = p^2 f (section 2.3) are accumulated in time x energy bins.
 *
 * Conventions for every entry point:
 *  - SI units throughout (m, s, kg, J, rad).
 *  - Every call returns fte_status; FTE_OK == 0.  On failure a message is
 *    available from fte_last_error() and the context is left unchanged
 *    (argument errors) or must be destroyed (FTE_EDEVICE).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it; fte_step_n and fte_inject return without
 *    waiting.  fte_load_grid, fte_bin_observers, fte_get_stats and
 *    fte_read_particles synchronise the stream before returning.
 *  - Device buffers are owned by the caller (allocated with the sizes from
 *    fte_query_sizes, e.g. as torch tensors) and must outlive the context.
 *    The library never allocates or frees device memory.  Host arrays passed
 *    in are only read during the call.
 *  - One context is used from one thread at a time.
 *  - Per-particle non-finite results are not errors: the particle is retired
 *    with status FTE_PS_NUMERIC and counted in fte_stats.
 */
#ifndef FTE_H
#define FTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fte_ctx fte_ctx;
typedef int fte_status;

enum {
    FTE_OK = 0,
    FTE_EINVAL = -1,   /* invalid argument or inconsistent description          */
    FTE_ESTATE = -2,   /* call out of order (e.g. step before load/inject)      */
    FTE_ENOMEM = -3,   /* a bound buffer is too small for the request           */
    FTE_EDEVICE = -4,  /* a HIP call failed                                     */
    FTE_ERANGE = -5    /* the requested steps leave the grid's time range       */
};

/* arithmetic of the step kernel */
enum {
    FTE_FP64 = 0,      /* all arithmetic and grid records in double precision   */
    FTE_MIXED = 1      /* float records and step arithmetic; position, time and
                          the radial boundary tests stay in double             */
};

/* pitch-angle diffusion coefficient D_mumu(mu) = A g(mu) (section 2.1) */
enum {
    FTE_DMM_ISO = 0,     /* g = 1 - mu^2                                        */
    FTE_DMM_EQ5 = 1,     /* g = (|mu|/(1+|mu|) + eps)(1 - mu^2), Eq. 5          */
    FTE_DMM_POWER_Q = 2  /* g = (1 - mu^2)|mu|^(q-1), 1 < q < 2                 */
};

/* particle status codes in the state buffers */
enum {
    FTE_PS_ACTIVE = 0,
    FTE_PS_ABSORBED_IN = 1,   /* crossed r < r_in                               */
    FTE_PS_ABSORBED_OUT = 2,  /* crossed r > r_out                              */
    FTE_PS_OUT_OF_DOMAIN = 3, /* colatitude left the grid's range               */
    FTE_PS_NUMERIC = 4,       /* non-finite state or vanishing b                */
    FTE_PS_DONE = 5           /* its run (ensemble) took all its steps          */
};

#define FTE_MAX_OBS 8
#define FTE_MAX_LEVELS 8
#define FTE_MAX_BATCH 64
#define FTE_MAX_RUNS 64

/* Observer: the radial x colatitude box of full widths dr, dtheta around
 * (r, theta), and n_phi (>= 1; 0 counts as 1) consecutive longitude bins of
 * width dphi, the first centred at phi + omega t (t the post-step time): a
 * spherical box (n_phi = 1, omega = 0), a ring of bins for longitudinal
 * profiles, or a corotating pattern (omega = the structure's rotation rate).
 * Each longitude bin is one observer bin of the sums. */
typedef struct {
    double r, theta, phi;
    double dr, dtheta, dphi;
    int n_phi;
    double omega;         /* rad/s                                                 */
} fte_observer;

/* One run of an ensemble: its own mean free path and cross-field ratio (the
 * other physics is shared), its own step count and Philox run id
 * (fte_params.run_id + its index), its own observer sums. */
typedef struct {
    double lambda_ref;    /* parallel mean free path at p_ref, m                   */
    double kperp_ratio;   /* kappa_perp / kappa_par (0: lambda_perp or none)        */
    uint64_t n_steps;     /* global steps 0 .. n_steps-1; then FTE_PS_DONE          */
} fte_run;

/* Physics and run parameters (fixed for the life of a context). */
typedef struct {
    double mass;          /* rest mass of the species, kg                          */
    int dmm_model;        /* FTE_DMM_*                                             */
    int dmm_norm;         /* 0: A = 3 v I / (8 lambda_par) so that lambda_par =
                             3 kappa_par / v with kappa_par = (v^2/8) Int (1-mu^2)^2/D;
                             1: A = v / lambda_par                                 */
    double lambda_ref;    /* parallel mean free path at momentum p_ref, m          */
    double p_ref;         /* reference momentum in units of m c                   */
    double alpha;         /* lambda_par = lambda_ref (p / p_ref)^alpha             */
    double q;             /* exponent of FTE_DMM_POWER_Q                           */
    double eps;           /* resonance-gap parameter of FTE_DMM_EQ5 (Eq. 5)        */
    double mu_floor;      /* |mu| floor inside |mu|^(q-2) of the POWER_Q drift     */
    double kperp_ratio;   /* kappa_perp = ratio * v lambda_par / 3 when > 0        */
    double lambda_perp;   /* otherwise kappa_perp = v lambda_perp / 3 when > 0     */
    double dt;            /* global time step, s                                   */
    double t0;            /* time of global step 0, s                              */
    double r_in, r_out;   /* absorbing spheres, m                                  */
    uint64_t seed;        /* Philox key                                            */
    int run_id;           /* 0..65535, part of the Philox counter                  */
    int precision;        /* FTE_FP64 or FTE_MIXED                                 */
    int n_obs;            /* 0..FTE_MAX_OBS                                        */
    fte_observer obs[FTE_MAX_OBS];
    double e_min;         /* lower kinetic-energy edge of bin 0, J                 */
    double dlne;          /* bin width in ln E                                     */
    int n_e;              /* energy bins                                           */
    double t_ref;         /* lower edge of time bin 0, s                           */
    double dT;            /* time-bin width, s                                     */
    int n_t;              /* time bins                                             */
    int n_batch;          /* 1..FTE_MAX_BATCH; batch = pid mod n_batch             */
    /* Kernel-smoothed intensities (on when sigma_x > 0): every post-step
     * state adds w v dt G3(x - x_o) G1(ln E - ln E_e) / E G1(t - t_t) to
     * J[o][e][t], x_o the observer centre, ln E_e = ln e_min + (e + 1/2) dlne
     * and t_t = t_ref + (t + 1/2) dT the bin centres, G3 / G1 normalised
     * Gaussians of widths sigma_x, sigma_lne, sigma_t, each dropped beyond 6
     * widths (1.5e-8 of the peak); J = sums / (4 pi W_inj).  A differentiable estimate of
     * j = p^2 f = v n_E / (4 pi) (section 2.3). */
    double sigma_x;       /* m                                                     */
    double sigma_lne;     /* ln E                                                  */
    double sigma_t;       /* s                                                     */
    int grad;             /* 1: also carry, per particle, the pathwise derivatives
                             of (x, mu, ln p) with respect to lambda_ref and
                             kperp_ratio (forward tangents driven by the same
                             noise) and d ln w / d gamma_inj, and accumulate dJ.
                             Needs sigma_x, sigma_lne, sigma_t > 0 and the
                             tangent buffers.                                     */
    /* Ensembles: n_runs > 0 runs share the grid, the clock and every other
     * parameter; each particle belongs to one run (fte_injection.run) and
     * takes that run's lambda_ref, kperp_ratio, step count and Philox run id
     * run_id + run; observer sums are kept per run.  A particle of run r
     * follows exactly the trajectory it has in a single-run context with
     * run_id + r and that run's lambda_ref and kperp_ratio.  n_runs = 0: a
     * single run with the fields above.  Not combined with sigma_x > 0.      */
    int n_runs;           /* 0..FTE_MAX_RUNS                                       */
    const fte_run *runs;  /* host, n_runs entries; copied by fte_create            */
    /* Gradient mode with FTE_DMM_EQ5: |mu| in Eq. 5 gives dD/dmu a jump of
     * 2A at mu = 0, which the derivative of each sampled step does not see
     * (a.e. d2D/dmu2 has no Dirac term).  kink_sigma > 0 adds to the
     * tangents' d2D/dmu2 the term 2A G(mu), G a normalised Gaussian of that
     * width standing for the Dirac (the local time at mu = 0 of the
     * continuous process); kink_sigma < 0 weights it by the time each step is
     * expected to spend at mu = 0 given its end points (a Brownian bridge with
     * the diffusion at mu = 0), no width; 0: the tangents are the exact
     * derivatives of each sampled path.  Trajectories are unchanged.          */
    double kink_sigma;
} fte_params;

/* Block-AMR spherical grid (section 2.4).  Coordinates (xi, theta, phi), with
 * xi = r - r_lo (xi_map 0) or ln(r / r_lo) (xi_map 1, radial stretching).
 * Level-1 cells are uniform in each coordinate; each level halves its parent
 * block along all three coordinates; every block holds bx[0] x bx[1] x bx[2]
 * cells.  Leaves must tile the domain and blocks touching face-wise or
 * diagonally may differ by at most one level.  bx[a] must be even and >= 4,
 * and divisible by 4 when n_levels >= 3; n1[a] must be a multiple of bx[a]. */
typedef struct {
    int xi_map;
    double r_lo, dxi;     /* radial origin (m) and level-1 width in xi            */
    double th_lo, dth;    /* colatitude origin and level-1 width, rad             */
    double ph_lo, dph;    /* longitude origin and level-1 width, rad              */
    int phi_periodic;     /* 1: n1[2] * dph spans 2 pi and phi wraps              */
    int n1[3];            /* level-1 cells along xi, theta, phi                   */
    int bx[3];            /* cells per block                                      */
    int n_levels;         /* 1..FTE_MAX_LEVELS                                    */
    int n_leaves;
    const int32_t *leaves;/* host, [n_leaves][4] = level, I, J, K (block index at
                             that level); list order defines leaf ids             */
    int n_snap;           /* snapshots; 1 = steady                                */
    double t_s0, dt_s;    /* snapshot k is at t_s0 + k dt_s                       */
    int n_slots;          /* snapshot records held on the device: 0 (or >= n_snap)
                             all of them (fte_load_grid); 2 .. n_snap-1 a ring
                             that fte_load_snapshot fills as the run advances  */
    int n_pool;           /* with a ring: 0 holds every leaf of each snapshot;
                             1 .. n_leaves holds at most that many leaf blocks
                             per slot, only those fte_plan_snapshot finds the
                             particles can reach (section 4: load only the
                             blocks that are needed)                          */
} fte_grid_desc;

/* Particle source for fte_inject (the synthetic workloads' injection; with
 * r_weight set it carries the r^-2 statistical weight of section 2.3, Eq. 6).
 * Draws use the injection Philox stream of each pid: isotropic mu, position
 * uniform in solid angle over [th_lo, th_hi] x [ph_lo, ph_hi] at radius r,
 * kinetic energy log-uniform on [e_lo, e_hi] (monoenergetic if equal) with
 * weight w0 (E/e_lo)^(1 - gamma_inj) (an E^-gamma_inj number spectrum),
 * and first step k0 + floor((pid - pid0 + u) n_inj_steps / n_total)
 * (stratified continuous injection; all at k0 when n_inj_steps == 0). */
typedef struct {
    double r;
    double th_lo, th_hi, ph_lo, ph_hi;
    double e_lo, e_hi;
    double gamma_inj;
    double w0;
    int r_weight;         /* 1: multiply the weight by (r_ref / r)^2              */
    double r_ref;
    uint64_t pid0;        /* first pid of the whole injection                     */
    uint64_t n_total;     /* particles of the whole injection (>= 1)              */
    uint32_t k0;
    uint32_t n_inj_steps;
    int run;              /* ensemble run the particles belong to (0 if none)     */
    /* The paper's law (section 2.3, Eq. 6) when region = 1: positions uniform
     * in volume over the shell sector r .. r_hi x [th_lo, th_hi] x
     * [ph_lo, ph_hi], kept where the leaf cell holding the point has
     * div V < divv_max at the snapshot nearest the particle's first step
     * (rejection sampling on the injection stream, counter steps 2, 3, ...; a
     * particle that finds no such point in max_tries attempts is retired with
     * FTE_PS_NUMERIC); with r_weight the weight is (r_ref / r)^2 at the drawn
     * radius. */
    int region;
    double r_hi;
    double divv_max;      /* 1/s                                                   */
    uint32_t max_tries;
} fte_injection;

/* Byte sizes of the caller-owned device buffers. */
typedef struct {
    uint64_t grid_bytes;    /* derived-field records of every snapshot             */
    uint64_t index_bytes;   /* block index and leaf table                          */
    uint64_t state_bytes;   /* one particle state buffer (two are bound)           */
    uint64_t hist_bytes;    /* observer batch sums                                 */
    uint64_t work_bytes;    /* counters, load-time workspace, finalize output,
                               smoothed-intensity sums                            */
    uint64_t tangent_bytes; /* one tangent buffer (two; gradient mode only)        */
} fte_sizes;

/* Device pointers, each at least the matching fte_sizes bytes, 256-byte
 * aligned.  tangent_a / tangent_b may be NULL when fte_params.grad == 0. */
typedef struct {
    void *grid, *index, *state_a, *state_b, *hist, *work, *tangent_a, *tangent_b;
} fte_buffers;

typedef struct {
    uint64_t n_live;          /* particles held (active or not yet started)     */
    uint64_t n_injected;
    uint64_t particle_steps;  /* steps taken by active particles                */
    uint64_t n_retired[6];    /* by FTE_PS_* (index 0 unused)                   */
    double w_injected;
    double w_retired[6];      /* weight of retired particles by FTE_PS_*        */
    uint64_t global_step;     /* next global step index                         */
    uint32_t device_flags;    /* nonzero: a kernel met an unsupported case (bit
                                 8: a step reached a leaf a streamed subset
                                 does not hold)                                 */
    uint32_t step_launches;   /* step-kernel launches timed since the last reset */
    double step_kernel_ms;    /* their summed duration (HIP events on `stream`) */
} fte_stats;

/* Record layout of the grid buffer (for readers of the raw buffer):
 * record(snap, leaf, pcell) at element ((snap * n_leaves + leaf) * pcells +
 * pcell) * stride, elements of double (FTE_FP64) or float (FTE_MIXED); the
 * stride is FTE_RECORD_STRIDE (10: fields 0-9) when kappa_perp is off and
 * FTE_RECORD_STRIDE_KPERP (13: fields 0-12) when it is on.
 * pcell = (i+1) + (bx+2) ((j+1) + (by+2)(k+1)) for local cell (i, j, k) in
 * [-1, bx] x [-1, by] x [-1, bz]: a one-cell ghost layer.
 * Record fields: 0-2 V (r, theta, phi components), 3-5 b = B/|B| (same),
 * 6 div V, 7 bb:grad V, 8 div b, 9 b . (dV/dt + (V . grad)V), 10-12
 * (b . grad) b (spherical components). */
#define FTE_RECORD_STRIDE 10
#define FTE_RECORD_STRIDE_KPERP 13
#define FTE_RECORD_FIELDS 13

/* Particle state buffer layout for capacity n_max: arrays of n_max entries
 * in this order: x, y, z, mu, lnp (ln of p / (m c)), w (all double), pid
 * (uint64), kinj (uint32), status (int32), run (uint16), each array starting
 * on a 256-byte boundary.  Tangent buffer layout: 13 double
 * arrays of n_max entries, in the order of fte_read_tangents. */

fte_status fte_create(fte_ctx **out, const fte_params *p);
void fte_destroy(fte_ctx *ctx);
const char *fte_last_error(const fte_ctx *ctx);

/* Buffer sizes for a grid and a particle capacity n_max (no device work). */
fte_status fte_query_sizes(const fte_params *p, const fte_grid_desc *g, uint64_t n_max, fte_sizes *out);

/* Attach the grid description (validated: tiling, 2:1 nesting, block shape)
 * and the caller's device buffers.  Resets particles and histograms. */
fte_status fte_bind_buffers(fte_ctx *ctx, const fte_grid_desc *g, uint64_t n_max, const fte_buffers *b);

/* Load the wind snapshots (section 2.4): vb_sph is DEVICE memory holding
 * double [n_snap][n_leaves][cells][6] = V_r, V_theta, V_phi, B_r, B_theta,
 * B_phi at leaf cell centres, cells ordered xi fastest, then theta, then phi
 * (cell centres at the midpoints in xi, theta, phi).  Builds the block index,
 * fills the ghost layers by the block-boundary value rule, derives the fields
 * of Eqs. 2-4 (gradients by central differences), and writes the records.
 * vb_sph is only read during the call.  Synchronises `stream`.  Returns
 * FTE_EINVAL if the data hold non-finite values or |B| = 0. */
fte_status fte_load_grid(fte_ctx *ctx, const double *vb_sph, void *stream);

/* Snapshot streaming (section 2.4 notes that reading whole data sets is the
 * bottleneck; the lock-step clock needs two snapshots at a time): with
 * n_slots < n_snap the grid buffer holds n_slots snapshots, snapshot k in
 * slot k mod n_slots, and this call derives snapshot k into its slot (the
 * first call also uploads the index and clears counters and sums, like
 * fte_load_grid).  raw[0..4] are DEVICE arrays [n_leaves][cells][6] (layout
 * of fte_load_grid) of snapshots k-2 .. k+2; the time derivative reads k-1
 * and k+1 (k, k+1, k+2 at k = 0 and k-2, k-1, k at the last snapshot; the
 * other one of two), the rest may be NULL.  fte_step_n returns FTE_ERANGE
 * while a snapshot its steps interpolate from is not resident, and a region
 * injection needs the snapshots nearest its first steps.  Loading a slot
 * replaces the snapshot it held; on the stream the steps run on, that is
 * ordered after them.  Records are bit-identical to those of fte_load_grid.
 * Synchronises. */
fte_status fte_load_snapshot(fte_ctx *ctx, int k, const double *const raw[5], void *stream);

/* Loading only the blocks the particles can reach (section 4 names this as
 * the remedy for the cost of reading whole snapshots).  With n_pool > 0,
 * snapshot k is loaded in two calls: this one decides which leaves its slot
 * holds, then fte_load_snapshot derives them.  Snapshot k serves the steps
 * between snapshots k-1 and k+1; over the time from the current clock to
 * snapshot k+1 a particle moves at most (1.5 v_max + wind_speed_max) times
 * that time, v_max the speed of the fastest held particle or source (1.5 an
 * allowance for acceleration).  The level-1 blocks within that distance of a
 * level-1 block holding a held particle (active or not yet started) or
 * overlapping a source region (each fte_injection: radius r, or r .. r_hi
 * with region = 1, x [th_lo, th_hi] x [ph_lo, ph_hi], energies up to e_hi)
 * hold the gather's set C of leaves; C and the leaves the ghost layers of C
 * read (within three cells of the next coarser level) are held; those and
 * the leaves their own ghost fill reads are the leaves whose input the load
 * reads.  counts[0..2] receive the leaves of
 * the three sets; leaves_out (HOST, may be NULL) the ids of the last, in
 * increasing order, so that the caller copies only their blocks into the
 * raw arrays of fte_load_snapshot (other leaves of those arrays are not
 * read).  FTE_ENOMEM when more than n_pool leaves must be held; FTE_EINVAL
 * without a pool.  A step that still reaches a leaf outside C retires the
 * particle as FTE_PS_NUMERIC and raises bit 8 of fte_stats.device_flags.
 * Not combined with smoothing or ensembles.
 * Synchronises. */
fte_status fte_plan_snapshot(fte_ctx *ctx, int k, const fte_injection *sources, int n_sources, double wind_speed_max,
                             int32_t *leaves_out, uint64_t cap, uint64_t counts[3], void *stream);

/* Append n particles with pids first_pid .. first_pid+n-1 drawn from `inj`
 * (see fte_injection).  Requires a loaded grid.  FTE_ENOMEM if the state
 * capacity would be exceeded. */
fte_status fte_inject(fte_ctx *ctx, const fte_injection *inj, uint64_t n, uint64_t first_pid, void *stream);

/* Advance every held particle through the next n_steps global steps
 * (Euler-Maruyama, lock-step clock t_n = t0 + n dt).  A particle takes step n
 * only when n >= its kinj.  Observer sums are accumulated in the same pass.
 * Retired particles are removed periodically.  FTE_ERANGE if a time-dependent
 * grid does not cover t_n for every step. */
fte_status fte_step_n(fte_ctx *ctx, uint32_t n_steps, void *stream);

/* Intensities j[o][e][t] = S / (4 pi dV dT dE W_inj) and their standard errors
 * from the n_batch batch sums, o running over the observer bins (n_obs_bins =
 * the sum of the observers' n_phi), written to HOST arrays of n_obs_bins*n_e*n_t doubles
 * (either may be NULL); for an ensemble [run][o][e][t] with each run's own
 * W_inj.  reset != 0 clears the sums afterwards.  Synchronises. */
fte_status fte_bin_observers(fte_ctx *ctx, double *j, double *sigma, int reset, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): fte_bin_observers with
 * the finalize output staged in a fixed device array the library holds
 * (2 x FTE_STATIC_BINS doubles, 4 MiB, on every GPU it runs on, until the
 * process ends) instead of the context's work buffer; same results and
 * arguments.  Allocates nothing.  FTE_EINVAL when the context has more than
 * FTE_STATIC_BINS observer bins (n_obs_bins * n_e * n_t, times the runs of
 * an ensemble).  Calls on one GPU share that array: calls that overlap in
 * time on one GPU (from several threads or streams) race.  Synchronises. */
#define FTE_STATIC_BINS 262144
fte_status fte_bin_observers_static(fte_ctx *ctx, double *j, double *sigma, int reset, void *stream);

/* Steady state of a Green's-function run (all particles started at one
 * time; section 2.3): the time integral of the intensity, J[o][e] =
 * sum_t S[o][e][t] / (4 pi dV dE W_inj), i.e. the intensity for a constant
 * injection of unit weight per unit time, and its standard error from the
 * batch sums; HOST arrays of n_obs_bins*n_e ([run][o][e] for an ensemble),
 * either may be NULL.  Synchronises. */
fte_status fte_bin_steady(fte_ctx *ctx, double *J, double *sigma, void *stream);

/* Raw batch sums S[o][e][t][batch] (host array of n_obs*n_e*n_t*n_batch;
 * [run][o][e][t][batch] for an ensemble) and the injected weight (host array
 * of max(n_runs, 1): per run).  Synchronises. */
fte_status fte_read_hist(fte_ctx *ctx, double *sums, double *w_injected, void *stream);

fte_status fte_get_stats(fte_ctx *ctx, fte_stats *out, void *stream);

/* Copy the held particles to HOST arrays of at least n_live entries (any may
 * be NULL); x3 is [n][3].  *n_out receives n_live.  Order is the storage
 * order (not pid order).  Synchronises. */
fte_status fte_read_particles(fte_ctx *ctx, double *x3, double *mu, double *lnp, double *w, uint64_t *pid,
                              uint32_t *kinj, int32_t *status, uint64_t cap, uint64_t *n_out, void *stream);

/* Smoothed intensities J (HOST array of n_obs*n_e*n_t; needs sigma_x > 0)
 * and, in gradient mode, their derivatives dJ (HOST array
 * [3][n_obs*n_e*n_t]) with respect to (lambda_ref, kperp_ratio, gamma_inj),
 * the last including the change of W_inj.  The derivatives are pathwise:
 * a hard absorption and the 6-width cut of the kernels are treated as fixed
 * events.
 * The kperp_ratio derivative is 0 unless kperp_ratio > 0.  Either array may
 * be NULL.  Synchronises. */
fte_status fte_bin_smoothed(fte_ctx *ctx, double *J, double *dJ, void *stream);

/* Gradient of a loss L(J) with respect to (lambda_ref, kperp_ratio,
 * gamma_inj): grad[k] = sum over bins of dL_dJ[bin] dJ[k][bin], contracted
 * on the device (gradient mode).  dL_dJ is a HOST array of n_obs*n_e*n_t;
 * grad a HOST array of 3.  Synchronises. */
fte_status fte_grad(fte_ctx *ctx, const double *dL_dJ, double grad[3], void *stream);

/* Tangents of the held particles (gradient mode), storage order as
 * fte_read_particles: HOST array [n_live][11] = dx, dy, dz, dmu, dlnp with
 * respect to lambda_ref, the same five with respect to kperp_ratio, and
 * d ln w / d gamma_inj.  cap is the row capacity of tan (FTE_ENOMEM if
 * below n_live); *n_out receives n_live.  Synchronises. */
fte_status fte_read_tangents(fte_ctx *ctx, double *tan, uint64_t cap, uint64_t *n_out, void *stream);

/* Checkpoint / resume.  A state blob holds the held particles (and tangents
 * in gradient mode), the global step, the device counters, the observer sums
 * and the smoothed sums; not the grid, which the resuming context loads
 * itself.  fte_state_size gives the blob size for the current state
 * (synchronises).  fte_save_state writes it to a HOST buffer of `bytes`
 * (FTE_ENOMEM if too small).  fte_load_state restores it into a context
 * with the same parameters (checked by a fingerprint of the parameters that
 * shape the trajectories and sums), the same grid shape and capacity >= the
 * saved particle count, after fte_load_grid; FTE_EINVAL on a mismatch or a
 * damaged blob.  Stepping on from a restored state gives the trajectories of
 * an uninterrupted run (they depend only on pid and step). */
fte_status fte_state_size(fte_ctx *ctx, uint64_t *bytes, void *stream);
fte_status fte_save_state(fte_ctx *ctx, void *host_blob, uint64_t bytes, void *stream);
fte_status fte_load_state(fte_ctx *ctx, const void *host_blob, uint64_t bytes, void *stream);

/* Drop all particles, observer sums, counters and timings and rewind the
 * global clock to step 0; the loaded grid stays.  Synchronises. */
fte_status fte_reset(fte_ctx *ctx, void *stream);

/* Record a HIP event pair around every step-kernel launch (on the stream the
 * launch uses); fte_get_stats then reports their summed duration. */
fte_status fte_set_timing(fte_ctx *ctx, int enable);

/* Launch shape: threads per block (64..256, multiple of 64), steps per
 * kernel launch, removal of retired particles every `compact_every` steps (a
 * multiple of steps_per_launch; 0 = never), and whether that removal also
 * regroups the live particles by leaf and cube of cells so that a wavefront
 * gathers from neighbouring records: spatial_sort 0 keeps the storage order,
 * 1, 2, 3 sort by cubes of 1, 2, 4 cells per edge.  Defaults 256 / 64 / 64 / 1. */
fte_status fte_set_launch(fte_ctx *ctx, int block, int steps_per_launch, int compact_every, int spatial_sort);

/* LDS record tile of the float (FTE_MIXED) step kernels on time-dependent
 * grids: each workgroup stages whole padded k-layers of one leaf for both
 * live snapshots in LDS, as many as tile_bytes holds (at least two layers,
 * else no tile), and reads the corners that lie in it from LDS instead of
 * through the cache.  Values, weights and summation order are those of the
 * global gather, so trajectories do not depend on it.  tile_bytes caps the
 * tile; the kernel also keeps it within the LDS that leaves two workgroups
 * per compute unit (three on a steady grid).  0 turns it off; default and
 * largest FTE_MAX_TILE_BYTES.  FTE_EINVAL outside 0..max. */
#define FTE_MAX_TILE_BYTES 131072
fte_status fte_set_record_tile(fte_ctx *ctx, int tile_bytes);

/* LDS-privatised observer histogram (where the residence-time sums behind
 * section 2.3's intensities accumulate): the observer time bins a step
 * launch can touch (its first to last post-step time) are accumulated in LDS when
 * their sums fit hist_bytes, and flushed with one global atomic per nonzero
 * bin at the end of the launch; otherwise every contribution is a global
 * atomic.  Counts are the same either way, sums equal up to the order of the
 * additions; the LDS it takes is no longer available to the record tile.
 * 0 (the default) keeps the sums in global memory.  FTE_EINVAL outside
 * 0..FTE_MAX_LDS_HIST_BYTES. */
#define FTE_MAX_LDS_HIST_BYTES 32768
fte_status fte_set_lds_histogram(fte_ctx *ctx, int hist_bytes);

/* Launch graphs for ensembles and repeated runs (a launch mechanism, not an
 * operation of the method): record what a sequence of fte_inject and
 * fte_step_n calls
 * enqueues on one stream as one HIP graph, then run it with a single launch
 * instead of one launch per kernel.
 *
 * fte_capture_begin starts a stream capture on `stream` (it first settles
 * the live count of the last compaction, which the recording cannot read
 * back).  Until fte_capture_end only fte_inject and fte_step_n may be called
 * on the context (the others return FTE_ESTATE); they validate their
 * arguments as usual and record their kernels without running them, with
 * launches sized by the particles injected so far (the recording skips the
 * live-count read-back and the per-launch timing events).  fte_capture_end
 * ends the capture on the same stream, instantiates the graph, returns it in
 * *out (owned by the caller, freed by fte_graph_destroy) and puts the
 * context back in the state it had at fte_capture_begin: nothing has run.
 * FTE_EDEVICE if HIP rejects the capture or the instantiation.
 *
 * fte_graph_launch runs the graph on `stream`.  The context must be at the
 * global step, particle buffer and compaction phase the recording began at
 * (checked, FTE_ESTATE otherwise), and its device state must be the one the
 * recording began from (not checked: e.g. record after fte_reset and launch
 * after another fte_reset).  The grid, launch shape and record tile are
 * those of the recording.  Afterwards the context is where the recorded
 * calls leave it.  Trajectories and sums are those of the same calls made
 * directly (the kernels are the same; only the launch sizes differ).
 * A graph refers to its context's buffers: destroy it before the context. */
typedef struct fte_graph fte_graph;
fte_status fte_capture_begin(fte_ctx *ctx, void *stream);
fte_status fte_capture_end(fte_ctx *ctx, void *stream, fte_graph **out);
fte_status fte_graph_launch(fte_ctx *ctx, fte_graph *graph, void *stream);
void fte_graph_destroy(fte_graph *graph);

/* Self-tuning of the launch shape: from the current state, run trial_steps
 * global steps under each candidate (block size x compaction interval, steps
 * per launch fixed), timing the step and compaction kernels with HIP events,
 * restoring the state (held in host memory) after each trial; then keep the
 * fastest and report it in best[0..2] = block, steps_per_launch,
 * compact_every (host array).  The run continues from the restored state, so
 * results do not depend on the tuning.  Synchronises. */
fte_status fte_autotune(fte_ctx *ctx, uint32_t trial_steps, int best[3], void *stream);

#ifdef __cplusplus
}
#endif
#endif
