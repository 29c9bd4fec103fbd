// Internal types shared by the host side of the library and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fte.h"

namespace fte {

constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr int kNF = FTE_RECORD_FIELDS;
constexpr int kRSPlain = FTE_RECORD_STRIDE;       // fields 0-9
constexpr int kRSKperp = FTE_RECORD_STRIDE_KPERP; // fields 0-12
// Smoothing kernels are dropped beyond this many widths, where a Gaussian has
// fallen to 1.5e-8 of its peak: the jump at the cut then adds no visible
// boundary term to the derivatives taken along trajectories.
constexpr double kKernelCut = 6.0;

// One run of an ensemble as the kernels see it.
struct DevRun {
    double lambda_ref, kperp_ratio;
    uint64_t step_end;       // first global step the run does not take
    int run_id;              // Philox run id
    int pad;
};

// Device-side copy of the run parameters, pre-digested on the host.
struct DevParams {
    double mass_c2;          // m c^2, J
    double dt, t0, r_in, r_out;
    double r_in2, r_out2;    // squared absorbing radii
    double lambda_ref, inv_p_ref, alpha;
    double q, eps, mu_floor;
    double dmm_scale;        // A = dmm_scale * v / lambda_par
    double kperp_ratio, lambda_perp;
    double e_min_ln, inv_dlne;   // ln(e_min), 1 / dlne
    double e_min, dlne, dT;
    double t_ref, inv_dT;
    double obs[FTE_MAX_OBS][6];  // r1, r2, th1, th2, phi centre of bin 0, bin width phi
    double obs_omega[FTE_MAX_OBS];   // rotation of each observer's pattern
    double obs_rsq[FTE_MAX_OBS][2];  // squared radial edges r1^2, r2^2
    int obs_nphi[FTE_MAX_OBS];       // longitude bins per observer
    double obs_u[6];                 // union of the observer boxes: r1, r2, r1^2, r2^2, th1, th2
    int obs_off[FTE_MAX_OBS];        // its first observer bin
    int n_obs_bins;
    // kernel-smoothed intensities (smooth != 0)
    double obs_xyz[FTE_MAX_OBS][3];  // observer centres, Cartesian
    double sx_cut2;          // (kKernelCut sigma_x)^2
    double inv_2sx2, inv_sx2, norm3;   // 1/(2 sx^2), 1/sx^2, (2 pi)^-3/2 sx^-3
    double sl_cut, inv_2sl2, inv_sl2, norm1;  // kKernelCut sl, 1/(2 sl^2), 1/sl^2, (2 pi)^-1/2 / sl
    double sig_t;            // time-kernel width
    double inv_lambda_ref, inv_kperp_ratio;   // explicit parameter derivatives
    long long win_lo;        // first global step of the smoothing window
    long long n_win;         // steps in the window
    int smooth, grad, nk;    // nk = sums per (step, observer, energy): 4 with grad, else 1
    const DevRun *runs;      // ensemble table (device), n_runs entries
    int n_runs;              // 0: single run
    int n_runs_eff;          // max(n_runs, 1): leading dimension of the sums
    int kperp_any;           // some run has kappa_perp: 13-field records, KPERP kernels
    double kink_norm, kink_inv_2s2;   // tangents: 2 / (sqrt(2 pi) s), 1 / (2 s^2) (0: off)
    int kink_bridge;                  // tangents: the bridge occupation at mu = 0 instead
    uint64_t seed;
    int dmm_model;
    int run_id;
    int n_obs, n_e, n_t, n_batch;
};

// Block-AMR grid as the kernels see it.
struct DevGrid {
    double r_lo, inv_dxi, th_lo, inv_dth, ph_lo, inv_dph;
    double inv_r_lo;
    double dxi, dth, dph;        // level-1 widths
    double th_hi;                // upper colatitude edge
    double t_s0, inv_dt_s, dt_s;
    int xi_map, periodic;
    int n1[3], bx[3], px[3];     // level-1 cells, block cells, padded block cells
    uint32_t bx_mag[3];          // ceil(2^32 / bx): c / bx as the high word of c * bx_mag
    int nb1[3];                  // level-1 blocks per dimension
    int n_levels, n_leaves, n_snap, n_base, n_child;
    int n_slots;                 // snapshot record slots held (snapshot k in slot k mod n_slots)
    int pcells;                  // padded cells per block
    int cells;                   // interior cells per block
    const int32_t *base;         // [nb1 product] node codes (>=0 leaf, <0 -(group+1))
    const int32_t *child;        // [n_groups][8] node codes
    const int32_t *leaf_info;    // [n_leaves][4] level, I, J, K
    const void *rec;             // records [slot][block][pcell][rs]
    int rs, nf;                  // record stride and stored fields (10/10 or 14/13)
    // Record blocks per slot: n_leaves (block = leaf id) or, when a subset of
    // leaves is streamed, the pool size n_pool with pool_map[slot][leaf] =
    // the leaf's block in that slot's pool (>= 0: resident and valid for the
    // gather; -2 - block: held only as a neighbour for the ghost fill; -1:
    // not held).  pool_map is NULL when every leaf is held.
    int n_blk;
    const int32_t *pool_map;
};

// Pool block of a leaf in a slot (any held block, also a neighbour-only one),
// or -1.
__host__ __device__ inline int pool_block(const DevGrid &g, int slot, int leaf) {
    if (!g.pool_map) return leaf;
    const int v = g.pool_map[(size_t)slot * g.n_leaves + leaf];
    return v >= 0 ? v : (v <= -2 ? -2 - v : -1);
}

// Particle state (struct of arrays, capacity n_max).
struct DevState {
    double *x, *y, *z, *mu, *lnp, *w;
    uint64_t *pid;
    uint32_t *kinj;
    int32_t *status;
    uint16_t *run;
};

// Tangent state of the gradient mode (struct of arrays, capacity n_max): 11
// double arrays of `stride` entries from `base`: d(x, y, z, mu, lnp)/d lambda_ref,
// the same with respect to kperp_ratio, and d ln w / d gamma_inj.
struct DevTan {
    double *base;
    uint64_t stride;
    __host__ __device__ double *col(int q) const { return base + (uint64_t)q * stride; }
};
enum : int { kTanLnw = 10, kTanCols = 11 };

// LDS plan of a step launch: observer time bins [it_lo, it_lo + n_tb) can be
// accumulated in LDS (histograms up to a budget, FTE_LDS_HIST_BYTES by
// default, fte_set_lds_histogram at run time; n_tb = 0: straight to the
// global histogram).  Off by default: observer hits are rare enough
// that the global atomics cost nothing measurable, and the record tile makes
// better use of the LDS (a fourth k-layer on the CIR workload, +3.5%).  The
// block index can be staged in LDS too (tables up to FTE_LDS_INDEX_BYTES); on
// the CIR workload its 10 KB stay resident in L1/L2 and staging cost 0.5%, so
// it is off unless the limit is raised at build time.
//
// Record tile: the float step kernels (histogram, smoothed and tangent
// modes, single runs and ensembles, with or without cross-field records)
// stage, per workgroup, whole padded k-layers of one leaf in LDS, for both
// live snapshots of a time-dependent grid or the one of a steady grid (as
// many as fit the budget, at least two; the budget is the LDS that leaves
// two workgroups per CU, three for the steady-grid kernels, capped by
// FTE_LDS_TILE_BYTES; 0 turns it off; fte_set_record_tile sets the cap at run
// time), anchored at the workgroup's middle particle (an odd number of
// layers centred on its cell); corners that lie in it are read from LDS, the
// others through the L1.  After the spatial sort a workgroup's particles sit
// in few k-layers of one leaf, and LDS serves such divergent reads several
// times faster than the L1.
struct StepLds {
    int it_lo, n_tb;
    int tile_layers;  // padded k-layers in the tile (0: no tile)
    int tile_off;     // byte offset of the tile in the dynamic LDS
};
#ifndef FTE_LDS_HIST_BYTES
#define FTE_LDS_HIST_BYTES 0
#endif
#ifndef FTE_LDS_INDEX_BYTES
#define FTE_LDS_INDEX_BYTES 0
#endif
#ifndef FTE_LDS_TILE_BYTES
#define FTE_LDS_TILE_BYTES 131072
#endif
constexpr size_t kLdsHistBytes = FTE_LDS_HIST_BYTES;
constexpr size_t kLdsTileBytes = FTE_LDS_TILE_BYTES;
constexpr size_t kLdsIndexBytes = FTE_LDS_INDEX_BYTES;

// Device counters (live in the work buffer).
struct DevCounters {
    unsigned long long n_live[2];
    unsigned long long steps;
    unsigned long long injected;
    unsigned long long retired[6];
    double w_retired[6];
    unsigned int flags;
    unsigned int pad;
    double w_inj[FTE_MAX_RUNS * FTE_MAX_BATCH];   // [run][batch]
    double w_inj_dgamma;     // sum of w d ln w / d gamma_inj
};

enum : unsigned int { kFlagAmrDepth = 1u, kFlagBadInput = 2u, kFlagNoLeaf = 4u, kFlagNotResident = 8u };

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

DevState state_view(void *base, uint64_t n_max);
size_t state_bytes(uint64_t n_max);
DevTan tangent_view(void *base, uint64_t n_max);
size_t tangent_bytes(uint64_t n_max);

// Kernel launchers (fte_kernels.hip).
// Raw input of snapshot k and its neighbours k-2 .. k+2 (NULL outside the
// run or where not needed), each a device array [leaf][cell][6] of double.
struct RawWin {
    const double *s[5];
    int k;
};
// A list of leaves the load kernels work on (NULL: every leaf).
struct LeafList {
    const int32_t *ids;
    int n;
};
hipError_t launch_raw_ghost(const DevGrid &g, const RawWin &w, double *work_cart, DevCounters *cnt, LeafList ll,
                            hipStream_t s);
hipError_t launch_derive(const DevGrid &g, const RawWin &w, const double *work_cart, void *rec, int fp32, LeafList ll,
                         hipStream_t s);
hipError_t launch_record_ghost(const DevGrid &g, int snap, void *rec, int fp32, DevCounters *cnt, LeafList ll,
                               hipStream_t s);
hipError_t launch_check_raw(const DevGrid &g, const double *raw, size_t n_snaps, DevCounters *cnt, hipStream_t s);
hipError_t launch_check_raw_leaves(const DevGrid &g, const double *raw, DevCounters *cnt, LeafList ll, hipStream_t s);
// Level-1 blocks that hold a live particle (occ[base block] = 1) and the
// largest ln p among them (as the ordered bits of a float in *lnp_bits).
hipError_t launch_occupancy(const DevGrid &g, DevState st, const DevCounters *cnt, int slot, uint64_t n_upper,
                            uint32_t *occ, uint32_t *lnp_bits, hipStream_t s);
hipError_t launch_inject(const DevParams &p, const DevGrid &g, int rec_fp32, const fte_injection &inj, DevState st,
                         DevTan tn, DevCounters *cnt, int slot, uint64_t n, uint64_t first_pid, hipStream_t s);
hipError_t launch_add_live(DevCounters *cnt, int slot, uint64_t n, hipStream_t s);
hipError_t launch_step(const DevParams &p, const DevGrid &g, DevState st, DevTan tn, DevCounters *cnt, int slot,
                       double *hist, double *sm, uint64_t n0, uint32_t n_steps, uint64_t n_upper, int block, int fp32,
                       size_t tile_bytes, size_t hist_bytes, hipStream_t s);
hipError_t launch_compact(DevState src, DevState dst, DevTan tsrc, DevTan tdst, DevCounters *cnt, int from,
                          uint64_t n_upper, int block, hipStream_t s);
hipError_t launch_zero_live(DevCounters *cnt, int slot, hipStream_t s);
// Key space of the spatial sort: (leaf >> leaf_shift, cube of 2^cube_shift
// cells per edge), n_keys keys, h[] cubes per block axis.
struct SortShape {
    int cube_shift, leaf_shift;
    int h[3];
    uint32_t n_sub, n_keys;
};
SortShape sort_shape_for(const DevGrid &g, int sort, uint64_t max_keys);
hipError_t launch_compact_sorted(const DevGrid &g, const SortShape &K, DevState src, DevState dst, DevTan tsrc,
                                 DevTan tdst, DevCounters *cnt, int from, uint64_t n_upper, uint32_t *keys,
                                 uint32_t *counts, uint32_t *tsum, hipStream_t s);
hipError_t launch_finalize(const DevParams &p, const double *hist, const DevCounters *cnt, double *j, double *sig,
                           hipStream_t s);
hipError_t launch_finalize_steady(const DevParams &p, const double *hist, const DevCounters *cnt, double *j,
                                  double *sig, hipStream_t s);
hipError_t launch_smooth_finalize(const DevParams &p, const double *sm, double *out, hipStream_t s);
hipError_t launch_grad_contract(const DevParams &p, const double *fin, const double *dl, double *out4, hipStream_t s);
hipError_t launch_zero(double *p, uint64_t n, hipStream_t s);
hipError_t launch_zero_counters(DevCounters *cnt, hipStream_t s);

}  // namespace fte
