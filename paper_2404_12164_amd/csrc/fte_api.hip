// Host side of the C ABI declared in include/fte.h: argument and grid
// validation, the block-AMR index, buffer carving, and the ordering of the
// kernel launches on the caller's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fte.h"
#include "fte_internal.hpp"

using namespace fte;

// Host-side stepping state that a recorded graph starts from and leaves.
struct HostClock {
    uint64_t global_step, since_compact, n_upper, injected_since;
    int cur;
};

struct fte_ctx {
    fte_params p{};
    std::vector<fte_run> runs;     // copy of the ensemble table
    DevParams dp{};
    bool bound = false, loaded = false, index_ready = false;
    std::vector<int> slot_snap;    // snapshot resident in each record slot (-1: none)
    // streamed subset of leaves (n_pool > 0): the plan of each slot
    struct SlotPlan {
        int snap = -1;
        std::vector<int32_t> map;          // [leaf]: pool block, -2 - block (neighbour only) or -1
        std::vector<int32_t> held, gather; // leaves held (pool order) and those the gather may read
        std::vector<int32_t> input;        // leaves whose input the load reads
    };
    std::vector<SlotPlan> plans;
    int32_t *d_lists = nullptr;    // device: held, gather and input lists of the load in progress
    double *scratch = nullptr;     // this device's copy of the static finalize scratch
    uint32_t *d_occ = nullptr;     // device: level-1 block occupancy + the largest ln p (last entry)
    fte_grid_desc g{};
    std::vector<int32_t> leaves, base, child, info;
    DevGrid dg{};
    uint64_t n_max = 0;
    fte_buffers b{};
    DevState st[2]{};
    DevTan tn[2]{};
    int cur = 0;
    DevCounters *cnt = nullptr;
    double *fin_j = nullptr, *fin_s = nullptr, *cart = nullptr;
    double *sm = nullptr, *fin_sm = nullptr, *dl = nullptr, *out4 = nullptr;
    uint64_t sm_n = 0;
    uint32_t *keys = nullptr, *counts = nullptr, *tsum = nullptr;
    uint32_t n_keys = 0;
    int sort = 1;
    uint64_t hist_n = 0;
    uint64_t n_upper = 0, injected_since = 0;
    unsigned long long *pinned = nullptr;
    hipEvent_t ev = nullptr;
    bool pending = false;
    uint64_t global_step = 0;
    // the launch shape measured best on every workload (CIR, ensemble autotuner,
    // largest, paper): 256 threads, 64 steps per launch, a per-cell sort every 64
    int block = 256, spl = 64, compact_every = 64;
    size_t tile_bytes = kLdsTileBytes;   // LDS record tile budget of the float step kernels
    size_t hist_bytes = kLdsHistBytes;   // LDS observer-histogram budget of the step kernels
    uint64_t since_compact = 0;
    bool timing = false;
    std::vector<hipEvent_t> tev;   // pairs: start, stop of each timed launch
    size_t tev_used = 0;
    double timed_ms = 0.0;
    uint32_t timed_launches = 0;
    // launch-graph recording (fte_capture_begin .. fte_capture_end)
    bool capturing = false;
    hipStream_t cap_stream = nullptr;
    HostClock graph_start{};
    std::string err;
};

struct fte_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    fte_ctx *ctx = nullptr;
    HostClock start{}, end{};
};

namespace {

fte_status fail(fte_ctx *c, fte_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

// Entry points that synchronise or read back refuse to run while a launch
// graph is being recorded (only fte_inject and fte_step_n are recorded).
#define NO_CAPTURE(ctx)                                                                            \
    do {                                                                                           \
        if ((ctx)->capturing)                                                                      \
            return fail(ctx, FTE_ESTATE, "only fte_inject and fte_step_n may run while recording a graph"); \
    } while (0)

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(ctx, FTE_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

int runs_eff(const fte_params *p) { return p->n_runs > 0 ? p->n_runs : 1; }

int obs_nphi(const fte_observer &o) { return o.n_phi > 1 ? o.n_phi : 1; }

int obs_bins(const fte_params *p) {
    int n = 0;
    for (int o = 0; o < p->n_obs; ++o) n += obs_nphi(p->obs[o]);
    return n;
}

// kappa_perp terms (and the 13-field records) are needed when any run has them
bool needs_kperp(const fte_params *p) {
    if (p->kperp_ratio > 0.0 || p->lambda_perp > 0.0) return true;
    for (int r = 0; r < p->n_runs; ++r)
        if (p->runs[r].kperp_ratio > 0.0) return true;
    return false;
}

// Global steps whose post-step time t0 + (n+1) dt can lie within the time
// kernel's cut of
// a time-bin centre (padded by a step on each side; the read-out applies the
// exact cut).
void smooth_window(const fte_params *p, long long *lo, long long *n) {
    const double cut = kKernelCut * p->sigma_t;
    const double t_lo = p->t_ref + 0.5 * p->dT - cut;
    const double t_hi = p->t_ref + ((double)p->n_t - 0.5) * p->dT + cut;
    double a = floor((t_lo - p->t0) / p->dt) - 2.0, b = floor((t_hi - p->t0) / p->dt) + 1.0;
    if (a < 0.0) a = 0.0;
    if (!(b >= a) || !isfinite(a) || !isfinite(b) || b - a > 1e12) {
        *lo = 0;
        *n = (isfinite(a) && isfinite(b) && b >= a) ? (long long)1e12 : 0;
        return;
    }
    *lo = (long long)a;
    *n = (long long)(b - a) + 1;
}

std::string check_params(const fte_params *p) {
    if (!p) return "params is NULL";
    if (!finite_pos(p->mass)) return "mass must be > 0";
    if (p->dmm_model < 0 || p->dmm_model > 2) return "unknown dmm_model";
    if (p->dmm_norm < 0 || p->dmm_norm > 1) return "dmm_norm must be 0 or 1";
    if (!finite_pos(p->lambda_ref)) return "lambda_ref must be > 0";
    if (p->alpha != 0.0 && !finite_pos(p->p_ref)) return "p_ref must be > 0 when alpha != 0";
    if (p->dmm_model == FTE_DMM_POWER_Q && !(p->q > 1.0 && p->q < 2.0)) return "power-law q must be in (1, 2)";
    if (p->dmm_model == FTE_DMM_POWER_Q && !finite_pos(p->mu_floor)) return "mu_floor must be > 0";
    if (p->dmm_model == FTE_DMM_EQ5 && !finite_pos(p->eps)) return "eps must be > 0 for Eq. 5";
    if (p->kperp_ratio < 0.0 || p->lambda_perp < 0.0) return "kappa_perp parameters must be >= 0";
    if (!finite_pos(p->dt)) return "dt must be > 0";
    if (!isfinite(p->t0)) return "t0 must be finite";
    if (!(p->r_in >= 0.0) || !(p->r_out > p->r_in)) return "need 0 <= r_in < r_out";
    if (p->run_id < 0 || p->run_id > 0xFFFF) return "run_id must fit 16 bits";
    if (p->precision != FTE_FP64 && p->precision != FTE_MIXED) return "unknown precision";
    if (p->n_obs < 0 || p->n_obs > FTE_MAX_OBS) return "n_obs out of range";
    if (p->n_batch < 1 || p->n_batch > FTE_MAX_BATCH) return "n_batch out of range";
    if (p->n_obs > 0) {
        if (!finite_pos(p->e_min) || !finite_pos(p->dlne) || p->n_e < 1) return "bad energy bins";
        if (!finite_pos(p->dT) || p->n_t < 1 || !isfinite(p->t_ref)) return "bad time bins";
        for (int o = 0; o < p->n_obs; ++o) {
            const fte_observer &ob = p->obs[o];
            if (!finite_pos(ob.r) || !finite_pos(ob.dr) || !finite_pos(ob.dtheta) || !finite_pos(ob.dphi) ||
                ob.dr >= 2 * ob.r || !isfinite(ob.theta) || !isfinite(ob.phi) || ob.dphi > 2 * kPi)
                return "bad observer box";
            if (ob.n_phi < 0 || ob.n_phi > 100000 || !isfinite(ob.omega)) return "bad observer ring";
            if ((ob.n_phi > 1 || ob.omega != 0.0) && p->sigma_x > 0.0)
                return "smoothed intensities need box observers (n_phi <= 1, omega = 0)";
        }
        if ((double)obs_bins(p) * p->n_e * p->n_t * p->n_batch * runs_eff(p) > 2e9) return "too many observer bins";
    }
    if (p->n_runs < 0 || p->n_runs > FTE_MAX_RUNS) return "n_runs out of range";
    if (p->n_runs > 0) {
        if (!p->runs) return "runs is NULL";
        if (p->run_id + p->n_runs - 1 > 0xFFFF) return "run ids must fit 16 bits";
        if (p->sigma_x > 0.0 || p->grad) return "ensembles do not combine with smoothed intensities";
        for (int r = 0; r < p->n_runs; ++r) {
            const fte_run &u = p->runs[r];
            if (!finite_pos(u.lambda_ref)) return "run lambda_ref must be > 0";
            if (!(u.kperp_ratio >= 0.0) || !isfinite(u.kperp_ratio)) return "run kperp_ratio must be >= 0";
            if (u.n_steps < 1 || u.n_steps >= (1ull << 48)) return "run n_steps out of range";
        }
    }
    if (!(p->sigma_x >= 0.0) || !isfinite(p->sigma_x)) return "sigma_x must be >= 0";
    if (!isfinite(p->kink_sigma)) return "kink_sigma must be finite";
    if (p->grad != 0 && p->grad != 1) return "grad must be 0 or 1";
    if (p->grad && !(p->sigma_x > 0.0)) return "the gradient needs the smoothed intensities (sigma_x > 0)";
    if (p->sigma_x > 0.0) {
        if (p->n_obs < 1) return "smoothed intensities need observers";
        if (!finite_pos(p->sigma_lne) || !finite_pos(p->sigma_t)) return "sigma_lne and sigma_t must be > 0";
        long long lo, n;
        smooth_window(p, &lo, &n);
        if ((double)n * p->n_obs * p->n_e * (p->grad ? 4 : 1) > 4e9) return "smoothing window too large";
    }
    return "";
}

// Build the block index from the leaf list and check that the leaves tile the
// domain and obey the 2:1 nesting rule.
std::string build_index(const fte_grid_desc *g, std::vector<int32_t> &base, std::vector<int32_t> &child,
                        std::vector<int32_t> &info) {
    if (!g) return "grid description is NULL";
    if (g->xi_map != 0 && g->xi_map != 1) return "xi_map must be 0 or 1";
    if (!finite_pos(g->r_lo) || !finite_pos(g->dxi) || !finite_pos(g->dth) || !finite_pos(g->dph))
        return "grid origin and widths must be > 0";
    if (g->n_levels < 1 || g->n_levels > FTE_MAX_LEVELS) return "n_levels out of range";
    for (int a = 0; a < 3; ++a) {
        if (g->bx[a] < 4 || (g->bx[a] & 1) || g->bx[a] > 64) return "block cells must be even, 4 .. 64";
        if (g->n_levels >= 3 && (g->bx[a] & 3)) return "block cells must be divisible by 4 with >= 3 levels";
        if (g->n1[a] < g->bx[a] || g->n1[a] % g->bx[a]) return "n1 must be a positive multiple of bx";
        if ((long)g->n1[a] << (g->n_levels - 1) > (1L << 26)) return "grid too fine";
    }
    if (!(g->th_lo >= 0.0) || !(g->th_lo + g->n1[1] * g->dth <= kPi + 1e-12)) return "colatitude range outside [0, pi]";
    if (g->phi_periodic && fabs(g->n1[2] * g->dph - 2 * kPi) > 1e-9) return "periodic phi must span 2 pi";
    if (g->n_snap < 1) return "n_snap must be >= 1";
    if (g->n_slots < 0 || g->n_slots == 1 || (g->n_slots > 0 && g->n_slots < g->n_snap && g->n_snap < 3))
        return "n_slots must be 0, >= 2, and streaming needs n_snap >= 3";
    if (g->n_snap >= 2 && !finite_pos(g->dt_s)) return "dt_s must be > 0";
    if (g->n_leaves < 1 || !g->leaves) return "no leaves";
    if (g->n_pool < 0 || g->n_pool > g->n_leaves) return "n_pool must be 0 .. n_leaves";
    if (g->n_pool > 0 && !(g->n_slots > 0 && g->n_slots < g->n_snap)) return "n_pool needs a snapshot ring (n_slots < n_snap)";
    const int nb1[3] = {g->n1[0] / g->bx[0], g->n1[1] / g->bx[1], g->n1[2] / g->bx[2]};
    const long nbase = (long)nb1[0] * nb1[1] * nb1[2];
    const int32_t EMPTY = INT_MIN;
    base.assign(nbase, EMPTY);
    child.clear();
    info.assign((size_t)g->n_leaves * 4, 0);
    for (int l = 0; l < g->n_leaves; ++l) {
        const int32_t *e = g->leaves + 4 * l;
        const int L = e[0];
        if (L < 1 || L > g->n_levels) return "leaf level out of range";
        for (int a = 0; a < 3; ++a)
            if (e[1 + a] < 0 || e[1 + a] >= (nb1[a] << (L - 1))) return "leaf block index out of range";
        for (int a = 0; a < 4; ++a) info[4 * l + a] = e[a];
        const int B0 = e[1] >> (L - 1), B1 = e[2] >> (L - 1), B2 = e[3] >> (L - 1);
        // slot = (which table, index): child may grow, so no pointers into it
        bool in_child = false;
        size_t at = B0 + (size_t)nb1[0] * (B1 + (size_t)nb1[1] * B2);
        for (int m = 1; m < L; ++m) {
            int32_t v = in_child ? child[at] : base[at];
            if (v >= 0) return "leaves overlap (a leaf covers a refined region)";
            if (v == EMPTY) {
                const int grp = (int)(child.size() / 8);
                child.insert(child.end(), 8, EMPTY);
                v = -(grp + 1);
                (in_child ? child[at] : base[at]) = v;
            }
            const int grp = -v - 1;
            const int sh = L - (m + 1);
            const int s = ((e[1] >> sh) & 1) | (((e[2] >> sh) & 1) << 1) | (((e[3] >> sh) & 1) << 2);
            in_child = true;
            at = (size_t)grp * 8 + s;
        }
        int32_t &slot = in_child ? child[at] : base[at];
        if (slot != EMPTY) return "leaves overlap";
        slot = l;
    }
    for (auto v : base)
        if (v == EMPTY) return "leaves do not cover the domain";
    for (auto v : child)
        if (v == EMPTY) return "leaves do not cover the domain";
    // 2:1 nesting across faces, edges and corners
    for (int l = 0; l < g->n_leaves; ++l) {
        const int32_t *e = g->leaves + 4 * l;
        const int L = e[0];
        if (L < 3) continue;
        const int nb[3] = {nb1[0] << (L - 1), nb1[1] << (L - 1), nb1[2] << (L - 1)};
        for (int dI = -1; dI <= 1; ++dI)
            for (int dJ = -1; dJ <= 1; ++dJ)
                for (int dK = -1; dK <= 1; ++dK) {
                    int q[3] = {e[1] + dI, e[2] + dJ, e[3] + dK};
                    if (q[0] < 0 || q[0] >= nb[0] || q[1] < 0 || q[1] >= nb[1]) continue;
                    if (q[2] < 0 || q[2] >= nb[2]) {
                        if (!g->phi_periodic) continue;
                        q[2] = (q[2] + nb[2]) % nb[2];
                    }
                    int32_t node = base[(q[0] >> (L - 1)) + (long)nb1[0] * ((q[1] >> (L - 1)) +
                                                                            (long)nb1[1] * (q[2] >> (L - 1)))];
                    int m = 1;
                    while (node < 0 && m < L) {
                        ++m;
                        const int sh = L - m;
                        const int s = ((q[0] >> sh) & 1) | (((q[1] >> sh) & 1) << 1) | (((q[2] >> sh) & 1) << 2);
                        node = child[(size_t)(-node - 1) * 8 + s];
                    }
                    if (node >= 0 && m < L - 1) return "2:1 nesting violated between neighbouring blocks";
                }
    }
    return "";
}

size_t rec_elem(const fte_params *p) { return p->precision == FTE_FP64 ? 8 : 4; }

int slots_of(const fte_grid_desc *g) { return (g->n_slots <= 0 || g->n_slots >= g->n_snap) ? g->n_snap : g->n_slots; }

struct Layout {
    size_t grid, index, state, hist, work, tangent;
    size_t off_child, off_info, off_map;
    size_t off_lists, off_occ;
    size_t off_j, off_s, off_cart, off_keys, off_counts, off_tsum;
    size_t off_sm, off_fin_sm, off_dl, off_out4, sm_n, off_runs;
    uint32_t n_keys;
    int pcells;
    int rs;
};

// Most keys of the spatial sort for a live-particle bound n: four per
// particle (at least 2^16, at most 2^31), so that a compaction's work is
// O(particles) whatever the grid's cell count.
uint64_t sort_key_bound(uint64_t n) { return std::min<uint64_t>(std::max<uint64_t>(4 * n, 1ull << 16), 1ull << 31); }

Layout layout(const fte_params *p, const fte_grid_desc *g, uint64_t n_max, size_t n_base, size_t n_child) {
    Layout L{};
    L.pcells = (g->bx[0] + 2) * (g->bx[1] + 2) * (g->bx[2] + 2);
    L.rs = needs_kperp(p) ? kRSKperp : kRSPlain;
    const size_t n_blk = g->n_pool > 0 ? (size_t)g->n_pool : (size_t)g->n_leaves;
    L.grid = (size_t)slots_of(g) * n_blk * L.pcells * L.rs * rec_elem(p);
    L.off_child = align256(n_base * 4);
    L.off_info = L.off_child + align256(std::max<size_t>(n_child, 8) * 4);
    L.off_map = L.off_info + align256((size_t)g->n_leaves * 16);
    L.index = L.off_map + (g->n_pool > 0 ? align256((size_t)slots_of(g) * g->n_leaves * 4) : 0);
    L.state = state_bytes(n_max);
    const size_t nbins = (size_t)p->n_obs * p->n_e * p->n_t;          // smoothed (box observers)
    const size_t nbr = (size_t)obs_bins(p) * p->n_e * p->n_t * runs_eff(p);
    L.hist = std::max<size_t>(nbr * p->n_batch * 8, 256);
    L.off_runs = align256(sizeof(DevCounters));
    L.off_j = L.off_runs + align256(FTE_MAX_RUNS * sizeof(DevRun));
    L.off_s = L.off_j + align256(std::max<size_t>(nbr, 1) * 8);
    L.off_cart = L.off_s + align256(std::max<size_t>(nbr, 1) * 8);
    L.off_keys = L.off_cart + align256((size_t)g->n_leaves * L.pcells * 6 * 8);
    // sort keys: the finest key space (one per leaf cell), bounded by the
    // particle capacity (see sort_key_bound)
    L.n_keys = (uint32_t)std::min<uint64_t>((uint64_t)g->n_leaves * g->bx[0] * g->bx[1] * g->bx[2],
                                            sort_key_bound(n_max));
    L.off_counts = L.off_keys + align256(n_max * 4);
    L.off_tsum = L.off_counts + align256(((size_t)L.n_keys + 1) * 4);
    L.off_sm = L.off_tsum + align256(((size_t)L.n_keys / 4096 + 2) * 4);
    L.sm_n = 0;
    if (p->sigma_x > 0.0) {
        long long lo, nw;
        smooth_window(p, &lo, &nw);
        L.sm_n = (size_t)nw * p->n_obs * p->n_e * (p->grad ? 4 : 1);
    }
    L.off_fin_sm = L.off_sm + align256(L.sm_n * 8);
    L.off_dl = L.off_fin_sm + align256(p->sigma_x > 0.0 ? 4 * nbins * 8 : 0);
    L.off_out4 = L.off_dl + align256(p->sigma_x > 0.0 ? nbins * 8 : 0);
    L.off_lists = L.off_out4 + 256;
    L.off_occ = L.off_lists + (g->n_pool > 0 ? align256((size_t)3 * g->n_leaves * 4) : 0);
    L.work = L.off_occ + (g->n_pool > 0 ? align256((n_base + 1) * 4) : 0);
    L.tangent = p->grad ? tangent_bytes(n_max) : 0;
    return L;
}

void make_devparams(const fte_params *p, DevParams *d) {
    memset(d, 0, sizeof(*d));
    d->mass_c2 = p->mass * kC * kC;
    d->dt = p->dt;
    d->t0 = p->t0;
    d->r_in = p->r_in;
    d->r_out = p->r_out;
    d->r_in2 = p->r_in * p->r_in;
    d->r_out2 = p->r_out * p->r_out;
    d->lambda_ref = p->lambda_ref;
    d->inv_p_ref = p->alpha != 0.0 ? 1.0 / p->p_ref : 1.0;
    d->alpha = p->alpha;
    d->q = p->q;
    d->eps = p->eps;
    d->mu_floor = p->mu_floor;
    // scale of D_mumu: A = dmm_scale * v / lambda_par
    double I;
    if (p->dmm_model == FTE_DMM_ISO) {
        I = 4.0 / 3.0;
    } else if (p->dmm_model == FTE_DMM_EQ5) {
        // I = 2 Int_0^1 (1-m)(1+m)^2 / ((1+eps) m + eps) dm in closed form:
        // substitute s = (1+eps) m + eps and integrate the resulting cubic / s
        const double a = 1.0 + p->eps, b = p->eps;
        // N(m) = 1 + m - m^2 - m^3 with m = (s - b)/a
        // coefficients of N as a polynomial in s
        const double ia = 1.0 / a;
        const double c3 = -ia * ia * ia;
        const double c2 = -ia * ia + 3.0 * b * ia * ia * ia;
        const double c1 = ia + 2.0 * b * ia * ia - 3.0 * b * b * ia * ia * ia;
        const double c0 = 1.0 - b * ia - b * b * ia * ia + b * b * b * ia * ia * ia;
        const double s0 = b, s1 = a + b;
        const double integ = c3 * (s1 * s1 * s1 - s0 * s0 * s0) / 3.0 + c2 * (s1 * s1 - s0 * s0) / 2.0 +
                             c1 * (s1 - s0) + c0 * log(s1 / s0);
        I = 2.0 * integ / a;
    } else {
        I = 4.0 / ((2.0 - p->q) * (4.0 - p->q));
    }
    d->dmm_scale = p->dmm_norm == 1 ? 1.0 : 3.0 * I / 8.0;
    d->kperp_ratio = p->kperp_ratio;
    d->lambda_perp = p->lambda_perp;
    d->e_min = p->e_min;
    d->dlne = p->dlne;
    d->dT = p->dT;
    d->e_min_ln = p->n_obs > 0 ? log(p->e_min) : 0.0;
    d->inv_dlne = p->n_obs > 0 ? 1.0 / p->dlne : 0.0;
    d->t_ref = p->t_ref;
    d->inv_dT = p->n_obs > 0 ? 1.0 / p->dT : 0.0;
    for (int o = 0; o < p->n_obs; ++o) {
        const fte_observer &ob = p->obs[o];
        d->obs[o][0] = ob.r - 0.5 * ob.dr;
        d->obs[o][1] = ob.r + 0.5 * ob.dr;
        d->obs_rsq[o][0] = d->obs[o][0] * d->obs[o][0];
        d->obs_rsq[o][1] = d->obs[o][1] * d->obs[o][1];
        d->obs[o][2] = ob.theta - 0.5 * ob.dtheta;
        d->obs[o][3] = ob.theta + 0.5 * ob.dtheta;
        d->obs[o][4] = ob.phi;
        d->obs[o][5] = ob.dphi;
        d->obs_nphi[o] = obs_nphi(ob);
        d->obs_omega[o] = ob.omega;
        d->obs_off[o] = d->n_obs_bins;
        d->n_obs_bins += d->obs_nphi[o];
    }
    // the smallest radial x colatitude box holding every observer box (a
    // particle outside it is in none)
    d->obs_u[0] = d->obs_u[2] = d->obs_u[4] = HUGE_VAL;
    d->obs_u[1] = d->obs_u[3] = d->obs_u[5] = -HUGE_VAL;
    for (int o = 0; o < p->n_obs; ++o) {
        d->obs_u[0] = std::min(d->obs_u[0], d->obs[o][0]);
        d->obs_u[1] = std::max(d->obs_u[1], d->obs[o][1]);
        d->obs_u[2] = std::min(d->obs_u[2], d->obs_rsq[o][0]);
        d->obs_u[3] = std::max(d->obs_u[3], d->obs_rsq[o][1]);
        d->obs_u[4] = std::min(d->obs_u[4], d->obs[o][2]);
        d->obs_u[5] = std::max(d->obs_u[5], d->obs[o][3]);
    }
    d->seed = p->seed;
    d->dmm_model = p->dmm_model;
    d->run_id = p->run_id;
    d->n_obs = p->n_obs;
    d->n_e = p->n_obs > 0 ? p->n_e : 1;
    d->n_t = p->n_obs > 0 ? p->n_t : 1;
    d->n_batch = p->n_batch;
    d->n_runs = p->n_runs;
    d->n_runs_eff = runs_eff(p);
    d->kperp_any = needs_kperp(p) ? 1 : 0;
    if (p->grad && p->dmm_model == FTE_DMM_EQ5 && p->kink_sigma > 0.0) {
        d->kink_norm = 2.0 / (sqrt(2.0 * kPi) * p->kink_sigma);
        d->kink_inv_2s2 = 1.0 / (2.0 * p->kink_sigma * p->kink_sigma);
    }
    if (p->grad && p->dmm_model == FTE_DMM_EQ5 && p->kink_sigma < 0.0) d->kink_bridge = 1;
    // kernel-smoothed intensities
    if (p->sigma_x > 0.0) {
        d->smooth = 1;
        d->grad = p->grad;
        d->nk = p->grad ? 4 : 1;
        for (int o = 0; o < p->n_obs; ++o) {
            const fte_observer &ob = p->obs[o];
            d->obs_xyz[o][0] = ob.r * sin(ob.theta) * cos(ob.phi);
            d->obs_xyz[o][1] = ob.r * sin(ob.theta) * sin(ob.phi);
            d->obs_xyz[o][2] = ob.r * cos(ob.theta);
        }
        const double sx = p->sigma_x, sl = p->sigma_lne;
        d->sx_cut2 = kKernelCut * kKernelCut * sx * sx;
        d->inv_2sx2 = 1.0 / (2.0 * sx * sx);
        d->inv_sx2 = 1.0 / (sx * sx);
        d->norm3 = 1.0 / (pow(2.0 * kPi, 1.5) * sx * sx * sx);
        d->sl_cut = kKernelCut * sl;
        d->inv_2sl2 = 1.0 / (2.0 * sl * sl);
        d->inv_sl2 = 1.0 / (sl * sl);
        d->norm1 = 1.0 / (sqrt(2.0 * kPi) * sl);
        d->sig_t = p->sigma_t;
        d->inv_lambda_ref = 1.0 / p->lambda_ref;
        d->inv_kperp_ratio = p->kperp_ratio > 0.0 ? 1.0 / p->kperp_ratio : 0.0;
        smooth_window(p, &d->win_lo, &d->n_win);
    }
}

}  // namespace

namespace fte {

size_t state_bytes(uint64_t n) {
    return 6 * align256(n * 8) + align256(n * 8) + align256(n * 4) + align256(n * 4) + align256(n * 2);
}

size_t tangent_bytes(uint64_t n) { return kTanCols * align256(n * 8); }

DevTan tangent_view(void *base, uint64_t n) {
    DevTan t{};
    t.base = (double *)base;
    t.stride = align256(n * 8) / 8;
    return t;
}

DevState state_view(void *base, uint64_t n) {
    char *c = (char *)base;
    DevState s;
    const size_t a8 = align256(n * 8), a4 = align256(n * 4);
    s.x = (double *)c;
    s.y = (double *)(c + a8);
    s.z = (double *)(c + 2 * a8);
    s.mu = (double *)(c + 3 * a8);
    s.lnp = (double *)(c + 4 * a8);
    s.w = (double *)(c + 5 * a8);
    s.pid = (uint64_t *)(c + 6 * a8);
    s.kinj = (uint32_t *)(c + 7 * a8);
    s.status = (int32_t *)(c + 7 * a8 + a4);
    s.run = (uint16_t *)(c + 7 * a8 + 2 * a4);
    return s;
}

}  // namespace fte

// Scratch of fte_bin_observers_static: the finalize kernel's output (j, then
// sigma) staged on the device before the copy to the caller's host arrays,
// in a file-scope array instead of the caller's work buffer.  Every GPU the
// library runs on holds its own copy until the process ends; its address on
// each device is looked up once, with that device current, and kept.
static __device__ __align__(256) double scratch[2 * FTE_STATIC_BINS];

namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch_of;   // by device id (nullptr: not looked up yet)

// The current device's address of `scratch` (looked up on first use).
hipError_t scratch_address(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_of.size() <= dev) g_scratch_of.resize(dev + 1, nullptr);
    if (!g_scratch_of[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_of[dev] = (double *)ptr;
    }
    *out = g_scratch_of[dev];
    return hipSuccess;
}
}  // namespace

extern "C" {

fte_status fte_create(fte_ctx **out, const fte_params *p) {
    if (!out) return FTE_EINVAL;
    *out = nullptr;
    const std::string e = check_params(p);
    if (!e.empty()) return FTE_EINVAL;
    fte_ctx *c = new (std::nothrow) fte_ctx();
    if (!c) return FTE_ENOMEM;
    c->p = *p;
    if (p->n_runs > 0) {
        c->runs.assign(p->runs, p->runs + p->n_runs);
        c->p.runs = c->runs.data();
    } else {
        c->p.runs = nullptr;
    }
    make_devparams(&c->p, &c->dp);
    if (hipHostMalloc((void **)&c->pinned, sizeof(unsigned long long)) != hipSuccess) {
        delete c;
        return FTE_EDEVICE;
    }
    if (hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(c->pinned);
        delete c;
        return FTE_EDEVICE;
    }
    if (scratch_address(&c->scratch) != hipSuccess) {
        (void)hipEventDestroy(c->ev);
        (void)hipHostFree(c->pinned);
        delete c;
        return FTE_EDEVICE;
    }
    *out = c;
    return FTE_OK;
}

void fte_destroy(fte_ctx *c) {
    if (!c) return;
    if (c->capturing) {
        // an unfinished recording: end it so that its stream is usable again
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    }
    if (c->ev) (void)hipEventDestroy(c->ev);
    for (auto e : c->tev) (void)hipEventDestroy(e);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
}

const char *fte_last_error(const fte_ctx *c) { return c ? c->err.c_str() : "null context"; }

fte_status fte_query_sizes(const fte_params *p, const fte_grid_desc *g, uint64_t n_max, fte_sizes *out) {
    if (!out) return FTE_EINVAL;
    if (!check_params(p).empty()) return FTE_EINVAL;
    std::vector<int32_t> base, child, info;
    if (!build_index(g, base, child, info).empty()) return FTE_EINVAL;
    const Layout L = layout(p, g, n_max, base.size(), child.size());
    out->grid_bytes = L.grid;
    out->index_bytes = L.index;
    out->state_bytes = L.state;
    out->hist_bytes = L.hist;
    out->work_bytes = L.work;
    out->tangent_bytes = L.tangent;
    return FTE_OK;
}

fte_status fte_bind_buffers(fte_ctx *c, const fte_grid_desc *g, uint64_t n_max, const fte_buffers *b) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!b) return fail(c, FTE_EINVAL, "buffers is NULL");
    std::vector<int32_t> base, child, info;
    const std::string e = build_index(g, base, child, info);
    if (!e.empty()) return fail(c, FTE_EINVAL, e);
    if (n_max == 0 || n_max > (1ull << 40)) return fail(c, FTE_EINVAL, "n_max out of range");
    const void *ptrs[6] = {b->grid, b->index, b->state_a, b->state_b, b->hist, b->work};
    for (int k = 0; k < 6; ++k)
        if (!ptrs[k] || ((uintptr_t)ptrs[k] & 255)) return fail(c, FTE_EINVAL, "buffers must be non-NULL, 256-byte aligned");
    if (c->p.grad && (!b->tangent_a || !b->tangent_b || ((uintptr_t)b->tangent_a & 255) ||
                      ((uintptr_t)b->tangent_b & 255)))
        return fail(c, FTE_EINVAL, "gradient mode needs 256-byte aligned tangent buffers");
    if (g->n_pool > 0 && (c->p.sigma_x > 0.0 || c->p.n_runs > 0))
        return fail(c, FTE_EINVAL, "a streamed subset (n_pool) is not combined with smoothing or ensembles");
    const Layout L = layout(&c->p, g, n_max, base.size(), child.size());
    c->g = *g;
    c->leaves.assign(g->leaves, g->leaves + 4 * (size_t)g->n_leaves);
    c->g.leaves = c->leaves.data();
    c->base.swap(base);
    c->child.swap(child);
    c->info.swap(info);
    c->n_max = n_max;
    c->b = *b;
    c->st[0] = state_view(b->state_a, n_max);
    c->st[1] = state_view(b->state_b, n_max);
    c->tn[0] = c->p.grad ? tangent_view(b->tangent_a, n_max) : DevTan{};
    c->tn[1] = c->p.grad ? tangent_view(b->tangent_b, n_max) : DevTan{};
    c->cur = 0;
    char *w = (char *)b->work;
    c->cnt = (DevCounters *)w;
    c->fin_j = (double *)(w + L.off_j);
    c->fin_s = (double *)(w + L.off_s);
    c->cart = (double *)(w + L.off_cart);
    c->keys = (uint32_t *)(w + L.off_keys);
    c->counts = (uint32_t *)(w + L.off_counts);
    c->tsum = (uint32_t *)(w + L.off_tsum);
    c->n_keys = L.n_keys;
    c->sm = (double *)(w + L.off_sm);
    c->sm_n = L.sm_n;
    c->fin_sm = (double *)(w + L.off_fin_sm);
    c->dl = (double *)(w + L.off_dl);
    c->out4 = (double *)(w + L.off_out4);
    c->hist_n = (uint64_t)obs_bins(&c->p) * c->p.n_e * c->p.n_t * c->p.n_batch * runs_eff(&c->p);
    c->dp.runs = (const DevRun *)(w + L.off_runs);

    DevGrid &d = c->dg;
    memset(&d, 0, sizeof(d));
    d.r_lo = g->r_lo;
    d.dxi = g->dxi;
    d.dth = g->dth;
    d.dph = g->dph;
    d.inv_dxi = 1.0 / g->dxi;
    d.inv_r_lo = 1.0 / g->r_lo;
    d.th_lo = g->th_lo;
    d.inv_dth = 1.0 / g->dth;
    d.ph_lo = g->ph_lo;
    d.inv_dph = 1.0 / g->dph;
    d.th_hi = g->th_lo + g->n1[1] * g->dth;
    d.t_s0 = g->t_s0;
    d.dt_s = g->n_snap >= 2 ? g->dt_s : 1.0;
    d.inv_dt_s = 1.0 / d.dt_s;
    d.xi_map = g->xi_map;
    d.periodic = g->phi_periodic;
    for (int a = 0; a < 3; ++a) {
        d.n1[a] = g->n1[a];
        d.bx[a] = g->bx[a];
        d.px[a] = g->bx[a] + 2;
        d.nb1[a] = g->n1[a] / g->bx[a];
        d.bx_mag[a] = (uint32_t)((0x100000000ull + g->bx[a] - 1) / g->bx[a]);
    }
    d.n_levels = g->n_levels;
    d.n_leaves = g->n_leaves;
    d.n_snap = g->n_snap;
    d.n_slots = slots_of(g);
    d.n_base = (int)c->base.size();
    d.n_child = (int)c->child.size();
    d.pcells = L.pcells;
    d.cells = g->bx[0] * g->bx[1] * g->bx[2];
    char *ix = (char *)b->index;
    d.base = (const int32_t *)ix;
    d.child = (const int32_t *)(ix + L.off_child);
    d.leaf_info = (const int32_t *)(ix + L.off_info);
    d.rec = b->grid;
    d.rs = L.rs;
    d.nf = L.rs == kRSKperp ? kNF : 10;
    d.n_blk = g->n_pool > 0 ? g->n_pool : g->n_leaves;
    d.pool_map = g->n_pool > 0 ? (const int32_t *)(ix + L.off_map) : nullptr;
    c->plans.assign(g->n_pool > 0 ? d.n_slots : 0, fte_ctx::SlotPlan{});
    c->d_lists = g->n_pool > 0 ? (int32_t *)(w + L.off_lists) : nullptr;
    c->d_occ = g->n_pool > 0 ? (uint32_t *)(w + L.off_occ) : nullptr;
    c->bound = true;
    c->loaded = false;
    c->index_ready = false;
    c->slot_snap.assign(d.n_slots, -1);
    c->global_step = 0;
    c->n_upper = 0;
    c->injected_since = 0;
    c->pending = false;
    c->since_compact = 0;
    c->err.clear();
    return FTE_OK;
}

// Index upload, counters and sums cleared, ensemble table: the start of a run.
static fte_status setup_grid(fte_ctx *c, hipStream_t s) {
    const DevGrid &d = c->dg;
    char *ix = (char *)c->b.index;
    HIPCHK(c, hipMemcpyAsync(ix, c->base.data(), c->base.size() * 4, hipMemcpyHostToDevice, s));
    if (!c->child.empty())
        HIPCHK(c, hipMemcpyAsync((void *)d.child, c->child.data(), c->child.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync((void *)d.leaf_info, c->info.data(), c->info.size() * 4, hipMemcpyHostToDevice, s));
    if (d.pool_map) {
        // no leaf held in any slot until its snapshot is loaded
        c->plans.assign(d.n_slots, fte_ctx::SlotPlan{});
        std::vector<int32_t> none((size_t)d.n_slots * d.n_leaves, -1);
        HIPCHK(c, hipMemcpyAsync((void *)d.pool_map, none.data(), none.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    HIPCHK(c, launch_zero_counters(c->cnt, s));
    if (c->hist_n) HIPCHK(c, launch_zero((double *)c->b.hist, c->hist_n, s));
    if (c->sm_n) HIPCHK(c, launch_zero(c->sm, c->sm_n, s));
    if (c->p.n_runs > 0) {
        std::vector<DevRun> dr(c->p.n_runs);
        for (int r = 0; r < c->p.n_runs; ++r) {
            dr[r].lambda_ref = c->runs[r].lambda_ref;
            dr[r].kperp_ratio = c->runs[r].kperp_ratio;
            dr[r].step_end = c->runs[r].n_steps;
            dr[r].run_id = c->p.run_id + r;
            dr[r].pad = 0;
        }
        HIPCHK(c, hipMemcpyAsync((void *)c->dp.runs, dr.data(), dr.size() * sizeof(DevRun), hipMemcpyHostToDevice, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    c->cur = 0;
    c->n_upper = 0;
    c->injected_since = 0;
    c->pending = false;
    c->global_step = 0;
    c->since_compact = 0;
    for (auto &v : c->slot_snap) v = -1;
    c->index_ready = true;
    return FTE_OK;
}

// Ghost fill, derived fields and record ghost fill of snapshot w.k into its slot.
static fte_status derive_snapshot(fte_ctx *c, const RawWin &w, hipStream_t s, LeafList held = LeafList{nullptr, 0},
                                  LeafList gath = LeafList{nullptr, 0}) {
    const DevGrid &d = c->dg;
    const int fp32 = c->p.precision == FTE_MIXED;
    HIPCHK(c, launch_raw_ghost(d, w, c->cart, c->cnt, held, s));
    HIPCHK(c, launch_derive(d, w, c->cart, c->b.grid, fp32, held, s));
    HIPCHK(c, launch_record_ghost(d, w.k % d.n_slots, c->b.grid, fp32, c->cnt, gath, s));
    return FTE_OK;
}

// Device flags raised while checking or deriving input; clears them.
static fte_status input_flags(fte_ctx *c, hipStream_t s) {
    unsigned int flags = 0;
    HIPCHK(c, hipMemcpyAsync(&flags, &c->cnt->flags, sizeof(flags), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (flags & (kFlagBadInput | kFlagAmrDepth | kFlagNotResident)) {
        HIPCHK(c, launch_zero_counters(c->cnt, s));
        HIPCHK(c, hipStreamSynchronize(s));
        c->loaded = false;
        c->index_ready = false;
        if (flags & kFlagBadInput) return fail(c, FTE_EINVAL, "wind data hold non-finite values or |B| = 0");
        if (flags & kFlagNotResident) return fail(c, FTE_EINVAL, "the ghost rule read a leaf the pool does not hold");
        return fail(c, FTE_EINVAL, "block-boundary rule needed more than one coarser level");
    }
    return FTE_OK;
}

// Snapshots the window needs for the time derivative of snapshot k.
static bool window_needs(int ns, int k, int j) {
    if (j == k) return true;
    if (ns == 2) return true;
    if (ns < 2) return false;
    if (k == 0) return j == 1 || j == 2;
    if (k == ns - 1) return j == ns - 2 || j == ns - 3;
    return j == k - 1 || j == k + 1;
}

fte_status fte_load_grid(fte_ctx *c, const double *vb, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->bound) return fail(c, FTE_ESTATE, "bind buffers before loading the grid");
    if (!vb) return fail(c, FTE_EINVAL, "wind data is NULL");
    const DevGrid &d = c->dg;
    if (d.n_slots < d.n_snap) return fail(c, FTE_ESTATE, "a streaming grid is loaded with fte_load_snapshot");
    hipStream_t s = (hipStream_t)stream;
    fte_status r = setup_grid(c, s);
    if (r != FTE_OK) return r;
    HIPCHK(c, launch_check_raw(d, vb, (size_t)d.n_snap, c->cnt, s));
    const size_t per = (size_t)d.n_leaves * d.cells * 6;
    for (int k = 0; k < d.n_snap; ++k) {
        RawWin w{};
        w.k = k;
        for (int i = 0; i < 5; ++i) {
            const int j = k - 2 + i;
            w.s[i] = (j >= 0 && j < d.n_snap) ? vb + (size_t)j * per : nullptr;
        }
        r = derive_snapshot(c, w, s);
        if (r != FTE_OK) return r;
        c->slot_snap[k] = k;
    }
    r = input_flags(c, s);
    if (r != FTE_OK) return r;
    c->loaded = true;
    return FTE_OK;
}

namespace {

// Cartesian bounding sphere of level-1 block (I, J, K): centre and radius
// from a 5 x 5 x 5 sample of the (xi, theta, phi) box, with 2% margin.
void block_sphere(const fte_grid_desc &g, int I, int J, int K, double c[3], double *rad) {
    double pts[125][3];
    int n = 0;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b)
            for (int e = 0; e < 5; ++e) {
                const double xi = (I + a / 4.0) * g.bx[0] * g.dxi;
                const double r = g.xi_map ? g.r_lo * exp(xi) : g.r_lo + xi;
                const double th = g.th_lo + (J + b / 4.0) * g.bx[1] * g.dth;
                const double ph = g.ph_lo + (K + e / 4.0) * g.bx[2] * g.dph;
                pts[n][0] = r * sin(th) * cos(ph);
                pts[n][1] = r * sin(th) * sin(ph);
                pts[n][2] = r * cos(th);
                ++n;
            }
    c[0] = c[1] = c[2] = 0.0;
    for (int q = 0; q < n; ++q)
        for (int a = 0; a < 3; ++a) c[a] += pts[q][a] / n;
    double m = 0.0;
    for (int q = 0; q < n; ++q) {
        const double dx = pts[q][0] - c[0], dy = pts[q][1] - c[1], dz = pts[q][2] - c[2];
        m = std::max(m, sqrt(dx * dx + dy * dy + dz * dz));
    }
    *rad = 1.02 * m;
}

bool ranges_overlap(double a0, double a1, double b0, double b1) { return a0 <= b1 && a1 >= b0; }

}  // namespace

extern "C" {

fte_status fte_plan_snapshot(fte_ctx *c, int k, const fte_injection *sources, int n_sources, double wind_speed_max,
                             int32_t *leaves_out, uint64_t cap, uint64_t counts[3], void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->bound) return fail(c, FTE_ESTATE, "bind buffers before planning snapshots");
    const DevGrid &d = c->dg;
    if (!d.pool_map) return fail(c, FTE_EINVAL, "the grid holds every leaf (n_pool = 0): nothing to plan");
    if (k < 0 || k >= d.n_snap) return fail(c, FTE_EINVAL, "snapshot index out of range");
    if (n_sources < 0 || (n_sources > 0 && !sources)) return fail(c, FTE_EINVAL, "bad source list");
    if (!(wind_speed_max >= 0.0) || !isfinite(wind_speed_max)) return fail(c, FTE_EINVAL, "wind_speed_max must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (!c->index_ready) {
        fte_status r = setup_grid(c, s);
        if (r != FTE_OK) return r;
    }
    const fte_grid_desc &g = c->g;
    const int nb[3] = {d.nb1[0], d.nb1[1], d.nb1[2]};
    const int n_base = nb[0] * nb[1] * nb[2];
    // level-1 blocks holding a held particle, and the fastest of them
    std::vector<uint32_t> occ((size_t)n_base + 1, 0u);
    HIPCHK(c, hipMemcpyAsync(c->d_occ, occ.data(), occ.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, launch_occupancy(d, c->st[c->cur], c->cnt, c->cur, c->n_upper, c->d_occ, c->d_occ + n_base, s));
    HIPCHK(c, hipMemcpyAsync(occ.data(), c->d_occ, occ.size() * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double P_max = 0.0;
    if (occ[n_base]) {
        float pos;
        memcpy(&pos, &occ[n_base], 4);
        P_max = exp((double)pos - 80.0);
    }
    const double mc2 = c->p.mass * kC * kC;
    for (int q = 0; q < n_sources; ++q) {
        const double eps = sources[q].e_hi / mc2;
        if (eps > 0.0) P_max = std::max(P_max, sqrt(eps * (eps + 2.0)));
    }
    const double v_max = kC * P_max / sqrt(1.0 + P_max * P_max);
    // snapshot k serves the steps from snapshot k-1 to k+1
    const double t_end = d.t_s0 + std::min(k + 1, d.n_snap - 1) * d.dt_s;
    const double t_now = c->p.t0 + (double)c->global_step * c->p.dt;
    const double horizon = std::max(t_end - t_now, 0.0) + c->p.dt;
    const double reach = (std::min(1.5 * v_max, kC) + wind_speed_max) * horizon;
    // seeds: occupied blocks and blocks overlapping a source region
    std::vector<double> cen((size_t)n_base * 3), rad(n_base);
    std::vector<char> seed(n_base, 0);
    for (int K = 0; K < nb[2]; ++K)
        for (int J = 0; J < nb[1]; ++J)
            for (int I = 0; I < nb[0]; ++I) {
                const int b = I + nb[0] * (J + nb[1] * K);
                block_sphere(g, I, J, K, &cen[3 * (size_t)b], &rad[b]);
                if (occ[b]) seed[b] = 1;
                const double xi0 = I * g.bx[0] * g.dxi, xi1 = (I + 1) * g.bx[0] * g.dxi;
                const double r0 = g.xi_map ? g.r_lo * exp(xi0) : g.r_lo + xi0;
                const double r1 = g.xi_map ? g.r_lo * exp(xi1) : g.r_lo + xi1;
                const double t0 = g.th_lo + J * g.bx[1] * g.dth, t1 = t0 + g.bx[1] * g.dth;
                const double p0 = g.ph_lo + K * g.bx[2] * g.dph, p1 = p0 + g.bx[2] * g.dph;
                for (int q = 0; q < n_sources && !seed[b]; ++q) {
                    const fte_injection &src = sources[q];
                    const double ra = src.r, rb = src.region ? std::max(src.r_hi, src.r) : src.r;
                    if (!ranges_overlap(ra, rb, r0, r1) || !ranges_overlap(src.th_lo, src.th_hi, t0, t1)) continue;
                    bool ph_ok = src.ph_hi - src.ph_lo >= 2 * kPi;
                    for (double sh : {-2 * kPi, 0.0, 2 * kPi}) ph_ok |= ranges_overlap(src.ph_lo + sh, src.ph_hi + sh, p0, p1);
                    if (ph_ok) seed[b] = 1;
                }
            }
    std::vector<int> seeds;
    for (int b = 0; b < n_base; ++b)
        if (seed[b]) seeds.push_back(b);
    // blocks within reach of a seed (3: the gather set)
    std::vector<char> lvl(n_base, 0);
    for (int b = 0; b < n_base; ++b) {
        if (seed[b]) {
            lvl[b] = 3;
            continue;
        }
        for (int q : seeds) {
            const double dx = cen[3 * (size_t)b] - cen[3 * (size_t)q], dy = cen[3 * (size_t)b + 1] - cen[3 * (size_t)q + 1],
                         dz = cen[3 * (size_t)b + 2] - cen[3 * (size_t)q + 2];
            if (sqrt(dx * dx + dy * dy + dz * dz) <= reach + rad[b] + rad[q]) {
                lvl[b] = 3;
                break;
            }
        }
    }
    // Leaves: the gather set holds the leaves under the level-1 blocks in
    // reach.  The ghost layer of a level-L leaf reads virtual values at its
    // ghost cell centres, which at a coarser neighbour interpolate level-(L-1)
    // values up to 2.5 level-L cells outside the leaf: every leaf within 3
    // level-(L-1) cells (one level-1 cell for L = 1) must be held, and the
    // input of each held leaf's own ghost fill reads as far again.
    const int F = g.n_levels;
    const int nper = d.periodic ? d.n1[2] << (F - 1) : 0;   // finest phi cells of a periodic grid
    auto leaf_range = [&](int l, long lo[3], long hi[3], long *e) {
        const int32_t *q = &c->info[4 * (size_t)l];
        const int L = q[0];
        for (int a2 = 0; a2 < 3; ++a2) {
            const long w = (long)g.bx[a2] << (F - L);
            lo[a2] = (long)q[1 + a2] * w;
            hi[a2] = lo[a2] + w;
        }
        *e = L >= 2 ? 3L << (F - L + 1) : 1L << (F - 1);
    };
    auto near = [&](int la, int lb) {   // lb within la's reach
        long lo[3], hi[3], lo2[3], hi2[3], e, e2;
        leaf_range(la, lo, hi, &e);
        leaf_range(lb, lo2, hi2, &e2);
        for (int a2 = 0; a2 < 2; ++a2)
            if (!(lo[a2] - e < hi2[a2] && hi[a2] + e > lo2[a2])) return false;
        bool ok = lo[2] - e < hi2[2] && hi[2] + e > lo2[2];
        if (nper) ok = ok || (lo[2] - e < hi2[2] + nper && hi[2] + e > lo2[2] + nper) ||
                       (lo[2] - e < hi2[2] - nper && hi[2] + e > lo2[2] - nper);
        return ok;
    };
    std::vector<std::vector<int>> in_block(n_base);
    std::vector<int> anc(d.n_leaves);
    for (int l = 0; l < d.n_leaves; ++l) {
        const int32_t *e = &c->info[4 * (size_t)l];
        const int sh = e[0] - 1;
        anc[l] = (e[1] >> sh) + nb[0] * ((e[2] >> sh) + nb[1] * (e[3] >> sh));
        in_block[anc[l]].push_back(l);
    }
    // the leaves within reach of any leaf of `from`: candidates in the 27
    // level-1 blocks around each
    auto grow = [&](const std::vector<char> &from) {
        std::vector<char> out = from;
        for (int la = 0; la < d.n_leaves; ++la) {
            if (!from[la]) continue;
            const int b = anc[la];
            const int I = b % nb[0], J = (b / nb[0]) % nb[1], K = b / (nb[0] * nb[1]);
            for (int dk = -1; dk <= 1; ++dk)
                for (int dj = -1; dj <= 1; ++dj)
                    for (int di = -1; di <= 1; ++di) {
                        int i2 = I + di, j2 = J + dj, k2 = K + dk;
                        if (i2 < 0 || i2 >= nb[0] || j2 < 0 || j2 >= nb[1]) continue;
                        if (k2 < 0 || k2 >= nb[2]) {
                            if (!d.periodic) continue;
                            k2 = (k2 + nb[2]) % nb[2];
                        }
                        for (int lb : in_block[i2 + nb[0] * (j2 + nb[1] * k2)])
                            if (!out[lb] && near(la, lb)) out[lb] = 1;
                    }
        }
        return out;
    };
    std::vector<char> in_c(d.n_leaves, 0);
    for (int l = 0; l < d.n_leaves; ++l) in_c[l] = lvl[anc[l]] == 3;
    const std::vector<char> in_h = grow(in_c);
    const std::vector<char> in_i = grow(in_h);
    fte_ctx::SlotPlan pl;
    pl.snap = k;
    pl.map.assign(d.n_leaves, -1);
    for (int l = 0; l < d.n_leaves; ++l) {
        if (in_i[l]) pl.input.push_back(l);
        if (in_h[l]) {
            const int blk = (int)pl.held.size();
            pl.held.push_back(l);
            pl.map[l] = in_c[l] ? blk : -2 - blk;
            if (in_c[l]) pl.gather.push_back(l);
        }
    }
    if ((int)pl.held.size() > c->g.n_pool)
        return fail(c, FTE_ENOMEM, "the particles can reach " + std::to_string(pl.held.size()) +
                                       " leaves, more than n_pool = " + std::to_string(c->g.n_pool));
    if (leaves_out && cap < pl.input.size()) return fail(c, FTE_ENOMEM, "leaves_out holds fewer than the input leaves");
    if (counts) {
        counts[0] = pl.gather.size();
        counts[1] = pl.held.size();
        counts[2] = pl.input.size();
    }
    if (leaves_out) memcpy(leaves_out, pl.input.data(), pl.input.size() * 4);
    c->plans[k % d.n_slots] = std::move(pl);
    return FTE_OK;
}

}  // extern "C"

fte_status fte_load_snapshot(fte_ctx *c, int k, const double *const raw[5], void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->bound) return fail(c, FTE_ESTATE, "bind buffers before loading snapshots");
    if (!raw) return fail(c, FTE_EINVAL, "raw is NULL");
    const DevGrid &d = c->dg;
    if (k < 0 || k >= d.n_snap) return fail(c, FTE_EINVAL, "snapshot index out of range");
    RawWin w{};
    w.k = k;
    for (int i = 0; i < 5; ++i) {
        const int j = k - 2 + i;
        const bool need = j >= 0 && j < d.n_snap && window_needs(d.n_snap, k, j);
        if (need && !raw[i]) return fail(c, FTE_EINVAL, "a snapshot the time derivative needs is NULL");
        w.s[i] = need ? raw[i] : nullptr;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!c->index_ready) {
        fte_status r = setup_grid(c, s);
        if (r != FTE_OK) return r;
    }
    fte_status r;
    if (d.pool_map) {
        // a streamed subset: the slot holds the leaves its plan chose
        fte_ctx::SlotPlan &pl = c->plans[k % d.n_slots];
        if (pl.snap != k) return fail(c, FTE_ESTATE, "plan snapshot k (fte_plan_snapshot) before loading it");
        const int nh = (int)pl.held.size(), ng = (int)pl.gather.size(), ni = (int)pl.input.size();
        HIPCHK(c, hipMemcpyAsync((void *)(d.pool_map + (size_t)(k % d.n_slots) * d.n_leaves), pl.map.data(),
                                 pl.map.size() * 4, hipMemcpyHostToDevice, s));
        if (nh) HIPCHK(c, hipMemcpyAsync(c->d_lists, pl.held.data(), (size_t)nh * 4, hipMemcpyHostToDevice, s));
        if (ng) HIPCHK(c, hipMemcpyAsync(c->d_lists + nh, pl.gather.data(), (size_t)ng * 4, hipMemcpyHostToDevice, s));
        if (ni)
            HIPCHK(c, hipMemcpyAsync(c->d_lists + nh + ng, pl.input.data(), (size_t)ni * 4, hipMemcpyHostToDevice, s));
        HIPCHK(c, launch_check_raw_leaves(d, raw[2], c->cnt, LeafList{c->d_lists + nh + ng, ni}, s));
        r = derive_snapshot(c, w, s, LeafList{c->d_lists, nh}, LeafList{c->d_lists + nh, ng});
    } else {
        HIPCHK(c, launch_check_raw(d, raw[2], 1, c->cnt, s));
        r = derive_snapshot(c, w, s);
    }
    if (r != FTE_OK) return r;
    r = input_flags(c, s);
    if (r != FTE_OK) return r;
    c->slot_snap[k % d.n_slots] = k;
    c->loaded = true;
    return FTE_OK;
}

// Snapshots the steps n0 .. n0+n-1 interpolate from must be resident.
static bool steps_resident(const fte_ctx *c, uint64_t n0, uint64_t n) {
    const DevGrid &d = c->dg;
    if (d.n_snap < 2) return c->slot_snap[0] == 0;
    auto ks_of = [&](uint64_t step) {
        const double t = c->p.t0 + (double)step * c->p.dt;
        double kf = floor((t - d.t_s0) * d.inv_dt_s);
        kf = kf < 0.0 ? 0.0 : (kf > (double)(d.n_snap - 2) ? (double)(d.n_snap - 2) : kf);
        return (int)kf;
    };
    const int a = ks_of(n0), b = ks_of(n0 + n - 1);
    for (int k = a; k <= b + 1; ++k)
        if (c->slot_snap[k % d.n_slots] != k) return false;
    return true;
}

static fte_status refresh_exact(fte_ctx *c, hipStream_t s) {
    unsigned long long n = 0;
    HIPCHK(c, hipMemcpyAsync(&n, &c->cnt->n_live[c->cur], sizeof(n), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    c->n_upper = n;
    c->pending = false;
    c->injected_since = 0;
    return FTE_OK;
}

// Sum the durations of the recorded launch pairs (waits for them).
static fte_status drain_timing(fte_ctx *c, hipStream_t s) {
    if (c->tev.empty()) {
        c->tev.resize(512);
        for (auto &e : c->tev) HIPCHK(c, hipEventCreate(&e));
        c->tev_used = 0;
        return FTE_OK;
    }
    if (c->tev_used == 0) return FTE_OK;
    HIPCHK(c, hipStreamSynchronize(s));
    for (size_t k = 0; k + 1 < c->tev_used; k += 2) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->tev[k], c->tev[k + 1]));
        c->timed_ms += ms;
        c->timed_launches += 1;
    }
    c->tev_used = 0;
    return FTE_OK;
}

fte_status fte_inject(fte_ctx *c, const fte_injection *inj, uint64_t n, uint64_t first_pid, void *stream) {
    if (!c) return FTE_EINVAL;
    if (!c->loaded) return fail(c, FTE_ESTATE, "load the grid before injecting");
    if (!inj) return fail(c, FTE_EINVAL, "injection is NULL");
    if (!finite_pos(inj->r) || !finite_pos(inj->e_lo) || !(inj->e_hi >= inj->e_lo) || !isfinite(inj->e_hi) ||
        !isfinite(inj->th_lo) || !isfinite(inj->th_hi) || !isfinite(inj->ph_lo) || !isfinite(inj->ph_hi) ||
        !isfinite(inj->gamma_inj) || !isfinite(inj->w0) || inj->n_total < 1 ||
        (inj->r_weight && !finite_pos(inj->r_ref)))
        return fail(c, FTE_EINVAL, "bad injection description");
    if (first_pid + n < first_pid || first_pid + n > (1ull << 60)) return fail(c, FTE_EINVAL, "pid out of range");
    if (inj->n_inj_steps > 0 && (first_pid < inj->pid0 || first_pid + n > inj->pid0 + inj->n_total))
        return fail(c, FTE_EINVAL, "pids outside the injection's range");
    if (inj->run < 0 || inj->run >= runs_eff(&c->p)) return fail(c, FTE_EINVAL, "injection run out of range");
    if (inj->region != 0 && inj->region != 1) return fail(c, FTE_EINVAL, "region must be 0 or 1");
    if (inj->region && (!(inj->r_hi >= inj->r) || !isfinite(inj->r_hi) || !isfinite(inj->divv_max) ||
                        inj->max_tries < 1 || !(inj->ph_hi >= inj->ph_lo) || !(inj->th_hi >= inj->th_lo)))
        return fail(c, FTE_EINVAL, "bad injection region");
    if (inj->region && c->dg.n_slots < c->dg.n_snap) {
        // the snapshots nearest the first steps of these pids
        const DevGrid &d = c->dg;
        const uint64_t k_hi = inj->n_inj_steps > 0 ? (uint64_t)inj->k0 + inj->n_inj_steps : inj->k0;
        for (uint64_t step : {(uint64_t)inj->k0, k_hi}) {
            const double t = c->p.t0 + (double)step * c->p.dt;
            double f = floor((t - d.t_s0) / d.dt_s + 0.5);
            f = f < 0.0 ? 0.0 : (f > (double)(d.n_snap - 1) ? (double)(d.n_snap - 1) : f);
            if (c->slot_snap[(int)f % d.n_slots] != (int)f)
                return fail(c, FTE_ERANGE, "region injection needs a snapshot that is not resident");
        }
    }
    if (n == 0) return FTE_OK;
    hipStream_t s = (hipStream_t)stream;
    if (c->n_upper + n > c->n_max) {
        if (c->capturing) return fail(c, FTE_ENOMEM, "particle capacity exceeded (while recording, retired "
                                                     "particles are not subtracted)");
        fte_status r = refresh_exact(c, s);
        if (r != FTE_OK) return r;
        if (c->n_upper + n > c->n_max) return fail(c, FTE_ENOMEM, "particle capacity exceeded");
    }
    HIPCHK(c, launch_inject(c->dp, c->dg, c->p.precision == FTE_MIXED, *inj, c->st[c->cur], c->tn[c->cur], c->cnt,
                            c->cur, n, first_pid, s));
    HIPCHK(c, launch_add_live(c->cnt, c->cur, n, s));
    c->n_upper += n;
    c->injected_since += n;
    return FTE_OK;
}

fte_status fte_step_n(fte_ctx *c, uint32_t n_steps, void *stream) {
    if (!c) return FTE_EINVAL;
    if (!c->loaded) return fail(c, FTE_ESTATE, "load the grid before stepping");
    if (n_steps == 0) return FTE_OK;
    const uint64_t last = c->global_step + n_steps - 1;
    if (last >= (1ull << 48)) return fail(c, FTE_ERANGE, "global step index exceeds 48 bits");
    if (c->g.n_snap >= 2) {
        const double t_last = c->p.t0 + (double)last * c->p.dt;
        const double t_end = c->g.t_s0 + (c->g.n_snap - 1) * c->g.dt_s;
        const double t_first = c->p.t0 + (double)c->global_step * c->p.dt;
        if (t_last > t_end * (1 + 1e-15) + 1e-9 || t_first < c->g.t_s0 - 1e-9)
            return fail(c, FTE_ERANGE, "steps leave the snapshot time range");
    }
    if (!steps_resident(c, c->global_step, n_steps))
        return fail(c, FTE_ERANGE, "a snapshot these steps interpolate from is not resident");
    hipStream_t s = (hipStream_t)stream;
    uint32_t left = n_steps;
    while (left > 0) {
        if (c->pending && hipEventQuery(c->ev) == hipSuccess) {
            c->n_upper = *c->pinned + c->injected_since;
            c->pending = false;
        }
        const uint32_t chunk = left < (uint32_t)c->spl ? left : (uint32_t)c->spl;
        // (a recorded graph carries no timing events and no read-back of
        // the live count: its launches are sized by the injected total)
        const bool timed = c->timing && !c->capturing;
        if (timed) {
            if (c->tev_used + 2 > c->tev.size()) {
                fte_status r = drain_timing(c, s);
                if (r != FTE_OK) return r;
            }
            HIPCHK(c, hipEventRecord(c->tev[c->tev_used], s));
        }
        HIPCHK(c, launch_step(c->dp, c->dg, c->st[c->cur], c->tn[c->cur], c->cnt, c->cur, (double *)c->b.hist, c->sm,
                              c->global_step, chunk, c->n_upper, c->block, c->p.precision == FTE_MIXED, c->tile_bytes, c->hist_bytes, s));
        if (timed) {
            HIPCHK(c, hipEventRecord(c->tev[c->tev_used + 1], s));
            c->tev_used += 2;
        }
        c->global_step += chunk;
        left -= chunk;
        c->since_compact += chunk;
        if (c->compact_every > 0 && c->since_compact >= (uint64_t)c->compact_every) {
            const int to = 1 - c->cur;
            if (c->sort) {
                const SortShape K = sort_shape_for(c->dg, c->sort, std::min<uint64_t>(c->n_keys, sort_key_bound(c->n_upper)));
                HIPCHK(c, launch_compact_sorted(c->dg, K, c->st[c->cur], c->st[to], c->tn[c->cur], c->tn[to], c->cnt,
                                                c->cur, c->n_upper, c->keys, c->counts, c->tsum, s));
            } else {
                HIPCHK(c, launch_zero_live(c->cnt, to, s));
                HIPCHK(c, launch_compact(c->st[c->cur], c->st[to], c->tn[c->cur], c->tn[to], c->cnt, c->cur,
                                         c->n_upper, 256, s));
            }
            c->cur = to;
            c->since_compact = 0;
            if (!c->capturing) {
                HIPCHK(c, hipMemcpyAsync(c->pinned, &c->cnt->n_live[to], sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, s));
                HIPCHK(c, hipEventRecord(c->ev, s));
                c->pending = true;
                c->injected_since = 0;
            }
        }
    }
    return FTE_OK;
}

fte_status fte_bin_observers(fte_ctx *c, double *j, double *sigma, int reset, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "nothing to bin before the grid is loaded");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)obs_bins(&c->p) * c->p.n_e * c->p.n_t * runs_eff(&c->p);
    if (nb > 0) {
        HIPCHK(c, launch_finalize(c->dp, (const double *)c->b.hist, c->cnt, c->fin_j, c->fin_s, s));
        if (j) HIPCHK(c, hipMemcpyAsync(j, c->fin_j, nb * 8, hipMemcpyDeviceToHost, s));
        if (sigma) HIPCHK(c, hipMemcpyAsync(sigma, c->fin_s, nb * 8, hipMemcpyDeviceToHost, s));
        if (reset) HIPCHK(c, launch_zero((double *)c->b.hist, c->hist_n, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    return FTE_OK;
}

fte_status fte_bin_observers_static(fte_ctx *c, double *j, double *sigma, int reset, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "nothing to bin before the grid is loaded");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)obs_bins(&c->p) * c->p.n_e * c->p.n_t * runs_eff(&c->p);
    if (nb > FTE_STATIC_BINS)
        return fail(c, FTE_EINVAL, std::to_string(nb) + " bins exceed the static scratch of " +
                                       std::to_string(FTE_STATIC_BINS) + "; use fte_bin_observers");
    if (nb > 0) {
        HIPCHK(c, launch_finalize(c->dp, (const double *)c->b.hist, c->cnt, c->scratch, c->scratch + FTE_STATIC_BINS, s));
        if (j) HIPCHK(c, hipMemcpyAsync(j, c->scratch, nb * 8, hipMemcpyDeviceToHost, s));
        if (sigma) HIPCHK(c, hipMemcpyAsync(sigma, c->scratch + FTE_STATIC_BINS, nb * 8, hipMemcpyDeviceToHost, s));
        if (reset) HIPCHK(c, launch_zero((double *)c->b.hist, c->hist_n, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    return FTE_OK;
}

fte_status fte_bin_steady(fte_ctx *c, double *J, double *sigma, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "nothing to bin before the grid is loaded");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)obs_bins(&c->p) * c->p.n_e * runs_eff(&c->p);
    if (nb > 0) {
        HIPCHK(c, launch_finalize_steady(c->dp, (const double *)c->b.hist, c->cnt, c->fin_j, c->fin_s, s));
        if (J) HIPCHK(c, hipMemcpyAsync(J, c->fin_j, nb * 8, hipMemcpyDeviceToHost, s));
        if (sigma) HIPCHK(c, hipMemcpyAsync(sigma, c->fin_s, nb * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    return FTE_OK;
}

fte_status fte_read_hist(fte_ctx *c, double *sums, double *w_injected, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    hipStream_t s = (hipStream_t)stream;
    if (sums && c->hist_n) HIPCHK(c, hipMemcpyAsync(sums, c->b.hist, c->hist_n * 8, hipMemcpyDeviceToHost, s));
    std::vector<double> w(FTE_MAX_RUNS * FTE_MAX_BATCH);
    HIPCHK(c, hipMemcpyAsync(w.data(), c->cnt->w_inj, w.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (w_injected)
        for (int r = 0; r < runs_eff(&c->p); ++r) {
            double t = 0.0;
            for (int b = 0; b < c->p.n_batch; ++b) t += w[r * c->p.n_batch + b];
            w_injected[r] = t;
        }
    return FTE_OK;
}

fte_status fte_get_stats(fte_ctx *c, fte_stats *out, void *stream) {
    if (!c || !out) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    hipStream_t s = (hipStream_t)stream;
    if (c->timing) {
        fte_status r = drain_timing(c, s);
        if (r != FTE_OK) return r;
    }
    DevCounters h;
    HIPCHK(c, hipMemcpyAsync(&h, c->cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    memset(out, 0, sizeof(*out));
    out->n_live = h.n_live[c->cur];
    out->n_injected = h.injected;
    out->particle_steps = h.steps;
    double wi = 0.0;
    for (int b = 0; b < c->p.n_batch * runs_eff(&c->p); ++b) wi += h.w_inj[b];
    out->w_injected = wi;
    for (int k = 0; k < 6; ++k) {
        out->n_retired[k] = h.retired[k];
        out->w_retired[k] = h.w_retired[k];
    }
    out->global_step = c->global_step;
    out->device_flags = h.flags;
    out->step_launches = c->timed_launches;
    out->step_kernel_ms = c->timed_ms;
    return FTE_OK;
}

fte_status fte_reset(fte_ctx *c, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, launch_zero_counters(c->cnt, s));
    if (c->hist_n) HIPCHK(c, launch_zero((double *)c->b.hist, c->hist_n, s));
    if (c->sm_n) HIPCHK(c, launch_zero(c->sm, c->sm_n, s));
    HIPCHK(c, hipStreamSynchronize(s));
    c->cur = 0;
    c->n_upper = 0;
    c->injected_since = 0;
    c->pending = false;
    c->global_step = 0;
    c->since_compact = 0;
    c->tev_used = 0;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    return FTE_OK;
}

fte_status fte_set_timing(fte_ctx *c, int enable) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (c->tev_used) return fail(c, FTE_ESTATE, "read the stats before switching timing");
    c->timing = enable != 0;
    if (c->timing && c->tev.empty()) {
        c->tev.resize(512);
        for (auto &e : c->tev) HIPCHK(c, hipEventCreate(&e));
    }
    return FTE_OK;
}

fte_status fte_read_particles(fte_ctx *c, double *x3, double *mu, double *lnp, double *w, uint64_t *pid,
                              uint32_t *kinj, int32_t *status, uint64_t cap, uint64_t *n_out, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long n = 0;
    HIPCHK(c, hipMemcpyAsync(&n, &c->cnt->n_live[c->cur], sizeof(n), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (n_out) *n_out = n;
    if (n > cap) return fail(c, FTE_ENOMEM, "host arrays too small");
    const DevState &d = c->st[c->cur];
    if (x3) {
        std::vector<double> tx(n), ty(n), tz(n);
        HIPCHK(c, hipMemcpyAsync(tx.data(), d.x, n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(ty.data(), d.y, n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(tz.data(), d.z, n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (size_t i = 0; i < n; ++i) {
            x3[3 * i] = tx[i];
            x3[3 * i + 1] = ty[i];
            x3[3 * i + 2] = tz[i];
        }
    }
    if (mu) HIPCHK(c, hipMemcpyAsync(mu, d.mu, n * 8, hipMemcpyDeviceToHost, s));
    if (lnp) HIPCHK(c, hipMemcpyAsync(lnp, d.lnp, n * 8, hipMemcpyDeviceToHost, s));
    if (w) HIPCHK(c, hipMemcpyAsync(w, d.w, n * 8, hipMemcpyDeviceToHost, s));
    if (pid) HIPCHK(c, hipMemcpyAsync(pid, d.pid, n * 8, hipMemcpyDeviceToHost, s));
    if (kinj) HIPCHK(c, hipMemcpyAsync(kinj, d.kinj, n * 4, hipMemcpyDeviceToHost, s));
    if (status) HIPCHK(c, hipMemcpyAsync(status, d.status, n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return FTE_OK;
}

// Smoothed sums -> fin_sm[k][bins] (k = 0: J numerators, 1-3: derivatives)
// and the injected weight and its gamma derivative.
static fte_status smoothed_sums(fte_ctx *c, hipStream_t s, double *W, double *dW) {
    HIPCHK(c, launch_smooth_finalize(c->dp, c->sm, c->fin_sm, s));
    double w[FTE_MAX_BATCH], dg = 0.0;
    HIPCHK(c, hipMemcpyAsync(w, c->cnt->w_inj, sizeof(w), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(&dg, &c->cnt->w_inj_dgamma, sizeof(dg), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double t = 0.0;
    for (int b = 0; b < c->p.n_batch; ++b) t += w[b];
    *W = t;
    *dW = dg;
    return FTE_OK;
}

fte_status fte_bin_smoothed(fte_ctx *c, double *J, double *dJ, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    if (!(c->p.sigma_x > 0.0)) return fail(c, FTE_ESTATE, "smoothed intensities are off (sigma_x = 0)");
    if (dJ && !c->p.grad) return fail(c, FTE_ESTATE, "derivatives need gradient mode");
    hipStream_t s = (hipStream_t)stream;
    double W = 0.0, dW = 0.0;
    fte_status r = smoothed_sums(c, s, &W, &dW);
    if (r != FTE_OK) return r;
    if (!(W > 0.0)) return fail(c, FTE_ESTATE, "no injected weight");
    const size_t nb = (size_t)c->p.n_obs * c->p.n_e * c->p.n_t;
    const int nk = c->p.grad ? 4 : 1;
    std::vector<double> f(nb * nk);
    HIPCHK(c, hipMemcpyAsync(f.data(), c->fin_sm, f.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const double inv = 1.0 / (4.0 * kPi * W);
    for (size_t b = 0; b < nb; ++b) {
        const double j = f[b] * inv;
        if (J) J[b] = j;
        if (dJ) {
            dJ[b] = f[nb + b] * inv;
            dJ[nb + b] = f[2 * nb + b] * inv;
            dJ[2 * nb + b] = f[3 * nb + b] * inv - j * dW / W;   // W_inj depends on gamma_inj
        }
    }
    return FTE_OK;
}

fte_status fte_grad(fte_ctx *c, const double *dL_dJ, double grad[3], void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    if (!c->p.grad) return fail(c, FTE_ESTATE, "gradient mode is off");
    if (!dL_dJ || !grad) return fail(c, FTE_EINVAL, "dL_dJ and grad must be non-NULL");
    hipStream_t s = (hipStream_t)stream;
    double W = 0.0, dW = 0.0;
    fte_status r = smoothed_sums(c, s, &W, &dW);
    if (r != FTE_OK) return r;
    if (!(W > 0.0)) return fail(c, FTE_ESTATE, "no injected weight");
    const size_t nb = (size_t)c->p.n_obs * c->p.n_e * c->p.n_t;
    HIPCHK(c, hipMemcpyAsync(c->dl, dL_dJ, nb * 8, hipMemcpyHostToDevice, s));
    HIPCHK(c, launch_grad_contract(c->dp, c->fin_sm, c->dl, c->out4, s));
    double o4[4];
    HIPCHK(c, hipMemcpyAsync(o4, c->out4, sizeof(o4), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const double inv = 1.0 / (4.0 * kPi * W);
    grad[0] = o4[1] * inv;
    grad[1] = o4[2] * inv;
    grad[2] = (o4[3] - o4[0] * dW / W) * inv;
    return FTE_OK;
}

fte_status fte_read_tangents(fte_ctx *c, double *tan, uint64_t cap, uint64_t *n_out, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    if (!c->p.grad) return fail(c, FTE_ESTATE, "gradient mode is off");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long n = 0;
    HIPCHK(c, hipMemcpyAsync(&n, &c->cnt->n_live[c->cur], sizeof(n), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (n_out) *n_out = n;
    if (n > cap) return fail(c, FTE_ENOMEM, "host array too small");
    if (!tan || n == 0) return FTE_OK;
    const DevTan &t = c->tn[c->cur];
    std::vector<double> col(n);
    for (int q = 0; q < kTanCols; ++q) {
        HIPCHK(c, hipMemcpyAsync(col.data(), t.col(q), n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (size_t i = 0; i < n; ++i) tan[kTanCols * i + q] = col[i];
    }
    return FTE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// checkpoint / resume
// ---------------------------------------------------------------------------
namespace {

constexpr uint64_t kStateMagic = 0x3145544154534654ull;   // "FTSTATE1"

struct StateHeader {
    uint64_t magic;
    uint64_t fingerprint;     // parameters and grid shape
    uint64_t n_live;
    uint64_t global_step;
    uint64_t hist_n, sm_n;
    uint32_t grad, pad;
    uint64_t total_bytes;
};

uint64_t fnv_mix(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

template <typename T>
uint64_t fnv_val(uint64_t h, T v) { return fnv_mix(h, &v, sizeof(v)); }

uint64_t state_fingerprint(const fte_ctx *c) {
    const fte_params &p = c->p;
    uint64_t h = 1469598103934665603ull;
    h = fnv_val(h, p.mass); h = fnv_val(h, p.dmm_model); h = fnv_val(h, p.dmm_norm);
    h = fnv_val(h, p.lambda_ref); h = fnv_val(h, p.p_ref); h = fnv_val(h, p.alpha); h = fnv_val(h, p.q);
    h = fnv_val(h, p.eps); h = fnv_val(h, p.mu_floor); h = fnv_val(h, p.kperp_ratio); h = fnv_val(h, p.lambda_perp);
    h = fnv_val(h, p.dt); h = fnv_val(h, p.t0); h = fnv_val(h, p.r_in); h = fnv_val(h, p.r_out);
    h = fnv_val(h, p.seed); h = fnv_val(h, p.run_id); h = fnv_val(h, p.precision); h = fnv_val(h, p.n_obs);
    for (int o = 0; o < p.n_obs; ++o) h = fnv_mix(h, &p.obs[o], sizeof(fte_observer));
    h = fnv_val(h, p.e_min); h = fnv_val(h, p.dlne); h = fnv_val(h, p.n_e); h = fnv_val(h, p.t_ref);
    h = fnv_val(h, p.dT); h = fnv_val(h, p.n_t); h = fnv_val(h, p.n_batch);
    h = fnv_val(h, p.sigma_x); h = fnv_val(h, p.sigma_lne); h = fnv_val(h, p.sigma_t); h = fnv_val(h, p.grad);
    h = fnv_val(h, p.n_runs);
    h = fnv_val(h, p.kink_sigma);
    for (int r = 0; r < p.n_runs; ++r) {
        h = fnv_val(h, c->runs[r].lambda_ref);
        h = fnv_val(h, c->runs[r].kperp_ratio);
        h = fnv_val(h, c->runs[r].n_steps);
    }
    h = fnv_val(h, c->g.n_leaves); h = fnv_val(h, c->g.n_snap); h = fnv_val(h, c->g.n_levels);
    for (int a = 0; a < 3; ++a) { h = fnv_val(h, c->g.n1[a]); h = fnv_val(h, c->g.bx[a]); }
    return h;
}

// SoA columns of the particle state: (device pointer, element bytes)
int state_columns(const DevState &d, void *col[10], size_t esz[10]) {
    void *v[10] = {d.x, d.y, d.z, d.mu, d.lnp, d.w, d.pid, d.kinj, d.status, d.run};
    const size_t e[10] = {8, 8, 8, 8, 8, 8, 8, 4, 4, 2};
    for (int k = 0; k < 10; ++k) { col[k] = v[k]; esz[k] = e[k]; }
    return 10;
}

uint64_t state_blob_bytes(const fte_ctx *c, uint64_t n) {
    uint64_t b = sizeof(StateHeader) + sizeof(DevCounters) + (c->hist_n + c->sm_n) * 8 + n * (6 * 8 + 8 + 4 + 4 + 2);
    if (c->p.grad) b += n * kTanCols * 8;
    return b;
}

}  // namespace

extern "C" {

fte_status fte_state_size(fte_ctx *c, uint64_t *bytes, void *stream) {
    if (!c || !bytes) return FTE_EINVAL;
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long n = 0;
    HIPCHK(c, hipMemcpyAsync(&n, &c->cnt->n_live[c->cur], sizeof(n), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *bytes = state_blob_bytes(c, n);
    return FTE_OK;
}

fte_status fte_save_state(fte_ctx *c, void *blob, uint64_t bytes, void *stream) {
    if (!c || !blob) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    hipStream_t s = (hipStream_t)stream;
    DevCounters h;
    HIPCHK(c, hipMemcpyAsync(&h, c->cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const uint64_t n = h.n_live[c->cur];
    const uint64_t need = state_blob_bytes(c, n);
    if (bytes < need) return fail(c, FTE_ENOMEM, "state blob too small");
    char *o = (char *)blob;
    StateHeader hd{};
    hd.magic = kStateMagic;
    hd.fingerprint = state_fingerprint(c);
    hd.n_live = n;
    hd.global_step = c->global_step;
    hd.hist_n = c->hist_n;
    hd.sm_n = c->sm_n;
    hd.grad = (uint32_t)c->p.grad;
    hd.total_bytes = need;
    // the counters as a compacted state: everything held sits in slot 0
    h.n_live[0] = n;
    h.n_live[1] = 0;
    memcpy(o, &hd, sizeof(hd));
    o += sizeof(hd);
    memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    if (c->hist_n) HIPCHK(c, hipMemcpyAsync(o, c->b.hist, c->hist_n * 8, hipMemcpyDeviceToHost, s));
    o += c->hist_n * 8;
    if (c->sm_n) HIPCHK(c, hipMemcpyAsync(o, c->sm, c->sm_n * 8, hipMemcpyDeviceToHost, s));
    o += c->sm_n * 8;
    void *col[10];
    size_t esz[10];
    const int nc = state_columns(c->st[c->cur], col, esz);
    for (int k = 0; k < nc; ++k) {
        if (n) HIPCHK(c, hipMemcpyAsync(o, col[k], n * esz[k], hipMemcpyDeviceToHost, s));
        o += n * esz[k];
    }
    if (c->p.grad)
        for (int q = 0; q < kTanCols; ++q) {
            if (n) HIPCHK(c, hipMemcpyAsync(o, c->tn[c->cur].col(q), n * 8, hipMemcpyDeviceToHost, s));
            o += n * 8;
        }
    HIPCHK(c, hipStreamSynchronize(s));
    return FTE_OK;
}

fte_status fte_load_state(fte_ctx *c, const void *blob, uint64_t bytes, void *stream) {
    if (!c || !blob) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "load the grid before restoring a state");
    if (bytes < sizeof(StateHeader)) return fail(c, FTE_EINVAL, "state blob too short");
    StateHeader hd;
    memcpy(&hd, blob, sizeof(hd));
    if (hd.magic != kStateMagic) return fail(c, FTE_EINVAL, "not a state blob");
    if (hd.fingerprint != state_fingerprint(c)) return fail(c, FTE_EINVAL, "state saved with other parameters or grid");
    if (hd.hist_n != c->hist_n || hd.sm_n != c->sm_n || hd.grad != (uint32_t)c->p.grad)
        return fail(c, FTE_EINVAL, "state layout differs from this context");
    if (hd.n_live > c->n_max) return fail(c, FTE_ENOMEM, "state holds more particles than the capacity");
    if (hd.total_bytes != state_blob_bytes(c, hd.n_live) || bytes < hd.total_bytes)
        return fail(c, FTE_EINVAL, "state blob size mismatch");
    if (hd.global_step >= (1ull << 48)) return fail(c, FTE_EINVAL, "bad global step");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipStreamSynchronize(s));
    const char *o = (const char *)blob + sizeof(hd);
    DevCounters h;
    memcpy(&h, o, sizeof(h));
    o += sizeof(h);
    if (h.n_live[0] != hd.n_live) return fail(c, FTE_EINVAL, "damaged state blob");
    const uint64_t n = hd.n_live;
    HIPCHK(c, hipMemcpyAsync(c->cnt, &h, sizeof(h), hipMemcpyHostToDevice, s));
    if (c->hist_n) HIPCHK(c, hipMemcpyAsync(c->b.hist, o, c->hist_n * 8, hipMemcpyHostToDevice, s));
    o += c->hist_n * 8;
    if (c->sm_n) HIPCHK(c, hipMemcpyAsync(c->sm, o, c->sm_n * 8, hipMemcpyHostToDevice, s));
    o += c->sm_n * 8;
    void *col[10];
    size_t esz[10];
    const int nc = state_columns(c->st[0], col, esz);
    for (int k = 0; k < nc; ++k) {
        if (n) HIPCHK(c, hipMemcpyAsync(col[k], o, n * esz[k], hipMemcpyHostToDevice, s));
        o += n * esz[k];
    }
    if (c->p.grad)
        for (int q = 0; q < kTanCols; ++q) {
            if (n) HIPCHK(c, hipMemcpyAsync(c->tn[0].col(q), o, n * 8, hipMemcpyHostToDevice, s));
            o += n * 8;
        }
    HIPCHK(c, hipStreamSynchronize(s));
    c->cur = 0;
    c->n_upper = n;
    c->injected_since = 0;
    c->pending = false;
    c->global_step = hd.global_step;
    c->since_compact = 0;
    c->tev_used = 0;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    return FTE_OK;
}

fte_status fte_autotune(fte_ctx *c, uint32_t trial_steps, int best[3], void *stream) {
    if (!c || !best) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "grid not loaded");
    if (trial_steps < 1) return fail(c, FTE_EINVAL, "trial_steps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    uint64_t bytes = 0;
    fte_status r = fte_state_size(c, &bytes, stream);
    if (r != FTE_OK) return r;
    std::vector<char> blob;
    try {
        blob.resize(bytes);
    } catch (...) {
        return fail(c, FTE_ENOMEM, "no host memory for the state copy");
    }
    r = fte_save_state(c, blob.data(), bytes, stream);
    if (r != FTE_OK) return r;
    const bool timing = c->timing;
    const int spl = c->spl, keep_block = c->block, keep_compact = c->compact_every;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    float best_ms = -1.f;
    int bb = keep_block, bc = keep_compact;
    const int blocks[3] = {64, 128, 256};
    const int mult[4] = {1, 2, 4, 8};
    c->timing = false;
    for (int ib = 0; ib < 3 && r == FTE_OK; ++ib)
        for (int im = 0; im < 4 && r == FTE_OK; ++im) {
            r = fte_load_state(c, blob.data(), bytes, stream);
            if (r != FTE_OK) break;
            c->block = blocks[ib];
            c->compact_every = spl * mult[im];
            if (hipEventRecord(e0, s) != hipSuccess) { r = fail(c, FTE_EDEVICE, "event record"); break; }
            r = fte_step_n(c, trial_steps, stream);
            if (r != FTE_OK) break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                r = fail(c, FTE_EDEVICE, "event wait");
                break;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { r = fail(c, FTE_EDEVICE, "event time"); break; }
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                bb = c->block;
                bc = c->compact_every;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = timing;
    c->block = keep_block;
    c->compact_every = keep_compact;
    // back to the state the caller had, with the winning shape
    fte_status r2 = fte_load_state(c, blob.data(), bytes, stream);
    if (r != FTE_OK) return r;
    if (r2 != FTE_OK) return r2;
    c->block = bb;
    c->compact_every = bc;
    best[0] = bb;
    best[1] = spl;
    best[2] = bc;
    return FTE_OK;
}

fte_status fte_set_launch(fte_ctx *c, int block, int steps_per_launch, int compact_every, int spatial_sort) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (block < 64 || block > 256 || (block & 63)) return fail(c, FTE_EINVAL, "block must be 64..256, multiple of 64");
    if (steps_per_launch < 1) return fail(c, FTE_EINVAL, "steps_per_launch must be >= 1");
    if (compact_every < 0 || (compact_every && compact_every % steps_per_launch))
        return fail(c, FTE_EINVAL, "compact_every must be a multiple of steps_per_launch");
    if (spatial_sort < 0 || spatial_sort > 3) return fail(c, FTE_EINVAL, "spatial_sort must be 0..3");
    for (int a = 0; a < 3 && spatial_sort > 1; ++a)
        if (c->bound && (c->g.bx[a] % (1 << (spatial_sort - 1))))
            return fail(c, FTE_EINVAL, "sort cube must divide the block");
    c->block = block;
    c->spl = steps_per_launch;
    c->compact_every = compact_every;
    c->sort = spatial_sort;
    return FTE_OK;
}

fte_status fte_set_record_tile(fte_ctx *c, int tile_bytes) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (tile_bytes < 0 || tile_bytes > FTE_MAX_TILE_BYTES)
        return fail(c, FTE_EINVAL, "tile_bytes must be 0.." + std::to_string(FTE_MAX_TILE_BYTES));
    c->tile_bytes = (size_t)tile_bytes;
    return FTE_OK;
}

fte_status fte_set_lds_histogram(fte_ctx *c, int hist_bytes) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (hist_bytes < 0 || hist_bytes > FTE_MAX_LDS_HIST_BYTES)
        return fail(c, FTE_EINVAL, "hist_bytes must be 0.." + std::to_string(FTE_MAX_LDS_HIST_BYTES));
    c->hist_bytes = (size_t)hist_bytes;
    return FTE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launch graphs
// ---------------------------------------------------------------------------
namespace {
HostClock clock_of(const fte_ctx *c) {
    return HostClock{c->global_step, c->since_compact, c->n_upper, c->injected_since, c->cur};
}
void set_clock(fte_ctx *c, const HostClock &k) {
    c->global_step = k.global_step;
    c->since_compact = k.since_compact;
    c->n_upper = k.n_upper;
    c->injected_since = k.injected_since;
    c->cur = k.cur;
}
}  // namespace

fte_status fte_capture_begin(fte_ctx *c, void *stream) {
    if (!c) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (!c->loaded) return fail(c, FTE_ESTATE, "load the grid before recording");
    hipStream_t s = (hipStream_t)stream;
    // settle the live count of the last compaction first: the recording
    // cannot read it back
    if (c->pending) {
        HIPCHK(c, hipEventSynchronize(c->ev));
        c->n_upper = *c->pinned + c->injected_since;
        c->pending = false;
    }
    HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    c->cap_stream = s;
    c->graph_start = clock_of(c);
    return FTE_OK;
}

fte_status fte_capture_end(fte_ctx *c, void *stream, fte_graph **out) {
    if (!c || !out) return FTE_EINVAL;
    *out = nullptr;
    if (!c->capturing) return fail(c, FTE_ESTATE, "no recording in progress");
    hipStream_t s = (hipStream_t)stream;
    if (s != c->cap_stream) return fail(c, FTE_EINVAL, "end the recording on the stream it began on");
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    c->capturing = false;
    const HostClock end = clock_of(c);
    set_clock(c, c->graph_start);      // nothing ran: back to where the recording began
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, FTE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(c, FTE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    fte_graph *g = new fte_graph;
    g->graph = graph;
    g->exec = exec;
    g->ctx = c;
    g->start = c->graph_start;
    g->end = end;
    *out = g;
    return FTE_OK;
}

fte_status fte_graph_launch(fte_ctx *c, fte_graph *g, void *stream) {
    if (!c || !g) return FTE_EINVAL;
    NO_CAPTURE(c);
    if (g->ctx != c) return fail(c, FTE_EINVAL, "the graph was recorded on another context");
    const HostClock k = clock_of(c);
    if (k.global_step != g->start.global_step || k.cur != g->start.cur || k.since_compact != g->start.since_compact)
        return fail(c, FTE_ESTATE, "the context is not at the global step, particle buffer and compaction phase "
                                   "the recording began at");
    hipStream_t s = (hipStream_t)stream;
    if (c->pending) {
        HIPCHK(c, hipEventSynchronize(c->ev));
        c->pending = false;
    }
    HIPCHK(c, hipGraphLaunch(g->exec, s));
    set_clock(c, g->end);
    return FTE_OK;
}

void fte_graph_destroy(fte_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}
