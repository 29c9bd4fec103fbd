/*
 * FP64 CPU oracle for the focused-transport pseudo-particle method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source, header,
 * table or helper with the GPU library; both follow the same written definition
 * of the method (the paper, section 2.1 "The PARADISE code", Eqs. 1-5, and
 * section 2.4 "Coupling of PARADISE to Icarus").
 *
 * Everything is double precision and written step by step in the order the
 * definition states it.  Nothing is blocked, fused or cached: every grid value
 * a particle needs is recomputed from the raw snapshot data on demand.
 *
 * Units are SI.  Positions are heliocentric inertial Cartesian metres (the
 * spatial coordinates of the mixed-coordinate FTE, section 2.1), mu is the
 * pitch-angle cosine and P = p/(m c) the momentum magnitude, both in the
 * solar-wind frame.  The state stores lnp = ln P.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_C   299792458.0
#define OR_PI  3.14159265358979323846

enum { OR_ACTIVE = 0, OR_ABS_IN = 1, OR_ABS_OUT = 2, OR_OUT_DOMAIN = 3, OR_NUMERIC = 4 };

enum { OR_DMM_ISO = 0, OR_DMM_EQ5 = 1, OR_DMM_POWER_Q = 2 };
enum { OR_BG_GRID = 0, OR_BG_UNIFORM = 1, OR_BG_PAR_FLOW = 2, OR_BG_PERP_FLOW = 3, OR_BG_RADIAL = 4 };

/* ------------------------------------------------------------------------- */
/* Parameters (mirrored field by field by the ctypes wrapper in __init__.py). */
/* ------------------------------------------------------------------------- */
typedef struct {
    double mass;          /* particle rest mass, kg                              */
    int    dmm_model;     /* OR_DMM_*                                            */
    int    dmm_norm;      /* 0: scale from lambda_par (MFP-consistent), 1: v/lambda */
    double lambda_ref;    /* parallel mean free path at P_ref, m                 */
    double p_ref;         /* reference momentum in units of m c                  */
    double alpha;         /* lambda_par = lambda_ref (P/P_ref)^alpha             */
    double q;             /* exponent of the power-law D_mumu model              */
    double eps;           /* resonance-gap filler of Eq. 5 (and of power law)    */
    double mu_floor;      /* floor on |mu| inside |mu|^(q-2)                     */
    double kperp_ratio;   /* kappa_perp = ratio * v lambda_par / 3 when > 0      */
    double lambda_perp;   /* else kappa_perp = v lambda_perp / 3 when > 0        */
    double dt, t0;        /* global step and clock origin, s                     */
    double r_in, r_out;   /* absorbing radii, m                                  */
    int    check_bounds;  /* apply r_in/r_out (and the theta range of a grid)    */
    int    run_id;
    uint64_t seed;
    int    n_obs;
    double obs[8][6];     /* r, theta, phi centre; dr, dtheta, dphi full widths  */
    int    obs_nphi[8];   /* longitude bins of width dphi (ring observer), >= 1  */
    double obs_omega[8];  /* rotation of the observer pattern, rad/s             */
    double e_min;         /* lower edge of energy bin 0, J                       */
    double dlne;          /* width of a bin in ln E                              */
    int    n_e;
    double t_ref, dT;     /* time-bin origin and width, s                        */
    int    n_t;
    int    n_batch;       /* batch = pid mod n_batch                             */
    int    bg_kind;       /* OR_BG_*                                             */
    double bg[16];        /* analytic background parameters                      */
    int    smooth;        /* accumulate the kernel-smoothed intensity sums       */
    double sig_x, sig_lne, sig_t;  /* Gaussian widths: space (m), ln E, time (s) */
} or_params;

/* Observer bins: observer o covers obs_nphi[o] consecutive longitude bins. */
static int or_nphi(const or_params *pp, int o) { return pp->obs_nphi[o] > 1 ? pp->obs_nphi[o] : 1; }

int or_obs_bins(const or_params *pp)
{
    int n = 0;
    for (int o = 0; o < pp->n_obs; ++o) n += or_nphi(pp, o);
    return n;
}

typedef struct {
    int    xi_map;        /* 0: xi = r - r_lo, 1: xi = ln(r / r_lo)             */
    double r_lo, dxi;     /* radial origin (m) and level-1 cell width in xi      */
    double th_lo, dth;    /* colatitude origin and level-1 width, rad            */
    double ph_lo, dph;    /* longitude origin and level-1 width, rad             */
    int    phi_periodic;
    int    n1[3];         /* level-1 cells along xi, theta, phi                  */
    int    bx[3];         /* cells per block along xi, theta, phi                */
    int    n_levels;
    int    n_leaves;
    const int32_t *leaves;/* [n_leaves][4] = level, I, J, K (block index)        */
    int    n_snap_total;  /* snapshots of the whole run                          */
    int    snap0;         /* first snapshot present in raw                       */
    int    n_snap_held;   /* snapshots present in raw                            */
    double t_s0, dt_s;    /* snapshot k sits at t_s0 + k dt_s                    */
    const double *raw;    /* [n_snap_held][n_leaves][cell][6] = Vr,Vth,Vph,Br,Bth,Bph */
} or_grid_desc;

typedef struct {
    or_grid_desc d;
    int32_t *map[8];      /* per level: block (I,J,K) -> leaf id, -1 if none     */
    int nb[8][3];         /* blocks per dimension at each level                  */
} or_grid;

/* ------------------------------------------------------------------------- */
/* Counter-based noise: Philox (Salmon, Moraes, Dror & Shaw, SC'11).          */
/* One round multiplies words 0 and 2 by the round constants, swaps the high  */
/* halves in with the key, and the key is bumped by the Weyl constants        */
/* between rounds.                                                            */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The 64-bit-word member of the same family; it exists so the shared round
 * structure can be checked against an independent library implementation. */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B97F4A7C15ull; k1 += 0xBB67AE8584CAA73Bull; }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout: word 0 = step index low 32 bits, word 1 = run id << 16 |
 * step index bits 32..47, word 2 = pid low 32 bits, word 3 = pid bits 32..59 |
 * stream tag << 28 (tag 0: step noise, tag 1: injection draws).  The key is
 * the 64-bit seed. */
void or_philox_words(uint64_t seed, int run_id, uint64_t n, uint64_t pid, int tag, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)(n & 0xFFFFFFFFu);
    ctr[1] = ((uint32_t)run_id << 16) | (uint32_t)((n >> 32) & 0xFFFFu);
    ctr[2] = (uint32_t)(pid & 0xFFFFFFFFu);
    ctr[3] = (uint32_t)((pid >> 32) & 0x0FFFFFFFu) | ((uint32_t)tag << 28);
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
    or_philox4x32_10(ctr, key, out);
}

/* Uniform on the open interval (0, 1): u = (k + 1/2) 2^-32. */
static double or_u01(uint32_t k) { return ((double)k + 0.5) * (1.0 / 4294967296.0); }

/* Four standard normals by the Box-Muller transform of the four words. */
void or_normals(uint64_t seed, int run_id, uint64_t n, uint64_t pid, double z[4])
{
    uint32_t k[4];
    or_philox_words(seed, run_id, n, pid, 0, k);
    double u0 = or_u01(k[0]), u1 = or_u01(k[1]), u2 = or_u01(k[2]), u3 = or_u01(k[3]);
    double ra = sqrt(-2.0 * log(u0)), rb = sqrt(-2.0 * log(u2));
    z[0] = ra * cos(2.0 * OR_PI * u1);
    z[1] = ra * sin(2.0 * OR_PI * u1);
    z[2] = rb * cos(2.0 * OR_PI * u3);
    z[3] = rb * sin(2.0 * OR_PI * u3);
}

/* ------------------------------------------------------------------------- */
/* Pitch-angle diffusion models (section 2.1, Eq. 5 and its power-law kin).   */
/* With D = A g(mu), kappa_par = (v^2/8) Int_{-1}^{1} (1-mu^2)^2 / D dmu and  */
/* lambda_par = 3 kappa_par / v give A = 3 v I / (8 lambda_par), where        */
/* I = Int_{-1}^{1} (1-mu^2)^2 / g dmu is returned here.                      */
/* ------------------------------------------------------------------------- */
double or_dmm_integral(int model, double q, double eps)
{
    if (model == OR_DMM_ISO) {
        /* g = 1 - mu^2:  I = Int (1 - mu^2) dmu = 4/3 */
        return 4.0 / 3.0;
    }
    if (model == OR_DMM_EQ5) {
        /* g = (|mu|/(1+|mu|) + eps)(1 - mu^2):
         * I = 2 Int_0^1 (1 - m)(1 + m)^2 / (a m + b) dm with a = 1 + eps, b = eps.
         * Long division of N(m) = 1 + m - m^2 - m^3 by (a m + b). */
        double a = 1.0 + eps, b = eps;
        double q2 = -1.0 / a;
        double q1 = (b / a - 1.0) / a;
        double q0 = (1.0 - q1 * b) / a;
        double rem = 1.0 - q0 * b;
        return 2.0 * (q2 / 3.0 + q1 / 2.0 + q0 + rem / a * log((a + b) / b));
    }
    /* power law g = (1 - mu^2) |mu|^(q-1):  I = 2 Int_0^1 (1 - m^2) m^(1-q) dm */
    return 2.0 * (1.0 / (2.0 - q) - 1.0 / (4.0 - q));
}

static double or_sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* D_mumu and dD_mumu/dmu for speed v and momentum P (units of m c). */
static void or_dmm(const or_params *pp, double v, double P, double mu, double *D, double *dD)
{
    double lam = pp->lambda_ref;
    if (pp->alpha != 0.0) lam *= pow(P / pp->p_ref, pp->alpha);
    double I = or_dmm_integral(pp->dmm_model, pp->q, pp->eps);
    double A = (pp->dmm_norm == 1) ? v / lam : 3.0 * v * I / (8.0 * lam);
    double am = fabs(mu), om = 1.0 - mu * mu;
    if (pp->dmm_model == OR_DMM_ISO) {
        *D = A * om;
        *dD = -2.0 * mu * A;
    } else if (pp->dmm_model == OR_DMM_EQ5) {
        double g = am / (1.0 + am) + pp->eps;
        *D = A * g * om;
        *dD = A * (or_sgn(mu) * om / ((1.0 + am) * (1.0 + am)) - 2.0 * mu * g);
    } else {
        double am_f = am > pp->mu_floor ? am : pp->mu_floor;
        double g = pow(am, pp->q - 1.0);
        *D = A * om * g;
        *dD = A * ((pp->q - 1.0) * or_sgn(mu) * pow(am_f, pp->q - 2.0) * om - 2.0 * mu * g);
    }
}

static double or_mfp(const or_params *pp, double P)
{
    double lam = pp->lambda_ref;
    if (pp->alpha != 0.0) lam *= pow(P / pp->p_ref, pp->alpha);
    return lam;
}

/* ------------------------------------------------------------------------- */
/* Block-AMR grid (section 2.4): every level halves its parent along each     */
/* coordinate; leaves tile the domain.  Coordinates are (xi, theta, phi) with */
/* xi = r - r_lo or ln(r / r_lo) (radial stretching); positions are measured  */
/* in level-1 cell units s, and a level-L cell index is floor(s 2^(L-1)).     */
/* ------------------------------------------------------------------------- */
void *or_grid_create(const or_grid_desc *d)
{
    or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
    g->d = *d;
    for (int L = 1; L <= d->n_levels; ++L) {
        long tot = 1;
        for (int a = 0; a < 3; ++a) {
            g->nb[L][a] = (d->n1[a] / d->bx[a]) << (L - 1);
            tot *= g->nb[L][a];
        }
        g->map[L] = (int32_t *)malloc(sizeof(int32_t) * tot);
        for (long i = 0; i < tot; ++i) g->map[L][i] = -1;
    }
    for (int l = 0; l < d->n_leaves; ++l) {
        const int32_t *e = d->leaves + 4 * l;
        int L = e[0];
        long idx = e[1] + (long)g->nb[L][0] * (e[2] + (long)g->nb[L][1] * e[3]);
        g->map[L][idx] = l;
    }
    return g;
}

void or_grid_destroy(void *gp)
{
    or_grid *g = (or_grid *)gp;
    if (!g) return;
    for (int L = 1; L <= g->d.n_levels; ++L) free(g->map[L]);
    free(g);
}

/* Number of level-L cells along dimension a. */
static long or_ncell(const or_grid *g, int L, int a) { return (long)g->d.n1[a] << (L - 1); }

/* Bring a level-L index into the domain: clamp along xi and theta (zero
 * gradient beyond the physical edges), wrap along a periodic phi. */
static void or_fold(const or_grid *g, int L, long c[3])
{
    for (int a = 0; a < 3; ++a) {
        long n = or_ncell(g, L, a);
        if (a == 2 && g->d.phi_periodic) {
            c[a] %= n;
            if (c[a] < 0) c[a] += n;
        } else {
            if (c[a] < 0) c[a] = 0;
            if (c[a] > n - 1) c[a] = n - 1;
        }
    }
}

/* The leaf that contains the point p (level-1 units).  Returns the leaf id,
 * its level and the point's level-M cell index; -1 if no leaf holds it. */
int or_find_leaf(const void *gp, const double p[3], int *level, long cell[3])
{
    const or_grid *g = (const or_grid *)gp;
    for (int M = 1; M <= g->d.n_levels; ++M) {
        double scale = ldexp(1.0, M - 1);
        long c[3], B[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (long)floor(p[a] * scale);
            long n = or_ncell(g, M, a);
            if (c[a] < 0) c[a] = 0;
            if (c[a] > n - 1) c[a] = n - 1;
            B[a] = c[a] / g->d.bx[a];
        }
        long idx = B[0] + (long)g->nb[M][0] * (B[1] + (long)g->nb[M][1] * B[2]);
        int leaf = g->map[M][idx];
        if (leaf >= 0) {
            *level = M;
            for (int a = 0; a < 3; ++a) cell[a] = c[a];
            return leaf;
        }
    }
    return -1;
}

/* Offset of a leaf cell inside the raw array for held snapshot k. */
static const double *or_raw_cell(const or_grid *g, int snap, int leaf, const long c[3])
{
    const int32_t *e = g->d.leaves + 4 * leaf;
    long li = c[0] - (long)e[1] * g->d.bx[0];
    long lj = c[1] - (long)e[2] * g->d.bx[1];
    long lk = c[2] - (long)e[3] * g->d.bx[2];
    long cells = (long)g->d.bx[0] * g->d.bx[1] * g->d.bx[2];
    long idx = li + g->d.bx[0] * (lj + (long)g->d.bx[1] * lk);
    long k = snap - g->d.snap0;
    return g->d.raw + ((k * g->d.n_leaves + leaf) * cells + idx) * 6;
}

typedef void (*or_cell_fn)(const or_grid *g, int snap, int leaf, int L, const long c[3], double *out);

/* Value of a level-L cell centre for any grid quantity (the paper leaves the
 * block-boundary treatment to case-by-case handling, section 2.4; this is the
 * rule used here):
 *   - the centre lies in a leaf of level L: that leaf's cell value;
 *   - the leaf is finer: the mean of the eight level-(L+1) children;
 *   - the leaf is coarser: trilinear interpolation, at the centre, of the
 *     level-(L-1) values of the eight surrounding level-(L-1) centres.
 * Indices are folded into the domain first. */
static void or_virtual(const or_grid *g, int snap, int L, const long cin[3], int ncomp,
                       or_cell_fn cellfn, double *out)
{
    long c[3] = {cin[0], cin[1], cin[2]};
    or_fold(g, L, c);
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = ((double)c[a] + 0.5) * ldexp(1.0, 1 - L);
    int M;
    long cm[3];
    int leaf = or_find_leaf(g, p, &M, cm);
    if (leaf < 0) {
        for (int k = 0; k < ncomp; ++k) out[k] = NAN;
        return;
    }
    if (M == L) {
        cellfn(g, snap, leaf, L, c, out);
        return;
    }
    double tmp[16];
    for (int k = 0; k < ncomp; ++k) out[k] = 0.0;
    if (M > L) {
        for (int d = 0; d < 8; ++d) {
            long ch[3] = {2 * c[0] + (d & 1), 2 * c[1] + ((d >> 1) & 1), 2 * c[2] + ((d >> 2) & 1)};
            or_virtual(g, snap, L + 1, ch, ncomp, cellfn, tmp);
            for (int k = 0; k < ncomp; ++k) out[k] += tmp[k];
        }
        for (int k = 0; k < ncomp; ++k) out[k] /= 8.0;
        return;
    }
    /* coarser leaf: centre of c in level-(L-1) units relative to the
     * level-(L-1) centres */
    long i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double u = ((double)c[a] + 0.5) / 2.0 - 0.5;
        i0[a] = (long)floor(u);
        f[a] = u - (double)i0[a];
    }
    for (int d = 0; d < 8; ++d) {
        int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
        long cc[3] = {i0[0] + e0, i0[1] + e1, i0[2] + e2};
        double w = (e0 ? f[0] : 1.0 - f[0]) * (e1 ? f[1] : 1.0 - f[1]) * (e2 ? f[2] : 1.0 - f[2]);
        or_virtual(g, snap, L - 1, cc, ncomp, cellfn, tmp);
        for (int k = 0; k < ncomp; ++k) out[k] += w * tmp[k];
    }
}

static void or_raw_leafcell(const or_grid *g, int snap, int leaf, int L, const long c[3], double *out)
{
    (void)L;
    if (snap < g->d.snap0 || snap >= g->d.snap0 + g->d.n_snap_held) {
        for (int k = 0; k < 6; ++k) out[k] = NAN;   /* snapshot not held */
        return;
    }
    const double *src = or_raw_cell(g, snap, leaf, c);
    for (int k = 0; k < 6; ++k) out[k] = src[k];
}

/* Raw (V, B) spherical components at a level-L cell centre. */
void or_raw_virtual(const void *gp, int snap, int L, const long c[3], double out[6])
{
    or_virtual((const or_grid *)gp, snap, L, c, 6, or_raw_leafcell, out);
}

/* Centre of a level-L cell: radius, colatitude, longitude. */
static void or_centre(const or_grid *g, int L, const long c[3], double *r, double *th, double *ph)
{
    double h = ldexp(1.0, 1 - L);
    double xi = ((double)c[0] + 0.5) * g->d.dxi * h;
    *r = (g->d.xi_map == 1) ? g->d.r_lo * exp(xi) : g->d.r_lo + xi;
    *th = g->d.th_lo + ((double)c[1] + 0.5) * g->d.dth * h;
    *ph = g->d.ph_lo + ((double)c[2] + 0.5) * g->d.dph * h;
}

/* Local unit vectors e_r, e_theta, e_phi as rows. */
static void or_basis(double th, double ph, double e[3][3])
{
    double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    e[0][0] = st * cp; e[0][1] = st * sp; e[0][2] = ct;
    e[1][0] = ct * cp; e[1][1] = ct * sp; e[1][2] = -st;
    e[2][0] = -sp;     e[2][1] = cp;      e[2][2] = 0.0;
}

static void or_sph_to_cart(const double e[3][3], const double s[3], double out[3])
{
    for (int a = 0; a < 3; ++a) out[a] = s[0] * e[0][a] + s[1] * e[1][a] + s[2] * e[2][a];
}

/* Cartesian V and unit b of a (folded) level-L cell centre, snapshot snap. */
static void or_cart_vb(const or_grid *g, int snap, int L, const long cin[3], double V[3], double b[3])
{
    long c[3] = {cin[0], cin[1], cin[2]};
    or_fold(g, L, c);
    double raw[6], r, th, ph, e[3][3];
    or_raw_virtual(g, snap, L, c, raw);
    or_centre(g, L, c, &r, &th, &ph);
    or_basis(th, ph, e);
    double Bn = sqrt(raw[3] * raw[3] + raw[4] * raw[4] + raw[5] * raw[5]);
    double bs[3] = {raw[3] / Bn, raw[4] / Bn, raw[5] / Bn};
    or_sph_to_cart(e, raw, V);
    or_sph_to_cart(e, bs, b);
}

/* Derivative along dimension a at level-L cell c of the six Cartesian
 * components (V, b): second-order central differences in the uniform
 * (xi, theta, phi) spacing, one-sided second order at physical edges. */
static void or_ddq(const or_grid *g, int snap, int L, const long c[3], int a, double h, double out[6])
{
    long n = or_ncell(g, L, a);
    double Va[3], ba[3], Vb[3], bb[3], Vc[3], bc[3];
    long c1[3] = {c[0], c[1], c[2]}, c2[3] = {c[0], c[1], c[2]};
    int periodic = (a == 2 && g->d.phi_periodic);
    if (!periodic && c[a] == 0) {
        c1[a] = c[a] + 1; c2[a] = c[a] + 2;
        or_cart_vb(g, snap, L, c, Va, ba);
        or_cart_vb(g, snap, L, c1, Vb, bb);
        or_cart_vb(g, snap, L, c2, Vc, bc);
        for (int k = 0; k < 3; ++k) {
            out[k] = (-3.0 * Va[k] + 4.0 * Vb[k] - Vc[k]) / (2.0 * h);
            out[3 + k] = (-3.0 * ba[k] + 4.0 * bb[k] - bc[k]) / (2.0 * h);
        }
    } else if (!periodic && c[a] == n - 1) {
        c1[a] = c[a] - 1; c2[a] = c[a] - 2;
        or_cart_vb(g, snap, L, c, Va, ba);
        or_cart_vb(g, snap, L, c1, Vb, bb);
        or_cart_vb(g, snap, L, c2, Vc, bc);
        for (int k = 0; k < 3; ++k) {
            out[k] = (3.0 * Va[k] - 4.0 * Vb[k] + Vc[k]) / (2.0 * h);
            out[3 + k] = (3.0 * ba[k] - 4.0 * bb[k] + bc[k]) / (2.0 * h);
        }
    } else {
        c1[a] = c[a] + 1; c2[a] = c[a] - 1;
        or_cart_vb(g, snap, L, c1, Vb, bb);
        or_cart_vb(g, snap, L, c2, Vc, bc);
        for (int k = 0; k < 3; ++k) {
            out[k] = (Vb[k] - Vc[k]) / (2.0 * h);
            out[3 + k] = (bb[k] - bc[k]) / (2.0 * h);
        }
    }
}

/* Cartesian V at a leaf cell of snapshot k (same cell, same angles). */
static void or_cart_v_snap(const or_grid *g, int snap, int L, const long c[3], double V[3])
{
    double b[3];
    or_cart_vb(g, snap, L, c, V, b);
}

/* Derived fields of a leaf cell (the quantities Eqs. 2-4 need, section 2.1):
 *   out[0..2]  V  (r, theta, phi components, as given)
 *   out[3..5]  b = B/|B|  (spherical components)
 *   out[6]     div V
 *   out[7]     bb : grad V = b_i b_j dV_i/dx_j
 *   out[8]     div b  (from b itself; div B is not assumed zero)
 *   out[9]     b . dV/dt with dV/dt = dV/dt|_x + (V . grad) V
 *   out[10..12] (b . grad) b  (spherical components)
 * Gradients: Cartesian components differenced in (xi, theta, phi), then the
 * chain rule grad u = u_xi xi'(r) e_r + u_theta e_theta / r + u_phi e_phi / (r sin theta). */
static void or_derived_leafcell(const or_grid *g, int snap, int leaf, int L, const long c[3], double *out)
{
    (void)leaf;
    double raw[6], r, th, ph, e[3][3];
    or_raw_virtual(g, snap, L, c, raw);
    or_centre(g, L, c, &r, &th, &ph);
    or_basis(th, ph, e);
    double Bn = sqrt(raw[3] * raw[3] + raw[4] * raw[4] + raw[5] * raw[5]);
    double bs[3] = {raw[3] / Bn, raw[4] / Bn, raw[5] / Bn};
    double V[3], b[3];
    or_sph_to_cart(e, raw, V);
    or_sph_to_cart(e, bs, b);

    double hL = ldexp(1.0, 1 - L);
    double dq[3][6];
    or_ddq(g, snap, L, c, 0, g->d.dxi * hL, dq[0]);
    or_ddq(g, snap, L, c, 1, g->d.dth * hL, dq[1]);
    or_ddq(g, snap, L, c, 2, g->d.dph * hL, dq[2]);
    double xip = (g->d.xi_map == 1) ? 1.0 / r : 1.0;
    double gq[3][3];   /* gradient of coordinate q, Cartesian components */
    for (int d = 0; d < 3; ++d) {
        gq[0][d] = xip * e[0][d];
        gq[1][d] = e[1][d] / r;
        gq[2][d] = e[2][d] / (r * sin(th));
    }
    double GV[3][3], Gb[3][3];  /* G[a][d] = d u_a / d x_d */
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
            GV[a][d] = dq[0][a] * gq[0][d] + dq[1][a] * gq[1][d] + dq[2][a] * gq[2][d];
            Gb[a][d] = dq[0][3 + a] * gq[0][d] + dq[1][3 + a] * gq[1][d] + dq[2][3 + a] * gq[2][d];
        }
    double divV = GV[0][0] + GV[1][1] + GV[2][2];
    double divb = Gb[0][0] + Gb[1][1] + Gb[2][2];
    double bbgV = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) bbgV += b[a] * b[d] * GV[a][d];

    /* explicit time derivative of V at this cell across snapshots */
    double dVdt[3] = {0.0, 0.0, 0.0};
    int ns = g->d.n_snap_total;
    if (ns == 2) {
        double V0[3], V1[3];
        or_cart_v_snap(g, 0, L, c, V0);
        or_cart_v_snap(g, 1, L, c, V1);
        for (int k = 0; k < 3; ++k) dVdt[k] = (V1[k] - V0[k]) / g->d.dt_s;
    } else if (ns >= 3) {
        double Va[3], Vb[3], Vc[3];
        if (snap == 0) {
            or_cart_v_snap(g, 0, L, c, Va);
            or_cart_v_snap(g, 1, L, c, Vb);
            or_cart_v_snap(g, 2, L, c, Vc);
            for (int k = 0; k < 3; ++k) dVdt[k] = (-3.0 * Va[k] + 4.0 * Vb[k] - Vc[k]) / (2.0 * g->d.dt_s);
        } else if (snap == ns - 1) {
            or_cart_v_snap(g, ns - 1, L, c, Va);
            or_cart_v_snap(g, ns - 2, L, c, Vb);
            or_cart_v_snap(g, ns - 3, L, c, Vc);
            for (int k = 0; k < 3; ++k) dVdt[k] = (3.0 * Va[k] - 4.0 * Vb[k] + Vc[k]) / (2.0 * g->d.dt_s);
        } else {
            or_cart_v_snap(g, snap + 1, L, c, Vb);
            or_cart_v_snap(g, snap - 1, L, c, Vc);
            for (int k = 0; k < 3; ++k) dVdt[k] = (Vb[k] - Vc[k]) / (2.0 * g->d.dt_s);
        }
    }
    double bDV = 0.0;
    for (int a = 0; a < 3; ++a) {
        double conv = GV[a][0] * V[0] + GV[a][1] * V[1] + GV[a][2] * V[2];
        bDV += b[a] * (dVdt[a] + conv);
    }
    double curv[3];
    for (int a = 0; a < 3; ++a) curv[a] = Gb[a][0] * b[0] + Gb[a][1] * b[1] + Gb[a][2] * b[2];

    out[0] = raw[0]; out[1] = raw[1]; out[2] = raw[2];
    out[3] = bs[0]; out[4] = bs[1]; out[5] = bs[2];
    out[6] = divV; out[7] = bbgV; out[8] = divb; out[9] = bDV;
    for (int a = 0; a < 3; ++a) out[10 + a] = curv[0] * e[a][0] + curv[1] * e[a][1] + curv[2] * e[a][2];
}

/* Derived fields at any level-L cell centre (the same virtual-value rule). */
void or_derived_virtual(const void *gp, int snap, int L, const long c[3], double out[13])
{
    or_virtual((const or_grid *)gp, snap, L, c, 13, or_derived_leafcell, out);
}

/* ------------------------------------------------------------------------- */
/* Background at a particle.                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    double V[3], b[3];     /* Cartesian */
    double divV, bbgV, divb, bDV;
    double curv[3];        /* Cartesian */
} or_fields;

/* Spherical coordinates of x and its level-1 grid coordinates s (folded into
 * the domain: clamped along xi and theta, wrapped along a periodic phi). */
static void or_grid_coords(const or_grid *g, const double x[3], double *r, double *th, double *ph, double s[3])
{
    *r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    *th = acos(x[2] / *r);
    *ph = atan2(x[1], x[0]);
    if (*ph < 0.0) *ph += 2.0 * OR_PI;
    s[0] = (g->d.xi_map == 1) ? log(*r / g->d.r_lo) / g->d.dxi : (*r - g->d.r_lo) / g->d.dxi;
    s[1] = (*th - g->d.th_lo) / g->d.dth;
    s[2] = (*ph - g->d.ph_lo) / g->d.dph;
    for (int a = 0; a < 2; ++a) {
        if (s[a] < 0.0) s[a] = 0.0;
        if (s[a] > g->d.n1[a]) s[a] = g->d.n1[a];
    }
    if (g->d.phi_periodic) {
        if (s[2] >= g->d.n1[2]) s[2] -= g->d.n1[2];
        if (s[2] < 0.0) s[2] += g->d.n1[2];
    } else {
        if (s[2] < 0.0) s[2] = 0.0;
        if (s[2] > g->d.n1[2]) s[2] = g->d.n1[2];
    }
}

/* Fields at position x and time t from the grid: trilinear interpolation of
 * the eight surrounding level-L centre values, L the level of the leaf that
 * holds x (section 2.4), each weighted linearly between the two snapshots
 * that bracket t.  Vector fields are interpolated in spherical components and
 * rotated with the particle's own basis; b is renormalised.  Returns 0, or
 * -1 when |b| vanishes. */
int or_grid_fields(const void *gp, const double x[3], double t, double out[16])
{
    const or_grid *g = (const or_grid *)gp;
    double r, th, ph, s[3];
    or_grid_coords(g, x, &r, &th, &ph, s);
    int L;
    long cm[3];
    int leaf = or_find_leaf(g, s, &L, cm);
    if (leaf < 0) return -2;
    long i[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double u = s[a] * ldexp(1.0, L - 1) - 0.5;
        i[a] = (long)floor(u);
        f[a] = u - (double)i[a];
    }
    int ns = g->d.n_snap_total, k = 0;
    double alpha = 0.0;
    if (ns >= 2) {
        double tau = (t - g->d.t_s0) / g->d.dt_s;
        k = (int)floor(tau);
        if (k < 0) k = 0;
        if (k > ns - 2) k = ns - 2;
        alpha = tau - (double)k;
    }
    double acc[13] = {0}, tmp[13];
    for (int sn = 0; sn < (ns >= 2 ? 2 : 1); ++sn) {
        double ws = (ns >= 2) ? (sn == 0 ? 1.0 - alpha : alpha) : 1.0;
        for (int d = 0; d < 8; ++d) {
            int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
            long cc[3] = {i[0] + e0, i[1] + e1, i[2] + e2};
            double w = (e0 ? f[0] : 1.0 - f[0]) * (e1 ? f[1] : 1.0 - f[1]) * (e2 ? f[2] : 1.0 - f[2]);
            or_derived_virtual(g, k + sn, L, cc, tmp);
            for (int m = 0; m < 13; ++m) acc[m] += ws * w * tmp[m];
        }
    }
    double e[3][3];
    or_basis(th, ph, e);
    double V[3], b[3], cv[3];
    or_sph_to_cart(e, acc + 0, V);
    or_sph_to_cart(e, acc + 3, b);
    or_sph_to_cart(e, acc + 10, cv);
    double bn = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    for (int a = 0; a < 3; ++a) { out[a] = V[a]; out[10 + a] = cv[a]; }
    out[6] = acc[6]; out[7] = acc[7]; out[8] = acc[8]; out[9] = acc[9];
    if (!(bn >= 1e-12)) {
        for (int a = 0; a < 3; ++a) out[3 + a] = 0.0;
        return -1;
    }
    for (int a = 0; a < 3; ++a) out[3 + a] = b[a] / bn;
    return 0;
}

/* Analytic backgrounds used to pin the SDE against closed forms. */
static int or_analytic_fields(const or_params *pp, const double x[3], or_fields *F)
{
    const double *bg = pp->bg;
    memset(F, 0, sizeof(*F));
    if (pp->bg_kind == OR_BG_UNIFORM) {
        /* bg[0..2] = V, bg[3..5] = B direction */
        double n = sqrt(bg[3] * bg[3] + bg[4] * bg[4] + bg[5] * bg[5]);
        for (int a = 0; a < 3; ++a) { F->V[a] = bg[a]; F->b[a] = bg[3 + a] / n; }
        return 0;
    }
    if (pp->bg_kind == OR_BG_PAR_FLOW || pp->bg_kind == OR_BG_PERP_FLOW) {
        /* V = U(z) z_hat, U = (U1+U2)/2 - (U1-U2)/2 tanh((z - z_s)/w);
         * bg[0] = U1, bg[1] = U2, bg[2] = w, bg[3] = z_s. */
        double U1 = bg[0], U2 = bg[1], w = bg[2], zs = bg[3];
        double th = tanh((x[2] - zs) / w);
        double U = 0.5 * (U1 + U2) - 0.5 * (U1 - U2) * th;
        double dU = -0.5 * (U1 - U2) * (1.0 - th * th) / w;
        F->V[2] = U;
        F->divV = dU;
        if (pp->bg_kind == OR_BG_PAR_FLOW) {
            F->b[2] = 1.0;           /* B along the flow */
            F->bbgV = dU;            /* b_z b_z dU/dz */
            F->bDV = U * dU;         /* b . (V . grad) V, steady */
        } else {
            F->b[0] = 1.0;           /* B across the flow */
        }
        return 0;
    }
    if (pp->bg_kind == OR_BG_RADIAL) {
        /* V = bg[0] r_hat, b = r_hat (bg[1] = +1) or -r_hat */
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        double sgn = bg[1] >= 0.0 ? 1.0 : -1.0;
        for (int a = 0; a < 3; ++a) { F->V[a] = bg[0] * x[a] / r; F->b[a] = sgn * x[a] / r; }
        F->divV = 2.0 * bg[0] / r;
        F->divb = sgn * 2.0 / r;
        return 0;
    }
    return -2;
}

static int or_fields_at(const or_params *pp, const void *g, const double x[3], double t, or_fields *F)
{
    if (pp->bg_kind != OR_BG_GRID) return or_analytic_fields(pp, x, F);
    double o[16];
    int st = or_grid_fields(g, x, t, o);
    for (int a = 0; a < 3; ++a) { F->V[a] = o[a]; F->b[a] = o[3 + a]; F->curv[a] = o[10 + a]; }
    F->divV = o[6]; F->bbgV = o[7]; F->divb = o[8]; F->bDV = o[9];
    return st;
}

/* ------------------------------------------------------------------------- */
/* One Euler-Maruyama step of the Ito SDEs equivalent to the FTE.             */
/*   dx   = [V + mu v b + div kappa_perp] dt + sqrt(2 kappa_perp)(I - bb) dW  */
/*   dmu  = [dmu/dt of Eq. 3 + dD_mumu/dmu] dt + sqrt(2 D_mumu) dW_mu         */
/*   dlnp = [(dp/dt)/p of Eq. 4] dt                                           */
/* with V_d = 0 (section 2.1), kappa_perp = kappa_perp (I - bb) spatially     */
/* uniform so div kappa_perp = -kappa_perp (div b b + (b . grad) b).          */
/* ------------------------------------------------------------------------- */
typedef struct {
    double x[3], mu, lnp, w;
    uint64_t pid;
    uint32_t kinj;
    int32_t status;
} or_particle;

static int or_finite3(const double *x) { return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]); }

/* Speed for P = p/(m c). */
static double or_speed(double P) { return OR_C * P / sqrt(1.0 + P * P); }

/* Kinetic energy for P: m c^2 (gamma - 1) = m c^2 P^2 / (gamma + 1). */
static double or_ekin(double mass, double P)
{
    double gam = sqrt(1.0 + P * P);
    return mass * OR_C * OR_C * P * P / (gam + 1.0);
}

#define OR_KCUT 6.0

/* Kernel-smoothed intensity sums: every post-step state adds
 *   w v dt G3(x - x_o) G1(ln E - ln E_e)/E G1(t - t_t)
 * to observer o, energy-bin centre E_e and time-bin centre t_t, where G3 and G1
 * are normalised Gaussians of widths sig_x, sig_lne, sig_t cut at OR_KCUT
 * widths (where they have fallen to 1.5e-8 of the peak, so that the jump at the
 * cut adds no visible boundary term to derivatives along a trajectory).
 * Divided by 4 pi W_inj this is a smooth estimate of j = v n_E / (4 pi)
 * (section 2.3) that is differentiable along each trajectory. */
static void or_smooth_add(const or_params *pp, const double x[3], double t1, double w, double P, double *sm)
{
    double gam = sqrt(1.0 + P * P), v = OR_C * P / gam;
    double E = pp->mass * OR_C * OR_C * P * P / (gam + 1.0), lnE = log(E);
    for (int o = 0; o < pp->n_obs; ++o) {
        const double *ob = pp->obs[o];
        double xo[3] = {ob[0] * sin(ob[1]) * cos(ob[2]), ob[0] * sin(ob[1]) * sin(ob[2]), ob[0] * cos(ob[1])};
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) d2 += (x[a] - xo[a]) * (x[a] - xo[a]);
        if (d2 > OR_KCUT * OR_KCUT * pp->sig_x * pp->sig_x) continue;
        double g3 = exp(-d2 / (2.0 * pp->sig_x * pp->sig_x)) /
                    (pow(2.0 * OR_PI, 1.5) * pp->sig_x * pp->sig_x * pp->sig_x);
        for (int e = 0; e < pp->n_e; ++e) {
            double ue = lnE - (log(pp->e_min) + (e + 0.5) * pp->dlne);
            if (fabs(ue) > OR_KCUT * pp->sig_lne) continue;
            double ke = exp(-ue * ue / (2.0 * pp->sig_lne * pp->sig_lne)) / (sqrt(2.0 * OR_PI) * pp->sig_lne) / E;
            for (int it = 0; it < pp->n_t; ++it) {
                double ut = t1 - (pp->t_ref + (it + 0.5) * pp->dT);
                if (fabs(ut) > OR_KCUT * pp->sig_t) continue;
                double kt = exp(-ut * ut / (2.0 * pp->sig_t * pp->sig_t)) / (sqrt(2.0 * OR_PI) * pp->sig_t);
                sm[((long)o * pp->n_e + e) * pp->n_t + it] += w * v * pp->dt * g3 * ke * kt;
            }
        }
    }
}

static void or_step(const or_params *pp, const void *g, or_particle *pt, uint64_t n, double *hist, double *sm)
{
    double t = pp->t0 + (double)n * pp->dt;
    or_fields F;
    int st = or_fields_at(pp, g, pt->x, t, &F);
    if (st != 0) { pt->status = OR_NUMERIC; return; }

    double mu = pt->mu;
    double P = exp(pt->lnp);
    double v = or_speed(P);
    double D, dD;
    or_dmm(pp, v, P, mu, &D, &dD);
    double kperp = 0.0;
    if (pp->kperp_ratio > 0.0) kperp = pp->kperp_ratio * v * or_mfp(pp, P) / 3.0;
    else if (pp->lambda_perp > 0.0) kperp = v * pp->lambda_perp / 3.0;

    double om = 1.0 - mu * mu;
    double a_x[3];
    for (int a = 0; a < 3; ++a)
        a_x[a] = F.V[a] + mu * v * F.b[a] - kperp * (F.divb * F.b[a] + F.curv[a]);
    double a_mu = 0.5 * om * (v * F.divb + mu * F.divV - 3.0 * mu * F.bbgV - (2.0 / v) * F.bDV) + dD;
    double a_lnp = 0.5 * (1.0 - 3.0 * mu * mu) * F.bbgV - 0.5 * om * F.divV - (mu / v) * F.bDV;

    double z[4];
    or_normals(pp->seed, pp->run_id, n, pt->pid, z);
    double xi[3] = {z[1], z[2], z[3]};
    double xib = xi[0] * F.b[0] + xi[1] * F.b[1] + xi[2] * F.b[2];
    double sx = sqrt(2.0 * kperp * pp->dt);
    double xn[3];
    for (int a = 0; a < 3; ++a) xn[a] = pt->x[a] + a_x[a] * pp->dt + sx * (xi[a] - xib * F.b[a]);
    double mun = mu + a_mu * pp->dt + sqrt(2.0 * D * pp->dt) * z[0];
    if (mun > 1.0) mun = 2.0 - mun;
    if (mun < -1.0) mun = -2.0 - mun;
    if (mun > 1.0) mun = 1.0;
    if (mun < -1.0) mun = -1.0;
    double lnpn = pt->lnp + a_lnp * pp->dt;

    if (!or_finite3(xn) || !isfinite(mun) || !isfinite(lnpn)) { pt->status = OR_NUMERIC; return; }
    pt->x[0] = xn[0]; pt->x[1] = xn[1]; pt->x[2] = xn[2];
    pt->mu = mun;
    pt->lnp = lnpn;

    double r = sqrt(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2]);
    if (pp->check_bounds) {
        if (r < pp->r_in) { pt->status = OR_ABS_IN; return; }
        if (r > pp->r_out) { pt->status = OR_ABS_OUT; return; }
        if (pp->bg_kind == OR_BG_GRID) {
            const or_grid *gg = (const or_grid *)g;
            double th = acos(xn[2] / r);
            double th_hi = gg->d.th_lo + gg->d.n1[1] * gg->d.dth;
            if (th < gg->d.th_lo || th > th_hi) { pt->status = OR_OUT_DOMAIN; return; }
        }
    }

    if (sm && pp->smooth && pp->n_obs > 0)
        or_smooth_add(pp, xn, pp->t0 + (double)(n + 1) * pp->dt, pt->w, exp(lnpn), sm);

    /* Residence-time estimator of the intensity j = p^2 f = v n_E / (4 pi)
     * (section 2.3): the post-step state adds w v dt to its bin.  Observer o
     * is the radial x colatitude box around (r, theta) and obs_nphi[o]
     * longitude bins of width dphi, the first centred at phi + omega t (t the
     * post-step time): a box, a ring of bins, or one that corotates. */
    if (hist && pp->n_obs > 0) {
        double th = acos(xn[2] / r);
        double ph = atan2(xn[1], xn[0]);
        if (ph < 0.0) ph += 2.0 * OR_PI;
        double Pn = exp(lnpn), vn = or_speed(Pn);
        double E = or_ekin(pp->mass, Pn);
        double ue = log(E / pp->e_min) / pp->dlne;
        double t1 = pp->t0 + (double)(n + 1) * pp->dt;
        double ut = (t1 - pp->t_ref) / pp->dT;
        if (ue >= 0.0 && ue < pp->n_e && ut >= 0.0 && ut < pp->n_t) {
            long ie = (long)floor(ue), it = (long)floor(ut);
            long ib = (long)(pt->pid % (uint64_t)pp->n_batch);
            int off = 0;
            for (int o = 0; o < pp->n_obs; ++o) {
                const double *ob = pp->obs[o];
                int np = or_nphi(pp, o);
                if (r >= ob[0] - 0.5 * ob[3] && r < ob[0] + 0.5 * ob[3] &&
                    th >= ob[1] - 0.5 * ob[4] && th < ob[1] + 0.5 * ob[4]) {
                    double u = fmod(ph - (ob[2] + pp->obs_omega[o] * t1 - 0.5 * ob[5]), 2.0 * OR_PI);
                    if (u < 0.0) u += 2.0 * OR_PI;
                    long k = (long)floor(u / ob[5]);
                    if (k < np) {
                        long idx = (((off + k) * (long)pp->n_e + ie) * pp->n_t + it) * pp->n_batch + ib;
                        hist[idx] += pt->w * vn * pp->dt;
                    }
                }
                off += np;
            }
        }
    }
}

/* Advance particles through global steps n0 .. n0+n_steps-1.  A particle
 * takes step n only while ACTIVE and n >= kinj.  hist (may be NULL) has
 * n_obs * n_e * n_t * n_batch entries and is accumulated into.  Returns the
 * number of particle-steps taken. */
uint64_t or_run(const or_params *pp, const void *g, long n, double *x, double *mu, double *lnp,
                double *w, const uint64_t *pid, const uint32_t *kinj, int32_t *status,
                uint64_t n0, uint32_t n_steps, double *hist, double *sm, int n_threads)
{
    long hsz = hist ? (long)or_obs_bins(pp) * pp->n_e * pp->n_t * pp->n_batch : 0;
    long ssz = sm ? (long)pp->n_obs * pp->n_e * pp->n_t : 0;
    uint64_t total = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#else
    n_threads = 1;
#endif
    double *priv = hist ? (double *)calloc((size_t)hsz * n_threads, sizeof(double)) : NULL;
    double *spriv = sm ? (double *)calloc((size_t)ssz * n_threads, sizeof(double)) : NULL;
#ifdef _OPENMP
#pragma omp parallel num_threads(n_threads) reduction(+ : total)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *h = priv ? priv + (long)tid * hsz : NULL;
        double *sp = spriv ? spriv + (long)tid * ssz : NULL;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long i = 0; i < n; ++i) {
            or_particle pt;
            pt.x[0] = x[3 * i]; pt.x[1] = x[3 * i + 1]; pt.x[2] = x[3 * i + 2];
            pt.mu = mu[i]; pt.lnp = lnp[i]; pt.w = w[i];
            pt.pid = pid[i]; pt.kinj = kinj[i]; pt.status = status[i];
            for (uint64_t s = n0; s < n0 + n_steps; ++s) {
                if (pt.status != OR_ACTIVE) break;
                if (s < pt.kinj) continue;
                or_step(pp, g, &pt, s, h, sp);
                total += 1;
            }
            x[3 * i] = pt.x[0]; x[3 * i + 1] = pt.x[1]; x[3 * i + 2] = pt.x[2];
            mu[i] = pt.mu; lnp[i] = pt.lnp; w[i] = pt.w; status[i] = pt.status;
        }
    }
    if (hist) {
        for (int t = 0; t < n_threads; ++t)
            for (long k = 0; k < hsz; ++k) hist[k] += priv[(long)t * hsz + k];
        free(priv);
    }
    if (sm) {
        for (int t = 0; t < n_threads; ++t)
            for (long k = 0; k < ssz; ++k) sm[k] += spriv[(long)t * ssz + k];
        free(spriv);
    }
    return total;
}

/* Fields the SDE sees at (x, t), flattened: V[3], b[3], divV, bbgV, divb,
 * bDV, curv[3].  Returns the status of the evaluation. */
int or_fields_public(const or_params *pp, const void *g, const double x[3], double t, double out[13])
{
    or_fields F;
    int st = or_fields_at(pp, g, x, t, &F);
    for (int a = 0; a < 3; ++a) { out[a] = F.V[a]; out[3 + a] = F.b[a]; out[10 + a] = F.curv[a]; }
    out[6] = F.divV; out[7] = F.bbgV; out[8] = F.divb; out[9] = F.bDV;
    return st;
}

/* D_mumu and its mu derivative for a particle of momentum P (tests). */
void or_dmm_public(const or_params *pp, double P, double mu, double out[2])
{
    or_dmm(pp, or_speed(P), P, mu, &out[0], &out[1]);
}

/* ------------------------------------------------------------------------- */
/* Injection (the synthetic workloads' source model; the paper's own law of  */
/* section 2.3, Eq. 6, is the shell/region variant with weight r^-2).        */
/* Draws come from the injection stream (tag 1) at counter step 0 and 1.      */
/* ------------------------------------------------------------------------- */
typedef struct {
    double r;                 /* injection radius, m                            */
    double th_lo, th_hi;      /* colatitude range, rad (uniform in solid angle) */
    double ph_lo, ph_hi;      /* longitude range, rad                           */
    double e_lo, e_hi;        /* kinetic energy range, J (e_lo == e_hi: mono)   */
    double gamma_inj;         /* number spectrum E^-gamma: weight (E/e_lo)^(1-gamma) */
    double w0;                /* weight scale                                   */
    int    r_weight;          /* 1: multiply the weight by (r_ref / r)^2        */
    double r_ref;
    uint64_t pid0;            /* first pid of this injection                    */
    uint64_t n_total;         /* particles in this injection                    */
    uint32_t k0;              /* first injection step                           */
    uint32_t n_inj_steps;     /* 0: all at k0; else stratified over this many   */
    int    region;            /* 1: uniform in volume where div V < divv_max    */
    double r_hi;              /* region: radii r .. r_hi                        */
    double divv_max;          /* region: threshold on the cell's div V, 1/s     */
    uint32_t max_tries;       /* region: attempts before giving up              */
} or_injection;

/* Region test of the paper's injection law: the leaf cell holding x has a
 * converging wind, div V < divv_max, at snapshot k (the cell's own derived
 * value, section 2.3: the region that traces the CIR shocks). */
static int or_in_region(const or_grid *g, const double x[3], int k, double divv_max)
{
    double r, th, ph, s[3];
    or_grid_coords(g, x, &r, &th, &ph, s);
    int L;
    long cm[3];
    int leaf = or_find_leaf(g, s, &L, cm);
    if (leaf < 0) return 0;
    double d[13];
    or_derived_leafcell(g, k, leaf, L, cm, d);
    return d[6] < divv_max;
}

void or_inject(const or_params *pp, const void *gp, const or_injection *inj, long n, uint64_t first_pid,
               double *x, double *mu, double *lnp, double *w, uint64_t *pid, uint32_t *kinj,
               int32_t *status)
{
    const or_grid *g = (const or_grid *)gp;
    double mc2 = pp->mass * OR_C * OR_C;
    for (long i = 0; i < n; ++i) {
        uint64_t p = first_pid + (uint64_t)i;
        uint32_t ka[4], kb[4];
        or_philox_words(pp->seed, pp->run_id, 0, p, 1, ka);
        or_philox_words(pp->seed, pp->run_id, 1, p, 1, kb);
        double u0 = or_u01(ka[0]), u1 = or_u01(ka[1]), u2 = or_u01(ka[2]), u3 = or_u01(ka[3]);
        /* first step: all at k0 or stratified over the injection window */
        if (inj->n_inj_steps > 0) {
            double j = (double)(p - inj->pid0);
            kinj[i] = inj->k0 + (uint32_t)floor((j + or_u01(kb[0])) * (double)inj->n_inj_steps / (double)inj->n_total);
        } else {
            kinj[i] = inj->k0;
        }
        status[i] = OR_ACTIVE;
        /* isotropic pitch-angle cosine */
        mu[i] = 2.0 * u0 - 1.0;
        double c1 = cos(inj->th_lo), c2 = cos(inj->th_hi);
        double rr = inj->r;
        if (!inj->region) {
            /* uniform in solid angle over the patch at radius r */
            double ct = c1 + u1 * (c2 - c1);
            double th = acos(ct);
            double ph = inj->ph_lo + u2 * (inj->ph_hi - inj->ph_lo);
            x[3 * i + 0] = rr * sin(th) * cos(ph);
            x[3 * i + 1] = rr * sin(th) * sin(ph);
            x[3 * i + 2] = rr * ct;
        } else {
            /* uniform in volume over the shell sector, kept where the wind
             * converges (rejection: attempt a uses counter step 2 + a) */
            int snap = 0;
            if (g->d.n_snap_total >= 2) {
                double t = pp->t0 + (double)kinj[i] * pp->dt;
                snap = (int)floor((t - g->d.t_s0) / g->d.dt_s + 0.5);
                if (snap < 0) snap = 0;
                if (snap > g->d.n_snap_total - 1) snap = g->d.n_snap_total - 1;
            }
            double r3a = inj->r * inj->r * inj->r, r3b = inj->r_hi * inj->r_hi * inj->r_hi;
            int ok = 0;
            for (uint32_t a = 0; a < inj->max_tries && !ok; ++a) {
                uint32_t kc[4];
                or_philox_words(pp->seed, pp->run_id, 2 + (uint64_t)a, p, 1, kc);
                rr = cbrt(r3a + or_u01(kc[0]) * (r3b - r3a));
                double ct = c1 + or_u01(kc[1]) * (c2 - c1);
                double st = sqrt(1.0 - ct * ct);
                double ph = inj->ph_lo + or_u01(kc[2]) * (inj->ph_hi - inj->ph_lo);
                x[3 * i + 0] = rr * st * cos(ph);
                x[3 * i + 1] = rr * st * sin(ph);
                x[3 * i + 2] = rr * ct;
                ok = or_in_region(g, x + 3 * i, snap, inj->divv_max);
            }
            if (!ok) status[i] = OR_NUMERIC;
        }
        /* energy: monoenergetic or log-uniform with a power-law weight */
        double E, wt = inj->w0;
        if (inj->e_hi > inj->e_lo) {
            E = exp(log(inj->e_lo) + u3 * (log(inj->e_hi) - log(inj->e_lo)));
            wt *= pow(E / inj->e_lo, 1.0 - inj->gamma_inj);
        } else {
            E = inj->e_lo;
        }
        /* the r^-2 weight of Eq. 6 */
        if (inj->r_weight) wt *= (inj->r_ref / rr) * (inj->r_ref / rr);
        double eps = E / mc2;
        lnp[i] = log(sqrt(eps * (eps + 2.0)));
        w[i] = wt;
        pid[i] = p;
    }
}

/* Intensities from the batch sums: j = S / (4 pi dV dT dE W_inj) per bin
 * and its standard error from the n_batch batch estimates. */
void or_finalize(const or_params *pp, const double *hist, double w_inj, double *j, double *sigma)
{
    int nb = pp->n_batch;
    long ob_i = 0;
    for (int o = 0; o < pp->n_obs; ++o) {
        const double *ob = pp->obs[o];
        double r1 = ob[0] - 0.5 * ob[3], r2 = ob[0] + 0.5 * ob[3];
        double t1 = ob[1] - 0.5 * ob[4], t2 = ob[1] + 0.5 * ob[4];
        double dV = (r2 * r2 * r2 - r1 * r1 * r1) / 3.0 * (cos(t1) - cos(t2)) * ob[5];
        for (int k = 0; k < or_nphi(pp, o); ++k, ++ob_i) {
            for (int e = 0; e < pp->n_e; ++e) {
                double dE = pp->e_min * (exp((e + 1) * pp->dlne) - exp(e * pp->dlne));
                double norm = 4.0 * OR_PI * dV * pp->dT * dE * w_inj;
                for (int t = 0; t < pp->n_t; ++t) {
                    const double *h = hist + ((ob_i * pp->n_e + e) * pp->n_t + t) * nb;
                    double s = 0.0;
                    for (int b = 0; b < nb; ++b) s += h[b];
                    double jm = s / norm;
                    double var = 0.0;
                    for (int b = 0; b < nb; ++b) {
                        double jb = nb * h[b] / norm;
                        var += (jb - jm) * (jb - jm);
                    }
                    long idx = (ob_i * pp->n_e + e) * pp->n_t + t;
                    j[idx] = jm;
                    sigma[idx] = nb > 1 ? sqrt(var / ((double)nb * (nb - 1))) : 0.0;
                }
            }
        }
    }
}

/* Steady state for a constant injection rate from a Green's-function run
 * (all particles injected at one time; section 2.3): the time integral of
 * the intensity, i.e. the sum over time bins of j dT,
 *   J[o][e] = sum_t S[o][e][t] / (4 pi dV dE W_inj),
 * per unit injected weight per unit time; sigma from the batch estimates of
 * the time-summed sums. */
void or_finalize_steady(const or_params *pp, const double *hist, double w_inj, double *j, double *sigma)
{
    int nb = pp->n_batch;
    long ob_i = 0;
    double *sb = (double *)calloc((size_t)nb, sizeof(double));
    for (int o = 0; o < pp->n_obs; ++o) {
        const double *ob = pp->obs[o];
        double r1 = ob[0] - 0.5 * ob[3], r2 = ob[0] + 0.5 * ob[3];
        double t1 = ob[1] - 0.5 * ob[4], t2 = ob[1] + 0.5 * ob[4];
        double dV = (r2 * r2 * r2 - r1 * r1 * r1) / 3.0 * (cos(t1) - cos(t2)) * ob[5];
        for (int k = 0; k < or_nphi(pp, o); ++k, ++ob_i) {
            for (int e = 0; e < pp->n_e; ++e) {
                double dE = pp->e_min * (exp((e + 1) * pp->dlne) - exp(e * pp->dlne));
                double norm = 4.0 * OR_PI * dV * dE * w_inj;
                for (int b = 0; b < nb; ++b) sb[b] = 0.0;
                for (int t = 0; t < pp->n_t; ++t) {
                    const double *h = hist + ((ob_i * pp->n_e + e) * pp->n_t + t) * nb;
                    for (int b = 0; b < nb; ++b) sb[b] += h[b];
                }
                double s = 0.0;
                for (int b = 0; b < nb; ++b) s += sb[b];
                double jm = s / norm;
                double var = 0.0;
                for (int b = 0; b < nb; ++b) {
                    double jb = nb * sb[b] / norm;
                    var += (jb - jm) * (jb - jm);
                }
                long idx = ob_i * pp->n_e + e;
                j[idx] = jm;
                sigma[idx] = nb > 1 ? sqrt(var / ((double)nb * (nb - 1))) : 0.0;
            }
        }
    }
    free(sb);
}

int or_abi_version(void) { return 1; }
