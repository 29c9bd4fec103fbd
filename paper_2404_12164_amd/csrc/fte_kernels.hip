// HIP kernels of the focused-transport pseudo-particle path (gfx950).
//
// Load time (once per snapshot): ghost-fill of the raw wind, derived fields,
// ghost-fill of the records.  Run time: injection, the fused step kernel
// (locate -> gather -> coefficients -> noise -> update -> boundaries ->
// observers, many steps per launch with the state in registers), compaction of
// retired particles, and the observer finalisation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fte_device.hpp"
#include "fte_internal.hpp"

namespace fte {

// ===========================================================================
// load time
// ===========================================================================
// raw input: [snap][leaf][cell][6] double, cell = i + bx (j + by k)
struct RawSrc {
    const double *p;             // this snapshot: [leaf][cell][6]
    const int32_t *leaf_info;
    int n_leaves, cells, bx0, bx1, bx2;
    __device__ void mean_cube(int leaf, const int cm[3], int k, double out[6]) const {
        const int4 li = reinterpret_cast<const int4 *>(leaf_info)[leaf];
        const int l0 = cm[0] - li.y * bx0, l1 = cm[1] - li.z * bx1, l2 = cm[2] - li.w * bx2;
        for (int q = 0; q < 6; ++q) out[q] = 0.0;
        if (l0 < 0 || l1 < 0 || l2 < 0 || l0 + k > bx0 || l1 + k > bx1 || l2 + k > bx2) {
            for (int q = 0; q < 6; ++q) out[q] = __builtin_nan("");
            return;
        }
        for (int c2 = 0; c2 < k; ++c2)
            for (int c1 = 0; c1 < k; ++c1)
                for (int c0 = 0; c0 < k; ++c0) {
                    const size_t idx = (l0 + c0) + (size_t)bx0 * ((l1 + c1) + (size_t)bx1 * (l2 + c2));
                    const double *src = p + ((size_t)leaf * cells + idx) * 6;
                    for (int q = 0; q < 6; ++q) out[q] += src[q];
                }
        const double inv = 1.0 / (double)(k * k * k);
        for (int q = 0; q < 6; ++q) out[q] *= inv;
    }
};

// records: [slot][block][pcell][rs] of R, interior at padded offset +1; the
// block of a leaf through the grid's pool map when a subset is held (a leaf
// not held reads as NaN, which the caller flags)
template <typename R>
struct RecSrc {
    const R *p;
    const DevGrid *g;
    int snap, pcells, px0, px1, bx0, bx1, bx2, rs, nf;
    __device__ void mean_cube(int leaf, const int cm[3], int k, double out[kNF]) const {
        const int4 li = reinterpret_cast<const int4 *>(g->leaf_info)[leaf];
        const int l0 = cm[0] - li.y * bx0, l1 = cm[1] - li.z * bx1, l2 = cm[2] - li.w * bx2;
        const int blk = pool_block(*g, snap, leaf);
        for (int q = 0; q < kNF; ++q) out[q] = 0.0;
        if (blk < 0 || l0 < 0 || l1 < 0 || l2 < 0 || l0 + k > bx0 || l1 + k > bx1 || l2 + k > bx2) {
            for (int q = 0; q < kNF; ++q) out[q] = __builtin_nan("");
            return;
        }
        for (int c2 = 0; c2 < k; ++c2)
            for (int c1 = 0; c1 < k; ++c1)
                for (int c0 = 0; c0 < k; ++c0) {
                    const size_t pc = (l0 + c0 + 1) + (size_t)px0 * ((l1 + c1 + 1) + (size_t)px1 * (l2 + c2 + 1));
                    const R *src = p + (((size_t)snap * g->n_blk + blk) * pcells + pc) * rs;
                    for (int q = 0; q < nf; ++q) out[q] += (double)src[q];
                }
        const double inv = 1.0 / (double)(k * k * k);
        for (int q = 0; q < kNF; ++q) out[q] *= inv;
    }
};

__device__ __forceinline__ void basis(double th, double ph, double e[3][3]) {
    double st, ct, sp, cp;
    ::sincos(th, &st, &ct);
    ::sincos(ph, &sp, &cp);
    e[0][0] = st * cp; e[0][1] = st * sp; e[0][2] = ct;
    e[1][0] = ct * cp; e[1][1] = ct * sp; e[1][2] = -st;
    e[2][0] = -sp;     e[2][1] = cp;      e[2][2] = 0.0;
}

__device__ __forceinline__ void centre(const DevGrid &G, int L, const int c[3], double *r, double *th, double *ph) {
    const double h = ::ldexp(1.0, 1 - L);
    const double xi = ((double)c[0] + 0.5) * G.dxi * h;
    *r = G.xi_map ? G.r_lo * ::exp(xi) : G.r_lo + xi;
    *th = G.th_lo + ((double)c[1] + 0.5) * G.dth * h;
    *ph = G.ph_lo + ((double)c[2] + 0.5) * G.dph * h;
}

// decode (leaf, padded cell) -> level, global level-L index, local index
__device__ __forceinline__ void decode_pcell(const DevGrid &G, int leaf, int pc, int *L, int c[3], int loc[3]) {
    const int4 li = reinterpret_cast<const int4 *>(G.leaf_info)[leaf];
    loc[0] = pc % G.px[0] - 1;
    loc[1] = (pc / G.px[0]) % G.px[1] - 1;
    loc[2] = pc / (G.px[0] * G.px[1]) - 1;
    *L = li.x;
    c[0] = li.y * G.bx[0] + loc[0];
    c[1] = li.z * G.bx[1] + loc[1];
    c[2] = li.w * G.bx[2] + loc[2];
}

// Flag non-finite values or a vanishing |B| in the raw input.
__global__ void k_check_raw(const double *raw, size_t n_cells, DevCounters *cnt) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_cells) return;
    const double *v = raw + i * 6;
    bool bad = false;
    for (int q = 0; q < 6; ++q) bad |= !isfinite(v[q]);
    bad |= !(v[3] * v[3] + v[4] * v[4] + v[5] * v[5] > 0.0);
    if (bad) atomicOr(&cnt->flags, kFlagBadInput);
}

__device__ __forceinline__ const double *raw_at(const RawWin &W, int j) { return W.s[j - W.k + 2]; }

// Padded Cartesian (V, b) of one snapshot: interior cells from the input,
// ghost cells by the block-boundary rule, then rotated with the angles of the
// (folded) cell centre.
__global__ void k_raw_ghost(DevGrid G, RawWin W, double *cart, DevCounters *cnt, LeafList ll) {
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = ll.ids ? ll.n : G.n_leaves;
    if (gid >= (size_t)nl * G.pcells) return;
    const int leaf = ll.ids ? ll.ids[gid / G.pcells] : (int)(gid / G.pcells), pc = (int)(gid % G.pcells);
    int L, c[3], loc[3];
    decode_pcell(G, leaf, pc, &L, c, loc);
    double v[6];
    const bool interior = loc[0] >= 0 && loc[0] < G.bx[0] && loc[1] >= 0 && loc[1] < G.bx[1] && loc[2] >= 0 &&
                          loc[2] < G.bx[2];
    if (interior) {
        const size_t idx = loc[0] + (size_t)G.bx[0] * (loc[1] + (size_t)G.bx[1] * loc[2]);
        const double *src = raw_at(W, W.k) + ((size_t)leaf * G.cells + idx) * 6;
        for (int q = 0; q < 6; ++q) v[q] = src[q];
    } else {
        RawSrc S{raw_at(W, W.k), G.leaf_info, G.n_leaves, G.cells, G.bx[0], G.bx[1], G.bx[2]};
        if (!virtual_value<6>(G, S, L, c, v)) {
            atomicOr(&cnt->flags, kFlagAmrDepth);
            for (int q = 0; q < 6; ++q) v[q] = __builtin_nan("");
        }
    }
    fold(G, L, c);
    double r, th, ph, e[3][3];
    centre(G, L, c, &r, &th, &ph);
    basis(th, ph, e);
    const double Bn = ::sqrt(v[3] * v[3] + v[4] * v[4] + v[5] * v[5]);
    const double bs[3] = {v[3] / Bn, v[4] / Bn, v[5] / Bn};
    double *dst = cart + ((size_t)leaf * G.pcells + pc) * 6;
    for (int a = 0; a < 3; ++a) {
        dst[a] = v[0] * e[0][a] + v[1] * e[1][a] + v[2] * e[2][a];
        dst[3 + a] = bs[0] * e[0][a] + bs[1] * e[1][a] + bs[2] * e[2][a];
    }
}

// Cartesian V of an interior cell taken straight from the input of snapshot k.
__device__ __forceinline__ void cart_v_input(const DevGrid &G, const double *snapshot, int leaf, size_t idx,
                                             const double e[3][3], double V[3]) {
    const double *s = snapshot + ((size_t)leaf * G.cells + idx) * 6;
    for (int a = 0; a < 3; ++a) V[a] = s[0] * e[0][a] + s[1] * e[1][a] + s[2] * e[2][a];
}

// Derived fields of every interior cell of one snapshot (the quantities of
// Eqs. 2-4): second-order central differences of the Cartesian (V, b) in the
// uniform (xi, theta, phi) spacing (one-sided at physical edges), chain rule
// with the analytic Jacobian at the centre, explicit dV/dt across snapshots.
template <typename R>
__global__ void k_derive(DevGrid G, RawWin W, const double *cart, R *rec, LeafList ll) {
    const int snap = W.k;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = ll.ids ? ll.n : G.n_leaves;
    if (gid >= (size_t)nl * G.cells) return;
    const int leaf = ll.ids ? ll.ids[gid / G.cells] : (int)(gid / G.cells);
    const int idx = (int)(gid % G.cells);
    const int loc[3] = {idx % G.bx[0], (idx / G.bx[0]) % G.bx[1], idx / (G.bx[0] * G.bx[1])};
    const int4 li = reinterpret_cast<const int4 *>(G.leaf_info)[leaf];
    const int L = li.x;
    const int c[3] = {li.y * G.bx[0] + loc[0], li.z * G.bx[1] + loc[1], li.w * G.bx[2] + loc[2]};
    const int pc = (loc[0] + 1) + G.px[0] * ((loc[1] + 1) + G.px[1] * (loc[2] + 1));
    const int stride[3] = {1, G.px[0], G.px[0] * G.px[1]};
    const double *U = cart + (size_t)leaf * G.pcells * 6;
    const double hL = ::ldexp(1.0, 1 - L);
    const double h[3] = {G.dxi * hL, G.dth * hL, G.dph * hL};

    double dq[3][6];
    for (int a = 0; a < 3; ++a) {
        const int n = ncell(G, L, a);
        const bool periodic = (a == 2) && G.periodic;
        const double *u0 = U + (size_t)pc * 6;
        if (!periodic && c[a] == 0) {
            const double *u1 = U + (size_t)(pc + stride[a]) * 6, *u2 = U + (size_t)(pc + 2 * stride[a]) * 6;
            for (int q = 0; q < 6; ++q) dq[a][q] = (-3.0 * u0[q] + 4.0 * u1[q] - u2[q]) / (2.0 * h[a]);
        } else if (!periodic && c[a] == n - 1) {
            const double *u1 = U + (size_t)(pc - stride[a]) * 6, *u2 = U + (size_t)(pc - 2 * stride[a]) * 6;
            for (int q = 0; q < 6; ++q) dq[a][q] = (3.0 * u0[q] - 4.0 * u1[q] + u2[q]) / (2.0 * h[a]);
        } else {
            const double *up = U + (size_t)(pc + stride[a]) * 6, *um = U + (size_t)(pc - stride[a]) * 6;
            for (int q = 0; q < 6; ++q) dq[a][q] = (up[q] - um[q]) / (2.0 * h[a]);
        }
    }
    double r, th, ph, e[3][3];
    centre(G, L, c, &r, &th, &ph);
    basis(th, ph, e);
    const double xip = G.xi_map ? 1.0 / r : 1.0;
    const double st = ::sin(th);
    double gq[3][3];
    for (int d = 0; d < 3; ++d) {
        gq[0][d] = xip * e[0][d];
        gq[1][d] = e[1][d] / r;
        gq[2][d] = e[2][d] / (r * st);
    }
    double GV[3][3], Gb[3][3];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
            GV[a][d] = dq[0][a] * gq[0][d] + dq[1][a] * gq[1][d] + dq[2][a] * gq[2][d];
            Gb[a][d] = dq[0][3 + a] * gq[0][d] + dq[1][3 + a] * gq[1][d] + dq[2][3 + a] * gq[2][d];
        }
    const double *u = U + (size_t)pc * 6;
    const double V[3] = {u[0], u[1], u[2]}, b[3] = {u[3], u[4], u[5]};
    const double divV = GV[0][0] + GV[1][1] + GV[2][2];
    const double divb = Gb[0][0] + Gb[1][1] + Gb[2][2];
    double bbgV = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) bbgV += b[a] * b[d] * GV[a][d];

    double dVdt[3] = {0.0, 0.0, 0.0};
    const int ns = G.n_snap;
    if (ns == 2) {
        double V0[3], V1[3];
        cart_v_input(G, raw_at(W, 0), leaf, idx, e, V0);
        cart_v_input(G, raw_at(W, 1), leaf, idx, e, V1);
        for (int a = 0; a < 3; ++a) dVdt[a] = (V1[a] - V0[a]) / G.dt_s;
    } else if (ns >= 3) {
        double Va[3], Vb[3], Vc[3];
        if (snap == 0) {
            cart_v_input(G, raw_at(W, 0), leaf, idx, e, Va);
            cart_v_input(G, raw_at(W, 1), leaf, idx, e, Vb);
            cart_v_input(G, raw_at(W, 2), leaf, idx, e, Vc);
            for (int a = 0; a < 3; ++a) dVdt[a] = (-3.0 * Va[a] + 4.0 * Vb[a] - Vc[a]) / (2.0 * G.dt_s);
        } else if (snap == ns - 1) {
            cart_v_input(G, raw_at(W, ns - 1), leaf, idx, e, Va);
            cart_v_input(G, raw_at(W, ns - 2), leaf, idx, e, Vb);
            cart_v_input(G, raw_at(W, ns - 3), leaf, idx, e, Vc);
            for (int a = 0; a < 3; ++a) dVdt[a] = (3.0 * Va[a] - 4.0 * Vb[a] + Vc[a]) / (2.0 * G.dt_s);
        } else {
            cart_v_input(G, raw_at(W, snap + 1), leaf, idx, e, Vb);
            cart_v_input(G, raw_at(W, snap - 1), leaf, idx, e, Vc);
            for (int a = 0; a < 3; ++a) dVdt[a] = (Vb[a] - Vc[a]) / (2.0 * G.dt_s);
        }
    }
    double bDV = 0.0;
    for (int a = 0; a < 3; ++a) bDV += b[a] * (dVdt[a] + GV[a][0] * V[0] + GV[a][1] * V[1] + GV[a][2] * V[2]);
    double curv[3];
    for (int a = 0; a < 3; ++a) curv[a] = Gb[a][0] * b[0] + Gb[a][1] * b[1] + Gb[a][2] * b[2];

    const double *s = raw_at(W, snap) + ((size_t)leaf * G.cells + idx) * 6;
    const double Bn = ::sqrt(s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
    const int slot = snap % G.n_slots;
    R *out = rec + (((size_t)slot * G.n_blk + pool_block(G, slot, leaf)) * G.pcells + pc) * G.rs;
    out[0] = (R)s[0];
    out[1] = (R)s[1];
    out[2] = (R)s[2];
    out[3] = (R)(s[3] / Bn);
    out[4] = (R)(s[4] / Bn);
    out[5] = (R)(s[5] / Bn);
    out[6] = (R)divV;
    out[7] = (R)bbgV;
    out[8] = (R)divb;
    out[9] = (R)bDV;
    if (G.nf > 10)
        for (int a = 0; a < 3; ++a) out[10 + a] = (R)(curv[0] * e[a][0] + curv[1] * e[a][1] + curv[2] * e[a][2]);
    for (int q = G.nf; q < G.rs; ++q) out[q] = (R)0;
}

// Ghost layer of the records by the block-boundary rule.
template <typename R>
__global__ void k_record_ghost(DevGrid G, int slot, R *rec, DevCounters *cnt, LeafList ll) {
    const int snap = slot;    // records are addressed by slot
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = ll.ids ? ll.n : G.n_leaves;
    if (gid >= (size_t)nl * G.pcells) return;
    const int leaf = ll.ids ? ll.ids[gid / G.pcells] : (int)(gid / G.pcells), pc = (int)(gid % G.pcells);
    int L, c[3], loc[3];
    decode_pcell(G, leaf, pc, &L, c, loc);
    const bool interior = loc[0] >= 0 && loc[0] < G.bx[0] && loc[1] >= 0 && loc[1] < G.bx[1] && loc[2] >= 0 &&
                          loc[2] < G.bx[2];
    if (interior) return;
    RecSrc<R> S{rec, &G, snap, G.pcells, G.px[0], G.px[1], G.bx[0], G.bx[1], G.bx[2], G.rs, G.nf};
    double v[kNF];
    R *out = rec + (((size_t)snap * G.n_blk + pool_block(G, snap, leaf)) * G.pcells + pc) * G.rs;
    if (!virtual_value<kNF>(G, S, L, c, v)) {
        atomicOr(&cnt->flags, kFlagAmrDepth);
        for (int q = 0; q < kNF; ++q) v[q] = __builtin_nan("");
    }
    if (G.pool_map) {
        // a neighbour the ghost rule reads is not held in the pool
        bool fin = true;
        for (int q = 0; q < G.nf; ++q) fin &= isfinite(v[q]);
        if (!fin) atomicOr(&cnt->flags, kFlagNotResident);
    }
    for (int q = 0; q < G.nf; ++q) out[q] = (R)v[q];
    for (int q = G.nf; q < G.rs; ++q) out[q] = (R)0;
}

static inline unsigned blocks_for(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_check_raw(const DevGrid &g, const double *raw, size_t n_snaps, DevCounters *cnt, hipStream_t s) {
    const size_t n = n_snaps * g.n_leaves * g.cells;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_raw, dim3(blocks_for(n, 256)), dim3(256), 0, s, raw, n, cnt);
    return hipGetLastError();
}

hipError_t launch_raw_ghost(const DevGrid &g, const RawWin &w, double *work_cart, DevCounters *cnt, LeafList ll,
                            hipStream_t s) {
    const size_t n = (size_t)(ll.ids ? ll.n : g.n_leaves) * g.pcells;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_raw_ghost, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, w, work_cart, cnt, ll);
    return hipGetLastError();
}

hipError_t launch_derive(const DevGrid &g, const RawWin &w, const double *work_cart, void *rec, int fp32, LeafList ll,
                         hipStream_t s) {
    const size_t n = (size_t)(ll.ids ? ll.n : g.n_leaves) * g.cells;
    if (n == 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_derive<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, w, work_cart, (float *)rec,
                           ll);
    else
        hipLaunchKernelGGL(k_derive<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, w, work_cart,
                           (double *)rec, ll);
    return hipGetLastError();
}

hipError_t launch_record_ghost(const DevGrid &g, int snap, void *rec, int fp32, DevCounters *cnt, LeafList ll,
                               hipStream_t s) {
    const size_t n = (size_t)(ll.ids ? ll.n : g.n_leaves) * g.pcells;
    if (n == 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_record_ghost<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, snap, (float *)rec,
                           cnt, ll);
    else
        hipLaunchKernelGGL(k_record_ghost<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, snap,
                           (double *)rec, cnt, ll);
    return hipGetLastError();
}

// Non-finite values or |B| = 0 in the cells of the listed leaves of one
// snapshot [leaf][cell][6].
__global__ void k_check_raw_leaves(const double *raw, int cells, LeafList ll, DevCounters *cnt) {
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)ll.n * cells) return;
    const double *v = raw + ((size_t)ll.ids[gid / cells] * cells + gid % cells) * 6;
    bool bad = false;
    for (int q = 0; q < 6; ++q) bad |= !isfinite(v[q]);
    bad |= !(v[3] * v[3] + v[4] * v[4] + v[5] * v[5] > 0.0);
    if (bad) atomicOr(&cnt->flags, kFlagBadInput);
}

hipError_t launch_check_raw_leaves(const DevGrid &g, const double *raw, DevCounters *cnt, LeafList ll, hipStream_t s) {
    const size_t n = (size_t)ll.n * g.cells;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_raw_leaves, dim3(blocks_for(n, 256)), dim3(256), 0, s, raw, g.cells, ll, cnt);
    return hipGetLastError();
}

// ===========================================================================
// the step kernel
// ===========================================================================
template <typename R>
struct Fields {
    R V[3], b[3], divV, bbgV, divb, bDV, curv[3];
};

// Level-1 grid coordinates of a position already reduced to (r, theta, phi),
// folded into the domain.
template <typename R>
__device__ __forceinline__ void grid_coords(const DevGrid &G, R r, R th, R ph, R s[3]);

template <>
__device__ __forceinline__ void grid_coords<double>(const DevGrid &G, double r, double th, double ph, double s[3]) {
    s[0] = G.xi_map ? ::log(r / G.r_lo) * G.inv_dxi : (r - G.r_lo) * G.inv_dxi;
    s[1] = (th - G.th_lo) * G.inv_dth;
    s[2] = (ph - G.ph_lo) * G.inv_dph;
}

template <>
__device__ __forceinline__ void grid_coords<float>(const DevGrid &G, float r, float th, float ph, float s[3]) {
    s[0] = G.xi_map ? __logf(r * (float)G.inv_r_lo) * (float)G.inv_dxi : (r - (float)G.r_lo) * (float)G.inv_dxi;
    s[1] = (th - (float)G.th_lo) * (float)G.inv_dth;
    s[2] = (ph - (float)G.ph_lo) * (float)G.inv_dph;
}

// Walk the block index from level 1 down to the leaf that holds the folded
// level-1 coordinates s.  S receives the coordinates in cells of the leaf's
// level, B the leaf's block index and *Lout (if given) its level; returns the
// leaf id or -1.
template <typename R>
__device__ __forceinline__ int descend(const DevGrid &G, const int32_t *base, const int32_t *child, const R s[3],
                                       R S[3], int B[3], int *Lout = nullptr) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int c = (int)M<R>::floor_(s[a]);
        c = c > G.n1[a] - 1 ? G.n1[a] - 1 : c;
        B[a] = div_bx(G, c, a);
        S[a] = s[a];
    }
    int node = base[B[0] + G.nb1[0] * (B[1] + G.nb1[1] * B[2])];
    int L = 1;
    while (node < 0) {
        const int grp = -node - 1;
        ++L;
        if (L > G.n_levels) return -1;
        int slot = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            S[a] = S[a] * (R)2;
            int c = (int)M<R>::floor_(S[a]);
            const int n = G.n1[a] << (L - 1);
            c = c > n - 1 ? n - 1 : c;
            B[a] = div_bx(G, c, a);
            slot |= (B[a] & 1) << a;
        }
        node = child[grp * 8 + slot];
    }
    if (Lout) *Lout = L;
    return node;
}

// Fold level-1 coordinates into the domain: clamp xi and theta (NaN -> 0),
// wrap a periodic phi.
template <typename R>
__device__ __forceinline__ void fold_s(const DevGrid &G, R s[3]) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const R n = (R)G.n1[a];
        s[a] = (s[a] >= (R)0) ? (s[a] > n ? n : s[a]) : (R)0;
    }
    const R n = (R)G.n1[2];
    if (G.periodic) {
        if (s[2] >= n) s[2] -= n;
        if (s[2] < (R)0) s[2] += n;
        if (!(s[2] >= (R)0 && s[2] < n)) s[2] = (R)0;
    } else {
        s[2] = (s[2] >= (R)0) ? (s[2] > n ? n : s[2]) : (R)0;
    }
}

// Level-1 blocks holding a held particle and the largest ln p among them (for
// planning which leaves a snapshot window needs).  Positive floats order like
// their bit patterns, so the maximum is an integer atomic.
__global__ void k_occupancy(DevGrid G, DevState st, const DevCounters *cnt, int slot, uint32_t *occ,
                            uint32_t *lnp_bits) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt->n_live[slot] || st.status[i] != FTE_PS_ACTIVE) return;
    const double x = st.x[i], y = st.y[i], z = st.z[i];
    const double r = ::sqrt(x * x + y * y + z * z);
    double ph = ::atan2(y, x);
    if (ph < 0.0) ph += 2.0 * kPi;
    double sc[3];
    grid_coords<double>(G, r, ::acos(z / r), ph, sc);
    fold_s<double>(G, sc);
    int B[3];
    for (int a = 0; a < 3; ++a) {
        int c = (int)::floor(sc[a]);
        c = c > G.n1[a] - 1 ? G.n1[a] - 1 : (c < 0 ? 0 : c);
        B[a] = div_bx(G, c, a);
    }
    occ[B[0] + G.nb1[0] * (B[1] + G.nb1[1] * B[2])] = 1u;
    const float lp = (float)st.lnp[i];
    const float pos = lp > -80.f ? lp + 80.f : 0.f;     // shifted to stay positive
    atomicMax(lnp_bits, __float_as_uint(pos));
}

hipError_t launch_occupancy(const DevGrid &g, DevState st, const DevCounters *cnt, int slot, uint64_t n_upper,
                            uint32_t *occ, uint32_t *lnp_bits, hipStream_t s) {
    if (n_upper == 0) return hipSuccess;
    hipLaunchKernelGGL(k_occupancy, dim3(blocks_for(n_upper, 256)), dim3(256), 0, s, g, st, cnt, slot, occ, lnp_bits);
    return hipGetLastError();
}

// ===========================================================================
// injection
// ===========================================================================
// Region test of the paper's injection law (section 2.3): the leaf cell
// holding x has div V < divv_max at snapshot k (its own record value).
__device__ bool in_region(const DevGrid &G, int rec_fp32, double x, double y, double z, int k, double divv_max,
                          unsigned int *flags) {
    const double r = ::sqrt(x * x + y * y + z * z);
    const double th = ::acos(z / r);
    double ph = ::atan2(y, x);
    if (ph < 0.0) ph += 2.0 * kPi;
    double s[3];
    grid_coords<double>(G, r, th, ph, s);
    fold_s<double>(G, s);
    int B[3], L;
    double S[3];
    const int leaf = descend<double>(G, G.base, G.child, s, S, B, &L);
    if (leaf < 0) return false;
    int loc[3];
    for (int a = 0; a < 3; ++a) {
        const int n = G.n1[a] << (L - 1);
        int c = (int)::floor(S[a]);
        c = c > n - 1 ? n - 1 : c;
        loc[a] = c - B[a] * G.bx[a];
    }
    const size_t pc = (size_t)(loc[0] + 1) + (size_t)G.px[0] * ((loc[1] + 1) + (size_t)G.px[1] * (loc[2] + 1));
    const int blk = pool_block(G, k % G.n_slots, leaf);
    if (blk < 0 || (G.pool_map && G.pool_map[(size_t)(k % G.n_slots) * G.n_leaves + leaf] < 0)) {
        atomicOr(flags, kFlagNotResident);     // a streamed subset without this leaf
        return false;
    }
    const size_t at = (((size_t)(k % G.n_slots) * G.n_blk + blk) * G.pcells + pc) * G.rs + 6;
    const double dv = rec_fp32 ? (double)reinterpret_cast<const float *>(G.rec)[at]
                               : reinterpret_cast<const double *>(G.rec)[at];
    return dv < divv_max;
}

__global__ void k_inject(DevParams P, DevGrid G, int rec_fp32, fte_injection inj, DevState st, DevTan tn,
                         DevCounters *cnt, int slot, uint64_t n, uint64_t first_pid) {
    __shared__ double wsum[FTE_MAX_BATCH];
    __shared__ double wdg;
    for (int b = threadIdx.x; b < FTE_MAX_BATCH; b += blockDim.x) wsum[b] = 0.0;
    if (threadIdx.x == 0) wdg = 0.0;
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint64_t base = cnt->n_live[slot];
        const uint64_t pid = first_pid + i;
        const int rid = P.n_runs > 0 ? P.runs[inj.run].run_id : P.run_id;
        const U4 ka = philox_words(P.seed, rid, 0, pid, 1u);
        const U4 kb = philox_words(P.seed, rid, 1, pid, 1u);
        const double u0 = M<double>::u01(ka.a), u1 = M<double>::u01(ka.b);
        const double u2 = M<double>::u01(ka.c), u3 = M<double>::u01(ka.d);
        // first step: all at k0 or stratified over the injection window
        uint32_t k = inj.k0;
        if (inj.n_inj_steps > 0) {
            const double jj = (double)(pid - inj.pid0);
            k = inj.k0 + (uint32_t)::floor((jj + M<double>::u01(kb.a)) * (double)inj.n_inj_steps /
                                           (double)inj.n_total);
        }
        const double mu = 2.0 * u0 - 1.0;
        const double c1 = ::cos(inj.th_lo), c2 = ::cos(inj.th_hi);
        double rr = inj.r, px, py, pz;
        int status = FTE_PS_ACTIVE;
        if (!inj.region) {
            // uniform in solid angle over the patch at radius r
            const double ct = c1 + u1 * (c2 - c1);
            const double th = ::acos(ct);
            const double ph = inj.ph_lo + u2 * (inj.ph_hi - inj.ph_lo);
            px = rr * ::sin(th) * ::cos(ph);
            py = rr * ::sin(th) * ::sin(ph);
            pz = rr * ct;
        } else {
            // uniform in volume over the shell sector, kept where the wind
            // converges; attempt a draws from counter step 2 + a
            int snap = 0;
            if (G.n_snap >= 2) {
                const double t = P.t0 + (double)k * P.dt;
                double f = ::floor((t - G.t_s0) / G.dt_s + 0.5);
                f = f < 0.0 ? 0.0 : (f > (double)(G.n_snap - 1) ? (double)(G.n_snap - 1) : f);
                snap = (int)f;
            }
            const double r3a = inj.r * inj.r * inj.r, r3b = inj.r_hi * inj.r_hi * inj.r_hi;
            bool ok = false;
            px = py = pz = 0.0;
            for (uint32_t a = 0; a < inj.max_tries && !ok; ++a) {
                const U4 kc = philox_words(P.seed, rid, 2 + (uint64_t)a, pid, 1u);
                rr = ::cbrt(r3a + M<double>::u01(kc.a) * (r3b - r3a));
                const double ct = c1 + M<double>::u01(kc.b) * (c2 - c1);
                const double stt = ::sqrt(1.0 - ct * ct);
                const double ph = inj.ph_lo + M<double>::u01(kc.c) * (inj.ph_hi - inj.ph_lo);
                px = rr * stt * ::cos(ph);
                py = rr * stt * ::sin(ph);
                pz = rr * ct;
                ok = in_region(G, rec_fp32, px, py, pz, snap, inj.divv_max, &cnt->flags);
            }
            if (!ok) status = FTE_PS_NUMERIC;
        }
        double E, wt = inj.w0, dlnw = 0.0;
        if (inj.e_hi > inj.e_lo) {
            E = ::exp(::log(inj.e_lo) + u3 * (::log(inj.e_hi) - ::log(inj.e_lo)));
            wt *= ::pow(E / inj.e_lo, 1.0 - inj.gamma_inj);
            dlnw = -::log(E / inj.e_lo);     // d ln w / d gamma_inj
        } else {
            E = inj.e_lo;
        }
        if (inj.r_weight) wt *= (inj.r_ref / rr) * (inj.r_ref / rr);
        const double eps = E / P.mass_c2;
        const uint64_t j = base + i;
        st.x[j] = px;
        st.y[j] = py;
        st.z[j] = pz;
        st.mu[j] = mu;
        st.lnp[j] = ::log(::sqrt(eps * (eps + 2.0)));
        st.w[j] = wt;
        st.pid[j] = pid;
        st.kinj[j] = k;
        st.status[j] = status;
        st.run[j] = (uint16_t)inj.run;
        if (status != FTE_PS_ACTIVE) {
            atomicAdd(&cnt->retired[status], 1ull);
            atomicAdd(&cnt->w_retired[status], wt);
        }
        atomicAdd(&wsum[pid % (uint64_t)P.n_batch], wt);
        if (P.grad) {
            for (int q = 0; q < kTanCols; ++q) tn.col(q)[j] = q == kTanLnw ? dlnw : 0.0;
            atomicAdd(&wdg, wt * dlnw);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < P.n_batch; b += blockDim.x)
        if (wsum[b] != 0.0) atomicAdd(&cnt->w_inj[inj.run * P.n_batch + b], wsum[b]);
    if (threadIdx.x == 0 && wdg != 0.0) atomicAdd(&cnt->w_inj_dgamma, wdg);
}

__global__ void k_add_live(DevCounters *cnt, int slot, uint64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt->n_live[slot] += n;
        cnt->injected += n;
    }
}

hipError_t launch_inject(const DevParams &p, const DevGrid &g, int rec_fp32, const fte_injection &inj, DevState st,
                         DevTan tn, DevCounters *cnt, int slot, uint64_t n, uint64_t first_pid, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_inject, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, g, rec_fp32, inj, st, tn, cnt, slot, n,
                       first_pid);
    return hipGetLastError();
}

hipError_t launch_add_live(DevCounters *cnt, int slot, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_add_live, dim3(1), dim3(64), 0, s, cnt, slot, n);
    return hipGetLastError();
}

// Locate the leaf holding level-1 coordinates s and gather + interpolate the
// records (trilinear in space, linear in time between snapshots k and k+1).
// TS2: the grid has two live snapshots and both are gathered in one unrolled
// pass, so that the loads of all 16 corners are in flight together.
// The workgroup's record tile (see StepLds): padded k-layers [k0, k0 +
// layers) of leaf `leaf` for the snapshot pair starting at ks, laid out as
// the leaf's own records, snapshot ks first.  The pointer is typed as LDS so
// that the compiler keeps the tile reads and the global gather apart (a
// generic pointer would turn both into flat loads).
typedef const __attribute__((address_space(3))) float lds_float;
struct RecTile {
    lds_float *lds;
    int leaf, k0, layers, ks;
};

// The first NF fields of the record at p in the tile.  Records of an even
// stride start on 8 bytes (the tile is 16-byte aligned and each snapshot's
// part holds whole records), so their fields are read in pairs, which the
// compiler issues as 8-byte LDS reads: on the CIR workload +9% over 4-byte
// reads, whose bank conflicts held the LDS 41% of the kernel's time.
#ifndef FTE_TILE_PAIRS
#define FTE_TILE_PAIRS 1
#endif
template <typename R, int NF, int RS>
__device__ __forceinline__ void tile_rec(lds_float *p, R out[NF]) {
    if constexpr (FTE_TILE_PAIRS && RS % 2 == 0) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        typedef const __attribute__((address_space(3))) f2v lds_f2v;
        lds_f2v *p2 = reinterpret_cast<lds_f2v *>(p);
#pragma unroll
        for (int q = 0; q < NF / 2; ++q) {
            const f2v u = p2[q];
            out[2 * q] = (R)u.x;
            out[2 * q + 1] = (R)u.y;
        }
        if constexpr (NF % 2 != 0) out[NF - 1] = (R)p[NF - 1];
    } else {
#pragma unroll
        for (int q = 0; q < NF; ++q) out[q] = (R)p[q];
    }
}

// Skip the block-index walk while a particle stays in its leaf (see
// descend_cached): CIR 2.66 -> 2.72 x 10^10 particle-steps/s, largest
// workload +2%.
#ifndef FTE_LEAF_CACHE
#define FTE_LEAF_CACHE 1
#endif
// Consecutive particle slices per XCD (see k_step).  Measured on the CIR
// workload: 1 (the hardware's own order) 2.61, 8 2.65, 32 2.66, 128 2.62,
// all (one contiguous share per XCD) 2.07 x 10^10 particle-steps/s; FP64
// 7.35, 32 8.36, 128 8.33 x 10^9.
#ifndef FTE_XCD_RUN
#define FTE_XCD_RUN 32
#endif
constexpr uint32_t kXcdRun = FTE_XCD_RUN;
// Float kernels with the record tile whose gather loads each lane's corners
// from its own source (tile or global) and interpolates once: the plain
// forward kernels with 10-field records, two snapshots (bit 1) or a steady
// grid (bit 2).  With the 13-field records (cross-field diffusion) it
// spills some 50 registers, even split into two passes over the fields, and
// runs a third slower; the ensemble instance fits but runs no faster; the
// leaf-pool instance gathers through its map.
#ifndef FTE_TILE_UNIFIED
#define FTE_TILE_UNIFIED 1
#endif
template <typename R, bool KPERP, int MODE, bool TS2, bool ENS, bool SUB>
constexpr bool unified_gather() {
    return std::is_same<R, float>::value && !KPERP && MODE == 0 && !ENS && !SUB &&
           (FTE_TILE_UNIFIED & (TS2 ? 1 : 2)) != 0;
}

// The leaf a particle's previous step found: its level and block index.
// A point whose block index at that level is the cached one lies in the same
// leaf (leaves partition the domain), with the same level coordinates the
// walk would compute (scaling by 2^(L-1) is exact), so the walk is skipped.
struct LeafCache {
    int leaf, L, B[3];
};
template <typename R>
__device__ __forceinline__ int descend_cached(const DevGrid &G, const int32_t *base, const int32_t *child, const R s[3],
                                              R S[3], int B[3], LeafCache &lc) {
    if (lc.leaf >= 0) {
        const R scale = (R)(1 << (lc.L - 1));
        bool same = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            S[a] = s[a] * scale;
            int c = (int)M<R>::floor_(S[a]);
            const int n = G.n1[a] << (lc.L - 1);
            c = c > n - 1 ? n - 1 : c;
            B[a] = div_bx(G, c, a);
            same = same && B[a] == lc.B[a];
        }
        if (same) return lc.leaf;
    }
    int L = 1;
    const int leaf = descend<R>(G, base, child, s, S, B, &L);
    lc.leaf = leaf;
    lc.L = L;
#pragma unroll
    for (int a = 0; a < 3; ++a) lc.B[a] = B[a];
    return leaf;
}

// Returns 0, or 1 when no leaf holds the point, 2 when (SUB: a streamed
// subset of leaves) the leaf's records are not resident in both slots.
template <typename R, bool KPERP, bool TS2, bool TILE = false, bool SUB = false, bool UNI = false>
__device__ __forceinline__ int gather(const DevGrid &G, const int32_t *ibase, const int32_t *ichild, R s[3], int ks,
                                      R alpha, R acc[kNF], const RecTile T = RecTile{nullptr, -1, 0, 0, -1},
                                      LeafCache *lc = nullptr) {
    constexpr int NF = KPERP ? 13 : 10;
    constexpr int RS = KPERP ? kRSKperp : kRSPlain;
    fold_s<R>(G, s);
    int B[3];
    R S[3];
    const int leaf = lc ? descend_cached<R>(G, ibase, ichild, s, S, B, *lc) : descend<R>(G, ibase, ichild, s, S, B);
    if (leaf < 0) return 1;
    // local cell relative to the first centre of the block, padded index
    int i[3];
    R f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R u = S[a] - (R)(B[a] * G.bx[a]) - (R)0.5;
        const R fl = M<R>::floor_(u);
        i[a] = (int)fl;
        f[a] = u - fl;
    }
    const size_t pc = (size_t)(i[0] + 1) + (size_t)G.px[0] * ((i[1] + 1) + (size_t)G.px[1] * (i[2] + 1));
    const size_t sx = 1, sy = G.px[0], sz = (size_t)G.px[0] * G.px[1];
    const R *rec = reinterpret_cast<const R *>(G.rec);
#pragma unroll
    for (int q = 0; q < NF; ++q) acc[q] = (R)0;
    if constexpr (TILE) {
        // both corner layers i[2] + 1 and i[2] + 2 in the tile: the same
        // values, weights and summation order as the global path below
        // (TS2: both live snapshots; otherwise a steady grid, one snapshot)
        constexpr int NS = TS2 ? 2 : 1;
        const bool in = (TS2 || G.n_snap < 2) && leaf == T.leaf && ks == T.ks && i[2] + 1 >= T.k0 &&
            i[2] + 2 < T.k0 + T.layers && i[0] >= -1 && i[0] + 2 < G.px[0] && i[1] >= -1 && i[1] + 2 < G.px[1];
        if constexpr (UNI) {
            // a wavefront whose particles are partly in the tile loads each
            // lane's corners from its own source into registers and
            // interpolates once (with a branch per source around the
            // interpolation too, such a wavefront would run it twice)
            if (TS2 || G.n_snap < 2) {
                static_assert(!SUB, "the leaf-pool kernels gather through the branches below");
                R v[NS][8][NF];
                if (in) {
                    const size_t tsnap = (size_t)T.layers * sz * RS;
                    lds_float *tb =
                        T.lds + ((size_t)(i[2] + 1 - T.k0) * sz + (size_t)(i[1] + 1) * sy + (size_t)(i[0] + 1)) * RS;
#pragma unroll
                    for (int sn = 0; sn < NS; ++sn)
#pragma unroll
                        for (int d = 0; d < 8; ++d) {
                            tile_rec<R, NF, RS>(
                                tb + sn * tsnap + ((d & 1) * sx + ((d >> 1) & 1) * sy + (d >> 2) * sz) * RS, v[sn][d]);
                        }
                } else {
#pragma unroll
                    for (int sn = 0; sn < NS; ++sn) {
                        const R *base =
                            rec + (((size_t)((ks + sn) % G.n_slots) * G.n_blk + leaf) * G.pcells + pc) * RS;
#pragma unroll
                        for (int d = 0; d < 8; ++d) {
                            const R *p = base + ((d & 1) * sx + ((d >> 1) & 1) * sy + (d >> 2) * sz) * RS;
#pragma unroll
                            for (int q = 0; q < NF; ++q) v[sn][d][q] = p[q];
                        }
                    }
                }
#pragma unroll
                for (int sn = 0; sn < NS; ++sn) {
                    const R ws = TS2 ? (sn == 0 ? (R)1 - alpha : alpha) : (R)1;
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        const int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
                        const R w =
                            ws * (e0 ? f[0] : (R)1 - f[0]) * (e1 ? f[1] : (R)1 - f[1]) * (e2 ? f[2] : (R)1 - f[2]);
#pragma unroll
                        for (int q = 0; q < NF; ++q) acc[q] += w * v[sn][d][q];
                    }
                }
                return 0;
            }
        }
        if (in) {
            const size_t tsnap = (size_t)T.layers * sz * RS;
            lds_float *tb = T.lds + ((size_t)(i[2] + 1 - T.k0) * sz + (size_t)(i[1] + 1) * sy + (size_t)(i[0] + 1)) * RS;
#pragma unroll
            for (int sn = 0; sn < NS; ++sn) {
                const R ws = TS2 ? (sn == 0 ? (R)1 - alpha : alpha) : (R)1;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
                    const R w = ws * (e0 ? f[0] : (R)1 - f[0]) * (e1 ? f[1] : (R)1 - f[1]) * (e2 ? f[2] : (R)1 - f[2]);
                    R u[NF];
                    tile_rec<R, NF, RS>(tb + sn * tsnap + (e0 * sx + e1 * sy + e2 * sz) * RS, u);
#pragma unroll
                    for (int q = 0; q < NF; ++q) acc[q] += w * u[q];
                }
            }
            return 0;
        }
    }
    // the record block of the leaf in each live slot
    int blk[2] = {leaf, leaf};
    if constexpr (SUB) {
#pragma unroll
        for (int sn = 0; sn < 2; ++sn) {
            blk[sn] = G.pool_map[(size_t)((ks + sn) % G.n_slots) * G.n_leaves + leaf];
            if (blk[sn] < 0) return 2;
        }
    }
    // the 8 corners of snapshot slot ks + sn, weighted by ws
    auto corners = [&](int sn, R ws) {
        const R *base = rec + (((size_t)((ks + sn) % G.n_slots) * G.n_blk + blk[sn]) * G.pcells + pc) * RS;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
            const R w = ws * (e0 ? f[0] : (R)1 - f[0]) * (e1 ? f[1] : (R)1 - f[1]) * (e2 ? f[2] : (R)1 - f[2]);
            const R *p = base + (e0 * sx + e1 * sy + e2 * sz) * RS;
#pragma unroll
            for (int q = 0; q < NF; ++q) acc[q] += w * p[q];
        }
    };
    if constexpr (TS2) {
#pragma unroll
        for (int sn = 0; sn < 2; ++sn) corners(sn, sn == 0 ? (R)1 - alpha : alpha);
    } else {
        const int nsn = G.n_snap >= 2 ? 2 : 1;
        for (int sn = 0; sn < nsn; ++sn) corners(sn, G.n_snap >= 2 ? (sn == 0 ? (R)1 - alpha : alpha) : (R)1);
    }
    return 0;
}

// Weight derivative of one corner along a tangent direction dS: every
// product and fused multiply-add written out, so that the tile and global
// paths (two copies of this code in one kernel) round identically whatever
// the compiler would contract on its own.
template <typename R>
__device__ __forceinline__ R corner_dw(R ws, R w0, R w1, R w2, R g0, R g1, R g2, const R dS[3]) {
#pragma clang fp contract(off)
    const R a0 = g0 * w1 * w2, a1 = w0 * g1 * w2, a2 = w0 * w1 * g2;
    return ws * M<R>::fma_(a2, dS[2], M<R>::fma_(a1, dS[1], a0 * dS[0]));
}

// Directional derivatives of the gathered (spherical-component) fields along
// ND tangent directions: ds[k] holds the derivative of the level-1
// coordinates along direction k; axes clamped by the fold contribute none.
template <typename R, bool KPERP, int ND, bool TILE = false>
__device__ __forceinline__ bool gather_d(const DevGrid &G, const int32_t *ibase, const int32_t *ichild, R s[3],
                                         const R ds[ND][3], int ks, R alpha, R acc[kNF], R dacc[ND][kNF],
                                         const RecTile T = RecTile{nullptr, -1, 0, 0, -1}) {
    constexpr int NF = KPERP ? 13 : 10;
    constexpr int RS = KPERP ? kRSKperp : kRSPlain;
    const R s_in[3] = {s[0], s[1], s[2]};
    fold_s<R>(G, s);
    bool live[3] = {s[0] == s_in[0], s[1] == s_in[1], G.periodic ? true : s[2] == s_in[2]};
    int B[3], L;
    R S[3];
    const int leaf = descend<R>(G, ibase, ichild, s, S, B, &L);
    if (leaf < 0) return false;
    const R scale = (R)(1 << (L - 1));
    R dS[ND][3];
#pragma unroll
    for (int k = 0; k < ND; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) dS[k][a] = live[a] ? ds[k][a] * scale : (R)0;
    int i[3];
    R f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R u = S[a] - (R)(B[a] * G.bx[a]) - (R)0.5;
        const R fl = M<R>::floor_(u);
        i[a] = (int)fl;
        f[a] = u - fl;
    }
    const size_t pc = (size_t)(i[0] + 1) + (size_t)G.px[0] * ((i[1] + 1) + (size_t)G.px[1] * (i[2] + 1));
    const size_t sx = 1, sy = G.px[0], sz = (size_t)G.px[0] * G.px[1];
    const R *rec = reinterpret_cast<const R *>(G.rec);
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        acc[q] = (R)0;
#pragma unroll
        for (int k = 0; k < ND; ++k) dacc[k][q] = (R)0;
    }
    const int nsn = G.n_snap >= 2 ? 2 : 1;
    if constexpr (TILE) {
        // both corner layers in the workgroup's tile (see gather): the same
        // values, weights and summation order as the loop below
        if (nsn == 2 && leaf == T.leaf && ks == T.ks && i[2] + 1 >= T.k0 && i[2] + 2 < T.k0 + T.layers &&
            i[0] >= -1 && i[0] + 2 < G.px[0] && i[1] >= -1 && i[1] + 2 < G.px[1]) {
            const size_t tsnap = (size_t)T.layers * sz * RS;
            lds_float *tb = T.lds + ((size_t)(i[2] + 1 - T.k0) * sz + (size_t)(i[1] + 1) * sy + (size_t)(i[0] + 1)) * RS;
#pragma unroll
            for (int sn = 0; sn < 2; ++sn) {
                const R ws = sn == 0 ? (R)1 - alpha : alpha;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
                    const R w0 = e0 ? f[0] : (R)1 - f[0], w1 = e1 ? f[1] : (R)1 - f[1], w2 = e2 ? f[2] : (R)1 - f[2];
                    const R g0 = e0 ? (R)1 : (R)-1, g1 = e1 ? (R)1 : (R)-1, g2 = e2 ? (R)1 : (R)-1;
                    const R w = ws * w0 * w1 * w2;
                    R dw[ND];
#pragma unroll
                    for (int k = 0; k < ND; ++k) dw[k] = corner_dw<R>(ws, w0, w1, w2, g0, g1, g2, dS[k]);
                    R u[NF];
                    tile_rec<R, NF, RS>(tb + sn * tsnap + (e0 * sx + e1 * sy + e2 * sz) * RS, u);
#pragma unroll
                    for (int q = 0; q < NF; ++q) {
                        const R v = u[q];
                        acc[q] = M<R>::fma_(w, v, acc[q]);
#pragma unroll
                        for (int k = 0; k < ND; ++k) dacc[k][q] = M<R>::fma_(dw[k], v, dacc[k][q]);
                    }
                }
            }
            return true;
        }
    }
    for (int sn = 0; sn < nsn; ++sn) {
        const R ws = (G.n_snap >= 2) ? (sn == 0 ? (R)1 - alpha : alpha) : (R)1;
        const R *base = rec + (((size_t)((ks + sn) % G.n_slots) * G.n_blk + leaf) * G.pcells + pc) * RS;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
            const R w0 = e0 ? f[0] : (R)1 - f[0], w1 = e1 ? f[1] : (R)1 - f[1], w2 = e2 ? f[2] : (R)1 - f[2];
            const R g0 = e0 ? (R)1 : (R)-1, g1 = e1 ? (R)1 : (R)-1, g2 = e2 ? (R)1 : (R)-1;
            const R w = ws * w0 * w1 * w2;
            R dw[ND];
#pragma unroll
            for (int k = 0; k < ND; ++k) dw[k] = corner_dw<R>(ws, w0, w1, w2, g0, g1, g2, dS[k]);
            const R *p = base + (e0 * sx + e1 * sy + e2 * sz) * RS;
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                const R v = p[q];
                acc[q] = M<R>::fma_(w, v, acc[q]);
#pragma unroll
                for (int k = 0; k < ND; ++k) dacc[k][q] = M<R>::fma_(dw[k], v, dacc[k][q]);
            }
        }
    }
    return true;
}

template <typename R>
__device__ __forceinline__ R sgn(R x) {
    return (R)((x > (R)0) - (x < (R)0));
}

// Rotate spherical components with the basis at the particle.
template <typename R>
__device__ __forceinline__ void to_cart(R st, R ct, R sp, R cp, const R s[3], R out[3]) {
    out[0] = s[0] * st * cp + s[1] * ct * cp - s[2] * sp;
    out[1] = s[0] * st * sp + s[1] * ct * sp + s[2] * cp;
    out[2] = s[0] * ct - s[1] * st;
}

// Derivative of a rotated vector field along a displacement with basis
// projections (tth, tph) = (e_theta . dx, e_phi . dx) / r: the change of its
// spherical components plus the turn of the local basis, rotated.
template <typename R>
__device__ __forceinline__ void d_to_cart(R st, R ct, R sp, R cp, R cot, R tth, R tph, const R a[3], const R da[3],
                                          R out[3]) {
    const R v[3] = {da[0] - a[1] * tth - a[2] * tph, da[1] + a[0] * tth - a[2] * cot * tph,
                    da[2] + a[0] * tph + a[1] * cot * tph};
    to_cart<R>(st, ct, sp, cp, v, out);
}

// Second derivative in mu of g(mu) (D_mumu = A g), the derivative of the drift
// term dD/dmu as the step evaluates it.
template <typename R>
__device__ __forceinline__ R dmm_g2(const DevParams &P, R mu) {
    const R am = mu < (R)0 ? -mu : mu;
    if (P.dmm_model == FTE_DMM_ISO) return (R)-2;
    if (P.dmm_model == FTE_DMM_EQ5) return (R)-2 * ((R)1 + (R)P.eps);
    const R q = (R)P.q;
    const R amf = am > (R)P.mu_floor ? am : (R)P.mu_floor;
    const R om = (R)1 - mu * mu;
    R g2 = (R)-2 * (q - (R)1) * am * M<R>::pow_(amf, q - (R)2) - (R)2 * q * M<R>::pow_(am, q - (R)1);
    if (am > (R)P.mu_floor) g2 += (q - (R)1) * (q - (R)2) * M<R>::pow_(amf, q - (R)3) * om;
    return g2;
}

// First derivative in mu of g(mu) itself (no floor): the change of D along
// a pitch-angle perturbation, for the noise amplitude.
template <typename R>
__device__ __forceinline__ R dmm_g1(const DevParams &P, R mu) {
    const R am = mu < (R)0 ? -mu : mu;
    const R om = (R)1 - mu * mu;
    if (P.dmm_model == FTE_DMM_ISO) return (R)-2 * mu;
    if (P.dmm_model == FTE_DMM_EQ5) {
        const R g = am / ((R)1 + am) + (R)P.eps;
        return sgn(mu) * om / (((R)1 + am) * ((R)1 + am)) - (R)2 * mu * g;
    }
    const R q = (R)P.q;
    const R amx = am > (R)0 ? am : (R)P.mu_floor;
    return (q - (R)1) * sgn(mu) * M<R>::pow_(amx, q - (R)2) * om - (R)2 * mu * M<R>::pow_(am, q - (R)1);
}

// Radius of a position and the cosine of its colatitude.  The FP64 path takes
// both in double.  The mixed path keeps the squared radius in double (the
// absorbing-sphere and observer-shell tests compare it with squared radii)
// and the radius in float for the grid coordinates and the local basis.
template <typename R>
__device__ __forceinline__ R radius_of(double r2) {
    if constexpr (std::is_same<R, double>::value) return ::sqrt(r2);
    else return M<float>::sqrt_((float)r2);
}
template <typename R>
__device__ __forceinline__ R cos_colat(double z, R r) {
    if constexpr (std::is_same<R, double>::value) return z / r;
    else return M<float>::div_((float)z, r);
}

// erfc(z) exp(z^2) for z >= 0: directly while erfc(z) stays a normal number,
// beyond that the asymptotic series to z^-7 (relative error below 7 z^-8).
template <typename R>
__device__ __forceinline__ R erfcx_pos(R z) {
    if (z < (std::is_same<R, float>::value ? (R)8 : (R)26)) {
        if constexpr (std::is_same<R, float>::value) return __expf(z * z) * erfcf(z);
        else return ::exp(z * z) * ::erfc(z);
    }
    const R t = M<R>::div_((R)1, z * z);
    return M<R>::div_((R)1, z * (R)1.7724538509055160273) * ((R)1 - (R)0.5 * t + (R)0.75 * t * t - (R)1.875 * t * t * t);
}

// Expected time a Brownian bridge of diffusion s2 (variance s2 h after a time
// h) from a to b spends per unit length at 0: the convolution of the two free
// densities through 0 over the bridge density,
// sqrt(2 pi h) / (2 s) erfcx((|a| + |b|) / (s sqrt(2 h))) exp(-(a b + |a b|) / (s2 h)).
template <typename R>
__device__ __forceinline__ R bridge_occupation(R a, R b, R s2, R h) {
    const R s = M<R>::sqrt_(s2);
    const R aa = a < (R)0 ? -a : a, ab = b < (R)0 ? -b : b;
    const R z = M<R>::div_(aa + ab, s * M<R>::sqrt_((R)2 * h));
    const R e = M<R>::exp_(-M<R>::div_(a * b + aa * ab, s2 * h));
    return M<R>::div_(M<R>::sqrt_((R)6.283185307179586477 * h), (R)2 * s) * erfcx_pos<R>(z) * e;
}

// MODE 0: histogram estimator only.  MODE 1: also the kernel-smoothed sums.
// MODE 2: also the pathwise tangents d(x, mu, ln p)/d(lambda_ref,
// kperp_ratio), propagated by the derivative of the same Euler-Maruyama map
// under the same Wiener increments, and the derivative sums of the smoothed
// estimator.
// Dynamic LDS of the step kernel: the observer histogram of the time bins
// this launch can touch (doubles, zeroed on entry, flushed with one global
// atomic per nonzero bin on exit), then the block index (base and child
// tables) when LIDX.
extern __shared__ __align__(16) unsigned char k_step_lds[];

// Minimum waves per SIMD the register allocation of the step kernel aims
// for (1 = no constraint).  Measured on the CIR workload: the double forward
// kernels gain 18% at 2 (one wave per SIMD otherwise; 3 or 4 spill hundreds
// of bytes); the float ones lose 5% when squeezed from 3 waves to 4.
#ifndef FTE_STEP_WPE_F32
#define FTE_STEP_WPE_F32 1
#endif
#ifndef FTE_STEP_WPE_F64
#define FTE_STEP_WPE_F64 2
#endif
template <typename R, bool KPERP, int MODE, bool TS2, bool ENS, bool SUB>
constexpr int step_wpe() {
    // the register-resident gather would otherwise take the allocator past
    // 256 registers (one wave per SIMD)
    if (unified_gather<R, KPERP, MODE, TS2, ENS, SUB>()) return 2;
    return MODE == 2 ? 1 : (std::is_same<R, float>::value ? FTE_STEP_WPE_F32 : FTE_STEP_WPE_F64);
}
// Most waves per SIMD the allocator plans for: 2 for the unrolled
// two-snapshot gather, so that the scheduler keeps its 40 loads in flight
// instead of trading them for a third wave.
#ifndef FTE_STEP_WPE_MAX_TS2
#define FTE_STEP_WPE_MAX_TS2 2
#endif
template <bool TS2>
constexpr int step_wpe_max() {
    return TS2 ? FTE_STEP_WPE_MAX_TS2 : 8;
}

template <typename R, bool KPERP, int MODE, bool LIDX, bool TS2, bool ENS, bool SUB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(step_wpe<R, KPERP, MODE, TS2, ENS, SUB>(), step_wpe_max<TS2>()))) void k_step(DevParams P, DevGrid G, DevState st, DevTan tn, DevCounters *cnt,
                                              int slot, double *hist, double *sm, uint64_t n0, uint32_t n_steps,
                                              StepLds LD) {
    constexpr int ND = MODE == 2 ? 2 : 1;
    // Workgroups are dealt to the eight XCDs in turn.  Give each XCD runs of
    // kXcdRun consecutive particle slices (the spatial sort makes them
    // neighbours in space), so that each XCD's own L2 sees a compact region
    // while the eight together still sweep one window of the sorted
    // particles through the shared Infinity Cache; the tail that does not
    // fill whole runs keeps its order.  A permutation of the slices: each
    // slice is stepped exactly as before.
    const uint32_t run8 = 8u * kXcdRun, full = gridDim.x / run8 * run8;
    uint32_t wg = blockIdx.x;
    if (wg < full) {
        const uint32_t xcd = wg & 7u, ix = wg >> 3;
        wg = ((ix / kXcdRun) * 8u + xcd) * kXcdRun + ix % kXcdRun;
    }
    const uint64_t i = (uint64_t)wg * blockDim.x + threadIdx.x;
    const uint64_t n_live = cnt->n_live[slot];
    unsigned long long my_steps = 0;
    double *lh = reinterpret_cast<double *>(k_step_lds);
    const int n_lh = LD.n_tb > 0 ? P.n_runs_eff * P.n_obs_bins * P.n_e * LD.n_tb * P.n_batch : 0;
    const int32_t *ibase = G.base, *ichild = G.child;
    if constexpr (LIDX) {
        int32_t *lb = reinterpret_cast<int32_t *>(k_step_lds + (size_t)n_lh * 8);
        int32_t *lc = lb + G.n_base;
        for (int k = threadIdx.x; k < G.n_base; k += blockDim.x) lb[k] = G.base[k];
        for (int k = threadIdx.x; k < G.n_child; k += blockDim.x) lc[k] = G.child[k];
        ibase = lb;
        ichild = lc;
    }
    for (int k = threadIdx.x; k < n_lh; k += blockDim.x) lh[k] = 0.0;
    if (LIDX || n_lh > 0) __syncthreads();
    // record tile (float kernels): anchored at the leaf and k-layer of the
    // workgroup's middle particle, for the snapshot pair of the launch's
    // first step (the one snapshot of a steady grid)
    constexpr bool kTile = std::is_same<R, float>::value && !LIDX;
    // each particle's leaf from its previous step (float kernels; the double
    // ones spill more with its registers and lost 4%)
    constexpr bool kLeafCache = FTE_LEAF_CACHE && std::is_same<R, float>::value;
    constexpr int kTileRS = KPERP ? kRSKperp : kRSPlain;
    RecTile tile{nullptr, -1, 0, 0, -1};
    if constexpr (kTile) {
        if (LD.tile_layers > 0) {
            __shared__ int anchor[2];
            if (threadIdx.x == 0) anchor[0] = -1;
            __syncthreads();
            const uint64_t im = (uint64_t)wg * blockDim.x + (blockDim.x >> 1);
            if (threadIdx.x == (blockDim.x >> 1) && im < n_live && st.status[im] == FTE_PS_ACTIVE) {
                const double ax = st.x[im], ay = st.y[im], az = st.z[im];
                const R ar = radius_of<R>(ax * ax + ay * ay + az * az);
                R aph = M<R>::atan2_((R)ay, (R)ax);
                if (aph < (R)0) aph += (R)(2.0 * kPi);
                R as[3], aS[3];
                int aB[3];
                grid_coords<R>(G, ar, M<R>::acos_(cos_colat<R>(az, ar)), aph, as);
                fold_s<R>(G, as);
                const int aleaf = descend<R>(G, ibase, ichild, as, aS, aB);
                if (aleaf >= 0) {
                    // the particles of cell c read padded layers c .. c + 2
                    // (c + 1 is the cell's own): an odd number of layers is
                    // centred on the cell, an even number on the middle
                    // particle's lower corner layer (the half of the cell
                    // it is in)
                    const R half = (LD.tile_layers & 1) ? (R)0 : (R)0.5;
                    anchor[0] = aleaf;
                    anchor[1] = (int)M<R>::floor_(aS[2] - (R)(aB[2] * G.bx[2]) - half) + 1;
                }
            }
            __syncthreads();
            if (anchor[0] >= 0) {
                const int TL = LD.tile_layers, pz = G.px[2];
                int k0 = anchor[1] - (TL - 1) / 2;
                k0 = k0 > pz - TL ? pz - TL : k0;
                k0 = k0 < 0 ? 0 : k0;
                // the snapshot pair of the launch's first step (one snapshot
                // on a steady grid)
                const int nst = G.n_snap >= 2 ? 2 : 1;
                int ks0 = 0;
                if (nst == 2) {
                    const double tau = (P.t0 + (double)n0 * P.dt - G.t_s0) * G.inv_dt_s;
                    double kf = ::floor(tau);
                    kf = kf < 0.0 ? 0.0 : (kf > (double)(G.n_snap - 2) ? (double)(G.n_snap - 2) : kf);
                    ks0 = (int)kf;
                }
                float *t = reinterpret_cast<float *>(k_step_lds + LD.tile_off);
                const size_t layer = (size_t)G.px[0] * G.px[1] * kTileRS;
                const size_t nfl = layer * TL;
                const float *recf = reinterpret_cast<const float *>(G.rec);
                // the anchor leaf's record block in each live slot (a
                // streamed subset: no tile unless it is resident in both)
                int ab[2] = {anchor[0], anchor[0]};
                if constexpr (SUB) {
                    for (int sn = 0; sn < 2; ++sn)
                        ab[sn] = G.pool_map[(size_t)((ks0 + sn) % G.n_slots) * G.n_leaves + anchor[0]];
                }
                if (ab[0] >= 0 && ab[1] >= 0) {
                for (int sn = 0; sn < nst; ++sn) {
                    const float *src = recf + (((size_t)((ks0 + sn) % G.n_slots) * G.n_blk + ab[sn]) * G.pcells) *
                                                  kTileRS + (size_t)k0 * layer;
                    if ((nfl & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
                        // 16-byte copies (the tile offset is 16-byte aligned)
                        const float4 *s4 = reinterpret_cast<const float4 *>(src);
                        float4 *t4 = reinterpret_cast<float4 *>(t + sn * nfl);
                        for (size_t q = threadIdx.x; q < (nfl >> 2); q += blockDim.x) t4[q] = s4[q];
                    } else {
                        for (size_t q = threadIdx.x; q < nfl; q += blockDim.x) t[sn * nfl + q] = src[q];
                    }
                }
                tile = RecTile{(lds_float *)t, anchor[0], k0, TL, ks0};
                }
            }
            __syncthreads();
        }
    }
    if (i < n_live && st.status[i] == FTE_PS_ACTIVE) {
        double x = st.x[i], y = st.y[i], z = st.z[i];
        R mu = (R)st.mu[i], lnp = (R)st.lnp[i];
        const double w = st.w[i];
        const uint64_t pid = st.pid[i];
        const uint32_t kinj = st.kinj[i];
        int status = FTE_PS_ACTIVE;
        const R dt = (R)P.dt;
        // this particle's run (ensembles): mean free path, cross-field ratio,
        // last step, Philox run id
        int run_r = 0, run_id = P.run_id;
        double lam_ref = P.lambda_ref, kratio = P.kperp_ratio;
        uint64_t step_end = ~0ull;
        if constexpr (ENS) {
            run_r = st.run[i];
            const DevRun rr = P.runs[run_r];
            lam_ref = rr.lambda_ref;
            kratio = rr.kperp_ratio;
            step_end = rr.step_end;
            run_id = rr.run_id;
        }
        // tangents (MODE 2)
        R TX[ND][3], TM[ND], TL[ND];
        R dlnw = (R)0;
        if constexpr (MODE == 2) {
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                TX[k][0] = (R)tn.col(5 * k + 0)[i];
                TX[k][1] = (R)tn.col(5 * k + 1)[i];
                TX[k][2] = (R)tn.col(5 * k + 2)[i];
                TM[k] = (R)tn.col(5 * k + 3)[i];
                TL[k] = (R)tn.col(5 * k + 4)[i];
            }
            dlnw = (R)tn.col(kTanLnw)[i];
        }
        // spherical coordinates of the current position
        constexpr bool kF64 = std::is_same<R, double>::value;
        double r2 = x * x + y * y + z * z;
        R r = radius_of<R>(r2);
        R th = M<R>::acos_(cos_colat<R>(z, r));
        R ph = M<R>::atan2_((R)y, (R)x);
        if (ph < (R)0) ph += (R)(2.0 * kPi);
        R Pcur = M<R>::exp_(lnp);
        R gcur = M<R>::sqrt_((R)1 + Pcur * Pcur);
        R vcur = M<R>::div_((R)kC * Pcur, gcur);
        const uint64_t n_win = n0 + n_steps;
        const uint64_t n_end = n_win < step_end ? n_win : step_end;
        uint64_t nstart = n0 > kinj ? n0 : kinj;
        LeafCache lcache{-1, 0, {0, 0, 0}};
        for (uint64_t n = nstart; n < n_end; ++n) {
            // ---- clock and snapshot pair (identical for every particle)
            int ks = 0;
            R alpha = (R)0;
            if (G.n_snap >= 2) {
                const double t = P.t0 + (double)n * P.dt;
                const double tau = (t - G.t_s0) * G.inv_dt_s;
                double kf = ::floor(tau);
                kf = kf < 0.0 ? 0.0 : (kf > (double)(G.n_snap - 2) ? (double)(G.n_snap - 2) : kf);
                ks = (int)kf;
                alpha = (R)(tau - kf);
            }
            // basis at the particle: before the gather only when the tangents
            // need it there (it would otherwise stay live across the gather)
            R st_, ct_, sp_, cp_;
            auto basis_at = [&]() {
                const R xf = (R)x, yf = (R)y, zf = (R)z;
                const R rho = M<R>::sqrt_(xf * xf + yf * yf);
                st_ = M<R>::div_(rho, r);
                ct_ = M<R>::div_(zf, r);
                sp_ = M<R>::div_(yf, rho);
                cp_ = M<R>::div_(xf, rho);
            };
            if constexpr (MODE == 2) basis_at();
            // ---- locate + gather + interpolate
            R s[3];
            grid_coords<R>(G, r, th, ph, s);
            R acc[kNF];
            R dacc[ND][kNF];
            R tth[ND], tph[ND], cot = (R)0;
            if constexpr (MODE == 2) {
                const R ir = M<R>::div_((R)1, r);
                cot = M<R>::div_(ct_, st_);
                R ds[ND][3];
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    const R ter = TX[k][0] * st_ * cp_ + TX[k][1] * st_ * sp_ + TX[k][2] * ct_;
                    tth[k] = (TX[k][0] * ct_ * cp_ + TX[k][1] * ct_ * sp_ - TX[k][2] * st_) * ir;
                    tph[k] = (-TX[k][0] * sp_ + TX[k][1] * cp_) * ir;
                    ds[k][0] = ter * (R)G.inv_dxi * (G.xi_map ? ir : (R)1);
                    ds[k][1] = tth[k] * (R)G.inv_dth;
                    ds[k][2] = M<R>::div_(tph[k], st_) * (R)G.inv_dph;
                }
                if (!gather_d<R, KPERP, ND, kTile>(G, ibase, ichild, s, ds, ks, alpha, acc, dacc, tile)) {
                    status = FTE_PS_NUMERIC;
                    break;
                }
            } else {
                const int gr = gather<R, KPERP, TS2, kTile, SUB, unified_gather<R, KPERP, MODE, TS2, ENS, SUB>()>(
                    G, ibase, ichild, s, ks, alpha, acc, tile, kLeafCache ? &lcache : nullptr);
                if (gr != 0) {
                    if (SUB && gr == 2) atomicOr(&cnt->flags, kFlagNotResident);
                    status = FTE_PS_NUMERIC;
                    break;
                }
                basis_at();
            }
            Fields<R> F;
            to_cart<R>(st_, ct_, sp_, cp_, acc + 0, F.V);
            R bt[3];
            to_cart<R>(st_, ct_, sp_, cp_, acc + 3, bt);
            const R bn = M<R>::sqrt_(bt[0] * bt[0] + bt[1] * bt[1] + bt[2] * bt[2]);
            if (!(bn >= (R)1e-12)) {
                status = FTE_PS_NUMERIC;
                break;
            }
            F.b[0] = M<R>::div_(bt[0], bn);
            F.b[1] = M<R>::div_(bt[1], bn);
            F.b[2] = M<R>::div_(bt[2], bn);
            F.divV = acc[6];
            F.bbgV = acc[7];
            F.divb = acc[8];
            F.bDV = acc[9];
            if (KPERP) {
                to_cart<R>(st_, ct_, sp_, cp_, acc + 10, F.curv);
            } else {
                F.curv[0] = F.curv[1] = F.curv[2] = (R)0;
            }
            // field derivatives along each tangent
            Fields<R> dF[ND];
            if constexpr (MODE == 2) {
                const R ibn = M<R>::div_((R)1, bn);
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    d_to_cart<R>(st_, ct_, sp_, cp_, cot, tth[k], tph[k], acc + 0, dacc[k] + 0, dF[k].V);
                    R dbt[3];
                    d_to_cart<R>(st_, ct_, sp_, cp_, cot, tth[k], tph[k], acc + 3, dacc[k] + 3, dbt);
                    const R bd = F.b[0] * dbt[0] + F.b[1] * dbt[1] + F.b[2] * dbt[2];
#pragma unroll
                    for (int a = 0; a < 3; ++a) dF[k].b[a] = (dbt[a] - F.b[a] * bd) * ibn;
                    dF[k].divV = dacc[k][6];
                    dF[k].bbgV = dacc[k][7];
                    dF[k].divb = dacc[k][8];
                    dF[k].bDV = dacc[k][9];
                    if (KPERP) {
                        d_to_cart<R>(st_, ct_, sp_, cp_, cot, tth[k], tph[k], acc + 10, dacc[k] + 10, dF[k].curv);
                    } else {
                        dF[k].curv[0] = dF[k].curv[1] = dF[k].curv[2] = (R)0;
                    }
                }
            }
            // ---- coefficients (Eqs. 2-5); P = p/(m c) and the speed are carried
            // from the previous update (the same values as exp(lnp) recomputed)
            const R Pm = Pcur;
            const R v = vcur;
            R lam = (R)lam_ref;
            if (P.alpha != 0.0) lam *= M<R>::pow_(Pm * (R)P.inv_p_ref, (R)P.alpha);
            const R A = (R)P.dmm_scale * v / lam;
            const R am = mu < (R)0 ? -mu : mu;
            const R om = (R)1 - mu * mu;
            R D, dD;
            if (P.dmm_model == FTE_DMM_ISO) {
                D = A * om;
                dD = (R)-2 * mu * A;
            } else if (P.dmm_model == FTE_DMM_EQ5) {
                const R g = am / ((R)1 + am) + (R)P.eps;
                D = A * g * om;
                dD = A * (sgn(mu) * om / (((R)1 + am) * ((R)1 + am)) - (R)2 * mu * g);
            } else {
                const R q = (R)P.q;
                const R amf = am > (R)P.mu_floor ? am : (R)P.mu_floor;
                const R g = M<R>::pow_(am, q - (R)1);
                D = A * om * g;
                dD = A * ((q - (R)1) * sgn(mu) * M<R>::pow_(amf, q - (R)2) * om - (R)2 * mu * g);
            }
            R kperp = (R)0;
            if (KPERP) {
                if (kratio > 0.0) kperp = (R)kratio * v * lam / (R)3;
                else kperp = v * (R)P.lambda_perp / (R)3;
            }
            R a_x[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) a_x[a] = F.V[a] + mu * v * F.b[a] - kperp * (F.divb * F.b[a] + F.curv[a]);
            const R Qm = v * F.divb + mu * F.divV - (R)3 * mu * F.bbgV - M<R>::div_((R)2, v) * F.bDV;
            const R a_mu = (R)0.5 * om * Qm + dD;
            const R a_lnp = (R)0.5 * ((R)1 - (R)3 * mu * mu) * F.bbgV - (R)0.5 * om * F.divV - M<R>::div_(mu, v) * F.bDV;
            // ---- Wiener increments: one Philox block, Box-Muller pairs
            const U4 k4 = philox_words(P.seed, run_id, n, pid, 0u);
            const R u0 = M<R>::u01(k4.a), u1 = M<R>::u01(k4.b), u2 = M<R>::u01(k4.c), u3 = M<R>::u01(k4.d);
            const R ra = M<R>::sqrt_((R)-2 * M<R>::log_(u0));
            const R rb = M<R>::sqrt_((R)-2 * M<R>::log_(u2));
            R c1, s1, c3, s3;
            M<R>::cs2pi(u1, &c1, &s1);
            M<R>::cs2pi(u3, &c3, &s3);
            const R z0 = ra * c1, z1 = ra * s1, z2 = rb * c3, z3 = rb * s3;
            // ---- Euler-Maruyama update
            double xn, yn, zn;
            R sxn = (R)0, xib = (R)0;
            {
                R dx[3];
                if (KPERP) {
                    xib = z1 * F.b[0] + z2 * F.b[1] + z3 * F.b[2];
                    sxn = M<R>::sqrt_((R)2 * kperp * dt);
                    dx[0] = a_x[0] * dt + sxn * (z1 - xib * F.b[0]);
                    dx[1] = a_x[1] * dt + sxn * (z2 - xib * F.b[1]);
                    dx[2] = a_x[2] * dt + sxn * (z3 - xib * F.b[2]);
                } else {
                    dx[0] = a_x[0] * dt;
                    dx[1] = a_x[1] * dt;
                    dx[2] = a_x[2] * dt;
                }
                xn = x + (double)dx[0];
                yn = y + (double)dx[1];
                zn = z + (double)dx[2];
            }
            const R nmu = M<R>::sqrt_((R)2 * D * dt) * z0;
            R mun = mu + a_mu * dt + nmu;
            const R mu_end = mun;     // before any reflection
            R flip = (R)1;
            if (mun > (R)1) {
                mun = (R)2 - mun;
                flip = -flip;
            }
            if (mun < (R)-1) {
                mun = (R)-2 - mun;
                flip = -flip;
            }
            if (mun > (R)1 || mun < (R)-1) flip = (R)0;
            mun = mun > (R)1 ? (R)1 : (mun < (R)-1 ? (R)-1 : mun);
            const R lnpn = lnp + a_lnp * dt;
            // ---- tangent update: derivative of the same map
            if constexpr (MODE == 2) {
                const R G2 = M<R>::div_((R)1, (R)1 + Pm * Pm);     // (d v / d ln p) / v
                const R g1 = dmm_g1<R>(P, mu);
                R g2 = dmm_g2<R>(P, mu);
                // Eq. 5's |mu| puts a jump of 2 into dg/dmu at mu = 0, i.e. a
                // Dirac term 2 delta(mu) into g'' (the local time at mu = 0 in
                // the tangent of the continuous process); with kink_norm > 0 a
                // Gaussian of width kink_sigma stands for it
                if (P.kink_norm > 0.0)
                    g2 += (R)P.kink_norm * M<R>::exp_(-mu * mu * (R)P.kink_inv_2s2);
                // with kink_bridge the Dirac term is weighted instead by the
                // time the step is expected to spend at mu = 0 given its end
                // points (a Brownian bridge with the diffusion 2 D(0) of mu = 0)
                R kink_step = (R)0;
                if (P.kink_bridge) kink_step = (R)2 * A * bridge_occupation<R>(mu, mu_end, (R)2 * A * (R)P.eps, dt);
                const R iv = M<R>::div_((R)1, v);
                const R halfD = D > (R)0 ? M<R>::div_(nmu, (R)2 * D) : (R)0;   // d noise / d D
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    const R dl = TL[k], dm = TM[k];
                    const R dv = v * G2 * dl;
                    R dlnA = (G2 - (R)P.alpha) * dl;
                    R dlnK = (G2 + (R)P.alpha) * dl;
                    if (k == 0) {
                        dlnA -= (R)P.inv_lambda_ref;
                        dlnK += (R)P.inv_lambda_ref;
                    } else {
                        dlnK += (R)P.inv_kperp_ratio;
                    }
                    if (!(P.kperp_ratio > 0.0)) dlnK = G2 * dl;    // kappa_perp = v lambda_perp / 3
                    const R dD_ = D * dlnA + A * g1 * dm;            // change of D
                    const R ddD = dD * dlnA + A * g2 * dm;           // change of dD/dmu
                    const Fields<R> &f = dF[k];
                    R dax[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        dax[a] = f.V[a] + (dm * v + mu * dv) * F.b[a] + mu * v * f.b[a];
                        if (KPERP)
                            dax[a] -= kperp * dlnK * (F.divb * F.b[a] + F.curv[a]) +
                                      kperp * (f.divb * F.b[a] + F.divb * f.b[a] + f.curv[a]);
                    }
                    const R dQ = dv * F.divb + v * f.divb + dm * F.divV + mu * f.divV - (R)3 * dm * F.bbgV -
                                 (R)3 * mu * f.bbgV + (R)2 * iv * iv * dv * F.bDV - (R)2 * iv * f.bDV;
                    const R damu = -mu * dm * Qm + (R)0.5 * om * dQ + ddD;
                    const R dalnp = (R)-3 * mu * dm * F.bbgV + (R)0.5 * ((R)1 - (R)3 * mu * mu) * f.bbgV +
                                    mu * dm * F.divV - (R)0.5 * om * f.divV - dm * iv * F.bDV +
                                    mu * dv * iv * iv * F.bDV - mu * iv * f.bDV;
                    R dnx[3] = {(R)0, (R)0, (R)0};
                    if (KPERP) {
                        const R xidb = z1 * f.b[0] + z2 * f.b[1] + z3 * f.b[2];
                        const R hk = (R)0.5 * dlnK;
                        const R zz[3] = {z1, z2, z3};
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            dnx[a] = sxn * (hk * (zz[a] - xib * F.b[a]) - xidb * F.b[a] - xib * f.b[a]);
                    }
#pragma unroll
                    for (int a = 0; a < 3; ++a) TX[k][a] += dax[a] * dt + dnx[a];
                    TM[k] = flip * (dm + damu * dt + halfD * dD_ + kink_step * dm);
                    TL[k] = dl + dalnp * dt;
                }
            }
            ++my_steps;
            if (!(isfinite(xn) && isfinite(yn) && isfinite(zn) && isfinite(mun) && isfinite(lnpn))) {
                status = FTE_PS_NUMERIC;
                break;
            }
            x = xn;
            y = yn;
            z = zn;
            mu = mun;
            lnp = lnpn;
            Pcur = M<R>::exp_(lnp);
            gcur = M<R>::sqrt_((R)1 + Pcur * Pcur);
            vcur = M<R>::div_((R)kC * Pcur, gcur);
            // ---- boundaries (radius in double on both paths)
            r2 = x * x + y * y + z * z;
            r = radius_of<R>(r2);
            if (kF64 ? (double)r < P.r_in : r2 < P.r_in2) {
                status = FTE_PS_ABSORBED_IN;
                break;
            }
            if (kF64 ? (double)r > P.r_out : r2 > P.r_out2) {
                status = FTE_PS_ABSORBED_OUT;
                break;
            }
            th = M<R>::acos_(cos_colat<R>(z, r));
            ph = M<R>::atan2_((R)y, (R)x);
            if (ph < (R)0) ph += (R)(2.0 * kPi);
            if (th < (R)G.th_lo || th > (R)G.th_hi) {
                status = FTE_PS_OUT_OF_DOMAIN;
                break;
            }
            // ---- kernel-smoothed sums of the post-step state, per global step
            // (the time kernel is applied when they are read out)
            if constexpr (MODE >= 1) {
                const long long m = (long long)n - P.win_lo;
                if (m >= 0 && m < P.n_win) {
                    const R lnE = M<R>::log_((R)P.mass_c2 * M<R>::div_(Pcur * Pcur, gcur + (R)1));
                    const R iE = M<R>::exp_(-lnE);
                    const R base_w = (R)w * vcur * dt;
                    const R dlE = M<R>::div_(gcur + (R)1, gcur);        // d ln E / d ln p
                    const R G2n = M<R>::div_((R)1, gcur * gcur);       // d ln v / d ln p
                    for (int o = 0; o < P.n_obs; ++o) {
                        const double ddx[3] = {x - P.obs_xyz[o][0], y - P.obs_xyz[o][1], z - P.obs_xyz[o][2]};
                        const double d2 = ddx[0] * ddx[0] + ddx[1] * ddx[1] + ddx[2] * ddx[2];
                        if (d2 > P.sx_cut2) continue;
                        const R g3 = M<R>::exp_((R)(-d2 * P.inv_2sx2)) * (R)P.norm3;
                        const R c0 = base_w * g3 * iE * (R)P.norm1;
                        R gx[ND];
                        if constexpr (MODE == 2) {
#pragma unroll
                            for (int k = 0; k < ND; ++k)
                                gx[k] = TL[k] * G2n - (R)((double)ddx[0] * (double)TX[k][0] + ddx[1] * (double)TX[k][1] +
                                                          ddx[2] * (double)TX[k][2]) * (R)P.inv_sx2;
                        }
                        // energy-bin centres within the cut: a range from the
                        // continuous centre index, the exact test per bin
                        const R uc = (lnE - (R)P.e_min_ln) * (R)P.inv_dlne - (R)0.5;
                        const R span = (R)P.sl_cut * (R)P.inv_dlne;
                        int e_a = (int)M<R>::floor_(uc - span) - 1, e_b = (int)M<R>::floor_(uc + span) + 2;
                        e_a = e_a < 0 ? 0 : e_a;
                        e_b = e_b > P.n_e - 1 ? P.n_e - 1 : e_b;
                        double *row = sm + ((size_t)m * P.n_obs + o) * (size_t)P.n_e * P.nk;
                        for (int e = e_a; e <= e_b; ++e) {
                            const R ue = lnE - (R)(P.e_min_ln + ((double)e + 0.5) * P.dlne);
                            if (!(ue <= (R)P.sl_cut && ue >= -(R)P.sl_cut)) continue;
                            const R c = c0 * M<R>::exp_(-ue * ue * (R)P.inv_2sl2);
                            double *cell = row + (size_t)e * P.nk;
                            atomicAdd(cell, (double)c);
                            if constexpr (MODE == 2) {
                                const R fe = (-ue * (R)P.inv_sl2 - (R)1) * dlE;
#pragma unroll
                                for (int k = 0; k < ND; ++k)
                                    atomicAdd(cell + 1 + k, (double)(c * (gx[k] + fe * TL[k])));
                                atomicAdd(cell + 3, (double)(c * dlnw));
                            }
                        }
                    }
                }
            }
            // ---- residence-time observer estimator, post-step state: the
            // radial and colatitude tests come first, then the longitude bin
            // of each observer (rotating with it), the energy bin only for a
            // particle inside one
            const bool in_obs_box = kF64 ? ((double)r >= P.obs_u[0] && (double)r < P.obs_u[1])
                                         : (r2 >= P.obs_u[2] && r2 < P.obs_u[3]);
            if (P.n_obs > 0 && in_obs_box && th >= (R)P.obs_u[4] && th < (R)P.obs_u[5]) {
                const double t = P.t0 + (double)n * P.dt;
                const double ut = (t + P.dt - P.t_ref) * P.inv_dT;
                const double t1 = P.t0 + (double)(n + 1) * P.dt;
                for (int o = 0; o < P.n_obs; ++o) {
                    const double *ob = P.obs[o];
                    const bool shell = kF64 ? ((double)r >= ob[0] && (double)r < ob[1])
                                            : (r2 >= P.obs_rsq[o][0] && r2 < P.obs_rsq[o][1]);
                    if (!(shell && th >= (R)ob[2] && th < (R)ob[3])) continue;
                    R u = M<R>::fmod_(ph - (R)(ob[4] + P.obs_omega[o] * t1 - 0.5 * ob[5]), (R)(2.0 * kPi));
                    if (u < (R)0) u += (R)(2.0 * kPi);
                    const int kb = (int)M<R>::floor_(M<R>::div_(u, (R)ob[5]));
                    if (!(kb >= 0 && kb < P.obs_nphi[o])) continue;
                    const int obin = P.obs_off[o] + kb;
                    const R lnE = M<R>::log_((R)P.mass_c2 * M<R>::div_(Pcur * Pcur, gcur + (R)1));
                    const R ue = (lnE - (R)P.e_min_ln) * (R)P.inv_dlne;
                    if (ue >= (R)0 && ue < (R)P.n_e && ut >= 0.0 && ut < (double)P.n_t) {
                        const int ie = (int)M<R>::floor_(ue);
                        const int it = (int)::floor(ut);
                        const int ib = (int)(pid % (uint64_t)P.n_batch);
                        const double add = w * (double)vcur * P.dt;
                        const int lt = it - LD.it_lo;
                        const size_t rob = (size_t)run_r * P.n_obs_bins + obin;
                        if (lt >= 0 && lt < LD.n_tb) {
                            atomicAdd(&lh[((rob * P.n_e + ie) * LD.n_tb + lt) * P.n_batch + ib], add);
                        } else {
                            atomicAdd(&hist[((rob * P.n_e + ie) * P.n_t + it) * P.n_batch + ib], add);
                        }
                    }
                }
            }
        }
        st.x[i] = x;
        st.y[i] = y;
        st.z[i] = z;
        st.mu[i] = (double)mu;
        st.lnp[i] = (double)lnp;
        if constexpr (MODE == 2) {
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                tn.col(5 * k + 0)[i] = (double)TX[k][0];
                tn.col(5 * k + 1)[i] = (double)TX[k][1];
                tn.col(5 * k + 2)[i] = (double)TX[k][2];
                tn.col(5 * k + 3)[i] = (double)TM[k];
                tn.col(5 * k + 4)[i] = (double)TL[k];
            }
        }
        if (status == FTE_PS_ACTIVE && n_win >= step_end) status = FTE_PS_DONE;
        if (status != FTE_PS_ACTIVE) {
            st.status[i] = status;
            atomicAdd(&cnt->retired[status], 1ull);
            atomicAdd(&cnt->w_retired[status], w);
        }
    }
    // block total of particle-steps, one atomic per block
    __shared__ unsigned long long red[1024 / 64];
    unsigned long long v = my_steps;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += red[k];
        if (tot) atomicAdd(&cnt->steps, tot);
    }
    // flush the block's histogram (the barrier above orders it after every
    // LDS accumulation)
    for (int k = threadIdx.x; k < n_lh; k += blockDim.x) {
        const double v = lh[k];
        if (v != 0.0) {
            const int ib = k % P.n_batch;
            const int lt = (k / P.n_batch) % LD.n_tb;
            const int oe = k / (P.n_batch * LD.n_tb);
            atomicAdd(&hist[((size_t)oe * P.n_t + LD.it_lo + lt) * P.n_batch + ib], v);
        }
    }
}

// Instances: the LDS block index only when the build allows it (it is off by
// default), so that the kernels of a plain run carry none of its code; the
// unrolled two-snapshot gather (TS2) on time-dependent grids, where the
// register peak it adds (2 waves per SIMD instead of 3 on the float path)
// pays for itself: +15% on the CIR workload, +10% on the kappa_perp
// ensemble, even on the largest workload, +2% on the double path (already at
// 2 waves).  The tangent kernels gather through their own path.
// Per-particle run parameters (ENS) only for ensembles: a single run's stay
// uniform, which frees vector registers (+6% on the double path).  Records
// through a leaf pool's map (SUB) only for streamed subsets.
template <typename R, bool KPERP, int MODE, bool LIDX, bool TS2>
static void launch_step_e(const DevParams &p, const DevGrid &g, DevState st, DevTan tn, DevCounters *cnt, int slot,
                          double *hist, double *sm, uint64_t n0, uint32_t n_steps, dim3 grid, dim3 blk, StepLds ld,
                          size_t shmem, hipStream_t s) {
    // ensembles (histogram mode only) read each particle's run parameters; a
    // single run keeps them uniform, in scalar registers
    if constexpr (MODE == 0) {
        if (p.n_runs > 0) {
            hipLaunchKernelGGL((k_step<R, KPERP, MODE, LIDX, TS2, true, false>), grid, blk, shmem, s, p, g, st, tn,
                               cnt, slot, hist, sm, n0, n_steps, ld);
            return;
        }
        // a streamed subset of leaves: records through the pool map
        if constexpr (TS2 && !LIDX) {
            if (g.pool_map) {
                hipLaunchKernelGGL((k_step<R, KPERP, MODE, LIDX, TS2, false, true>), grid, blk, shmem, s, p, g, st,
                                   tn, cnt, slot, hist, sm, n0, n_steps, ld);
                return;
            }
        }
    }
    hipLaunchKernelGGL((k_step<R, KPERP, MODE, LIDX, TS2, false, false>), grid, blk, shmem, s, p, g, st, tn, cnt,
                       slot, hist, sm, n0, n_steps, ld);
}

template <typename R, bool KPERP, int MODE, bool LIDX>
static void launch_step_ts(const DevParams &p, const DevGrid &g, DevState st, DevTan tn, DevCounters *cnt, int slot,
                           double *hist, double *sm, uint64_t n0, uint32_t n_steps, dim3 grid, dim3 blk, StepLds ld,
                           size_t shmem, hipStream_t s) {
    if constexpr (MODE < 2) {
        if (g.n_snap >= 2) {
            launch_step_e<R, KPERP, MODE, LIDX, true>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld,
                                                      shmem, s);
            return;
        }
    }
    launch_step_e<R, KPERP, MODE, LIDX, false>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem,
                                               s);
}

template <typename R, bool KPERP, int MODE>
static void launch_step_m(const DevParams &p, const DevGrid &g, DevState st, DevTan tn, DevCounters *cnt, int slot,
                          double *hist, double *sm, uint64_t n0, uint32_t n_steps, dim3 grid, dim3 blk, StepLds ld,
                          size_t shmem, bool lidx, hipStream_t s) {
    if constexpr (kLdsIndexBytes > 0) {
        if (lidx) {
            launch_step_ts<R, KPERP, MODE, true>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem,
                                                 s);
            return;
        }
    }
    launch_step_ts<R, KPERP, MODE, false>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, s);
}

template <typename R, bool KPERP>
static void launch_step_t(const DevParams &p, const DevGrid &g, DevState st, DevTan tn, DevCounters *cnt, int slot,
                          double *hist, double *sm, uint64_t n0, uint32_t n_steps, dim3 grid, dim3 blk, StepLds ld,
                          size_t shmem, bool lidx, hipStream_t s) {
    if (p.grad)
        launch_step_m<R, KPERP, 2>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, lidx, s);
    else if (p.smooth)
        launch_step_m<R, KPERP, 1>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, lidx, s);
    else
        launch_step_m<R, KPERP, 0>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, lidx, s);
}

// LDS plan of one launch: the time bins its post-step times fall in (the
// kernel's own floor of (t + dt - t_ref) / dT at the first and last step),
// when their histogram fits hist_bytes; the block index when it fits
// kLdsIndexBytes.
StepLds plan_step_lds(const DevParams &p, const DevGrid &g, uint64_t n0, uint32_t n_steps, size_t hist_bytes,
                      size_t *shmem, bool *lidx) {
    StepLds ld{0, 0, 0, 0};
    if (p.n_obs > 0 && n_steps > 0) {
        const double t_a = p.t0 + (double)n0 * p.dt, t_b = p.t0 + (double)(n0 + n_steps - 1) * p.dt;
        double fa = ::floor((t_a + p.dt - p.t_ref) * p.inv_dT), fb = ::floor((t_b + p.dt - p.t_ref) * p.inv_dT);
        fa = fa < 0.0 ? 0.0 : fa;
        fb = fb > (double)(p.n_t - 1) ? (double)(p.n_t - 1) : fb;
        if (fb >= fa) {
            const int ntb = (int)(fb - fa) + 1;
            const size_t bytes = (size_t)p.n_runs_eff * p.n_obs_bins * p.n_e * ntb * p.n_batch * 8;
            if (bytes <= hist_bytes) {
                ld.it_lo = (int)fa;
                ld.n_tb = ntb;
            }
        }
    }
    const size_t hb = ld.n_tb > 0 ? (size_t)p.n_runs_eff * p.n_obs_bins * p.n_e * ld.n_tb * p.n_batch * 8 : 0;
    const size_t ib = ((size_t)g.n_base + g.n_child) * 4;
    *lidx = ib <= kLdsIndexBytes;
    *shmem = hb + (*lidx ? ib : 0);
    return ld;
}

hipError_t launch_step(const DevParams &p, const DevGrid &g, DevState st, DevTan tn, DevCounters *cnt, int slot,
                       double *hist, double *sm, uint64_t n0, uint32_t n_steps, uint64_t n_upper, int block, int fp32,
                       size_t tile_bytes, size_t hist_bytes, hipStream_t s) {
    if (n_upper == 0 || n_steps == 0) return hipSuccess;
    const bool kp = p.kperp_any != 0;
    dim3 grid(blocks_for(n_upper, block)), blk(block);
    size_t shmem = 0;
    bool lidx = false;
    StepLds ld = plan_step_lds(p, g, n0, n_steps, hist_bytes, &shmem, &lidx);
    if (fp32 && !lidx && (g.n_snap >= 2 || !p.grad) && tile_bytes > 0) {
        // as many whole padded k-layers of the live snapshots (two, or the
        // one of a steady grid) as fit, at least two
        const size_t nst = g.n_snap >= 2 ? 2 : 1;
        const size_t layer_bytes = (size_t)g.px[0] * g.px[1] * (kp ? kRSKperp : kRSPlain) * sizeof(float);
        // LDS of two workgroups per CU within its 160 KB (the two-snapshot
        // kernels run 2 waves per SIMD), of three for the steady-grid kernel
        // (3 waves per SIMD); 1 KB of each share is left to the kernel's
        // static LDS and the allocation granule
        const size_t share = (size_t)160 * 1024 / (nst == 1 ? 3 : 2);
        const size_t fit = share > shmem + 1024 ? share - shmem - 1024 : 0;
        const size_t budget = tile_bytes < fit ? tile_bytes : fit;
        size_t tl = budget / (nst * layer_bytes);
        if (tl > (size_t)g.px[2]) tl = (size_t)g.px[2];
        if (tl >= 2) {
            ld.tile_off = (int)((shmem + 15) & ~(size_t)15);
            ld.tile_layers = (int)tl;
            shmem = (size_t)ld.tile_off + nst * tl * layer_bytes;
        }
    }
    if (fp32) {
        if (kp) launch_step_t<float, true>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, lidx, s);
        else launch_step_t<float, false>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, lidx, s);
    } else {
        if (kp) launch_step_t<double, true>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, lidx, s);
        else launch_step_t<double, false>(p, g, st, tn, cnt, slot, hist, sm, n0, n_steps, grid, blk, ld, shmem, lidx, s);
    }
    return hipGetLastError();
}

// ===========================================================================
// compaction: wavefront ballot + in-wave prefix, one atomic per wave
// ===========================================================================
__global__ void k_zero_live(DevCounters *cnt, int slot) {
    if (threadIdx.x == 0 && blockIdx.x == 0) cnt->n_live[slot] = 0;
}

__device__ __forceinline__ void copy_tangent(const DevTan &a, const DevTan &b, uint64_t i, uint64_t j) {
    if (!a.base) return;
#pragma unroll
    for (int q = 0; q < kTanCols; ++q) b.col(q)[j] = a.col(q)[i];
}

__global__ void k_compact(DevState src, DevState dst, DevTan tsrc, DevTan tdst, DevCounters *cnt, int from) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n_live = cnt->n_live[from];
    const bool alive = i < n_live && src.status[i] == FTE_PS_ACTIVE;
    const unsigned long long mask = __ballot(alive);
    const int lane = threadIdx.x & 63;
    const int prefix = __popcll(mask & ((1ull << lane) - 1ull));
    const int total = __popcll(mask);
    unsigned long long base = 0;
    if (lane == 0 && total > 0) base = atomicAdd(&cnt->n_live[1 - from], (unsigned long long)total);
    base = __shfl(base, 0, 64);
    if (alive) {
        const uint64_t j = base + prefix;
        dst.x[j] = src.x[i];
        dst.y[j] = src.y[i];
        dst.z[j] = src.z[i];
        dst.mu[j] = src.mu[i];
        dst.lnp[j] = src.lnp[i];
        dst.w[j] = src.w[i];
        dst.pid[j] = src.pid[i];
        dst.kinj[j] = src.kinj[i];
        dst.status[j] = FTE_PS_ACTIVE;
        dst.run[j] = src.run[i];
        copy_tangent(tsrc, tdst, i, j);
    }
}

hipError_t launch_zero_live(DevCounters *cnt, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_live, dim3(1), dim3(64), 0, s, cnt, slot);
    return hipGetLastError();
}

hipError_t launch_compact(DevState src, DevState dst, DevTan tsrc, DevTan tdst, DevCounters *cnt, int from,
                          uint64_t n_upper, int block, hipStream_t s) {
    if (n_upper == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(blocks_for(n_upper, block)), dim3(block), 0, s, src, dst, tsrc, tdst, cnt,
                       from);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compaction with a spatial counting sort: live particles are regrouped by
// (leaf, cube of cells) so that a wavefront gathers from neighbouring
// records; order inside a key is arbitrary (results depend only on pid, not
// on storage order).  The key space is bounded by the particle count, not by
// the grid: the host picks the cube edge (and, on grids with more leaves than
// that bound allows, groups of consecutive leaves) per compaction
// (sort_shape_for), so zeroing and scanning the per-key counts costs
// O(live particles) however many cells the grid has.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell_key(const DevGrid &G, const SortShape &K, double x, double y, double z) {
    const double r = ::sqrt(x * x + y * y + z * z);
    float ph = ::atan2f((float)y, (float)x);
    if (ph < 0.f) ph += (float)(2.0 * kPi);
    float s[3];
    grid_coords<float>(G, r, ::acosf((float)(z / r)), ph, s);
    fold_s<float>(G, s);
    float S[3];
    int B[3];
    const int leaf = descend<float>(G, G.base, G.child, s, S, B);
    if (leaf < 0) return 0u;
    int sub[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int l = (int)::floorf(S[a]) - B[a] * G.bx[a];
        l = l < 0 ? 0 : (l > G.bx[a] - 1 ? G.bx[a] - 1 : l);
        sub[a] = l >> K.cube_shift;
    }
    return ((uint32_t)leaf >> K.leaf_shift) * K.n_sub + (uint32_t)(sub[0] + K.h[0] * (sub[1] + K.h[1] * sub[2]));
}

__global__ void k_sort_key(DevGrid G, SortShape K, DevState src, const DevCounters *cnt, int from, uint32_t *keys,
                           uint32_t *counts) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt->n_live[from]) return;
    if (src.status[i] != FTE_PS_ACTIVE) {
        keys[i] = 0xFFFFFFFFu;
        return;
    }
    const uint32_t k = cell_key(G, K, src.x[i], src.y[i], src.z[i]);
    keys[i] = k;
    atomicAdd(&counts[k], 1u);
}

// Exclusive scan of counts[0..nk) in three passes: tiles of 4096 scanned by
// one workgroup each (tile totals to tsum), the tile totals by one
// workgroup, then the tile offsets added back.  The total becomes the
// destination's live count.
constexpr int kScanTile = 4096;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    const int t = threadIdx.x, nt = blockDim.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const uint32_t a = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    const uint32_t incl = sh[t];
    *total = sh[nt - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(1024) k_scan_tiles(uint32_t *counts, uint32_t nk, uint32_t *tsum) {
    __shared__ uint32_t sh[1024];
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * 4;
    uint32_t c[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c[q] = base + q < nk ? counts[base + q] : 0u;
        sum += c[q];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(sum, sh, &tot);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < nk) counts[base + q] = run;
        run += c[q];
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_totals(uint32_t *tsum, uint32_t nt, DevCounters *cnt, int to) {
    __shared__ uint32_t sh[1024];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nt; b0 += blockDim.x) {
        const uint32_t k = b0 + threadIdx.x;
        const uint32_t v = k < nt ? tsum[k] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, sh, &tot);
        if (k < nt) tsum[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) cnt->n_live[to] = carry;
}

__global__ void k_scan_add(uint32_t *counts, uint32_t nk, const uint32_t *tsum) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nk) counts[i] += tsum[i / kScanTile];
}

__global__ void k_sort_scatter(DevState src, DevState dst, DevTan tsrc, DevTan tdst, const DevCounters *cnt,
                               int from, const uint32_t *keys, uint32_t *cursor) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt->n_live[from]) return;
    const uint32_t k = keys[i];
    if (k == 0xFFFFFFFFu) return;
    const uint64_t j = atomicAdd(&cursor[k], 1u);
    dst.x[j] = src.x[i];
    dst.y[j] = src.y[i];
    dst.z[j] = src.z[i];
    dst.mu[j] = src.mu[i];
    dst.lnp[j] = src.lnp[i];
    dst.w[j] = src.w[i];
    dst.pid[j] = src.pid[i];
    dst.kinj[j] = src.kinj[i];
    dst.status[j] = FTE_PS_ACTIVE;
    dst.run[j] = src.run[i];
    copy_tangent(tsrc, tdst, i, j);
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Cubes of 2^(sort-1) cells or coarser, and groups of 2^leaf_shift
// consecutive leaves, so that the key space fits max_keys.
SortShape sort_shape_for(const DevGrid &g, int sort, uint64_t max_keys) {
    SortShape K{};
    const int bmax = g.bx[0] > g.bx[1] ? (g.bx[0] > g.bx[2] ? g.bx[0] : g.bx[2]) : (g.bx[1] > g.bx[2] ? g.bx[1] : g.bx[2]);
    for (K.cube_shift = sort - 1;; ++K.cube_shift) {
        const int e = 1 << K.cube_shift;
        for (int a = 0; a < 3; ++a) K.h[a] = (g.bx[a] + e - 1) >> K.cube_shift;
        K.n_sub = (uint32_t)(K.h[0] * K.h[1] * K.h[2]);
        if ((uint64_t)g.n_leaves * K.n_sub <= max_keys || e >= bmax) break;
    }
    for (K.leaf_shift = 0;; ++K.leaf_shift) {
        const uint64_t groups = ((uint64_t)g.n_leaves + (1ull << K.leaf_shift) - 1) >> K.leaf_shift;
        K.n_keys = (uint32_t)(groups * K.n_sub);
        if (groups * K.n_sub <= max_keys) break;
    }
    return K;
}

hipError_t launch_compact_sorted(const DevGrid &g, const SortShape &K, DevState src, DevState dst, DevTan tsrc,
                                 DevTan tdst, DevCounters *cnt, int from, uint64_t n_upper, uint32_t *keys,
                                 uint32_t *counts, uint32_t *tsum, hipStream_t s) {
    const uint32_t nk = K.n_keys;
    const uint32_t ntile = (nk + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(nk, 256)), dim3(256), 0, s, counts, nk);
    if (n_upper > 0)
        hipLaunchKernelGGL(k_sort_key, dim3(blocks_for(n_upper, 256)), dim3(256), 0, s, g, K, src, cnt, from, keys,
                           counts);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntile), dim3(1024), 0, s, counts, nk, tsum);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, tsum, ntile, cnt, 1 - from);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(nk, 256)), dim3(256), 0, s, counts, nk, tsum);
    if (n_upper > 0)
        hipLaunchKernelGGL(k_sort_scatter, dim3(blocks_for(n_upper, 256)), dim3(256), 0, s, src, dst, tsrc, tdst, cnt,
                           from, keys, counts);
    return hipGetLastError();
}

// ===========================================================================
// finalisation: j = S / (4 pi dV dT dE W_inj), standard error from batches
// ===========================================================================
// observer owning observer bin ob
__device__ __forceinline__ int obs_of_bin(const DevParams &P, int ob) {
    int o = 0;
    while (o + 1 < P.n_obs && ob >= P.obs_off[o + 1]) ++o;
    return o;
}

__device__ __forceinline__ double obs_volume(const DevParams &P, int o) {
    const double *ob = P.obs[o];
    return (ob[1] * ob[1] * ob[1] - ob[0] * ob[0] * ob[0]) / 3.0 * (::cos(ob[2]) - ::cos(ob[3])) * ob[5];
}

__global__ void k_finalize(DevParams P, const double *hist, const DevCounters *cnt, double *j, double *sig) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = P.n_obs_bins * P.n_e * P.n_t;
    if (idx >= nb * P.n_runs_eff) return;
    const int run = idx / nb;
    const int obin = (idx % nb) / (P.n_e * P.n_t);
    const int e = (idx / P.n_t) % P.n_e;
    double W = 0.0;
    for (int b = 0; b < P.n_batch; ++b) W += cnt->w_inj[run * P.n_batch + b];
    const double dV = obs_volume(P, obs_of_bin(P, obin));
    const double dE = P.e_min * (::exp((e + 1) * P.dlne) - ::exp(e * P.dlne));
    const double norm = 4.0 * kPi * dV * P.dT * dE * W;
    const double *h = hist + (size_t)idx * P.n_batch;
    double s = 0.0;
    for (int b = 0; b < P.n_batch; ++b) s += h[b];
    const double jm = W > 0.0 ? s / norm : 0.0;
    double var = 0.0;
    for (int b = 0; b < P.n_batch; ++b) {
        const double jb = W > 0.0 ? P.n_batch * h[b] / norm : 0.0;
        var += (jb - jm) * (jb - jm);
    }
    j[idx] = jm;
    sig[idx] = P.n_batch > 1 ? ::sqrt(var / ((double)P.n_batch * (P.n_batch - 1))) : 0.0;
}

// Steady state of a Green's-function run: time-summed sums per batch, then
// J = S / (4 pi dV dE W_inj) and the batch standard error.
__global__ void k_finalize_steady(DevParams P, const double *hist, const DevCounters *cnt, double *j, double *sig) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = P.n_obs_bins * P.n_e;
    if (idx >= nb * P.n_runs_eff) return;
    const int run = idx / nb;
    const int obin = (idx % nb) / P.n_e;
    const int e = idx % P.n_e;
    double W = 0.0;
    for (int b = 0; b < P.n_batch; ++b) W += cnt->w_inj[run * P.n_batch + b];
    const double dV = obs_volume(P, obs_of_bin(P, obin));
    const double dE = P.e_min * (::exp((e + 1) * P.dlne) - ::exp(e * P.dlne));
    const double norm = 4.0 * kPi * dV * dE * W;
    const double *h = hist + (size_t)idx * P.n_t * P.n_batch;
    double sb[FTE_MAX_BATCH];
    for (int b = 0; b < P.n_batch; ++b) sb[b] = 0.0;
    for (int t = 0; t < P.n_t; ++t)
        for (int b = 0; b < P.n_batch; ++b) sb[b] += h[(size_t)t * P.n_batch + b];
    double s = 0.0;
    for (int b = 0; b < P.n_batch; ++b) s += sb[b];
    const double jm = W > 0.0 ? s / norm : 0.0;
    double var = 0.0;
    for (int b = 0; b < P.n_batch; ++b) {
        const double jb = W > 0.0 ? P.n_batch * sb[b] / norm : 0.0;
        var += (jb - jm) * (jb - jm);
    }
    j[idx] = jm;
    sig[idx] = P.n_batch > 1 ? ::sqrt(var / ((double)P.n_batch * (P.n_batch - 1))) : 0.0;
}

hipError_t launch_finalize_steady(const DevParams &p, const double *hist, const DevCounters *cnt, double *j,
                                  double *sig, hipStream_t s) {
    const int n = p.n_obs_bins * p.n_e * p.n_runs_eff;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_steady, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, hist, cnt, j, sig);
    return hipGetLastError();
}

hipError_t launch_finalize(const DevParams &p, const double *hist, const DevCounters *cnt, double *j, double *sig,
                           hipStream_t s) {
    const int n = p.n_obs_bins * p.n_e * p.n_t * p.n_runs_eff;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, hist, cnt, j, sig);
    return hipGetLastError();
}

// ===========================================================================
// smoothed intensities: time kernel over the per-step sums
// ===========================================================================
// out[k][o][e][t] = sum over the window's steps n of
//   G1(t0 + (n+1) dt - t_t) sums[n][o][e][k], dropping |.| > kKernelCut sigma_t.
__global__ void k_smooth_finalize(DevParams P, const double *sm, double *out) {
    const int nb = P.n_obs * P.n_e * P.n_t;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb * P.nk) return;
    const int k = idx / nb, b = idx % nb;
    const int o = b / (P.n_e * P.n_t), e = (b / P.n_t) % P.n_e, it = b % P.n_t;
    const double tc = P.t_ref + ((double)it + 0.5) * P.dT;
    const double cut = kKernelCut * P.sig_t;
    long long na = (long long)::floor((tc - cut - P.t0) / P.dt) - 2;
    long long nb_ = (long long)::ceil((tc + cut - P.t0) / P.dt) + 1;
    na = na < P.win_lo ? P.win_lo : na;
    nb_ = nb_ > P.win_lo + P.n_win - 1 ? P.win_lo + P.n_win - 1 : nb_;
    const double norm = 1.0 / (::sqrt(2.0 * kPi) * P.sig_t);
    double s = 0.0;
    for (long long n = na; n <= nb_; ++n) {
        const double ut = (P.t0 + (double)(n + 1) * P.dt) - tc;
        if (::fabs(ut) > cut) continue;
        const double kt = ::exp(-ut * ut / (2.0 * P.sig_t * P.sig_t)) * norm;
        s += kt * sm[(((size_t)(n - P.win_lo) * P.n_obs + o) * P.n_e + e) * P.nk + k];
    }
    out[idx] = s;
}

hipError_t launch_smooth_finalize(const DevParams &p, const double *sm, double *out, hipStream_t s) {
    const int n = p.n_obs * p.n_e * p.n_t * p.nk;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_smooth_finalize, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, sm, out);
    return hipGetLastError();
}

// out4[k] = sum over bins of dl[bin] fin[k][bin], k = 0..3 (one workgroup).
__global__ void __launch_bounds__(256) k_grad_contract(int nb, const double *fin, const double *dl, double *out4) {
    __shared__ double red[4][256];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double g = dl[b];
        for (int k = 0; k < 4; ++k) a[k] += g * fin[(size_t)k * nb + b];
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) out4[threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_grad_contract(const DevParams &p, const double *fin, const double *dl, double *out4, hipStream_t s) {
    const int nb = p.n_obs * p.n_e * p.n_t;
    hipLaunchKernelGGL(k_grad_contract, dim3(1), dim3(256), 0, s, nb, fin, dl, out4);
    return hipGetLastError();
}

__global__ void k_zero(double *p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t launch_zero(double *p, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

__global__ void k_zero_counters(DevCounters *cnt) {
    const int t = threadIdx.x;
    unsigned int *w = reinterpret_cast<unsigned int *>(cnt);
    const int nw = (int)(sizeof(DevCounters) / sizeof(unsigned int));
    for (int k = t; k < nw; k += blockDim.x) w[k] = 0u;
}

hipError_t launch_zero_counters(DevCounters *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, cnt);
    return hipGetLastError();
}

}  // namespace fte
