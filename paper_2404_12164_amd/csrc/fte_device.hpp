// Device building blocks: counter-based noise, precision-generic math, and the
// block-AMR index walk used by the load-time and stepping kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fte_internal.hpp"

namespace fte {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 32x32
// multiplies with the high halves mixed into the other words and the key,
// Weyl-incremented key between rounds.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox10(U4 ctr, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply each (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * ctr.a;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr.c;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        U4 nx;
        nx.a = hi1 ^ ctr.b ^ k0;
        nx.b = lo1;
        nx.c = hi0 ^ ctr.d ^ k1;
        nx.d = lo0;
        ctr = nx;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        // the round keys are uniform: bump them in scalar registers each
        // round rather than let the compiler hoist all twenty out of the
        // step loop, where they spill to vector lanes and cost a read each
        asm volatile("" : "+s"(k0), "+s"(k1));
    }
    return ctr;
}

// Stream layout: step index (48 bits), run id (16 bits), pid (60 bits), tag
// (4 bits; 0 = step noise, 1 = injection draws); key = seed.
__device__ __forceinline__ U4 philox_words(uint64_t seed, int run_id, uint64_t n, uint64_t pid, uint32_t tag) {
    U4 c;
    c.a = (uint32_t)n;
    c.b = ((uint32_t)run_id << 16) | ((uint32_t)(n >> 32) & 0xFFFFu);
    c.c = (uint32_t)pid;
    c.d = ((uint32_t)(pid >> 32) & 0x0FFFFFFFu) | (tag << 28);
    return philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// precision-generic math
// ---------------------------------------------------------------------------
template <typename R>
struct M;

template <>
struct M<double> {
    static __device__ __forceinline__ double sqrt_(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double log_(double x) { return ::log(x); }
    static __device__ __forceinline__ double exp_(double x) { return ::exp(x); }
    static __device__ __forceinline__ double pow_(double x, double y) { return ::pow(x, y); }
    static __device__ __forceinline__ double acos_(double x) { return ::acos(x); }
    static __device__ __forceinline__ double atan2_(double y, double x) { return ::atan2(y, x); }
    static __device__ __forceinline__ double floor_(double x) { return ::floor(x); }
    static __device__ __forceinline__ double fma_(double a, double b, double c) { return ::fma(a, b, c); }
    static __device__ __forceinline__ double fmod_(double x, double y) { return ::fmod(x, y); }
    // quotients in the double path stay correctly rounded
    static __device__ __forceinline__ double div_(double a, double b) { return a / b; }
    static __device__ __forceinline__ double u01(uint32_t k) { return ((double)k + 0.5) * (1.0 / 4294967296.0); }
    // (cos, sin)(2 pi u)
    static __device__ __forceinline__ void cs2pi(double u, double *c, double *s) { ::sincospi(2.0 * u, s, c); }
};

template <>
struct M<float> {
    // hardware square root (1 ulp) instead of the correctly rounded sequence
    // (a scaled estimate corrected by two fused multiply-adds).  The empty asm
    // hides the result's origin from the optimizer: it would otherwise fold
    // some reciprocals of it into reciprocal square roots and not others, so
    // that the same quantity computed at two places (at launch start and in
    // the step loop) could round differently.
    static __device__ __forceinline__ float sqrt_(float x) {
        float r = __builtin_amdgcn_sqrtf(x);
        asm("" : "+v"(r));
        return r;
    }
    static __device__ __forceinline__ float log_(float x) { return __logf(x); }
    static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
    static __device__ __forceinline__ float pow_(float x, float y) { return __expf(y * __logf(x)); }
    static __device__ __forceinline__ float acos_(float x) { return ::acosf(x); }
    static __device__ __forceinline__ float atan2_(float y, float x) { return ::atan2f(y, x); }
    static __device__ __forceinline__ float floor_(float x) { return ::floorf(x); }
    static __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float fmod_(float x, float y) { return ::fmodf(x, y); }
    // quotients in the float path: hardware reciprocal (1 ulp) times numerator
    static __device__ __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    // top 24 bits: strictly inside (0, 1) in float
    static __device__ __forceinline__ float u01(uint32_t k) { return ((float)(k >> 8) + 0.5f) * (1.0f / 16777216.0f); }
    // the hardware sine/cosine take their argument in revolutions
    static __device__ __forceinline__ void cs2pi(float u, float *c, float *s) {
        *c = __builtin_amdgcn_cosf(u);
        *s = __builtin_amdgcn_sinf(u);
    }
};

// ---------------------------------------------------------------------------
// block-AMR index
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ncell(const DevGrid &G, int L, int a) { return G.n1[a] << (L - 1); }

// c / bx[a] for 0 <= c: the high word of c ceil(2^32 / bx).  With
// e = ceil(2^32 / bx) - 2^32 / bx in [0, 1) the product exceeds c / bx by
// c e / 2^32 < 1 / bx as long as c bx < 2^32 (cell indices below 2^26, blocks
// of at most 64 cells), so the floor is exact.
__device__ __forceinline__ int div_bx(const DevGrid &G, int c, int a) {
    return (int)__umulhi((uint32_t)c, G.bx_mag[a]);
}

// Bring a level-L index into the domain: clamp xi and theta, wrap a periodic phi.
__device__ __forceinline__ void fold(const DevGrid &G, int L, int c[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int n = ncell(G, L, a);
        if (a == 2 && G.periodic) {
            c[a] %= n;
            if (c[a] < 0) c[a] += n;
        } else {
            c[a] = c[a] < 0 ? 0 : (c[a] > n - 1 ? n - 1 : c[a]);
        }
    }
}

// Leaf holding the (folded) level-L cell c.  *M receives the leaf level and
// cm the level-M index of c (its ancestor when M <= L, its first descendant
// when M > L; all descendants of c then lie in that one leaf).
__device__ __forceinline__ int find_leaf_cell(const DevGrid &G, int L, const int c[3], int *M, int cm[3]) {
    int cc[3], B[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cc[a] = c[a] >> (L - 1);
        B[a] = div_bx(G, cc[a], a);
    }
    int node = G.base[B[0] + G.nb1[0] * (B[1] + G.nb1[1] * B[2])];
    int m = 1;
    while (node < 0) {
        const int grp = -node - 1;
        ++m;
        if (m > G.n_levels) return -1;
        int slot = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cc[a] = (m <= L) ? (c[a] >> (L - m)) : (c[a] << (m - L));
            const int Bn = div_bx(G, cc[a], a);
            slot |= (Bn & 1) << a;
        }
        node = G.child[grp * 8 + slot];
    }
    *M = m;
#pragma unroll
    for (int a = 0; a < 3; ++a) cm[a] = cc[a];
    return node;
}

// Value of a level-L cell centre for any per-cell quantity held by `Src`
// (the block-boundary rule): same level -> the cell value; finer leaf -> mean
// of the descendants; coarser leaf -> trilinear interpolation, at the centre,
// of the level-(L-1) values around it.  With 2:1 nesting every coarser
// stencil value resolves without a further level change; otherwise the
// function reports failure.
template <int NC, class Src>
__device__ bool virtual_value(const DevGrid &G, const Src &S, int L, const int cin[3], double out[NC]) {
    int c[3] = {cin[0], cin[1], cin[2]};
    fold(G, L, c);
    int Mlev, cm[3];
    int leaf = find_leaf_cell(G, L, c, &Mlev, cm);
    if (leaf < 0) return false;
    if (Mlev >= L) {
        S.mean_cube(leaf, cm, 1 << (Mlev - L), out);
        return true;
    }
    int i0[3];
    double f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = ((double)c[a] + 0.5) / 2.0 - 0.5;
        i0[a] = (int)::floor(u);
        f[a] = u - (double)i0[a];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) out[k] = 0.0;
    for (int d = 0; d < 8; ++d) {
        const int e0 = d & 1, e1 = (d >> 1) & 1, e2 = (d >> 2) & 1;
        int cc[3] = {i0[0] + e0, i0[1] + e1, i0[2] + e2};
        const double w = (e0 ? f[0] : 1.0 - f[0]) * (e1 ? f[1] : 1.0 - f[1]) * (e2 ? f[2] : 1.0 - f[2]);
        fold(G, L - 1, cc);
        int M2, cm2[3];
        const int lf2 = find_leaf_cell(G, L - 1, cc, &M2, cm2);
        if (lf2 < 0 || M2 < L - 1) return false;
        double tmp[NC];
        S.mean_cube(lf2, cm2, 1 << (M2 - (L - 1)), tmp);
#pragma unroll
        for (int k = 0; k < NC; ++k) out[k] += w * tmp[k];
    }
    return true;
}

}  // namespace fte
