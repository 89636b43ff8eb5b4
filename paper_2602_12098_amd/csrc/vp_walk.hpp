// Path-walk primitives shared by the path-search kernels (per-call search
// and batched search): the start residual, the walk of one position vector
// down the tree with its PED, and the argmin key reduction.  Every search
// kernel uses these, so a path evaluated anywhere performs bit-identical
// float32 arithmetic (Sec. II-B PED recursion, Sec. III-A-2 DEMAP).
#pragma once

#include "vp_internal.hpp"

#ifndef VP_LUT_STORAGE
#define VP_LUT_STORAGE static __constant__
#endif
#include "vp_device.hpp"

namespace vp {

// s-tilde_i / tau = (sum_{j<=i} W_ij s_{pi_j}) / tau for one vector.
template <int N>
__device__ __forceinline__ float2 stilde_over_tau(const float2 *__restrict__ Wc, const uint8_t *__restrict__ pm,
                                                  const float2 *__restrict__ s, size_t v, size_t n_vec, int i,
                                                  float inv_tau) {
    float re = 0.f, im = 0.f;
    // every load is issued up front (vp_pidx(N, i, j) stays inside the packed
    // triangle for all j < N); the terms j > i are skipped
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float2 w = Wc[vp_pidx(N, i, j)];
        const int u = pm[j] < N ? pm[j] : N - 1;   // a corrupt permutation must not index out of bounds
        const float2 x = s[(size_t)u * n_vec + v];
        if (j <= i) {
            re = fmaf(w.x, x.x, fmaf(-w.y, x.y, re));
            im = fmaf(w.x, x.y, fmaf(w.y, x.x, im));
        }
    }
    return make_float2(re * inv_tau, im * inv_tau);
}

// Walk one path over levels [LO, HI).  r: residuals / tau (in: their values
// after level LO-1, destroyed), linv_i = 1 / W_ii, wdiag_i = W_ii, ped: the
// PED so far.  Returns ped + sum_{LO<=i<HI} |r_i + W_ii l_i|^2; with REC the
// chosen offsets.  A walk split into consecutive ranges performs exactly the
// arithmetic of the whole walk.
// Hides a wave-uniform pointer from loop-invariant code motion, so that the W
// column of each level is scalar-loaded where it is used instead of all 240
// coefficients being hoisted (and spilled) at once.  Loads through the
// constant address space are selected as scalar (SMEM) loads.
typedef const __attribute__((address_space(4))) float cfloat;   // constant space: scalar loads

// The dependence on `after` keeps a load from being issued before that value
// exists (the level's DEMAP result, or the chunk two steps back), which bounds
// the scalar registers held by W to two chunks.
__device__ __forceinline__ cfloat *opaque_uniform(const float2 *p, float after) {
    asm volatile("" : "+s"(p) : "v"(after));
    return (cfloat *)p;
}

template <int N, bool UNIFORM_TIERS, bool REC, int LO = 0, int HI = N>
__device__ __forceinline__ float walk(const float2 *__restrict__ W0, const float *linv, const float *wdiag, float2 (&r)[N],
                                      unsigned long long word, const uint8_t *lut, float *ra, float *rb,
                                      float ped = 0.f) {
    constexpr int CH = 4;   // W rows per scalar load (8 dwords)
#pragma unroll
    for (int i = LO; i < HI; ++i) {
        const int rank = (int)((word >> (4 * i)) & 15ull);
        const float li = linv[i];
        const float cx = -(r[i].x * li);
        const float cy = -(r[i].y * li);
        float a, b;
        if (UNIFORM_TIERS) {   // the cheapest variant that serves every lane of the wave
            if (!__any(rank != 0)) vp_demap0(cx, cy, a, b);
            else if (!__any(rank > 1)) vp_demap1(cx, cy, rank, a, b);
            else if (!__any(rank > 2)) vp_demap2(cx, cy, rank, a, b);
            else vp_demapN(cx, cy, rank, lut, a, b);
        } else {
            vp_demapN(cx, cy, rank, lut, a, b);
        }
        if (REC) {
            ra[i] = a;
            rb[i] = b;
        }
        const float wii = wdiag[i];
        const float ex = fmaf(wii, a, r[i].x);
        const float ey = fmaf(wii, b, r[i].y);
        ped = fmaf(ex, ex, ped);
        ped = fmaf(ey, ey, ped);
#pragma unroll
        for (int m0 = i + 1; m0 < N; m0 += CH) {
            float2 w[CH];
            if (UNIFORM_TIERS) {
                // chunk c may load once chunk c-1 has started at this level
                const float dep = (m0 > i + 1) ? r[m0 - CH].y : a;
                cfloat *Wk = opaque_uniform(W0, dep);
#pragma unroll
                for (int q = 0; q < CH; ++q)
                    if (m0 + q < N) {
                        w[q].x = Wk[2 * vp_pidx(N, m0 + q, i)];
                        w[q].y = Wk[2 * vp_pidx(N, m0 + q, i) + 1];
                    }
            } else {
#pragma unroll
                for (int q = 0; q < CH; ++q)
                    if (m0 + q < N) w[q] = W0[vp_pidx(N, m0 + q, i)];
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int m = m0 + q;
                if (m < N) {
                    r[m].x = fmaf(w[q].x, a, fmaf(-w[q].y, b, r[m].x));
                    r[m].y = fmaf(w[q].x, b, fmaf(w[q].y, a, r[m].y));
                }
            }
        }
    }
    return ped;
}

__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_min(unsigned long long x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = umin64(x, __shfl_xor(x, off));
    return x;
}

// Rank nibbles of path k (level i at bits 4i..4i+3).
template <int N>
__device__ __forceinline__ unsigned long long load_word(const uint8_t *__restrict__ P, int k) {
    unsigned long long wd = 0;
    if (N == 16 && ((reinterpret_cast<uintptr_t>(P) & 15) == 0)) {
        const uint4 q = *reinterpret_cast<const uint4 *>(P + (size_t)k * 16);
        const uint32_t d[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) wd |= (unsigned long long)((d[i >> 2] >> (8 * (i & 3))) & 15u) << (4 * i);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) wd |= (unsigned long long)(P[(size_t)k * N + i] & 15) << (4 * i);
    }
    return wd;
}


// Workgroups are dispatched to the 8 XCDs of the chip in turn (workgroup b to
// XCD b mod 8), and every XCD has its own L2.  This bijection of [0, n) gives
// each XCD one contiguous range of indices, so that consecutive vectors --
// the symbols of one subcarrier, which read the same W, path table and path
// orders -- meet in one L2 instead of being fetched by up to eight.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n) {
    constexpr uint32_t kXcd = 8;
    const uint32_t per = n / kXcd, rem = n % kXcd;
    const uint32_t x = b % kXcd, i = b / kXcd;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

}  // namespace vp
