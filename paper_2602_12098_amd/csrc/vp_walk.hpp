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

// stilde_over_tau in two steps for kernels that stage the symbols in LDS:
// the W row i (all N loads issued up front, as above), then the sum over the
// permuted symbols x[pm[j]] with the same arithmetic in the same order, so
// the result has the same bits.
template <int N>
__device__ __forceinline__ void stilde_row(const float2 *__restrict__ Wc, int i, float2 (&w)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) w[j] = Wc[vp_pidx(N, i, j)];
}

template <int N>
__device__ __forceinline__ float2 stilde_staged(const float2 (&w)[N], const uint8_t *pm, const float2 *x_user, int i,
                                                float inv_tau) {
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int u = pm[j] < N ? pm[j] : N - 1;   // a corrupt permutation must not index out of bounds
        const float2 x = x_user[u];
        if (j <= i) {
            re = fmaf(w[j].x, x.x, fmaf(-w[j].y, x.y, re));
            im = fmaf(w[j].x, x.y, fmaf(w[j].y, x.x, im));
        }
    }
    return make_float2(re * inv_tau, im * inv_tau);
}

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

// How a walk picks its DEMAP variant at each level.
enum : int {
    kTierLut = 0,    // always the table (any rank): the re-walks that write l
    kTierAny = 1,    // the cheapest variant serving every lane of the wave, found by wave votes
    kTierTherm = 2   // from a wave-uniform thermometer word (rank_tiers below), no votes
};

// Per level i, bits 4i, 4i+1, 4i+2 of the result: the path's rank at that
// level is >= 1, >= 2, >= 3.  The OR of these words over a wave's paths
// tells, per level, the largest rank any lane needs there (capped at 3).
// Formed on the two 32-bit halves (eight levels each).
__device__ __forceinline__ uint32_t rank_tiers32(uint32_t w) {
    constexpr uint32_t M = 0x11111111u;
    const uint32_t w1 = w >> 1, w2 = w >> 2, w3 = w >> 3;
    const uint32_t ge1 = (w | w1 | w2 | w3) & M;
    const uint32_t ge2 = (w1 | w2 | w3) & M;
    const uint32_t ge3 = (w2 | w3 | (w & w1)) & M;
    return ge1 | (ge2 << 1) | (ge3 << 2);
}

__device__ __forceinline__ unsigned long long rank_tiers(unsigned long long w) {
    return ((unsigned long long)rank_tiers32((uint32_t)(w >> 32)) << 32) | rank_tiers32((uint32_t)w);
}

// OR over each half (32 lanes) of a wave by DPP moves; lanes 31 and 63 end
// with the OR of their half (the other lanes with partial results).
__device__ __forceinline__ uint32_t half_wave_or(uint32_t x) {
    const int v = (int)x;
    int r = v;
    r |= __builtin_amdgcn_update_dpp(0, r, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
    r |= __builtin_amdgcn_update_dpp(0, r, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
    r |= __builtin_amdgcn_update_dpp(0, r, 0x141, 0xF, 0xF, false);   // row_half_mirror
    r |= __builtin_amdgcn_update_dpp(0, r, 0x140, 0xF, 0xF, false);   // row_mirror
    r |= __builtin_amdgcn_update_dpp(0, r, 0x142, 0xA, 0xF, false);   // row_bcast:15 into rows 1, 3
    return (uint32_t)r;
}

// OR over the 64 lanes of a wave, returned wave-uniform (in scalar registers).
__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    lo = wave_reduce(lo, 0u, [](uint32_t p, uint32_t q) { return p | q; });
    hi = wave_reduce(hi, 0u, [](uint32_t p, uint32_t q) { return p | q; });
    return ((unsigned long long)__builtin_amdgcn_readfirstlane(hi) << 32) | __builtin_amdgcn_readfirstlane(lo);
}

// Walk one path over levels [LO, HI).  r: residuals / tau (in: their values
// after level LO-1, destroyed), nlinv_i = -1 / W_ii, wdiag_i = W_ii, ped: the
// PED so far.  Returns ped + sum_{LO<=i<HI} |r_i + W_ii l_i|^2; with REC the
// chosen offsets.  The level centre c_i = -r_i / W_ii enters DEMAP as
// cp = c - 1/2, one fused multiply-add, and (above rank 0) as c.  A walk split
// into consecutive ranges performs exactly the arithmetic of the whole walk,
// and every tier mode gives the same bits.
// RLUT: the children of rank >= 1 come from the paper's region table
// (vp_demap_region) instead of the exact order; rank 0 is the same in both.
template <int N, int TIERS, bool REC, int LO = 0, int HI = N, bool RLUT = false>
__device__ __forceinline__ float walk(const float2 *__restrict__ W0, const float *nlinv, const float *wdiag,
                                      float2 (&r)[N], unsigned long long word, unsigned long long therm,
                                      const uint8_t *lut, float *ra, float *rb, float ped = 0.f) {
    constexpr int CH = 4;   // W rows per scalar load (8 dwords)
#pragma unroll
    for (int i = LO; i < HI; ++i) {
        const float nl = nlinv[i];
        const float cpx = fmaf(r[i].x, nl, -0.5f);
        const float cpy = fmaf(r[i].y, nl, -0.5f);
        float a, b;
        if (TIERS == kTierTherm) {
            const uint32_t th = (uint32_t)(therm >> (4 * i)) & 7u;   // wave-uniform
            if (th == 0u) {
                vp_demap0(cpx, cpy, a, b);
            } else {
                const int rank = (int)((word >> (4 * i)) & 15ull);
                const float cx = r[i].x * nl, cy = r[i].y * nl;
                if (RLUT) vp_demap_region(cpx, cpy, cx, cy, rank, VP_REGION_LUT, a, b);
                else if (th == 1u) vp_demap1(cpx, cpy, cx, cy, rank, a, b);
                else if (th == 3u) vp_demap2(cpx, cpy, cx, cy, rank, a, b);
                else vp_demapN(cpx, cpy, cx, cy, rank, lut, a, b);
            }
        } else if (TIERS == kTierAny) {
            const int rank = (int)((word >> (4 * i)) & 15ull);
            if (!__any(rank != 0)) {
                vp_demap0(cpx, cpy, a, b);
            } else {
                const float cx = r[i].x * nl, cy = r[i].y * nl;
                if (RLUT) vp_demap_region(cpx, cpy, cx, cy, rank, VP_REGION_LUT, a, b);
                else if (!__any(rank > 1)) vp_demap1(cpx, cpy, cx, cy, rank, a, b);
                else if (!__any(rank > 2)) vp_demap2(cpx, cpy, cx, cy, rank, a, b);
                else vp_demapN(cpx, cpy, cx, cy, rank, lut, a, b);
            }
        } else {
            const int rank = (int)((word >> (4 * i)) & 15ull);
            if (RLUT) vp_demap_region(cpx, cpy, r[i].x * nl, r[i].y * nl, rank, VP_REGION_LUT, a, b);
            else vp_demapN(cpx, cpy, r[i].x * nl, r[i].y * nl, rank, lut, a, b);
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
            if (TIERS != kTierLut) {
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

// Rank nibbles of path k (level i at bits 4i..4i+3): each byte's low nibble.
// For N = 16 the row is one 16-byte load; per dword the two ranks of each
// byte pair are merged into one byte (t | t >> 4), and a byte permute
// gathers bytes 0 and 2 of two such dwords into one dword.
template <int N>
__device__ __forceinline__ unsigned long long load_word(const uint8_t *__restrict__ P, int k) {
    unsigned long long wd = 0;
    if (N == 16 && ((reinterpret_cast<uintptr_t>(P) & 15) == 0)) {
        const uint4 q = *reinterpret_cast<const uint4 *>(P + (size_t)k * 16);
        auto merge = [](uint32_t x) {
            const uint32_t t = x & 0x0F0F0F0Fu;
            return t | (t >> 4);   // byte 0: ranks 0 | 1 << 4, byte 2: ranks 2 | 3 << 4
        };
        const uint32_t lo = __builtin_amdgcn_perm(merge(q.y), merge(q.x), 0x06040200u);
        const uint32_t hi = __builtin_amdgcn_perm(merge(q.w), merge(q.z), 0x06040200u);
        wd = ((unsigned long long)hi << 32) | lo;
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
