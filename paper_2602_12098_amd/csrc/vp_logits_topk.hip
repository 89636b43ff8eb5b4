// The proposal network's last layer fused with its top-64 and softmax mass:
// z = X Wt^T + bias over the whole vocabulary, reduced to the 64 largest
// entries per row (value descending, column ascending, IEEE total order) and
// sum_sel exp(z - max) / sum_all exp(z - max), without writing z to memory.
//
// A bound below each row's 64th largest logit is known only once the row is
// complete, so the logits are computed twice:
//   pass 1  the vocabulary is split four ways by 32-row blocks (split q takes
//           blocks b with b % 4 == q) and, inside a split, into 32 groups by
//           the row within the block: 128 disjoint groups per row.  Every
//           group's two largest logits are kept (256 distinct entries) and
//           stored as 16-bit truncated order keys.
//   bound   per row, the value of the 64th largest of those 256 keys: a
//           truncated key is never above its value's key, so at least 64
//           logits are at or above it and no logit below it is among the 64
//           largest.  Also the row's maximum (at the top of its truncation
//           interval).
//   pass 2  the logits again: sum of exp(z - max) per split, and every logit
//           at or above the bound (or NaN) appended to the split's candidate
//           list (about 65 per row on trained and on random logits).
//   select  the candidates ranked exactly against each other.  A row with
//           more candidates than its lists hold is queued for
//   exact   one wave recomputes that row's logits with the same matrix-core
//           instruction sequence (so bit-identical values) and ranks all of
//           them.
//
// Matrix cores: v_mfma_f32_32x32x16_bf16 with a 32-row vocabulary block as A
// and 32 rows of X as B: lane l then holds, for row l % 32 of X, the logits of
// vocabulary rows 8 (r / 4) + 4 (l / 32) + r % 4 of the block (r < 16), the
// k-steps summed in increasing order as the unfused GEMM does.  A wave keeps
// the B fragments of its 64 rows of X (two 32-column tiles, k = 256) in
// registers for the whole pass; the four waves of a workgroup share each
// 32 x 256 vocabulary block through a ring of four LDS slots, and each
// matrix-core instruction runs beside one value of the previous block's
// epilogue.
#include <math.h>
#include "vp_internal.hpp"
#include "vp_learn.h"

namespace vp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kLT = 256;         // threads per pass workgroup
constexpr int kKD = 256;         // inner dimension (hidden width)
constexpr int kLDK = kKD + 8;    // padded LDS row of a vocabulary block (bf16)
constexpr int kNQ = 4;           // vocabulary splits
constexpr int kCQ = 64;          // candidate list length per (row, split)
constexpr int kMaxCand = 128;    // candidates per row the selection ranks directly
constexpr int kRowsWG = 256;     // rows of X per pass workgroup (4 waves x 64)
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ uint32_t okey(float f) {   // increasing in the IEEE total order
    const uint32_t u = __float_as_uint(f);
    return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}
__device__ __forceinline__ float key_value(uint32_t k) {   // inverse of okey
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__device__ __forceinline__ int ballot_count(bool p) { return __popcll(__ballot(p)); }
__device__ __forceinline__ uint32_t wave_sum_u(uint32_t x) {
    return wave_reduce(x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

// Per-value work on the 2 x 16 logits a lane holds (block m of split q):
// pass 1 updates the groups' two largest; pass 2 sums exp(z - max) and marks
// the candidates (branch-free, so that it interleaves with the matrix-core
// instructions of the next block), then appends them.
template <int MODE>
struct PassState {
    float m1[2][16], m2[2][16];   // pass 1: the two largest of each group
    float T[2], off[2], esum[2];  // pass 2: bound, -max * log2(e), sum of exp
    bool valid[2];
};

template <int MODE>
__device__ __forceinline__ void epi_one(PassState<MODE> &st, const f32x16 (&acc)[2], const float (&bb)[16],
                                        uint32_t (&cm)[2], int u, int r) {
    if (MODE == 0) {
        // NaN counts as -inf here (it is always a candidate in pass 2)
        const float z = fmaxf(acc[u][r] + bb[r], -INFINITY);
        st.m2[u][r] = __builtin_amdgcn_fmed3f(st.m1[u][r], st.m2[u][r], z);
        st.m1[u][r] = fmaxf(st.m1[u][r], z);
        // an empty asm keeps the result where it is computed, so the pure
        // arithmetic is not moved away from the matrix-core instruction it
        // is meant to run beside
        asm volatile("" : "+v"(st.m1[u][r]), "+v"(st.m2[u][r]));
    } else if (MODE == 1) {
        const float z = acc[u][r] + bb[r];
        st.esum[u] += __builtin_amdgcn_exp2f(fmaf(z, kLog2e, st.off[u]));
        cm[u] |= (!(z < st.T[u]) ? 1u : 0u) << r;
        asm volatile("" : "+v"(st.esum[u]), "+v"(cm[u]));
    } else {   // pass 2 without the softmax mass: the candidates only
        const float z = acc[u][r] + bb[r];
        cm[u] |= (!(z < st.T[u]) ? 1u : 0u) << r;
        asm volatile("" : "+v"(cm[u]));
    }
}

// Appends the marked logits of block m to the row's list for split q.  A lane
// with candidates stages its 16 logits of the tile in LDS and loops over its
// set bits only (candidates are about 2 % of the logits).
template <int MODE>
__device__ __forceinline__ void epi_append(const PassState<MODE> &st, const f32x16 (&acc)[2], const float (&bb)[16],
                                           const uint32_t (&cm)[2], int m, int q, int h, int rbase, int j, int wv,
                                           int *s_cnt, float *zst, uint2 *__restrict__ cand) {
    const int c0 = 32 * (q + kNQ * m) + 4 * h;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (cm[u] && st.valid[u]) {
#pragma unroll
            for (int r = 0; r < 16; r += 4)
                *reinterpret_cast<float4 *>(&zst[r]) = make_float4(acc[u][r] + bb[r], acc[u][r + 1] + bb[r + 1],
                                                                   acc[u][r + 2] + bb[r + 2], acc[u][r + 3] + bb[r + 3]);
            const int row = rbase + 32 * u + j;
            int p = atomicAdd(&s_cnt[wv * 64 + 32 * u + j], __popc(cm[u]));
            uint2 *dst = cand + ((size_t)row * kNQ + q) * kCQ;
            for (uint32_t bits = cm[u]; bits; bits &= bits - 1u, ++p) {
                const int r = __builtin_ctz(bits);
                if (p < kCQ) dst[p] = make_uint2(~(uint32_t)(c0 + 8 * (r >> 2) + (r & 3)), okey(zst[r]));
            }
        }
    }
}

constexpr int kSlots = 4;   // LDS ring of vocabulary blocks: m, m + 1, m + 2 (m + 3 in registers)

struct PassLds {
    uint16_t w[kSlots][32][kLDK];   // vocabulary blocks
    float b[kSlots][32];            // their bias
    int cnt[kRowsWG];               // pass 2: candidates per row of the workgroup
    float zst[kLT][20];             // pass 2: a lane's 16 logits while it appends (padded row)
};

// A block of the split on its way from memory to LDS: thread t carries
// vocabulary row t / 8, elements 32 (t % 8) .. + 31, and lanes < 32 the bias
// of row t.
struct BlockRegs {
    uint4 x0, x1, x2, x3;
    float b;
};

__device__ __forceinline__ void load_block(BlockRegs &p, const uint16_t *__restrict__ Wt,
                                           const float *__restrict__ bias, int q, int mb, int t) {
    const uint4 *src = reinterpret_cast<const uint4 *>(Wt + (size_t)(32 * (q + kNQ * mb) + (t >> 3)) * kKD + (t & 7) * 32);
    p.x0 = src[0];
    p.x1 = src[1];
    p.x2 = src[2];
    p.x3 = src[3];
    p.b = bias[32 * (q + kNQ * mb) + (t & 31)];   // every lane loads (no branch); lanes < 32 store
}

// LDS position (in 16-byte units of the row) of the row's 16-byte piece u:
// inside each 64-byte chunk c the four pieces are rotated by (c / 2) % 4, so
// that the eight threads that stage one row (chunks 0..7) write eight
// different bank groups, while a fragment read (every lane the same piece of
// its own row, rows 528 bytes apart) stays conflict-free.
__device__ __forceinline__ int lds_unit(int u) { return (u & ~3) | (((u >> 3) + u) & 3); }

__device__ __forceinline__ void store_block(PassLds &L, const BlockRegs &p, int mb, int t) {
    const int slot = mb % kSlots;
    uint16_t *row = &L.w[slot][t >> 3][0];
    const int u0 = (t & 7) * 4;   // the thread's pieces u0 .. u0 + 3
    *reinterpret_cast<uint4 *>(row + 8 * lds_unit(u0)) = p.x0;
    *reinterpret_cast<uint4 *>(row + 8 * lds_unit(u0 + 1)) = p.x1;
    *reinterpret_cast<uint4 *>(row + 8 * lds_unit(u0 + 2)) = p.x2;
    *reinterpret_cast<uint4 *>(row + 8 * lds_unit(u0 + 3)) = p.x3;
    if (t < 32) L.b[slot][t] = p.b;
}

__device__ __forceinline__ void read_bias(const PassLds &L, int slot, int h, float (&bb)[16]) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float4 b4 = *reinterpret_cast<const float4 *>(&L.b[slot][8 * g + 4 * h]);
        bb[4 * g] = b4.x;
        bb[4 * g + 1] = b4.y;
        bb[4 * g + 2] = b4.z;
        bb[4 * g + 3] = b4.w;
    }
}

// One block step.  On entry fa holds the A fragments of block m (k = 16 s +
// 8 h .. + 7 of vocabulary row j) and `stage` block m + 2; the 32
// matrix-core instructions of block m each run beside one value of the
// epilogue of block m - 1 (its logits in acc_prev; for m = 0 a neutral -inf
// block), and after k-step s the fragment s of block m + 1 (in LDS) replaces
// fa[s].  Block m + 3 is read from memory into `fetch` meanwhile; block m + 2
// is staged into LDS at the end.
template <int MODE>
__device__ __forceinline__ void pass_block(int m, int nb, int q, int t, int h, int j, int wv, int rbase,
                                           const uint16_t *__restrict__ Wt, const float *__restrict__ bias,
                                           PassLds &L, const uint4 (&fb)[2][16], bf16x8 (&fa)[16],
                                           f32x16 (&acc)[2], float (&bb_next)[16], const f32x16 (&acc_prev)[2],
                                           const float (&bb_prev)[16], const BlockRegs &stage, BlockRegs &fetch,
                                           PassState<MODE> &st, uint2 *__restrict__ cand) {
    load_block(fetch, Wt, bias, q, m + 3 < nb ? m + 3 : nb - 1, t);   // past the end: in range, never staged
    const int nslot = (m + 1 < nb ? m + 1 : m) % kSlots;
    const uint16_t *nrow = &L.w[nslot][j][0];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[u][r] = 0.f;
    uint32_t cm[2] = {0u, 0u};
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], as_bf16x8(fb[0][s]), acc[0], 0, 0, 0);
        epi_one<MODE>(st, acc_prev, bb_prev, cm, s >> 3, 2 * (s & 7));
        __builtin_amdgcn_sched_barrier(0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], as_bf16x8(fb[1][s]), acc[1], 0, 0, 0);
        fa[s] = *reinterpret_cast<const bf16x8 *>(nrow + 8 * lds_unit(2 * s + h));
        epi_one<MODE>(st, acc_prev, bb_prev, cm, s >> 3, 2 * (s & 7) + 1);
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (MODE >= 1) {
        if (m > 0) epi_append(st, acc_prev, bb_prev, cm, m - 1, q, h, rbase, j, wv, L.cnt, L.zst[t], cand);
    }
    read_bias(L, nslot, h, bb_next);   // after the last use of bb_prev: the two may be one array
    if (m + 2 < nb) store_block(L, stage, m + 2, t);
    __syncthreads();
}

template <int MODE>
__device__ __forceinline__ void pass_last(PassState<MODE> &st, const f32x16 (&acc)[2], const float (&bb)[16], int m,
                                          int q, int h, int rbase, int j, int wv, PassLds &L, int t,
                                          uint2 *__restrict__ cand) {
    uint32_t cm[2] = {0u, 0u};
#pragma unroll
    for (int i = 0; i < 32; ++i) epi_one<MODE>(st, acc, bb, cm, i >> 4, i & 15);
    if constexpr (MODE >= 1) epi_append(st, acc, bb, cm, m, q, h, rbase, j, wv, L.cnt, L.zst[t], cand);
}

// Pass 1 (MODE 0) and pass 2 (MODE 1, or 2 without the softmax mass's sums).
// One workgroup per (256 rows, split);
// a one-dimensional grid ordered so that the four splits of a row group are
// consecutive workgroups of one XCD (workgroup i runs on XCD i % 8), which
// then read its rows of X through one L2.
template <int MODE>
__global__ __launch_bounds__(kLT) void k_lt_pass(const uint16_t *__restrict__ X, int rows,
                                                 const uint16_t *__restrict__ Wt, const float *__restrict__ bias,
                                                 int V, uint16_t *__restrict__ stats, const float2 *__restrict__ thr,
                                                 uint2 *__restrict__ cand, int32_t *__restrict__ cnt,
                                                 float *__restrict__ qsum) {
    __shared__ __attribute__((aligned(16))) PassLds L;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, h = lane >> 5, j = lane & 31;
    const int xcd = blockIdx.x % 8, k = blockIdx.x / 8;
    const int rg = xcd + 8 * (k / kNQ), q = k % kNQ;
    if (rg * kRowsWG >= rows) return;
    const int nb = V / (32 * kNQ);   // at least 2
    const int rbase = rg * kRowsWG + wv * 64;   // tile u of the wave: rows rbase + 32 u + j

    uint4 fb[2][16];   // B fragments: row rbase + 32 u + j, k = 16 s + 8 h .. + 7
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int row = rbase + 32 * u + j;
#pragma unroll
        for (int s = 0; s < 16; ++s)
            fb[u][s] = row < rows ? *reinterpret_cast<const uint4 *>(X + (size_t)row * kKD + 16 * s + 8 * h)
                                  : make_uint4(0, 0, 0, 0);
    }
    PassState<MODE> st;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int row = rbase + 32 * u + j;
        st.valid[u] = row < rows;
        if (MODE == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) st.m1[u][r] = st.m2[u][r] = -INFINITY;
        } else {
            const float2 tm = st.valid[u] ? thr[row] : make_float2(INFINITY, 0.f);
            st.T[u] = tm.x;
            st.off[u] = -tm.y * kLog2e;
            st.esum[u] = 0.f;
        }
    }
    if (MODE >= 1) L.cnt[t] = 0;
    BlockRegs pE, pO;
    load_block(pE, Wt, bias, q, 0, t);
    store_block(L, pE, 0, t);
    load_block(pO, Wt, bias, q, 1, t);
    store_block(L, pO, 1, t);
    load_block(pE, Wt, bias, q, nb > 2 ? 2 : 1, t);   // block 2, staged by step 0
    __syncthreads();
    bf16x8 fa[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) fa[s] = *reinterpret_cast<const bf16x8 *>(&L.w[0][j][8 * lds_unit(2 * s + h)]);
    f32x16 accE[2], accO[2];   // logits of the even / odd blocks
    float bbE[16], bbO[16];
    read_bias(L, 0, h, bbE);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 16; ++r) accO[u][r] = -INFINITY;   // block -1: leaves every statistic as it is
#pragma unroll
    for (int r = 0; r < 16; ++r) bbO[r] = 0.f;
    // even steps stage pE and fetch into pO, odd steps the reverse
    int m = 0;
    for (; m + 1 < nb; m += 2) {
        pass_block<MODE>(m, nb, q, t, h, j, wv, rbase, Wt, bias, L, fb, fa, accE, bbO, accO, bbO, pE, pO, st, cand);
        pass_block<MODE>(m + 1, nb, q, t, h, j, wv, rbase, Wt, bias, L, fb, fa, accO, bbE, accE, bbE, pO, pE, st,
                         cand);
    }
    if (m < nb) {
        pass_block<MODE>(m, nb, q, t, h, j, wv, rbase, Wt, bias, L, fb, fa, accE, bbO, accO, bbO, pE, pO, st, cand);
        pass_last<MODE>(st, accE, bbE, nb - 1, q, h, rbase, j, wv, L, t, cand);
    } else {
        pass_last<MODE>(st, accO, bbO, nb - 1, q, h, rbase, j, wv, L, t, cand);
    }
    if (MODE >= 1) __syncthreads();   // every append of the workgroup is counted
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int row = rbase + 32 * u + j;
        if (MODE == 0) {
            // the groups' two largest as 16-bit order keys, truncated (never
            // above the value's own key, so a bound taken from them stays a
            // valid one)
            if (st.valid[u]) {
                uint32_t w[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) w[r] = (okey(st.m1[u][r]) >> 16) | (okey(st.m2[u][r]) & 0xffff0000u);
                uint4 *dst = reinterpret_cast<uint4 *>(stats + ((size_t)row * kNQ + q) * 64 + 32 * h);
#pragma unroll
                for (int i = 0; i < 4; ++i) dst[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
            }
        } else {
            const float e = MODE == 1 ? st.esum[u] + __shfl_xor(st.esum[u], 32) : 0.f;
            if (st.valid[u] && h == 0) {
                if (MODE == 1) qsum[(size_t)row * kNQ + q] = e;
                cnt[(size_t)row * kNQ + q] = L.cnt[wv * 64 + 32 * u + j];
            }
        }
    }
}

// Bound and maximum per row from the 256 truncated keys; one wave per row,
// four rows per workgroup.  Also clears the count of queued rows for the
// selection.  The bound is the value of the 64th largest truncated key
// (every truncated key is at most its value's key, so at least 64 logits lie
// at or above it); the maximum is taken at the top of its truncation
// interval, so that it is at least the row's largest logit.
__global__ __launch_bounds__(256) void k_lt_bound(const uint16_t *__restrict__ stats, int rows,
                                                  float2 *__restrict__ thr, int32_t *__restrict__ n_exact) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_exact = 0;
    if (row >= rows) return;
    const uint2 v = reinterpret_cast<const uint2 *>(stats + (size_t)row * kNQ * 64)[lane];
    const uint32_t k0 = v.x & 0xffffu, k1 = v.x >> 16, k2 = v.y & 0xffffu, k3 = v.y >> 16;
    uint32_t T = 0;
    for (int b = 15; b >= 0; --b) {
        const uint32_t c = T | (1u << b);
        if (ballot_count(k0 >= c) + ballot_count(k1 >= c) + ballot_count(k2 >= c) + ballot_count(k3 >= c) >= 64) T = c;
    }
    uint32_t mk = max(max(k0, k1), max(k2, k3));
    mk = wave_reduce(mk, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
    const float mx = fminf(key_value((mk << 16) | 0xffffu), 3.402823466e38f);
    if (lane == 0) thr[row] = make_float2(key_value(T << 16), mx);
}

// Ranks the candidates of each row (one wave per row): a candidate's position
// is the number of candidates with a larger (key, ~column) pair.  Rows with a
// full list or more than 128 candidates go to the exact queue (as would a row
// with fewer than 64, which the bound rules out).
__global__ __launch_bounds__(64) void k_lt_select(int rows, const float2 *__restrict__ thr,
                                                  const uint2 *__restrict__ cand, const int32_t *__restrict__ cnt,
                                                  const float *__restrict__ qsum, int32_t *__restrict__ idx_out,
                                                  float *__restrict__ mass_out, int32_t *__restrict__ n_exact,
                                                  int32_t *__restrict__ queue) {
    __shared__ unsigned long long s_c[kMaxCand];
    const int row = blockIdx.x, lane = threadIdx.x;
    int n[kNQ], total = 0;
    bool full = false;
#pragma unroll
    for (int q = 0; q < kNQ; ++q) {
        n[q] = cnt[(size_t)row * kNQ + q];
        full |= n[q] > kCQ;
        total += n[q];
    }
    if (full || total > kMaxCand || total < 64) {
        if (lane == 0) queue[atomicAdd(n_exact, 1)] = row;
        return;
    }
    // candidate p of the row: split q, entry p - (n[0] + .. + n[q-1])
    unsigned long long c[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int p = lane + 64 * i;
        c[i] = 0ull;
        if (p < total) {
            int q = 0, o = p;
            while (o >= n[q]) {
                o -= n[q];
                ++q;
            }
            const uint2 e = cand[((size_t)row * kNQ + q) * kCQ + o];
            c[i] = ((unsigned long long)e.y << 32) | e.x;
            s_c[p] = c[i];
        }
    }
    __syncthreads();
    uint32_t r0 = 0, r1 = 0;
    for (int p = 0; p < total; ++p) {
        const unsigned long long v = s_c[p];
        r0 += v > c[0] ? 1u : 0u;
        r1 += v > c[1] ? 1u : 0u;
    }
    const float mx = thr[row].y, off = -mx * kLog2e;
    float e = 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int p = lane + 64 * i;
        const uint32_t r = i ? r1 : r0;
        if (p < total && r < 64u) {
            idx_out[(size_t)row * 64 + r] = (int32_t)~(uint32_t)c[i];
            e += __builtin_amdgcn_exp2f(fmaf(key_value((uint32_t)(c[i] >> 32)), kLog2e, off));
        }
    }
    if (mass_out) {
        e = wave_sum_f(e);
        float all = 0.f;
#pragma unroll
        for (int q = 0; q < kNQ; ++q) all += qsum[(size_t)row * kNQ + q];
        if (lane == 0) mass_out[row] = all > 0.f ? e / all : 0.f;
    }
}

// The queued rows, one wave each (a grid-stride loop over the queue): all V
// logits of the row with the pass kernels' instruction sequence (the row in
// column 0 of a 32-column tile), kept in LDS, then ranked exactly: the 64th
// largest key by a bitwise search, the keys above it and the equal keys of
// smallest column, ordered by counting.
__global__ __launch_bounds__(64) void k_lt_exact(const uint16_t *__restrict__ X, const uint16_t *__restrict__ Wt,
                                                 const float *__restrict__ bias, int V,
                                                 const float2 *__restrict__ thr,
                                                 const int32_t *__restrict__ n_exact,
                                                 const int32_t *__restrict__ queue, int32_t *__restrict__ idx_out,
                                                 float *__restrict__ mass_out) {
    __shared__ uint32_t s_k[VP_MAX_VOCAB];
    __shared__ unsigned long long s_sel[64];
    const int lane = threadIdx.x, h = lane >> 5, j = lane & 31;
    const int nq = *n_exact;
    for (int qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const int row = queue[qi];
        uint4 fb[16];
#pragma unroll
        for (int s = 0; s < 16; ++s)
            fb[s] = j == 0 ? *reinterpret_cast<const uint4 *>(X + (size_t)row * kKD + 16 * s + 8 * h)
                           : make_uint4(0, 0, 0, 0);
        for (int b = 0; b < V / 32; ++b) {
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const uint4 a = *reinterpret_cast<const uint4 *>(Wt + (size_t)(32 * b + j) * kKD + 16 * s + 8 * h);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a), as_bf16x8(fb[s]), acc, 0, 0, 0);
            }
            if (j == 0) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int c = 32 * b + 8 * (r >> 2) + 4 * h + (r & 3);
                    s_k[c] = okey(acc[r] + bias[c]);
                }
            }
        }
        __syncthreads();
        // the exact 64th largest key
        uint32_t T = 0;
        for (int bt = 31; bt >= 0; --bt) {
            const uint32_t c = T | (1u << bt);
            uint32_t k = 0;
            for (int i = lane; i < V; i += 64) k += s_k[i] >= c ? 1u : 0u;
            if (wave_sum_u(k) >= 64u) T = c;
        }
        // keys above T, then keys equal to T by increasing column
        uint32_t above = 0;
        for (int i = lane; i < V; i += 64) above += s_k[i] > T ? 1u : 0u;
        uint32_t incl = wave_scan_incl(above);
        uint32_t pos = incl - above;
        const uint32_t n_above = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        for (int i = lane; i < V; i += 64)
            if (s_k[i] > T) s_sel[pos++] = ((unsigned long long)s_k[i] << 32) | ~(uint32_t)i;
        uint32_t run = n_above;
        for (int i0 = 0; i0 < V && run < 64u; i0 += 64) {
            const int i = i0 + lane;
            const bool eq = i < V && s_k[i] == T;
            const uint32_t p = run + (uint32_t)__popcll(__ballot(eq) & ((1ull << lane) - 1ull));
            if (eq && p < 64u) s_sel[p] = ((unsigned long long)T << 32) | ~(uint32_t)i;
            run += (uint32_t)ballot_count(eq);
        }
        __syncthreads();
        const unsigned long long a = s_sel[lane];
        uint32_t r = 0;
        for (int p = 0; p < 64; ++p) r += s_sel[p] > a ? 1u : 0u;
        idx_out[(size_t)row * 64 + r] = (int32_t)~(uint32_t)a;
        if (mass_out) {
            const float off = -thr[row].y * kLog2e;
            float all = 0.f;
            for (int i = lane; i < V; i += 64) all += __builtin_amdgcn_exp2f(fmaf(key_value(s_k[i]), kLog2e, off));
            all = wave_sum_f(all);
            const float e = wave_sum_f(__builtin_amdgcn_exp2f(fmaf(key_value((uint32_t)(a >> 32)), kLog2e, off)));
            if (lane == 0) mass_out[row] = all > 0.f ? e / all : 0.f;
        }
        __syncthreads();
    }
}

}  // namespace

size_t logits_top64_work_bytes(int rows) {
    const size_t r = (size_t)(rows > 0 ? rows : 0);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return al(r * kNQ * kCQ * sizeof(uint2)) + al(r * sizeof(float2)) + al(r * kNQ * sizeof(int32_t)) +
           al(r * kNQ * sizeof(float)) + al(r * sizeof(int32_t)) + 256;
}

int launch_logits_top64(const uint16_t *X, int rows, const uint16_t *Wt, const float *bias, int V, int32_t *idx,
                        float *mass, void *work, hipStream_t st) {
    if (rows == 0) return VP_OK;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t r = (size_t)rows;
    char *w = static_cast<char *>(work);
    // the candidate lists reuse the pass-1 statistics' memory (read by the
    // bound kernel before pass 2 starts)
    uint2 *cand = reinterpret_cast<uint2 *>(w);
    uint16_t *stats = reinterpret_cast<uint16_t *>(w);
    w += al(r * kNQ * kCQ * sizeof(uint2));
    float2 *thr = reinterpret_cast<float2 *>(w);
    w += al(r * sizeof(float2));
    int32_t *cnt = reinterpret_cast<int32_t *>(w);
    w += al(r * kNQ * sizeof(int32_t));
    float *qsum = reinterpret_cast<float *>(w);
    w += al(r * kNQ * sizeof(float));
    int32_t *queue = reinterpret_cast<int32_t *>(w);
    w += al(r * sizeof(int32_t));
    int32_t *n_exact = reinterpret_cast<int32_t *>(w);
    const int n_rg = (rows + kRowsWG - 1) / kRowsWG;
    const dim3 grid((unsigned)(8 * ((n_rg + 7) / 8) * kNQ));   // workgroups beyond the rows exit at once
    hipLaunchKernelGGL(k_lt_pass<0>, grid, dim3(kLT), 0, st, X, rows, Wt, bias, V, stats, nullptr, nullptr, nullptr,
                       nullptr);
    hipLaunchKernelGGL(k_lt_bound, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, stats, rows, thr, n_exact);
    if (mass)
        hipLaunchKernelGGL(k_lt_pass<1>, grid, dim3(kLT), 0, st, X, rows, Wt, bias, V, nullptr, thr, cand, cnt, qsum);
    else   // no softmax mass asked for: pass 2 leaves out the sums of exp
        hipLaunchKernelGGL(k_lt_pass<2>, grid, dim3(kLT), 0, st, X, rows, Wt, bias, V, nullptr, thr, cand, cnt,
                           nullptr);
    hipLaunchKernelGGL(k_lt_select, dim3((unsigned)rows), dim3(64), 0, st, rows, thr, cand, cnt, qsum, idx, mass,
                       n_exact, queue);
    hipLaunchKernelGGL(k_lt_exact, dim3(256), dim3(64), 0, st, X, Wt, bias, V, thr, n_exact, queue, idx, mass);
    return launch_status();
}

}  // namespace vp
