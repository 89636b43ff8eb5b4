// Per-vector path search and argmin (Sec. II-B PED recursion, Sec. III-A-2
// level centres and DEMAP, Alg. 2 parallel post-processing over K paths).
//
// k_search: one 256-thread workgroup per vector, one path per lane.  The
// subcarrier's W column entries are wave-uniform (scalar loads), the
// per-vector start residual s-tilde / tau is computed once and broadcast
// through LDS, and each lane reads its path's ranks as one 16-byte load.
// Down the tree each lane keeps its residuals r_m = (s-tilde_m + tau
// sum_{j<i} W_mj l_j) / tau in registers, so a level costs one DEMAP and a
// rank-1 update of the residuals below it (4 FMAs per entry: l is a
// Gaussian integer in the box).  The DEMAP work is picked per wave and
// level from the largest rank the wave needs there (rank 0 is plain
// rounding).  The cost of each path is ||W (s_pi + tau l)||^2 =
// tau^2 sum_i |r_i + W_ii l_i|^2; the argmin over paths packs
// (cost bits, k) into one 64-bit key and reduces it across the wave and the
// workgroup.
//
// k_search_finalize re-walks the winning path of each vector with the very
// same arithmetic to materialise l in user order.
#include <mutex>

#include "vp_walk.hpp"

namespace vp {
namespace {

constexpr int kT = 256;

// The vectors a search serves: all of them (mass == nullptr), or those whose
// proposal mass is not at least theta (a NaN mass counts as not confident).
// Kernels take it with a compile-time MASKED flag, so that the plain search
// carries no trace of it.
struct VecMask {
    const float *mass;
    float theta;
    __device__ __forceinline__ bool on(size_t v) const { return !mass || !(mass[v] >= theta); }
};

template <int N, bool MASKED, bool RLUT>
__global__ __launch_bounds__(kT) void k_search(const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                               const float2 *__restrict__ s, const float *__restrict__ taus,
                                               const uint8_t *__restrict__ paths, int K, long long pstride,
                                               int n_sym, unsigned flags, float *__restrict__ cost_out,
                                               int32_t *__restrict__ kidx_out, VecMask mask) {
    __shared__ float2 s_r0[N];
    __shared__ float s_nlinv[N];
    __shared__ float s_wdiag[N];
    __shared__ uint8_t s_perm[N];
    __shared__ unsigned long long s_red[kT / 64];

    constexpr int NP = VP_PACKED(N);
    const size_t v = xcd_contiguous(blockIdx.x, gridDim.x);   // one vector per workgroup
    if (MASKED && !mask.on(v)) return;
    const int sc = (int)(v / n_sym);
    const int t = threadIdx.x;
    const size_t n_vec = (size_t)gridDim.x;
    const float2 *__restrict__ Wc = W + (size_t)sc * NP;
    const float w00 = Wc[0].x;
    const float tau = taus[sc];
    if (!(w00 > 0.f) || !isfinite(w00) || !(tau > 0.f) || !isfinite(tau)) {   // failed subcarrier: l = 0, cost = NaN
        if (t == 0) {
            cost_out[v] = __int_as_float(0x7fc00000);
            kidx_out[v] = -1;
        }
        return;
    }
    if (t < N) {
        s_wdiag[t] = Wc[vp_pidx(N, t, t)].x;
        s_nlinv[t] = -(1.0f / s_wdiag[t]);
        s_perm[t] = perm[(size_t)sc * N + t];
    }
    __syncthreads();
    if (t < N) s_r0[t] = stilde_over_tau<N>(Wc, s_perm, s, v, n_vec, t, 1.0f / tau);
    __syncthreads();

    const uint8_t *P = paths + ((flags & VP_PATHS_PER_VECTOR) ? v : (size_t)sc) * pstride;
    unsigned long long best = ~0ull;
    for (int k = t; k < K; k += kT) {
        const unsigned long long wd = load_word<N>(P, k);
        float2 r[N];
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = s_r0[i];
        const float ped = walk<N, kTierAny, false, 0, N, RLUT>(Wc, s_nlinv, s_wdiag, r, wd, 0ull, VP_DEMAP_LUT, nullptr, nullptr);
        best = umin64(best, ((unsigned long long)__float_as_uint(ped * (tau * tau)) << 32) | (unsigned)k);
    }
    if ((flags & VP_INCLUDE_ZERO) && t == 0) {
        float z = 0.f;
        for (int i = 0; i < N; ++i) {
            z = fmaf(s_r0[i].x, s_r0[i].x, z);
            z = fmaf(s_r0[i].y, s_r0[i].y, z);
        }
        best = umin64(best, ((unsigned long long)__float_as_uint(z * (tau * tau)) << 32) | (unsigned)K);
    }
    best = wave_min(best);
    if ((t & 63) == 0) s_red[t >> 6] = best;
    __syncthreads();
    if (t == 0) {
        unsigned long long b = s_red[0];
        for (int w = 1; w < kT / 64; ++w) b = umin64(b, s_red[w]);
        cost_out[v] = __uint_as_float((unsigned)(b >> 32));
        kidx_out[v] = (int32_t)(b & 0xffffffffull);
    }
}

// Prefix-sharing search (path orders from vp_paths_mop: lexicographic, and
// deepest level most significant).
// Stage 1: each distinct prefix of levels [0, P1) is walked once per vector,
// one lane per (vector, prefix), and its residuals below P1 and its PED are
// kept in LDS.  Stage 2: each path continues from its prefix's state over
// levels [P1, N), taken in deepest-level-first order so that the paths of a
// wave mostly need the same DEMAP work; the two vectors of the workgroup are
// interleaved over the lanes (lane 2j + h: vector h, path j of the order), so
// that a wave holds 32 paths, and each wave's DEMAP variant per level comes
// from a tier word of its 32 paths built once in the set-up (no votes in the
// walk).  A table with more than kMaxPrefix distinct prefixes is done in
// chunks of kMaxPrefix prefixes (their paths are contiguous in lexicographic
// order).  Every path sees exactly the arithmetic of a direct walk.
//
// Occupancy: the walk is a long chain of dependent VALU work, so it runs best
// with five waves per SIMD (at most 96 VGPRs, and at most a fifth of the
// CU's 160 KiB LDS per workgroup: 120 stage-1 states of two vectors and the
// K = 512 tables come to 31 KiB).
constexpr int kTT = 128;          // threads of the prefix-sharing search, per vector
constexpr int kMaxPrefix = 120;   // stage-1 prefixes held in LDS at a time
constexpr int kTrieWaves = 5;     // waves per SIMD the register budget is set for

template <int N>
constexpr int prefix_levels() { return N >= 4 ? N / 4 : 1; }

constexpr int kVPB = 2;                 // vectors of one subcarrier per workgroup (they share its table)
constexpr int kTB = kTT * kVPB;         // threads of the prefix-sharing search
constexpr int kBatch = 64 / kVPB;       // distinct paths per wave in stage 2
static_assert(kVPB == 2 && 2 * kMaxPrefix <= kTB, "stage 1 packs both vectors' prefixes over the workgroup");

// Bytes of dynamic LDS of k_search_trie for a table of K paths.
inline size_t trie_lds_bytes(int K) {
    const size_t nb = (size_t)(K + kBatch - 1) / kBatch;
    return (size_t)K * sizeof(unsigned long long) + nb * sizeof(unsigned long long) +
           (size_t)(3 * K + 1) * sizeof(uint16_t);
}

// Minimum over the lanes of one parity (lane & 1) of a wave: lane 0 ends with
// the minimum of the even lanes, lane 1 with that of the odd lanes.
__device__ __forceinline__ unsigned long long wave_min_by_parity(unsigned long long x) {
#pragma unroll
    for (int off = 32; off > 1; off >>= 1) x = umin64(x, __shfl_xor(x, off));
    return x;
}

template <int N, bool MASKED, bool RLUT>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(kTrieWaves))) void k_search_trie(
    const float2 *__restrict__ W, const uint8_t *__restrict__ perm, const float2 *__restrict__ s,
    const float *__restrict__ taus, const uint8_t *__restrict__ paths, const uint16_t *__restrict__ order, int K,
    long long pstride, int n_sym, size_t n_vec, unsigned flags, float *__restrict__ cost_out,
    int32_t *__restrict__ kidx_out, VecMask mask) {
    constexpr int P1 = prefix_levels<N>();
    constexpr int SW = 2 * (N - P1) + 1;   // stage-1 state: residuals of levels P1..N-1 and the PED
    const int NB = (K + kBatch - 1) / kBatch;
    extern __shared__ unsigned long long s_words[];                 // [K] rank nibbles of path k
    unsigned long long *s_therm = s_words + K;                      // [NB] tier words of stage-2 batches
    uint16_t *s_k = reinterpret_cast<uint16_t *>(s_therm + NB);     // [K] path index of lex position
    uint16_t *s_node = s_k + K;                                     // [K] stage-1 prefix of path k
    uint16_t *s_first = s_node + K;                                 // [K + 1] first lex position of a prefix
    __shared__ __align__(16) float s_state[kVPB][kMaxPrefix * SW];
    // the workgroup's symbol vectors in user order [kVPB][N], read once after
    // the first barrier, in the stage-1 state area (first written after two
    // more barriers)
    float2 *s_x = reinterpret_cast<float2 *>(&s_state[0][0]);
    __shared__ float2 s_r0[kVPB][N];
    __shared__ float s_nlinv[N];
    __shared__ float s_wdiag[N];
    __shared__ uint8_t s_perm[N];
    __shared__ uint32_t s_scan[kTB / 64];
    __shared__ unsigned long long s_red[kTB / 64][kVPB];

    constexpr int NP = VP_PACKED(N);
    const int slots = (n_sym + kVPB - 1) / kVPB;
    const uint32_t blk = xcd_contiguous(blockIdx.x, gridDim.x);
    const int sc = (int)(blk / slots);
    const int t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    // the workgroup's vectors: symbols 2 j and 2 j + 1 of its subcarrier
    // (j = blk mod slots); in a masked search of up to 64 symbols per
    // subcarrier, the j-th pair of the subcarrier's served symbols instead, so
    // that served vectors are not left paired with skipped ones (a workgroup
    // left without a pair returns at once)
    const int j_pair = (int)(blk % slots);
    int sym0 = j_pair * kVPB, sym1 = sym0 + 1;
    int nlive = min(kVPB, n_sym - sym0);   // live vectors of this workgroup
    bool on0 = true, on1 = nlive > 1;      // the live vectors it serves (the same in every thread)
    if (MASKED) {
        if (n_sym <= 64) {
            const int lane = t & 63;
            const bool f = lane < n_sym && mask.on((size_t)sc * n_sym + lane);
            unsigned long long bal = __ballot(f);   // every wave forms the same word
            const int nf = __popcll(bal);
            if (kVPB * j_pair >= nf) return;
            nlive = min(kVPB, nf - kVPB * j_pair);
            for (int q = 0; q < kVPB * j_pair; ++q) bal &= bal - 1ull;   // drop the pairs before this one
            sym0 = __builtin_ctzll(bal);
            bal &= bal - 1ull;
            sym1 = nlive > 1 ? __builtin_ctzll(bal) : sym0;
            on1 = nlive > 1;
        } else {
            on0 = mask.on((size_t)sc * n_sym + sym0);
            on1 = nlive > 1 && mask.on((size_t)sc * n_sym + sym1);
            if (!on0 && !on1) return;
        }
    }
    const size_t vsel0 = (size_t)sc * n_sym + sym0, vsel1 = (size_t)sc * n_sym + (nlive > 1 ? sym1 : sym0);
    auto vsel = [&](int h) { return h == 0 ? vsel0 : vsel1; };   // a select, not an indexed array
    const float2 *__restrict__ Wc = W + (size_t)sc * NP;
    const float w00 = Wc[0].x;
    const float tau = taus[sc];
    if (!(w00 > 0.f) || !isfinite(w00) || !(tau > 0.f) || !isfinite(tau)) {   // failed subcarrier (all its vectors)
        if (t < nlive && (t == 0 ? on0 : on1)) {
            cost_out[vsel(t)] = __int_as_float(0x7fc00000);
            kidx_out[vsel(t)] = -1;
        }
        return;
    }
    const uint8_t *P = paths + (size_t)sc * pstride;
    const uint16_t *LX = order + (size_t)sc * 2 * K;        // lexicographic
    const uint16_t *SX = LX + K;                            // deepest level most significant
    // every global read of the set-up is issued here, before the first
    // barrier, and none waits on another: for the start residuals, thread
    // (h, i) (vector h, level i) reads W row i and user i's symbol of vector h,
    // and the sum over the permuted symbols is formed from LDS after the
    // barrier; then the level order, the table and both orders (the
    // deepest-level-first positions t + kTB it are the ones the tier words
    // below take, kept in registers)
    const int h0 = t / kTT, i0 = t % kTT;
    const bool r0_thread = i0 < N && h0 < nlive;
    float2 wrow[N];
    if (r0_thread) {
        s_x[h0 * N + i0] = s[(size_t)i0 * n_vec + vsel(h0)];
        stilde_row<N>(Wc, i0, wrow);
    }
    if (t < N) {
        s_wdiag[t] = Wc[vp_pidx(N, t, t)].x;
        s_nlinv[t] = -(1.0f / s_wdiag[t]);
        s_perm[t] = perm[(size_t)sc * N + t];
    }
    constexpr int kPre = 2;   // deepest-level-first positions t + kTB it, it < kPre, read here
    int sx[kPre];
#pragma unroll
    for (int it = 0; it < kPre; ++it) sx[it] = 0;
    for (int j = t, it = 0; j < K; j += kTB, ++it) {
        int k = LX[j];
        k = k < K ? k : K - 1;   // a corrupt order must not index out of bounds
        s_k[j] = (uint16_t)k;
        s_words[j] = load_word<N>(P, j);
        if (it < kPre) {
            k = SX[j];
            k = k < K ? k : K - 1;
            if (it == 0) sx[0] = k;
            else sx[1] = k;
        }
    }
    __syncthreads();
    if (r0_thread) s_r0[h0][i0] = stilde_staged<N>(wrow, s_perm, s_x + h0 * N, i0, 1.0f / tau);   // read in stage 1, two barriers on
    // stage-2 tier words: batch b holds the paths at positions [32 b, 32 b + 32)
    // of the deepest-level-first order; OR of their per-level rank thermometers
    static_assert(kBatch == 32 && kTB % kBatch == 0, "a batch is one half of a wave");
    for (int b0 = 0, it = 0; b0 < NB; b0 += kTB / kBatch, ++it) {
        const int b = b0 + t / kBatch, q = b * kBatch + t % kBatch;   // q = t + kTB it
        unsigned long long w = 0ull;
        if (q < K) {
            int k;
            if (it < kPre) {
                k = it == 0 ? sx[0] : sx[1];
            } else {
                k = SX[q];
                k = k < K ? k : K - 1;
            }
            w = s_words[k];
        }
        const uint32_t lo = half_wave_or(rank_tiers32((uint32_t)w));
        const uint32_t hi = half_wave_or(rank_tiers32((uint32_t)(w >> 32)));
        if (t % kBatch == kBatch - 1 && b < NB) s_therm[b] = ((unsigned long long)hi << 32) | lo;
    }
    // prefix boundaries: contiguous chunk of lex positions per thread, then a block scan
    constexpr unsigned long long PMASK = P1 >= 16 ? ~0ull : ((1ull << (4 * P1)) - 1ull);
    const int chunk = (K + kTB - 1) / kTB;
    const int j0 = t * chunk, j1 = min(K, j0 + chunk);
    uint32_t cnt = 0;
    // the word of lex position j is s_words[s_k[j]]
    unsigned long long prev = j0 > 0 && j0 < j1 ? s_words[s_k[j0 - 1]] : 0ull;
    for (int j = j0; j < j1; ++j) {
        const unsigned long long wj = s_words[s_k[j]];
        cnt += (j == 0 || ((wj ^ prev) & PMASK) != 0ull) ? 1u : 0u;
        prev = wj;
    }
    uint32_t incl = wave_scan_incl(cnt);
    {
        const int lane = t & 63;
        if (lane == 63) s_scan[wv] = incl;
        __syncthreads();
        for (int q = 0; q < wv; ++q) incl += s_scan[q];
    }
    uint32_t n1 = 0;
    for (int q = 0; q < kTB / 64; ++q) n1 += s_scan[q];
    uint32_t node = incl - cnt;
    prev = j0 > 0 && j0 < j1 ? s_words[s_k[j0 - 1]] : 0ull;
    for (int j = j0; j < j1; ++j) {
        const unsigned long long wj = s_words[s_k[j]];
        if (j == 0 || ((wj ^ prev) & PMASK) != 0ull) s_first[node++] = (uint16_t)j;
        s_node[s_k[j]] = (uint16_t)(node - 1);
        prev = wj;
    }
    if (t == 0) s_first[n1] = (uint16_t)K;
    __syncthreads();
    const float tau2 = tau * tau;
    // stage-2 lane roles: vector hv, path slot t / 2 of each group of kTB / 2
    const int hv = t & 1;
    const bool hv_on = hv < nlive && (hv == 0 ? on0 : on1);
    unsigned long long best = ~0ull;
    for (uint32_t base = 0; base < n1; base += kMaxPrefix) {
        const uint32_t nc = min(n1 - base, (uint32_t)kMaxPrefix);
        // stage 1: one lane per (vector, distinct prefix), the vectors' prefixes
        // packed one after the other over the workgroup (2 nc <= kTB)
        const int hh = t >= (int)nc ? 1 : 0, pp = t - hh * (int)nc;
        if (hh < nlive && (hh == 0 ? on0 : on1) && pp < (int)nc) {
            float2 r[N];
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] = s_r0[hh][i];
            const float ped = walk<N, kTierAny, false, 0, P1, RLUT>(Wc, s_nlinv, s_wdiag, r,
                                                             s_words[s_k[s_first[base + pp]]], 0ull, VP_DEMAP_LUT,
                                                             nullptr, nullptr);
            float *st = s_state[hh] + pp * SW;
#pragma unroll
            for (int i = P1; i < N; ++i) {
                st[2 * (i - P1)] = r[i].x;
                st[2 * (i - P1) + 1] = r[i].y;
            }
            st[SW - 1] = ped;
        }
        __syncthreads();
        // stage 2: all paths at once in deepest-level-first order with the tier
        // words of the set-up, or (chunked case) the contiguous lexicographic
        // range of this chunk's prefixes with tier words formed per wave
        const bool whole = (n1 <= (uint32_t)kMaxPrefix);
        const int q0 = whole ? 0 : s_first[base];
        const int q1 = whole ? K : s_first[base + nc];
        for (int it = 0; q0 + it * (kTB / kVPB) < q1; ++it) {
            const int q = q0 + it * (kTB / kVPB) + (t >> 1);
            const bool on = hv_on && q < q1;
            int k = 0;
            if (on) {
                k = whole ? SX[q] : s_k[q];
                k = k < K ? k : K - 1;   // a corrupt order must not index out of bounds
            }
            const unsigned long long wd = s_words[k];
            unsigned long long therm;
            if (whole) {
                // a wave whose paths all lie beyond K (its batch >= NB) walks nothing
                const int bt = it * (kTB / 64) + wv;
                therm = bt < NB ? s_therm[bt] : 0ull;
                therm = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(therm >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)therm);
            } else {
                therm = wave_or64(on ? rank_tiers(wd) : 0ull);
            }
            if (on) {
                int nd = (int)s_node[k] - (int)base;   // in [0, nc) unless the order is corrupt
                nd = nd < 0 ? 0 : (nd < (int)nc ? nd : (int)nc - 1);
                const float *st = s_state[hv] + nd * SW;
                float2 r[N];
#pragma unroll
                for (int i = 0; i < P1; ++i) r[i] = make_float2(0.f, 0.f);
#pragma unroll
                for (int i = P1; i < N; ++i) r[i] = make_float2(st[2 * (i - P1)], st[2 * (i - P1) + 1]);
                const float ped = walk<N, kTierTherm, false, P1, N, RLUT>(Wc, s_nlinv, s_wdiag, r, wd, therm,
                                                                    VP_DEMAP_LUT, nullptr, nullptr, st[SW - 1]);
                best = umin64(best, ((unsigned long long)__float_as_uint(ped * tau2) << 32) | (unsigned)k);
            }
        }
        __syncthreads();
    }
    if ((flags & VP_INCLUDE_ZERO) && t < kVPB && hv_on) {
        float z = 0.f;
        for (int i = 0; i < N; ++i) {
            z = fmaf(s_r0[hv][i].x, s_r0[hv][i].x, z);
            z = fmaf(s_r0[hv][i].y, s_r0[hv][i].y, z);
        }
        best = umin64(best, ((unsigned long long)__float_as_uint(z * tau2) << 32) | (unsigned)K);
    }
    best = wave_min_by_parity(best);
    if ((t & 63) < kVPB) s_red[wv][t & 63] = best;
    __syncthreads();
    if (t < kVPB && hv_on) {
        unsigned long long b = s_red[0][t];
        for (int w = 1; w < kTB / 64; ++w) b = umin64(b, s_red[w][t]);
        cost_out[vsel(t)] = __uint_as_float((unsigned)(b >> 32));
        kidx_out[vsel(t)] = (int32_t)(b & 0xffffffffull);
    }
}

// Small path tables (K up to a few hundred, e.g. per-vector proposals): one
// wave per vector, four vectors per workgroup, so that no lane idles on a
// table shorter than the workgroup.
constexpr int kWV = 4;          // vectors (waves) per workgroup
constexpr int kWaveMaxK = 192;  // tables up to this size use one wave per vector

template <int N, bool MASKED, bool RLUT>
__global__ __launch_bounds__(64 * kWV) void k_search_wave(const float2 *__restrict__ W,
                                                          const uint8_t *__restrict__ perm,
                                                          const float2 *__restrict__ s,
                                                          const float *__restrict__ taus,
                                                          const uint8_t *__restrict__ paths, int K,
                                                          long long pstride, int n_sym, size_t n_vec,
                                                          unsigned flags, float *__restrict__ cost_out,
                                                          int32_t *__restrict__ kidx_out, VecMask mask) {
    __shared__ float2 s_r0[kWV][N];
    __shared__ float s_nlinv[kWV][N];
    __shared__ float s_wdiag[kWV][N];
    __shared__ uint8_t s_perm[kWV][N];
    __shared__ float2 s_x[kWV][N];   // each vector's symbols, user order

    constexpr int NP = VP_PACKED(N);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = threadIdx.x & 63;
    const size_t v0 = (size_t)xcd_contiguous(blockIdx.x, gridDim.x) * kWV + wv;
    const bool live = v0 < n_vec && (!MASKED || mask.on(v0));   // the last workgroup may hold fewer vectors
    const size_t v = live ? v0 : n_vec - 1;
    const int sc = (int)(v / n_sym);
    const float2 *__restrict__ Wc = W + (size_t)sc * NP;
    const float w00 = Wc[0].x;
    const float tau = taus[sc];
    const bool ok = (w00 > 0.f) && isfinite(w00) && (tau > 0.f) && isfinite(tau);
    const uint8_t *P = paths + ((flags & VP_PATHS_PER_VECTOR) ? v : (size_t)sc) * pstride;
    // every global read of the set-up is issued before any is waited for: the
    // diagonal and level order, lane t's W row and symbol of user t (the start
    // residuals are summed from LDS after the barrier, so no read waits on the
    // level order), and lane t's first path
    float2 wrow[N];
    float2 xs = make_float2(0.f, 0.f);
    float wdg = 1.f;
    uint8_t pmv = 0;
    if (t < N) {
        wdg = Wc[vp_pidx(N, t, t)].x;
        pmv = perm[(size_t)sc * N + t];
        xs = s[(size_t)t * n_vec + v];
        stilde_row<N>(Wc, t, wrow);
    }
    const unsigned long long wd0 = t < K ? load_word<N>(P, t) : 0ull;
    if (t < N) {
        s_wdiag[wv][t] = wdg;
        s_nlinv[wv][t] = -(1.0f / wdg);
        s_perm[wv][t] = pmv;
        s_x[wv][t] = xs;
    }
    __syncthreads();
    if (t < N) s_r0[wv][t] = stilde_staged<N>(wrow, s_perm[wv], s_x[wv], t, 1.0f / tau);
    __syncthreads();
    if (!live) return;
    if (!ok) {   // failed preprocessing: l = 0, cost = NaN
        if (t == 0) {
            cost_out[v] = __int_as_float(0x7fc00000);
            kidx_out[v] = -1;
        }
        return;
    }

    const float tau2 = tau * tau;
    unsigned long long best = ~0ull;
    for (int k = t; k < K; k += 64) {
        const unsigned long long wd = k == t ? wd0 : load_word<N>(P, k);
        float2 r[N];
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = s_r0[wv][i];
        const float ped = walk<N, kTierAny, false, 0, N, RLUT>(Wc, s_nlinv[wv], s_wdiag[wv], r, wd, 0ull, VP_DEMAP_LUT, nullptr, nullptr);
        best = umin64(best, ((unsigned long long)__float_as_uint(ped * tau2) << 32) | (unsigned)k);
    }
    if ((flags & VP_INCLUDE_ZERO) && t == 0) {
        float z = 0.f;
        for (int i = 0; i < N; ++i) {
            z = fmaf(s_r0[wv][i].x, s_r0[wv][i].x, z);
            z = fmaf(s_r0[wv][i].y, s_r0[wv][i].y, z);
        }
        best = umin64(best, ((unsigned long long)__float_as_uint(z * tau2) << 32) | (unsigned)K);
    }
    best = wave_min(best);
    if (t == 0) {
        cost_out[v] = __uint_as_float((unsigned)(best >> 32));
        kidx_out[v] = (int32_t)(best & 0xffffffffull);
    }
}

template <int N, bool RLUT>
__global__ __launch_bounds__(kT) void k_search_finalize(const float2 *__restrict__ W,
                                                        const uint8_t *__restrict__ perm,
                                                        const float2 *__restrict__ s,
                                                        const float *__restrict__ taus,
                                                        const uint8_t *__restrict__ paths, int K,
                                                        long long pstride, int n_sc, int n_sym, unsigned flags,
                                                        const int32_t *__restrict__ kidx,
                                                        int8_t *__restrict__ l_out) {
    constexpr int NP = VP_PACKED(N);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t v = (size_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n_vec) return;
    const int sc = (int)(v / n_sym);
    const int k = kidx[v];
    const uint8_t *pm = perm + (size_t)sc * N;
    float ra[N], rb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) ra[i] = rb[i] = 0.f;
    if (k >= 0 && k < K) {
        const float2 *__restrict__ Wc = W + (size_t)sc * NP;
        float nlinv[N], wdiag[N];
        float2 r[N];
        const float inv_tau = 1.0f / taus[sc];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            wdiag[i] = Wc[vp_pidx(N, i, i)].x;
            nlinv[i] = -(1.0f / wdiag[i]);
            r[i] = stilde_over_tau<N>(Wc, pm, s, v, n_vec, i, inv_tau);
        }
        const uint8_t *P = paths + ((flags & VP_PATHS_PER_VECTOR) ? v : (size_t)sc) * pstride + (size_t)k * N;
        unsigned long long wd = 0;
        for (int i = 0; i < N; ++i) wd |= (unsigned long long)(P[i] & 15) << (4 * i);
        (void)walk<N, kTierLut, true, 0, N, RLUT>(Wc, nlinv, wdiag, r, wd, 0ull, VP_DEMAP_LUT, ra, rb);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int u = pm[i] < N ? pm[i] : N - 1;
        int8_t *o = l_out + ((size_t)u * n_vec + v) * 2;
        o[0] = (int8_t)ra[i];
        o[1] = (int8_t)rb[i];
    }
}

// Fallback merge: a vector the fixed-table search served takes that result
// where its cost is below the one already held (the proposal's), with l from
// a re-walk of the winning fixed path (the arithmetic of k_search_finalize).
template <int N>
__global__ __launch_bounds__(kT) void k_fallback_merge(const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                                       const float2 *__restrict__ s, const float *__restrict__ taus,
                                                       const uint8_t *__restrict__ paths, int K, long long pstride,
                                                       int n_sc, int n_sym, VecMask mask,
                                                       const float *__restrict__ cost_fix,
                                                       const int32_t *__restrict__ kidx_fix, int32_t kidx_base,
                                                       int8_t *__restrict__ l_out, float *__restrict__ cost_io,
                                                       int32_t *__restrict__ kidx_io) {
    constexpr int NP = VP_PACKED(N);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t v = (size_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n_vec || !mask.on(v)) return;
    const float c = cost_fix[v];
    if (!(c < cost_io[v])) return;   // ties and NaN keep the proposal's result
    const int sc = (int)(v / n_sym);
    const int k = kidx_fix[v];
    const uint8_t *pm = perm + (size_t)sc * N;
    float ra[N], rb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) ra[i] = rb[i] = 0.f;
    if (k >= 0 && k < K) {
        const float2 *__restrict__ Wc = W + (size_t)sc * NP;
        float nlinv[N], wdiag[N];
        float2 r[N];
        const float inv_tau = 1.0f / taus[sc];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            wdiag[i] = Wc[vp_pidx(N, i, i)].x;
            nlinv[i] = -(1.0f / wdiag[i]);
            r[i] = stilde_over_tau<N>(Wc, pm, s, v, n_vec, i, inv_tau);
        }
        const uint8_t *P = paths + (size_t)sc * pstride + (size_t)k * N;
        unsigned long long wd = 0;
        for (int i = 0; i < N; ++i) wd |= (unsigned long long)(P[i] & 15) << (4 * i);
        (void)walk<N, kTierLut, true>(Wc, nlinv, wdiag, r, wd, 0ull, VP_DEMAP_LUT, ra, rb);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int u = pm[i] < N ? pm[i] : N - 1;
        int8_t *o = l_out + ((size_t)u * n_vec + v) * 2;
        o[0] = (int8_t)ra[i];
        o[1] = (int8_t)rb[i];
    }
    cost_io[v] = c;
    kidx_io[v] = kidx_base + k;
}

// Static LDS of a kernel (0 if the runtime cannot tell).
template <typename Kern>
size_t static_lds_bytes(Kern *kernel) {
    hipFuncAttributes a{};
    return hipFuncGetAttributes(&a, (const void *)kernel) == hipSuccess ? a.sharedSizeBytes : 0;
}

// LDS one workgroup may hold on the current device (0 if unknown).
inline size_t max_lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    return (size_t)v;
}

// The search kernel for a table shape: prefix sharing with orders, one wave
// per vector for short tables, else one workgroup per vector.  A table too
// large for the prefix-sharing kernel's LDS (static plus K-sized dynamic part
// beyond what a workgroup may hold) takes the per-path kernels, which give
// the same results.
template <int N, bool MASKED, bool RLUT>
void launch_search_kernel(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, const uint8_t *paths,
                          const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, uint32_t flags,
                          VecMask mask, float *cost, int32_t *kidx, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    constexpr size_t kDynMax = 64 * 1024;
    static const bool lds_ok = allow_dynamic_lds(k_search_trie<N, MASKED, RLUT>, kDynMax);
    static const size_t trie_static = static_lds_bytes(k_search_trie<N, MASKED, RLUT>);
    const size_t smem = trie_lds_bytes(K);
    if (order && lds_ok && smem <= kDynMax && trie_static + smem <= max_lds_per_block()) {
        const unsigned blocks = (unsigned)n_sc * (unsigned)((n_sym + kVPB - 1) / kVPB);
        hipLaunchKernelGGL((k_search_trie<N, MASKED, RLUT>), dim3(blocks), dim3(kTB), smem, st, W, perm, s, tau, paths,
                           order, K, (long long)pstride, n_sym, n_vec, flags, cost, kidx, mask);
    } else if (K <= kWaveMaxK) {
        hipLaunchKernelGGL((k_search_wave<N, MASKED, RLUT>), dim3((unsigned)((n_vec + kWV - 1) / kWV)), dim3(64 * kWV),
                           0, st, W, perm, s, tau, paths, K, (long long)pstride, n_sym, n_vec, flags, cost, kidx,
                           mask);
    } else {
        hipLaunchKernelGGL((k_search<N, MASKED, RLUT>), dim3((unsigned)n_vec), dim3(kT), 0, st, W, perm, s, tau, paths,
                           K, (long long)pstride, n_sym, flags, cost, kidx, mask);
    }
}

template <int N, bool RLUT>
int launch_search_nr(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, const uint8_t *paths,
                     const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, uint32_t flags, int8_t *l,
                     float *cost, int32_t *kidx, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    launch_search_kernel<N, false, RLUT>(W, perm, s, tau, paths, order, K, pstride, n_sc, n_sym, flags,
                                         VecMask{nullptr, 0.f}, cost, kidx, st);
    hipLaunchKernelGGL((k_search_finalize<N, RLUT>), dim3((unsigned)((n_vec + kT - 1) / kT)), dim3(kT), 0, st, W,
                       perm, s, tau, paths, K, (long long)pstride, n_sc, n_sym, flags, kidx, l);
    return launch_status();
}

template <int N>
int launch_search_n(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, const uint8_t *paths,
                    const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, uint32_t flags, int8_t *l,
                    float *cost, int32_t *kidx, hipStream_t st) {
    if (flags & VP_DEMAP_REGION)
        return launch_search_nr<N, true>(W, perm, s, tau, paths, order, K, pstride, n_sc, n_sym, flags, l, cost,
                                         kidx, st);
    return launch_search_nr<N, false>(W, perm, s, tau, paths, order, K, pstride, n_sc, n_sym, flags, l, cost, kidx,
                                      st);
}

template <int N>
int launch_fallback_n(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, const uint8_t *paths,
                      const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, uint32_t flags,
                      const float *mass, float theta, int32_t kidx_base, int8_t *l, float *cost, int32_t *kidx,
                      void *work, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    float *cost_fix = static_cast<float *>(work);
    int32_t *kidx_fix = reinterpret_cast<int32_t *>(cost_fix + n_vec);
    const VecMask mask{mass, theta};
    launch_search_kernel<N, true, false>(W, perm, s, tau, paths, order, K, pstride, n_sc, n_sym, flags, mask,
                                         cost_fix, kidx_fix, st);
    hipLaunchKernelGGL(k_fallback_merge<N>, dim3((unsigned)((n_vec + kT - 1) / kT)), dim3(kT), 0, st, W, perm, s,
                       tau, paths, K, (long long)pstride, n_sc, n_sym, mask, cost_fix, kidx_fix, kidx_base, l, cost,
                       kidx);
    return launch_status();
}

}  // namespace

int launch_search(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, const uint8_t *paths,
                  const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, int N, uint32_t flags,
                  int8_t *l, float *cost, int32_t *kidx, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    switch (N) {
#define VP_CASE(n)                                                                                            \
    case n:                                                                                                   \
        return launch_search_n<n>(W, perm, s, tau, paths, order, K, pstride, n_sc, n_sym, flags, l, cost, \
                                  kidx, st);
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: return VP_EUNSUPPORTED;
    }
}

int launch_search_fallback(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, const uint8_t *paths,
                           const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, int N, uint32_t flags,
                           const float *mass, float theta, int32_t kidx_base, int8_t *l, float *cost, int32_t *kidx,
                           void *work, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    switch (N) {
#define VP_CASE(n)                                                                                              \
    case n:                                                                                                     \
        return launch_fallback_n<n>(W, perm, s, tau, paths, order, K, pstride, n_sc, n_sym, flags, mass, theta, \
                                    kidx_base, l, cost, kidx, work, st);
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: return VP_EUNSUPPORTED;
    }
}

// Workspace of the allocation-free fallback: the fixed-set search's cost and
// path index per vector (8 bytes each), for up to kNoAllocVectors vectors.
// One copy per GPU, alive until the process ends.  In host code `scratch` is
// only a handle for hipGetSymbolAddress; its device address, which differs
// per GPU, is looked up once per device and kept in g_scratch below.
static __device__ __align__(256) unsigned char scratch[kNoAllocVectors * 8];

namespace {
std::mutex g_scratch_mutex;
void *g_scratch[kMaxDevices];   // device address of `scratch` per device, nullptr until looked up
}  // namespace

// Device address of this GPU's workspace (the current device's), looked up
// with that device current on the first call that needs it.
static void *scratch_address(int *err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = (int)(e != hipSuccess ? e : hipErrorInvalidDevice);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

int launch_search_fallback_noalloc(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau,
                                   const uint8_t *paths, const uint16_t *order, int K, int64_t pstride, int n_sc,
                                   int n_sym, int N, uint32_t flags, const float *mass, float theta,
                                   int32_t kidx_base, int8_t *l, float *cost, int32_t *kidx, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    int err = 0;
    void *work = scratch_address(&err);
    if (!work) {
        record_hip_error(err);
        return VP_ELAUNCH;
    }
    // every vector the fixed search serves writes its own cost and index
    // before the merge reads them: nothing in the workspace must start at zero
    return launch_search_fallback(W, perm, s, tau, paths, order, K, pstride, n_sc, n_sym, N, flags, mass, theta,
                                  kidx_base, l, cost, kidx, work, st);
}

}  // namespace vp
