// Most-promising-path selection (Sec. III-A-2, eq_mop): the K position
// vectors r in {0..8}^N with the smallest Metric of Promise
// M(r) = sum_i w_i r_i (float64, level order), ties in lexicographic order.
// One 256-thread workgroup per subcarrier.
//
// k_mop_thr (main path).  Because M is a sum of non-negative per-level
// terms, the K smallest vectors are exactly the K smallest of
// S(T) = {r : M(r) <= T} for any T with |S(T)| >= K, and every prefix of a
// member of S(T) is itself a member padded with zeros.  So: (1) a counting
// recursion over a discretised metric (each term rounded up to a grid of
// step h, which can only under-count) picks the smallest grid threshold T
// with at least K members, on a grid over [0, 0.625 U] for an upper bound U
// of the K-th smallest M (over [0, 1.25 U] if that grid never reaches K);
// (2) S(T) is enumerated level by level, keeping every prefix whose partial
// metric is <= T (the frontier never exceeds |S(T)|); (3) S(T) is
// bucket-sorted by M over [0, T] and each member placed inside its bucket by
// its rank under the exact key (M, lexicographic r); the first K are the
// result.  This
// does one enumeration and one sort instead of a K-way selection per
// level.  A subcarrier whose S(T) does not fit the buffer (clustered or
// equal weights) is marked and handled by the K-best kernel below.
//
// k_mop (fallback): the paper's breadth-first K-best search.  At level l the K survivors P (sorted by (M, lexicographic prefix)) expand
// into nine candidate lists L_r = P + w_l r, r = 0..8.  Each list is already
// sorted, and its a-th element is preceded by at least (a+1)(r+1)-1
// candidates, so only its first floor(K/(r+1)) elements can survive.  The
// K smallest of the union are formed by eight merge-path merges in LDS
// (each truncated to K), then the survivors' lexicographic ranks are
// refreshed with a presence scan.  Keys are (M as float64, lexicographic
// key), both exact and unique, so the result equals the K smallest
// position vectors of the whole tree ordered by (M, r).
#include "vp_internal.hpp"

namespace vp {
namespace {

constexpr int kT = 256;

constexpr uint8_t kRedo = 0xFF;   // first byte of a subcarrier's table: K-best must redo it

struct MopSmem {
    double pm[kMaxKMop];                 // survivors: metric
    uint16_t plex[kMaxKMop];             // survivors: lexicographic rank among survivors
    unsigned long long pword[kMaxKMop];  // survivors: rank nibbles, level i at bits 4i..4i+3
    double tm[2][kMaxKMop];              // merge ping-pong: metric
    uint32_t ttag[2][kMaxKMop];          // merge ping-pong: lexkey | parent << 14
    uint16_t scan[kMaxKMop * 9];         // presence flags -> exclusive prefix
    uint32_t part[kT];
};

// In-LDS bitonic sort of n (a power of two) 64-bit keys with 16-bit payloads
// by a workgroup of TPB threads.
template <int TPB = kT>
__device__ void block_bitonic_sort(unsigned long long *key, uint16_t *val, int n) {
    const int t = threadIdx.x;
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < (n >> 1); i += TPB) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const unsigned long long a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                    const uint16_t x = val[lo];
                    val[lo] = val[hi];
                    val[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

// Writes order[1]: the path indices sorted with the deepest level most
// significant.  word(k) must return path k's rank nibbles (level i at bits 4i),
// which is exactly that key.  key/val are LDS scratch of >= pow2(K) entries.
// Compare-exchange with the partner element: keep the smaller (take_min) or
// the larger of the two (key, value) pairs.
__device__ __forceinline__ void bitonic_keep(unsigned long long &k, uint32_t &v, unsigned long long ok, uint32_t ov,
                                             bool take_min) {
    const bool take = take_min ? (ok < k) : (k < ok);
    k = take ? ok : k;
    v = take ? ov : v;
}

template <int TPB = kT, class WordFn>
__device__ void write_suffix_order(WordFn word, int K, unsigned long long *key, uint16_t *val,
                                   uint16_t *__restrict__ out) {
    const int t = threadIdx.x;
    int n = 1;
    while (n < K) n <<= 1;
    if (n <= 2 * TPB) {
        // Bitonic sort with elements 2t and 2t + 1 in thread t's registers:
        // partners at distance 1 are in the same thread, at 2..64 in lane
        // t ^ (stride / 2) of the same wave, further ones are exchanged
        // through LDS.  Positions n..2 TPB - 1 hold sentinels sorted among
        // themselves.
        const int e0 = 2 * t;
        unsigned long long k0 = e0 < K ? word(e0) : ~0ull, k1 = e0 + 1 < K ? word(e0 + 1) : ~0ull;
        uint32_t v0 = (uint32_t)e0, v1 = (uint32_t)e0 + 1;
        for (int size = 2; size <= n; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                const bool asc = (e0 & size) == 0;
                if (stride == 1) {
                    if (asc ? (k1 < k0) : (k0 < k1)) {
                        const unsigned long long tk = k0;
                        k0 = k1;
                        k1 = tk;
                        const uint32_t tv = v0;
                        v0 = v1;
                        v1 = tv;
                    }
                    continue;
                }
                const bool take_min = ((e0 & stride) == 0) == asc;   // e0 and e0 + 1 share both bits
                unsigned long long o0, o1;
                uint32_t w0, w1;
                if (stride <= 64) {
                    const int j = stride >> 1;
                    o0 = __shfl_xor(k0, j);
                    o1 = __shfl_xor(k1, j);
                    w0 = __shfl_xor(v0, j);
                    w1 = __shfl_xor(v1, j);
                } else {
                    key[e0] = k0;
                    key[e0 + 1] = k1;
                    val[e0] = (uint16_t)v0;
                    val[e0 + 1] = (uint16_t)v1;
                    __syncthreads();
                    o0 = key[e0 ^ stride];
                    o1 = key[(e0 + 1) ^ stride];
                    w0 = val[e0 ^ stride];
                    w1 = val[(e0 + 1) ^ stride];
                    __syncthreads();
                }
                bitonic_keep(k0, v0, o0, w0, take_min);
                bitonic_keep(k1, v1, o1, w1, take_min);
            }
        }
        if (e0 < K) out[e0] = (uint16_t)v0;
        if (e0 + 1 < K) out[e0 + 1] = (uint16_t)v1;
        __syncthreads();
        return;
    }
    for (int k = t; k < n; k += TPB) {
        key[k] = k < K ? word(k) : ~0ull;
        val[k] = (uint16_t)k;
    }
    __syncthreads();
    block_bitonic_sort<TPB>(key, val, n);
    for (int k = t; k < K; k += TPB) out[k] = val[k];
    __syncthreads();
}

// The N rank nibbles of a path word in reverse level order (nibble i <-> N-1-i):
// swap the nibbles of every byte, reverse the bytes, drop the unused levels.
__device__ __forceinline__ unsigned long long nibble_reverse(unsigned long long x, int N) {
    x = ((x & 0x0F0F0F0F0F0F0F0Full) << 4) | ((x >> 4) & 0x0F0F0F0F0F0F0F0Full);
    return __builtin_bswap64(x) >> (4 * (16 - N));
}

__device__ __forceinline__ bool key_less(double ma, uint32_t ta, double mb, uint32_t tb) {
    return ma < mb || (ma == mb && (ta & 0x3fffu) < (tb & 0x3fffu));
}

// Element a of candidate list r.
__device__ __forceinline__ void list_elem(const MopSmem &S, double wl, int r, int a, double &m, uint32_t &tag) {
    m = S.pm[a] + wl * (double)r;
    tag = (uint32_t)(S.plex[a] * 9 + r) | ((uint32_t)a << 14);
}

// One subcarrier: w2 its N weights, out its [K][N] table, order its [2][K]
// orders or NULL.  With only_marked, a table not marked for redoing is left.
__device__ __forceinline__ void mop_kbest_one(MopSmem &S, const float *__restrict__ w2, int N, int K, uint8_t *__restrict__ out,
                              uint16_t *__restrict__ order, int only_marked) {
    const int t = threadIdx.x;
    if (only_marked && out[0] != kRedo) return;
    __syncthreads();   // every thread has read the marker before it is overwritten

    if (t == 0) {
        S.pm[0] = 0.0;
        S.plex[0] = 0;
        S.pword[0] = 0ull;
    }
    int n = 1;
    __syncthreads();

    for (int lvl = 0; lvl < N; ++lvl) {
        const double wl = (double)w2[lvl];
        // list 0 -> buffer 0
        int len0 = n < K ? n : K;
        for (int a = t; a < len0; a += kT) list_elem(S, wl, 0, a, S.tm[0][a], S.ttag[0][a]);
        __syncthreads();
        int cur = 0, lenT = len0;
        for (int r = 1; r < 9; ++r) {
            int lenB = K / (r + 1);
            if (lenB > n) lenB = n;
            if (lenB == 0) break;
            const int total = (lenT + lenB < K) ? lenT + lenB : K;
            const int per = (total + kT - 1) / kT;
            const int start = t * per;
            if (start < total) {
                const int end = (start + per < total) ? start + per : total;
                // co-rank: number i of T elements among the first `start` outputs
                int lo = start - lenB > 0 ? start - lenB : 0;
                int hi = start < lenT ? start : lenT;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;       // i = mid: is T[mid] < B[start-mid-1]?
                    double bm;
                    uint32_t bt;
                    list_elem(S, wl, r, start - mid - 1, bm, bt);
                    if (key_less(S.tm[cur][mid], S.ttag[cur][mid], bm, bt)) lo = mid + 1;
                    else hi = mid;
                }
                int ia = lo, ib = start - lo;
                for (int o = start; o < end; ++o) {
                    bool takeA;
                    double bm = 0.0;
                    uint32_t bt = 0;
                    if (ib < lenB) list_elem(S, wl, r, ib, bm, bt);
                    if (ia >= lenT) takeA = false;
                    else if (ib >= lenB) takeA = true;
                    else takeA = key_less(S.tm[cur][ia], S.ttag[cur][ia], bm, bt);
                    if (takeA) {
                        S.tm[cur ^ 1][o] = S.tm[cur][ia];
                        S.ttag[cur ^ 1][o] = S.ttag[cur][ia];
                        ++ia;
                    } else {
                        S.tm[cur ^ 1][o] = bm;
                        S.ttag[cur ^ 1][o] = bt;
                        ++ib;
                    }
                }
            }
            __syncthreads();
            cur ^= 1;
            lenT = total;
        }
        // survivors T[0..lenT): refresh lexicographic ranks (lexkey space is 9n)
        const int nk = 9 * n;
        for (int q = t; q < nk; q += kT) S.scan[q] = 0;
        __syncthreads();
        for (int o = t; o < lenT; o += kT) S.scan[S.ttag[cur][o] & 0x3fffu] = 1;
        __syncthreads();
        {
            const int chunk = (nk + kT - 1) / kT;
            const int q0 = t * chunk;
            uint32_t sum = 0;
            for (int q = q0; q < q0 + chunk && q < nk; ++q) sum += S.scan[q];
            S.part[t] = sum;
            __syncthreads();
            if (t == 0) {   // exclusive scan of the 256 partial sums
                uint32_t acc = 0;
                for (int u = 0; u < kT; ++u) {
                    const uint32_t v = S.part[u];
                    S.part[u] = acc;
                    acc += v;
                }
            }
            __syncthreads();
            uint32_t acc = S.part[t];
            for (int q = q0; q < q0 + chunk && q < nk; ++q) {
                const uint32_t v = S.scan[q];
                S.scan[q] = (uint16_t)acc;
                acc += v;
            }
        }
        __syncthreads();
        // new survivors (read parents before overwriting them)
        double nm[kMaxKMop / kT];
        uint16_t nl[kMaxKMop / kT];
        unsigned long long nw[kMaxKMop / kT];
        int cnt = 0;
        for (int o = t; o < lenT; o += kT, ++cnt) {
            const uint32_t tag = S.ttag[cur][o];
            const uint32_t lk = tag & 0x3fffu;
            const int a = (int)(tag >> 14);
            const int r = (int)(lk % 9u);
            nm[cnt] = S.tm[cur][o];
            nl[cnt] = S.scan[lk];
            nw[cnt] = S.pword[a] | ((unsigned long long)r << (4 * lvl));
        }
        __syncthreads();
        cnt = 0;
        for (int o = t; o < lenT; o += kT, ++cnt) {
            S.pm[o] = nm[cnt];
            S.plex[o] = nl[cnt];
            S.pword[o] = nw[cnt];
        }
        n = lenT;
        __syncthreads();
    }
    for (int idx = t; idx < K * N; idx += kT) {
        const int k = idx / N, i = idx % N;
        out[idx] = (uint8_t)((S.pword[k] >> (4 * i)) & 15ull);
    }
    if (order) {   // survivors carry their lexicographic rank
        for (int k = t; k < K; k += kT) order[S.plex[k]] = (uint16_t)k;
        __syncthreads();
        write_suffix_order([&](int k) { return S.pword[k]; }, K,
                           reinterpret_cast<unsigned long long *>(S.tm[0]), S.scan, order + K);
    }
}

// Collects the indices `idx` of the threads with `mark` into s_list[0..*s_cnt).
__device__ __forceinline__ void marked_list(bool mark, int idx, int *s_list, int *s_cnt) {
    if (threadIdx.x == 0) *s_cnt = 0;
    __syncthreads();
    if (mark) s_list[atomicAdd(s_cnt, 1)] = idx;
    __syncthreads();
}

__global__ __launch_bounds__(kT) void k_mop(const float *__restrict__ w2, int n_sc, int N, int K,
                                            uint8_t *__restrict__ paths, uint16_t *__restrict__ order,
                                            int only_marked) {
    extern __shared__ unsigned char smem_raw[];
    MopSmem &S = *reinterpret_cast<MopSmem *>(smem_raw);
    if (!only_marked) {
        const int sc = blockIdx.x;
        mop_kbest_one(S, w2 + (size_t)sc * N, N, K, paths + (size_t)sc * K * N,
                      order ? order + (size_t)sc * 2 * K : nullptr, 0);
        return;
    }
    // marked tables only: each pass checks kT markers at once, then redoes
    // the marked subcarriers one after the other
    __shared__ int s_list[kT];
    __shared__ int s_cnt;
    for (int base = blockIdx.x * kT; base < n_sc; base += gridDim.x * kT) {
        marked_list(base + threadIdx.x < n_sc && paths[(size_t)(base + threadIdx.x) * K * N] == kRedo,
                    base + threadIdx.x, s_list, &s_cnt);
        for (int q = 0; q < s_cnt; ++q) {
            const int sc = s_list[q];
            mop_kbest_one(S, w2 + (size_t)sc * N, N, K, paths + (size_t)sc * K * N,
                          order ? order + (size_t)sc * 2 * K : nullptr, 1);
        }
        __syncthreads();   // s_list and s_cnt are rewritten by the next pass
    }
}


// ---------------------------------------------------------------------------
// threshold + enumeration + bucket sort
// ---------------------------------------------------------------------------


// Exclusive scan of one value per thread across the workgroup; returns the
// prefix and writes the total to *total.
// With FENCE = false the closing barrier (which lets the next scan reuse
// `scratch`) is left out: the caller then alternates two scratch buffers and
// has a barrier of its own between two scans on the same one.
template <bool FENCE = true, int TPB = kT>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *scratch, uint32_t *total) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t incl = wave_scan_incl(v);
    if (lane == 63) scratch[wv] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < TPB / 64; ++q) {
        const uint32_t x = scratch[q];
        if (q < wv) base += x;
        tot += x;
    }
    *total = tot;
    if (FENCE) __syncthreads();
    return base + incl - v;
}

// Counting recursion on a grid of NB bins of width h (NB = kT or 2 kT: one
// or two adjacent bins per thread): after levels l..N-1, count[b] = number of
// rank suffixes whose metric, with every term w_i r_i rounded up to whole
// bins, is at most b bins (an under-count of the true |S(b h)|).  Returns the
// smallest b with count >= K, or -1.  The two buffers (cur, next) carry NB
// zero bins on their left so that shifted reads need no bounds test; counts
// saturate at 2^20 (>= K, all that is compared).  buf: 2 x 2 NB uint32 of
// LDS; dtab: kMaxN x 9 ints of LDS.
template <int NB, int TPB = kT>
__device__ int dp_threshold(const double *w, int N, int K, double h, uint32_t *buf, int *sbest, int (*dtab)[9]) {
    constexpr int BPT = NB / TPB;   // bins per thread
    static_assert(BPT * TPB == NB && (BPT == 1 || BPT == 2), "one or two bins per thread");
    constexpr uint32_t kSat = 1u << 20;
    const int t = threadIdx.x;
    const double inv_h = (1.0 + 0x1p-40) / h;   // the tiny excess keeps every term rounded up
    uint32_t *b0 = buf, *b1 = buf + 2 * NB;
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
        b0[BPT * t + e] = 0u;
        b1[BPT * t + e] = 0u;
        b0[NB + BPT * t + e] = 1u;
    }
    if (t == 0) *sbest = NB;
    // the shifts ceil(w_l r / h) depend only on the level: one thread each
    for (int q = t; q < N * 9; q += TPB) {
        const int l = q / 9, r = q % 9;
        const double x = ceil((w[l] * inv_h) * (double)r);
        dtab[l][r] = x < (double)NB ? (int)x : NB;
    }
    __syncthreads();
    uint32_t *cur = b0, *nxt = b1;
    const int lane = t & 63;
    for (int l = N - 1; l >= 0; --l) {
        const uint32_t *src = cur + NB + BPT * t;
        // the level's nine shifts: one LDS read by lanes 0..8, then scalar copies
        const int dl = dtab[l][lane < 9 ? lane : 0];
        uint32_t a[BPT];
#pragma unroll
        for (int e = 0; e < BPT; ++e) a[e] = 0u;
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const int d = __builtin_amdgcn_readlane(dl, r);
#pragma unroll
            for (int e = 0; e < BPT; ++e) a[e] += src[e - d];
        }
#pragma unroll
        for (int e = 0; e < BPT; ++e) nxt[NB + BPT * t + e] = min(a[e], kSat);
        __syncthreads();
        uint32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    int mine = NB;
#pragma unroll
    for (int e = BPT - 1; e >= 0; --e)
        if (cur[NB + BPT * t + e] >= (uint32_t)K) mine = BPT * t + e;
    atomicMin(sbest, mine);
    __syncthreads();
    const int r = *sbest;
    __syncthreads();
    return r < NB ? r : -1;
}

constexpr int kNBCount = 256;   // grid points of the counting recursion (one per thread)
constexpr int kNB = 512;   // buckets of the sort by metric

// An upper bound on the K-th smallest M: for per-level rank limits a_i the
// box {r : r_i <= a_i} holds prod (a_i + 1) position vectors, each with
// M <= sum a_i w_i.  The limits are raised greedily, each time at the level
// with the smallest cost per gained log-count, w_i / ln((a_i + 2) / (a_i + 1)),
// until the box holds K vectors (K <= 9^N).  0 for K = 1.  Run by the whole
// of wave 0, lane i holding level i: each step is a 16-lane argmin by DPP
// moves (xor 1, xor 2, half-row mirror, row mirror).
__device__ __forceinline__ float dpp_f(float x, int ctrl_sel) {
    const int v = __float_as_int(x);
    int r;
    switch (ctrl_sel) {
        case 0: r = __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false); break;    // quad_perm [1,0,3,2]
        case 1: r = __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false); break;    // quad_perm [2,3,0,1]
        case 2: r = __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false); break;   // row_half_mirror
        default: r = __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false); break; // row_mirror
    }
    return __int_as_float(r);
}

__device__ __forceinline__ int dpp_i(int v, int ctrl_sel) {
    switch (ctrl_sel) {
        case 0: return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);
        case 1: return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);
        case 2: return __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);
        default: return __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);
    }
}

constexpr int kRankMax = 8;   // ranks 0..8 per level (the 3 x 3 box)

// Wave 0 only (all 64 lanes active); returns the bound in every lane.
__device__ double product_set_bound(const double *w, int N, int K) {
    const int lane = threadIdx.x & 63;
    const bool mine = lane < N;
    const double wl = mine ? w[lane] : 0.0;
    int a = 0;   // this level's limit
    // 1 / ln((a + 2) / (a + 1)) for a = 0..7
    auto inv_gain = [](int a) {
        const float g[kRankMax] = {1.4426950f, 2.4663035f, 3.4760595f, 4.4814201f,
                                   5.4848149f, 6.4871592f, 7.4888757f, 8.4901870f};
        float v = g[0];
#pragma unroll
        for (int q = 1; q < kRankMax; ++q) v = a == q ? g[q] : v;
        return v;
    };
    const float kInf = __int_as_float(0x7f800000);
    float c = mine ? (float)wl * inv_gain(0) : kInf;
    long long count = 1;
    double U = 0.0;
    while (count < (long long)K) {
        float m = c;
        int mi = lane;
#pragma unroll
        for (int s = 0; s < 4; ++s) {   // (cost, level) minimum over the 16 lanes of each row
            const float om = dpp_f(m, s);
            const int oi = dpp_i(mi, s);
            const bool take = (om < m) | ((om == m) & (oi < mi));
            m = take ? om : m;
            mi = take ? oi : mi;
        }
        const int best = __builtin_amdgcn_readfirstlane(mi);
        if (!(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m))) < kInf)) break;
        const int ab = __builtin_amdgcn_readlane(a, best);
        count = count / (ab + 1) * (ab + 2);
        U += w[best];
        if (lane == best) {
            ++a;
            c = a < kRankMax ? (float)wl * inv_gain(a) : kInf;
        }
    }
    return U;
}

// A cheaper bound of the same kind when K <= 2^N: the box with limit 1 on
// the m = ceil(log2 K) levels of smallest weight holds 2^m >= K vectors, so
// the K-th smallest M is at most the sum of those m weights.  One step for
// the whole wave instead of the greedy's chain of dependent ones; looser (it
// never raises a limit to 2), which only widens the counting grid.  Wave 0
// only (all 64 lanes active); returns the bound in every lane.
__device__ double smallest_weights_bound(const double *w, int N, int m) {
    const int lane = threadIdx.x & 63;
    double x = 0.0;
    if (lane < N) {
        const double wl = w[lane];
        int rank = 0;   // position of this level among the weights (ties: smaller level first)
        for (int j = 0; j < N; ++j) {
            const double wj = w[j];
            rank += (wj < wl || (wj == wl && j < lane)) ? 1 : 0;
        }
        x = rank < m ? wl : 0.0;
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) x += __shfl_xor(x, off);   // levels live in lanes 0..15
    return __shfl(x, 0);
}

template <int CAP, int NBK = kNB, int TPB = kT>
struct ThrSmem {
    // fm and fw, adjacent, first hold the counting recursion's two buffers
    double fm[CAP];               // S(T) members / frontier: metric
    unsigned long long fw[CAP];   // rank nibbles (level i at bits 4i), later the lexicographic key
    uint16_t fe[CAP];             // enumeration (= lexicographic) position, carried through the sort
    uint16_t rank_of[CAP];        // enumeration position -> MoP rank (or 0xffff beyond K)
    uint32_t dp[2][NBK];          // bucket starts / cursors
    double w[kMaxN];
    int dtab[kMaxN][9];           // bin shifts of the counting recursion
    uint32_t scan[TPB / 64];
    uint32_t lscan[2][TPB / 64];  // the enumeration's scans, alternating by level
    int best;
    double ubound;

    __device__ uint32_t *count_buffers() {
        static_assert(2 * CAP * sizeof(double) >= 4 * kNBCount * sizeof(uint32_t), "fm and fw hold the counting buffers");
        return reinterpret_cast<uint32_t *>(fm);
    }
};

// Frontier capacity of the threshold pass for tables of up to 512 paths: the
// enumerated set exceeds K by a few members for spread weights (513 to 522
// for K = 512 on 16 x 16 Rayleigh channels); a larger set sends the table to
// the K-best kernel.  20 KiB of LDS, eight workgroups per CU.
constexpr int kCap512 = 768;

// The same for tables of up to 256 paths on 128-thread workgroups: 384
// frontier entries and 256 metric buckets, 10 KiB of LDS, so that a CU holds
// fifteen workgroups and a whole slot's subcarriers are resident at once.
constexpr int kCap256 = 384, kNB256 = 256, kT256 = 128;

// One subcarrier (pointers as for mop_kbest_one).  Marks the table for the
// K-best kernel when the threshold enumeration does not fit.
template <int CAP, int NBK = kNB, int TPB = kT>
__device__ __forceinline__ void mop_thr_one(ThrSmem<CAP, NBK, TPB> &S, const float *__restrict__ w2, int N, int K,
                                            uint8_t *__restrict__ out, uint16_t *__restrict__ order) {
    constexpr int PER = CAP / TPB;   // frontier entries held per thread
    const int t = threadIdx.x;

    if (t < N) S.w[t] = (double)w2[t];
    __syncthreads();
    bool valid = true;
    for (int i = 0; i < N; ++i) {
        valid &= (S.w[i] > 0.0) && isfinite(S.w[i]);
    }
    if (!valid) {   // failed preprocessing: a deterministic all-zero table
        for (int idx = t; idx < K * N; idx += TPB) out[idx] = 0;
        if (order)
            for (int k = t; k < 2 * K; k += TPB) order[k] = (uint16_t)(k % K);
        return;
    }
    // (1) threshold: the smallest grid point whose count reaches K.  U bounds
    // the K-th smallest M from above; the grid first spans [0, 0.625 U] (the
    // K-th smallest is typically U / 2.5), and the guaranteed [0, 1.25 U] only
    // when that one never reaches K.
    if (t < 64) {
        int m = 0;   // ceil(log2 K)
        while ((1 << m) < K) ++m;
        const double U0 = m <= N ? smallest_weights_bound(S.w, N, m) : product_set_bound(S.w, N, K);
        if (t == 0) S.ubound = U0;
    }
    __syncthreads();
    const double U = S.ubound;
    double T = 0.0;   // K = 1: the zero path alone
    if (U > 0.0) {
        double h = 0.625 * U / (double)(kNBCount - 1);
        int b = dp_threshold<kNBCount, TPB>(S.w, N, K, h, S.count_buffers(), &S.best, S.dtab);
        if (b < 0) {
            h = 1.25 * U / (double)(kNBCount - 1);
            b = dp_threshold<kNBCount, TPB>(S.w, N, K, h, S.count_buffers(), &S.best, S.dtab);
        }
        T = (b < 0 ? (double)(kNBCount - 1) : (double)b) * h;
    }
    // (2) enumerate S(T) level by level, in place: every thread first takes its
    // contiguous share of the frontier into registers, then writes the children
    if (t == 0) {
        S.fm[0] = 0.0;
        S.fw[0] = 0ull;
    }
    uint32_t n = 1;
    bool fail = false;
    __syncthreads();
    for (int l = 0; l < N; ++l) {
        const double wl = S.w[l];
        double wr[9];   // the level's metric steps w_l r, formed once
#pragma unroll
        for (int r = 0; r < 9; ++r) wr[r] = wl * (double)r;
        const uint32_t chunk = (n + TPB - 1) / TPB;
        const uint32_t j0 = t * chunk;
        double m[PER];
        unsigned long long wd[PER];
        int R[PER];
        uint32_t cnt = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            R[q] = 0;
            if ((uint32_t)q < chunk && j0 + q < n) {
                m[q] = S.fm[j0 + q];
                wd[q] = S.fw[j0 + q];
                int r = 1;   // children r = 0 .. R-1 stay within T (the steps increase with r)
#pragma unroll
                for (int rr = 1; rr < 9; ++rr) r += (m[q] + wr[rr] <= T) ? 1 : 0;
                R[q] = r;
                cnt += r;
            }
        }
        uint32_t total;
        // (its barrier also orders this level's frontier reads before the
        // children's writes; the barrier closing the level separates two
        // scans on one buffer)
        uint32_t off = block_scan_excl<false, TPB>(cnt, S.lscan[l & 1], &total);
        if (total > (uint32_t)CAP) {
            fail = true;
            break;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {   // children r = 0 .. R-1 (R = 0 past the frontier)
            const double mq = m[q];
            const unsigned long long wq = wd[q];
            for (int r = 0; r < R[q]; ++r) {
                S.fm[off] = mq + wl * (double)r;   // the step w_l r formed as above
                S.fw[off] = wq | ((unsigned long long)r << (4 * l));
                ++off;
            }
        }
        __syncthreads();
        n = total;
    }
    if (fail || n < (uint32_t)K) {
        if (t == 0) out[0] = kRedo;
        return;
    }
    // (3) bucket sort by M over [0, T], then exact (M, lexicographic r) inside buckets
    // bucket of M: NBK (M / T)^4, monotone in M.  The members of S(T) grow
    // steeply towards T (|S(x)| rises like a power of x), and the fourth power
    // spreads them nearly evenly, which keeps every bucket's ranking short.
    const double invT = T > 0.0 ? 1.0 / T : 0.0;
    for (int b = t; b < NBK; b += TPB) S.dp[0][b] = 0u;
    double m[PER];
    unsigned long long lex[PER];
    int bk[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t j = t + q * TPB;
        bk[q] = -1;
        if (j < n) {
            S.rank_of[j] = 0xffff;
            m[q] = S.fm[j];
            const unsigned long long wd = S.fw[j];
            lex[q] = nibble_reverse(wd, N);   // level 0 in the most significant nibble
            const double x = m[q] * invT, x2 = x * x;
            bk[q] = min(NBK - 1, (int)(x2 * x2 * (double)NBK));
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (bk[q] >= 0) atomicAdd(&S.dp[0][bk[q]], 1u);
    __syncthreads();
    {
        constexpr int BPT = NBK / TPB;
        uint32_t loc = 0;
        for (int q = 0; q < BPT; ++q) loc += S.dp[0][t * BPT + q];
        uint32_t tot;
        uint32_t base = block_scan_excl<true, TPB>(loc, S.scan, &tot);
        for (int q = 0; q < BPT; ++q) {
            const uint32_t c = S.dp[0][t * BPT + q];
            S.dp[0][t * BPT + q] = base;   // bucket start
            S.dp[1][t * BPT + q] = base;   // fill cursor
            base += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (bk[q] >= 0) {
            const uint32_t pos = atomicAdd(&S.dp[1][bk[q]], 1u);
            S.fm[pos] = m[q];
            S.fw[pos] = lex[q];
        }
    __syncthreads();
    // inside its bucket, each member's place is the number of members with a
    // smaller (M, lexicographic r) key (the keys are distinct: r is); every
    // thread ranks its own members, then all write them to their places
    uint32_t dst[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        dst[q] = 0xffffffffu;
        if (bk[q] >= 0) {
            const uint32_t lo = S.dp[0][bk[q]], hi = S.dp[1][bk[q]];
            uint32_t below = 0;
            for (uint32_t a = lo; a < hi; ++a) {
                const double ma = S.fm[a];
                below += (ma < m[q] || (ma == m[q] && S.fw[a] < lex[q])) ? 1u : 0u;
            }
            dst[q] = lo + below;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (bk[q] >= 0) {
            S.fm[dst[q]] = m[q];
            S.fw[dst[q]] = lex[q];
            S.fe[dst[q]] = (uint16_t)(t + q * TPB);
        }
    __syncthreads();
    for (int k = t; k < K; k += TPB) {   // one path per thread: its N rank bytes
        const unsigned long long w = nibble_reverse(S.fw[k], N);   // level i at bits 4i
        uint8_t *o = out + (size_t)k * N;
        if (N == 16 && (reinterpret_cast<uintptr_t>(o) & 15) == 0) {
            uint32_t d[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t n4 = (uint32_t)(w >> (16 * q));   // levels 4q .. 4q+3
                d[q] = (n4 & 15u) | ((n4 >> 4) & 15u) << 8 | ((n4 >> 8) & 15u) << 16 | ((n4 >> 12) & 15u) << 24;
            }
            *reinterpret_cast<uint4 *>(o) = make_uint4(d[0], d[1], d[2], d[3]);
        } else {
            for (int i = 0; i < N; ++i) o[i] = (uint8_t)((w >> (4 * i)) & 15ull);
        }
    }
    if (order) {
        uint16_t *lexorder = order;
        // the enumeration visited S(T) in lexicographic order: the selected
        // paths, in enumeration order, are the path table in lexicographic order
        for (int k = t; k < K; k += TPB) S.rank_of[S.fe[k]] = (uint16_t)k;
        __syncthreads();
        uint32_t sel[PER];
        uint32_t cnt = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t j = t * PER + q;
            sel[q] = (j < n && S.rank_of[j] != 0xffff) ? 1u : 0u;
            cnt += sel[q];
        }
        uint32_t tot;
        uint32_t pos = block_scan_excl<true, TPB>(cnt, S.scan, &tot);
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (sel[q]) lexorder[pos++] = S.rank_of[t * PER + q];
        // suffix-major order: the nibble reversal of the lexicographic key
        const int NN = N;
        write_suffix_order<TPB>(
            [&](int k) { return nibble_reverse(S.fw[k], NN); },
            K, reinterpret_cast<unsigned long long *>(S.fm), S.fe, lexorder + K);
    }
}

template <int CAP, int NBK = kNB, int TPB = kT>
__global__ __launch_bounds__(TPB) void k_mop_thr(const float *__restrict__ w2, int N, int K,
                                                 uint8_t *__restrict__ paths, uint16_t *__restrict__ order) {
    extern __shared__ unsigned char smem_raw[];
    ThrSmem<CAP, NBK, TPB> &S = *reinterpret_cast<ThrSmem<CAP, NBK, TPB> *>(smem_raw);
    const int sc = blockIdx.x;
    mop_thr_one<CAP, NBK, TPB>(S, w2 + (size_t)sc * N, N, K, paths + (size_t)sc * K * N,
                               order ? order + (size_t)sc * 2 * K : nullptr);
}

// Batched: one workgroup per subcarrier of any group (K <= 512, or the
// 128-thread form when every group has K <= 256), then the K-best kernel for
// the tables the threshold pass marked.
template <int CAP, int NBK = kNB, int TPB = kT>
__global__ __launch_bounds__(TPB) void k_batch_mop_thr(const BatchGroup *__restrict__ groups,
                                                       const int32_t *__restrict__ sc_group,
                                                       const float *__restrict__ w2, uint8_t *__restrict__ paths) {
    extern __shared__ unsigned char smem_raw[];
    ThrSmem<CAP, NBK, TPB> &S = *reinterpret_cast<ThrSmem<CAP, NBK, TPB> *>(smem_raw);
    const int sc = blockIdx.x;
    const BatchGroup g = groups[sc_group[sc]];
    const long long j = sc - g.sc0;
    mop_thr_one<CAP, NBK, TPB>(S, w2 + g.offN + j * g.U, g.U, g.K, paths + g.offP + j * g.K * g.U, nullptr);
}

__global__ __launch_bounds__(kT) void k_batch_mop_kbest(const BatchGroup *__restrict__ groups,
                                                        const int32_t *__restrict__ sc_group, int n_sc_total,
                                                        const float *__restrict__ w2, uint8_t *__restrict__ paths) {
    extern __shared__ unsigned char smem_raw[];
    MopSmem &S = *reinterpret_cast<MopSmem *>(smem_raw);
    __shared__ int s_list[kT];
    __shared__ int s_cnt;
    for (int base = blockIdx.x * kT; base < n_sc_total; base += gridDim.x * kT) {
        const int sc = base + threadIdx.x;
        bool mark = false;
        if (sc < n_sc_total) {
            const BatchGroup g = groups[sc_group[sc]];
            mark = paths[g.offP + (sc - g.sc0) * g.K * g.U] == kRedo;
        }
        marked_list(mark, sc, s_list, &s_cnt);
        for (int q = 0; q < s_cnt; ++q) {
            const int sm = s_list[q];
            const BatchGroup g = groups[sc_group[sm]];
            const long long j = sm - g.sc0;
            mop_kbest_one(S, w2 + g.offN + j * g.U, g.U, g.K, paths + g.offP + j * g.K * g.U, nullptr, 1);
        }
        __syncthreads();
    }
}

}  // namespace

void prepare_batch_kernels() {
    (void)allow_dynamic_lds(k_batch_mop_thr<kCap512>, sizeof(ThrSmem<kCap512>));
    (void)allow_dynamic_lds(k_batch_mop_thr<kCap256, kNB256, kT256>, sizeof(ThrSmem<kCap256, kNB256, kT256>));
    (void)allow_dynamic_lds(k_batch_mop_kbest, sizeof(MopSmem));
}

int launch_batch_mop(const BatchGroup *groups, const int32_t *sc_group, int n_sc_total, int max_K, const float *w2,
                     uint8_t *paths, hipStream_t st) {
    if (n_sc_total == 0) return VP_OK;
    if (max_K <= 256)
        hipLaunchKernelGGL((k_batch_mop_thr<kCap256, kNB256, kT256>), dim3(n_sc_total), dim3(kT256),
                           sizeof(ThrSmem<kCap256, kNB256, kT256>), st, groups, sc_group, w2, paths);
    else
        hipLaunchKernelGGL(k_batch_mop_thr<kCap512>, dim3(n_sc_total), dim3(kT), sizeof(ThrSmem<kCap512>), st, groups,
                           sc_group, w2, paths);
    hipLaunchKernelGGL(k_batch_mop_kbest, dim3((unsigned)((n_sc_total + kT - 1) / kT)), dim3(kT), sizeof(MopSmem), st,
                       groups, sc_group, n_sc_total, w2, paths);
    return launch_status();
}

int launch_mop(const float *w2, int n_sc, int N, int K, uint8_t *paths, uint16_t *order, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    static const int lds_ok = (int)allow_dynamic_lds(k_mop, sizeof(MopSmem)) +
                              (int)allow_dynamic_lds(k_mop_thr<kCap512>, sizeof(ThrSmem<kCap512>)) +
                              (int)allow_dynamic_lds(k_mop_thr<2048>, sizeof(ThrSmem<2048>));
    (void)lds_ok;
    using Small = ThrSmem<kCap256, kNB256, kT256>;
    if (K <= 256)
        hipLaunchKernelGGL((k_mop_thr<kCap256, kNB256, kT256>), dim3(n_sc), dim3(kT256), sizeof(Small), st, w2, N, K,
                           paths, order);
    else if (K <= 512)
        hipLaunchKernelGGL(k_mop_thr<kCap512>, dim3(n_sc), dim3(kT), sizeof(ThrSmem<kCap512>), st, w2, N, K, paths,
                           order);
    else
        hipLaunchKernelGGL(k_mop_thr<2048>, dim3(n_sc), dim3(kT), sizeof(ThrSmem<2048>), st, w2, N, K, paths,
                           order);
    hipLaunchKernelGGL(k_mop, dim3((unsigned)((n_sc + kT - 1) / kT)), dim3(kT), sizeof(MopSmem), st, w2, n_sc, N, K,
                       paths, order, 1);
    return launch_status();
}

int launch_mop_kbest(const float *w2, int n_sc, int N, int K, uint8_t *paths, uint16_t *order, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    hipLaunchKernelGGL(k_mop, dim3(n_sc), dim3(kT), sizeof(MopSmem), st, w2, n_sc, N, K, paths, order, 0);
    return launch_status();
}

}  // namespace vp
