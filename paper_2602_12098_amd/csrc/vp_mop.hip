// Most-promising-path selection (Sec. III-A-2, eq_mop): the paper's
// breadth-first K-best search over the Metric of Promise
// M(r) = sum_i w_i r_i, one 256-thread workgroup per subcarrier.
//
// At level l the K survivors P (sorted by (M, lexicographic prefix)) expand
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

struct MopSmem {
    double pm[kMaxKMop];                 // survivors: metric
    uint16_t plex[kMaxKMop];             // survivors: lexicographic rank among survivors
    unsigned long long pword[kMaxKMop];  // survivors: rank nibbles, level i at bits 4i..4i+3
    double tm[2][kMaxKMop];              // merge ping-pong: metric
    uint32_t ttag[2][kMaxKMop];          // merge ping-pong: lexkey | parent << 14
    uint16_t scan[kMaxKMop * 9];         // presence flags -> exclusive prefix
    uint32_t part[kT];
};

__device__ __forceinline__ bool key_less(double ma, uint32_t ta, double mb, uint32_t tb) {
    return ma < mb || (ma == mb && (ta & 0x3fffu) < (tb & 0x3fffu));
}

// Element a of candidate list r.
__device__ __forceinline__ void list_elem(const MopSmem &S, double wl, int r, int a, double &m, uint32_t &tag) {
    m = S.pm[a] + wl * (double)r;
    tag = (uint32_t)(S.plex[a] * 9 + r) | ((uint32_t)a << 14);
}

__global__ __launch_bounds__(kT) void k_mop(const float *__restrict__ w2, int N, int K, uint8_t *__restrict__ paths) {
    extern __shared__ unsigned char smem_raw[];
    MopSmem &S = *reinterpret_cast<MopSmem *>(smem_raw);
    const int sc = blockIdx.x;
    const int t = threadIdx.x;

    if (t == 0) {
        S.pm[0] = 0.0;
        S.plex[0] = 0;
        S.pword[0] = 0ull;
    }
    int n = 1;
    __syncthreads();

    for (int lvl = 0; lvl < N; ++lvl) {
        const double wl = (double)w2[(size_t)sc * N + lvl];
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
    uint8_t *out = paths + (size_t)sc * K * N;
    for (int idx = t; idx < K * N; idx += kT) {
        const int k = idx / N, i = idx % N;
        out[idx] = (uint8_t)((S.pword[k] >> (4 * i)) & 15ull);
    }
}

}  // namespace

int launch_mop(const float *w2, int n_sc, int N, int K, uint8_t *paths, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    const size_t smem = sizeof(MopSmem);
    static const int attr_once =
        (hipFuncSetAttribute((const void *)k_mop, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem), 0);
    (void)attr_once;
    hipLaunchKernelGGL(k_mop, dim3(n_sc), dim3(kT), smem, st, w2, N, K, paths);
    return launch_status();
}

}  // namespace vp
