// Learned path proposal: kernels for a small MLP that scores a vocabulary of
// position vectors per vector (features -> 256 -> 256 -> V logits, ReLU),
// its training (softmax cross-entropy, hand-written backward) and its use
// (top-64 per vector -> per-vector path table for the path search).
//
// The proposal only chooses which position vectors the search walks; the
// search itself (Sec. II-B PED, Sec. III-A-2 DEMAP, Alg. 2 argmin) is
// unchanged, so l stays an exact Gaussian integer.  Labels are the position
// vectors of the exact (sphere-encoder) solutions: the rank of each level's
// exact symbol in the DEMAP order of that level's centre.
//
// GEMM: bf16 operands, fp32 accumulation on the matrix cores
// (v_mfma_f32_32x32x16_bf16), 64x64 tiles per 256-thread workgroup, one
// 32x32 block per wave, K staged through LDS in steps of 32.
#include "vp_internal.hpp"

#define VP_LUT_STORAGE static __constant__
#include "vp_device.hpp"

namespace vp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// GEMM  C[M][N] = epi(alpha A[M][K] B[K][N] + bias[N])
//   TA: A is stored as [K][M] (lda = row stride of the stored matrix)
//   TB: B is stored as [N][K]
// 128 x 128 tile per workgroup, 2 x 2 waves of 64 x 64 (2 x 2 MFMA blocks of
// 32 x 32 each), K in steps of 32 through LDS ([row][k] with a padded row),
// the global loads of step s + 1 issued before the MFMAs of step s.
// ---------------------------------------------------------------------------
constexpr int GT = 256, BM = 128, BN = 128, BK = 32, LDK = BK + 8;

// 8 consecutive elements of a stored row starting at `start` (< limit), zero
// beyond `limit`; one 16-byte load when the row is 16-byte aligned there.
__device__ __forceinline__ uint4 load8(const uint16_t *__restrict__ row, int start, int limit, bool vec) {
    if (vec && start + 8 <= limit) return *reinterpret_cast<const uint4 *>(row + start);
    uint16_t e[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) e[j] = (start + j < limit) ? row[start + j] : (uint16_t)0;
    uint4 r;
    r.x = e[0] | ((uint32_t)e[1] << 16);
    r.y = e[2] | ((uint32_t)e[3] << 16);
    r.z = e[4] | ((uint32_t)e[5] << 16);
    r.w = e[6] | ((uint32_t)e[7] << 16);
    return r;
}

// A ROWS x BK tile of op(X) (rows = m or n) in two steps, so that the global
// loads of the next K step are in flight while the current one is computed:
// fetch() loads this thread's 8-element chunks into registers, put() stores
// them to S[row][k].  CONTIG_K: the stored matrix is contiguous along k
// (X[row][k]); else along rows (X[k][row]).
template <bool CONTIG_K, int ROWS>
struct TileRegs {
    static constexpr int Q = ROWS * BK / 8 / GT;   // chunks per thread
    uint4 x[Q];
};

template <bool CONTIG_K, int ROWS>
__device__ __forceinline__ void fetch(TileRegs<CONTIG_K, ROWS> &R, const uint16_t *__restrict__ X, long long ld, int r0,
                                      int nrows, int k0, int K, bool vec, int t) {
#pragma unroll
    for (int q = 0; q < R.Q; ++q) {
        const int c = q * GT + t;
        uint4 x = make_uint4(0, 0, 0, 0);
        if (CONTIG_K) {
            const int rr = c / (BK / 8), kk = (c % (BK / 8)) * 8;
            const int gr = r0 + rr;
            if (gr < nrows && k0 + kk < K) x = load8(X + (size_t)gr * ld, k0 + kk, K, vec);
        } else {
            const int kk = c / (ROWS / 8), rr = (c % (ROWS / 8)) * 8;
            const int gk = k0 + kk;
            if (gk < K && r0 + rr < nrows) x = load8(X + (size_t)gk * ld, r0 + rr, nrows, vec);
        }
        R.x[q] = x;
    }
}

template <bool CONTIG_K, int ROWS>
__device__ __forceinline__ void put(uint16_t (*S)[LDK], const TileRegs<CONTIG_K, ROWS> &R, int t) {
#pragma unroll
    for (int q = 0; q < R.Q; ++q) {
        const int c = q * GT + t;
        const uint4 x = R.x[q];
        if (CONTIG_K) {
            const int rr = c / (BK / 8), kk = (c % (BK / 8)) * 8;
            *reinterpret_cast<uint4 *>(&S[rr][kk]) = x;
        } else {
            const int kk = c / (ROWS / 8), rr = (c % (ROWS / 8)) * 8;
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                S[rr + 2 * j][kk] = (uint16_t)(w[j] & 0xffffu);
                S[rr + 2 * j + 1][kk] = (uint16_t)(w[j] >> 16);
            }
        }
    }
}

// Four waves per SIMD: the accumulators then sit in ordinary VGPRs (128 in
// all, with the registers of the next step's loads) instead of 144 VGPRs + 64
// accumulation registers at two waves, which hides more of each K step's load
// latency.
template <bool TA, bool TB>
__global__ __launch_bounds__(GT) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm(int M, int N, int K, const uint16_t *__restrict__ A, long long lda,
                                             const uint16_t *__restrict__ B, long long ldb, int vec_a, int vec_b,
                                             float *__restrict__ Cf, uint16_t *__restrict__ Cb, long long ldc,
                                             const float *__restrict__ bias, int relu,
                                             const uint16_t *__restrict__ mask, long long ldm, float alpha) {
    __shared__ __attribute__((aligned(16))) uint16_t As[BM][LDK];   // [m][k]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LDK];   // [n][k]
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
    TileRegs<!TA, BM> ra;
    TileRegs<TB, BN> rb;
    fetch<!TA, BM>(ra, A, lda, m0, M, 0, K, vec_a != 0, t);
    fetch<TB, BN>(rb, B, ldb, n0, N, 0, K, vec_b != 0, t);
    for (int k0 = 0; k0 < K; k0 += BK) {
        put<!TA, BM>(As, ra, t);
        put<TB, BN>(Bs, rb, t);
        __syncthreads();
        if (k0 + BK < K) {   // the next step's loads, in flight during this step's MFMAs
            fetch<!TA, BM>(ra, A, lda, m0, M, k0 + BK, K, vec_a != 0, t);
            fetch<TB, BN>(rb, B, ldb, n0, N, k0 + BK, K, vec_b != 0, t);
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            // lane l: row (l % 32) of a 32-row block, k = kk + 8 (l / 32) .. +7
            const int kl = kk + 8 * (lane >> 5);
            bf16x8 fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = *reinterpret_cast<const bf16x8 *>(&As[wm + 32 * a + (lane & 31)][kl]);
#pragma unroll
            for (int b = 0; b < 2; ++b) fb[b] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 32 * b + (lane & 31)][kl]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // D layout of a 32 x 32 block: register r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int gm = m0 + wm + 32 * a + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int gn = n0 + wn + 32 * b + (lane & 31);
                if (gm < M && gn < N) {
                    float v = alpha * acc[a][b][r];
                    if (bias) v += bias[gn];
                    if (relu) v = fmaxf(v, 0.f);
                    if (mask && !(bf2f(mask[(size_t)gm * ldm + gn]) > 0.f)) v = 0.f;
                    if (Cf) Cf[(size_t)gm * ldc + gn] = v;
                    if (Cb) Cb[(size_t)gm * ldc + gn] = f2bf(v);
                }
            }
}

// ---------------------------------------------------------------------------
// features: 64 per vector
//   [0,16)  W_ii / mean_j W_jj                  (the MoP weights, Sec. III-A-2)
//   [16,32) Re c0_i, [32,48) Im c0_i           c0_i = -(s-tilde_i / tau) / W_ii, the
//                                                level centres of the zero perturbation
//   [48,64) w_i |c0_i - round_box(c0_i)|^2 / mean w   (rank-0 PED share per level)
// levels beyond N are zero.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(64) void k_features(const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                                 const float2 *__restrict__ s, float tau, int n_sc, int n_sym,
                                                 uint16_t *__restrict__ feat) {
    constexpr int NP = VP_PACKED(N);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t v = (size_t)blockIdx.x * 64 + threadIdx.x;
    if (v >= n_vec) return;
    const int sc = (int)(v / n_sym);
    const float2 *Wc = W + (size_t)sc * NP;
    const uint8_t *pm = perm + (size_t)sc * N;
    uint16_t *f = feat + v * 64;
    float wd[N], mean = 0.f, wmean = 0.f;
    for (int i = 0; i < N; ++i) {
        wd[i] = Wc[vp_pidx(N, i, i)].x;
        mean += wd[i];
        wmean += wd[i] * wd[i];
    }
    mean /= N;
    wmean /= N;
    const bool ok = (wd[0] > 0.f) && isfinite(wd[0]) && (mean > 0.f) && isfinite(mean) && isfinite(wmean);
    const float inv_tau = 1.0f / tau;
    for (int i = 0; i < 16; ++i) {
        float a = 0.f, cx = 0.f, cy = 0.f, d0 = 0.f;
        if (i < N && ok) {
            float re = 0.f, im = 0.f;
            for (int j = 0; j <= i; ++j) {
                const float2 w = Wc[vp_pidx(N, i, j)];
                const int u = pm[j] < N ? pm[j] : N - 1;
                const float2 x = s[(size_t)u * n_vec + v];
                re = fmaf(w.x, x.x, fmaf(-w.y, x.y, re));
                im = fmaf(w.x, x.y, fmaf(w.y, x.x, im));
            }
            a = wd[i] / mean;
            cx = -(re * inv_tau) / wd[i];
            cy = -(im * inv_tau) / wd[i];
            const float ex = cx - vp_o0(cx - 0.5f), ey = cy - vp_o0(cy - 0.5f);
            d0 = wd[i] * wd[i] * (ex * ex + ey * ey) / wmean;
        }
        f[i] = f2bf(a);
        f[16 + i] = f2bf(cx);
        f[32 + i] = f2bf(cy);
        f[48 + i] = f2bf(d0);
    }
}

// features along the rank-0 walk (kind VP_FEAT_RANK0_WALK): the centres c_i
// of the path that takes the nearest box point b_i at every level (the same
// float32 walk as the search's rank-0 path), and per level
//   [i]     W_ii / mean W_jj
//   [16+i]  Re (c_i - b_i),  [32+i]  Im (c_i - b_i)
//   [48+i]  W_ii^2 (d1_i - d0_i) / mean W_jj^2, d0 / d1 the squared distances
//           of c_i to its nearest and second-nearest box points (the PED cost,
//           in units of tau^2, of taking rank 1 instead of rank 0 at level i)
// Four lanes per vector (lane q: levels q, q + 4, q + 8, q + 12), sixteen
// vectors per wave: every lane keeps its levels' residuals in registers, the
// lane of level k decides b_k and hands it to the other lanes of its vector,
// which update their residuals below k; each lane writes its levels' four
// features.  The operations of each level (and the mean weights, summed in
// level order) are exactly those of a one-thread-per-vector walk, with a chain
// N steps long and four times the lanes in flight.
constexpr int kFeatLPV = 4;                 // lanes per vector
constexpr int kFeatVPB = 256 / kFeatLPV;    // vectors per 256-thread workgroup

template <int N>
__global__ __launch_bounds__(256) void k_features_walk(const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                                       const float2 *__restrict__ s, float tau, int n_sc, int n_sym,
                                                       uint16_t *__restrict__ feat) {
    constexpr int T = (N + kFeatLPV - 1) / kFeatLPV;   // levels per lane
    __shared__ float s_wd[kFeatVPB][16];
    constexpr int NP = VP_PACKED(N);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const int vl = threadIdx.x / kFeatLPV, q = threadIdx.x % kFeatLPV;
    const size_t v0 = (size_t)blockIdx.x * kFeatVPB + vl;
    const bool live = v0 < n_vec;
    const size_t v = live ? v0 : n_vec - 1;   // dead lanes shadow the last vector (no writes)
    const int sc = (int)(v / n_sym);
    const float2 *Wc = W + (size_t)sc * NP;
    const uint8_t *pm = perm + (size_t)sc * N;
    const int src0 = (threadIdx.x & 63) & ~(kFeatLPV - 1);   // lane of level 0 of this vector, within the wave
    float wdv[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int i = q + kFeatLPV * t;
        wdv[t] = i < N ? Wc[vp_pidx(N, i < N ? i : 0, i < N ? i : 0)].x : 0.f;
    }
#pragma unroll
    for (int t = 0; t < 16 / kFeatLPV; ++t) s_wd[vl][q + kFeatLPV * t] = t < T ? wdv[t < T ? t : 0] : 0.f;
    __syncthreads();
    float mean = 0.f, wmean = 0.f;   // in level order, as a sequential loop forms them
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float w = s_wd[vl][j];
        mean += w;
        wmean += w * w;
    }
    mean /= N;
    wmean /= N;
    const float wd0 = s_wd[vl][0];
    const bool ok = (wd0 > 0.f) && isfinite(wd0) && (mean > 0.f) && isfinite(mean) && isfinite(wmean);
    uint16_t *f = feat + v * 64;
    if (!ok) {
        if (live)
#pragma unroll
            for (int t = 0; t < 16 / kFeatLPV; ++t) {
                const int i = q + kFeatLPV * t;
                f[i] = f[16 + i] = f[32 + i] = f[48 + i] = 0;
            }
        return;   // the same for all lanes of the vector
    }
    const float inv_tau = 1.0f / tau;
    float2 r[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int i = q + kFeatLPV * t;
        float re = 0.f, im = 0.f;
        if (i < N) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (j <= i) {
                    const float2 w = Wc[vp_pidx(N, i, j)];
                    const int u = pm[j] < N ? pm[j] : N - 1;
                    const float2 x = s[(size_t)u * n_vec + v];
                    re = fmaf(w.x, x.x, fmaf(-w.y, x.y, re));
                    im = fmaf(w.x, x.y, fmaf(w.y, x.x, im));
                }
            }
        }
        r[t] = make_float2(re * inv_tau, im * inv_tau);
    }
    float fa[T], fx[T], fy[T], fd[T];
#pragma unroll
    for (int t = 0; t < T; ++t) fa[t] = fx[t] = fy[t] = fd[t] = 0.f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        constexpr int L = kFeatLPV;
        const int tk = k / L;
        // level k's lane: the centre as the search's walk forms it
        // (cp = c - 1/2 in one fma), its nearest and second-nearest box points
        float a = 0.f, b = 0.f;
        if (q == k % L) {
            const float wdk = wdv[tk];
            const float nlinv = -(1.0f / wdk);
            const float cpx = fmaf(r[tk].x, nlinv, -0.5f), cpy = fmaf(r[tk].y, nlinv, -0.5f);
            const float cx = r[tk].x * nlinv, cy = r[tk].y * nlinv;
            float a1, b1;
            vp_demap0(cpx, cpy, a, b);
            vp_demap1(cpx, cpy, cx, cy, 1, a1, b1);
            const float ex = cx - a, ey = cy - b;
            const float gx = cx - a1, gy = cy - b1;
            const float d0 = ex * ex + ey * ey, d1 = gx * gx + gy * gy;
            fa[tk] = wdk / mean;
            fx[tk] = ex;
            fy[tk] = ey;
            fd[tk] = wdk * wdk * (d1 - d0) / wmean;
        }
        a = __shfl(a, src0 + k % L);
        b = __shfl(b, src0 + k % L);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int i = q + L * t;
            if (i > k && i < N) {
                const float2 w = Wc[vp_pidx(N, i, k)];
                r[t].x = fmaf(w.x, a, fmaf(-w.y, b, r[t].x));
                r[t].y = fmaf(w.x, b, fmaf(w.y, a, r[t].y));
            }
        }
    }
    if (live)
#pragma unroll
        for (int t = 0; t < 16 / kFeatLPV; ++t) {
            const int i = q + kFeatLPV * t;
            f[i] = f2bf(t < T ? fa[t < T ? t : 0] : 0.f);
            f[16 + i] = f2bf(t < T ? fx[t < T ? t : 0] : 0.f);
            f[32 + i] = f2bf(t < T ? fy[t < T ? t : 0] : 0.f);
            f[48 + i] = f2bf(t < T ? fd[t < T ? t : 0] : 0.f);
        }
}

// ---------------------------------------------------------------------------
// ranks of a given perturbation along the tree (labels): at each level the
// rank r with DEMAP(c_i, r) == l_i, the same DEMAP the search uses; 15 if the
// symbol is not in the box.  Walks with the search's arithmetic.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(64) void k_ranks(const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                              const float2 *__restrict__ s, float tau, int n_sc, int n_sym,
                                              const int8_t *__restrict__ l, uint8_t *__restrict__ ranks) {
    constexpr int NP = VP_PACKED(N);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t v = (size_t)blockIdx.x * 64 + threadIdx.x;
    if (v >= n_vec) return;
    const int sc = (int)(v / n_sym);
    const float2 *Wc = W + (size_t)sc * NP;
    const uint8_t *pm = perm + (size_t)sc * N;
    const float inv_tau = 1.0f / tau;
    float2 r[N];
    for (int i = 0; i < N; ++i) {
        float re = 0.f, im = 0.f;
        for (int j = 0; j <= i; ++j) {
            const float2 w = Wc[vp_pidx(N, i, j)];
            const int u = pm[j] < N ? pm[j] : N - 1;
            const float2 x = s[(size_t)u * n_vec + v];
            re = fmaf(w.x, x.x, fmaf(-w.y, x.y, re));
            im = fmaf(w.x, x.y, fmaf(w.y, x.x, im));
        }
        r[i] = make_float2(re * inv_tau, im * inv_tau);
    }
    for (int i = 0; i < N; ++i) {
        const int u = pm[i] < N ? pm[i] : N - 1;
        const int8_t *li = l + ((size_t)u * n_vec + v) * 2;
        const float la = (float)li[0], lb = (float)li[1];
        const float wii = Wc[vp_pidx(N, i, i)].x;
        const float nlinv = -(1.0f / wii);
        const float cpx = fmaf(r[i].x, nlinv, -0.5f), cpy = fmaf(r[i].y, nlinv, -0.5f);   // as the search's walk
        const float cx = r[i].x * nlinv, cy = r[i].y * nlinv;
        int rk = 15;
        for (int q = 8; q >= 0; --q) {
            float a, b;
            vp_demapN(cpx, cpy, cx, cy, q, VP_DEMAP_LUT, a, b);
            if (a == la && b == lb) rk = q;
        }
        ranks[v * N + i] = (uint8_t)rk;
        for (int m = i + 1; m < N; ++m) {
            const float2 w = Wc[vp_pidx(N, m, i)];
            r[m].x = fmaf(w.x, la, fmaf(-w.y, lb, r[m].x));
            r[m].y = fmaf(w.x, lb, fmaf(w.y, la, r[m].y));
        }
    }
}

// ---------------------------------------------------------------------------
// top-64 of each row of fp32 scores [rows][C] (64 <= C <= 4096): columns
// ordered by (score desc, column asc) in the IEEE total order, and the softmax
// mass of the selected 64.  One wave per row; lane L keeps the columns
// 256 q + 4 L + e (q < 16, e < 4) as order-preserving keys in registers
// (absent columns: key 0, below every present one that the searches try).
//   bound:   the 64th largest of the 128 keys made of every lane's two largest
//            is at most the row's 64th largest key, since those are 128
//            distinct entries; a bitwise search with wave ballots finds it
//   select:  the keys at or above the bound (64 to 128 in the usual case) are
//            packed as (key, ~column), so that one unsigned order is the
//            selection order, and each is ranked against all the others
//   others:  (short rows, more than 128 candidates, ties over many columns)
//            the exact 64th key by a bitwise search over all keys, the keys
//            above it and the equal keys of smallest column, ranked the same way
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t okey(float f) {   // larger float -> larger key
    const uint32_t u = __float_as_uint(f);
    return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k) {   // inverse of okey
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

constexpr int kTopQ = 16;          // float4 column blocks per lane
constexpr int kTopV = 4 * kTopQ;   // keys per lane
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t x) {
    return wave_reduce(x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ __forceinline__ int ballot_count(bool p) { return __popcll(__ballot(p)); }

__device__ __forceinline__ uint64_t topk_pack(uint32_t key, uint32_t ncol) {
    return ((uint64_t)key << 32) | ncol;
}

// candidate p: key and ~column in two arrays, so that the registers holding
// the keys need not pair with a column register
struct TopkCand {
    uint32_t key[128];
    uint32_t ncol[128];
    __device__ __forceinline__ void put(uint32_t p, uint32_t k, uint32_t nc) {
        key[p] = k;
        ncol[p] = nc;
    }
    __device__ __forceinline__ uint64_t get(int p) const { return topk_pack(key[p], ncol[p]); }
};

template <bool FULL, bool VEC4>
__global__ __launch_bounds__(64) void k_topk64(const float *__restrict__ S, int C, int32_t *__restrict__ idx_out,
                                               float *__restrict__ mass_out) {
    __shared__ TopkCand cand;
    __shared__ uint32_t sel[64];
    const int row = blockIdx.x, lane = threadIdx.x;
    const float *x = S + (size_t)row * C;
    const uint32_t ncol0 = ~(uint32_t)(4 * lane);   // ~column of value 0; value i = 4 q + e is ncol0 - (256 q + e)
    uint32_t key[kTopV];
#pragma unroll
    for (int q = 0; q < kTopQ; ++q) {
        const int c = 256 * q + 4 * lane;
        if (VEC4) {
            float4 v = make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
            if (FULL || c < C) v = *reinterpret_cast<const float4 *>(x + c);
            key[4 * q + 0] = __float_as_uint(v.x);
            key[4 * q + 1] = __float_as_uint(v.y);
            key[4 * q + 2] = __float_as_uint(v.z);
            key[4 * q + 3] = __float_as_uint(v.w);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) key[4 * q + e] = __float_as_uint((FULL || c + e < C) ? x[c + e] : -INFINITY);
        }
    }
    // softmax denominator around the lane's maximum, rescaled to the row's
    float lmx = -INFINITY;
#pragma unroll
    for (int i = 0; i < kTopV; ++i) lmx = fmaxf(lmx, __uint_as_float(key[i]));
    const float mx = wave_max_f(lmx);
    float sall = 0.f;
    if (mass_out) {
        const float off = -lmx * kLog2e;
        float se = 0.f;
#pragma unroll
        for (int i = 0; i < kTopV; ++i) se += __builtin_amdgcn_exp2f(fmaf(__uint_as_float(key[i]), kLog2e, off));
        se = (lmx > -INFINITY) ? se * __builtin_amdgcn_exp2f((lmx - mx) * kLog2e) : 0.f;
        sall = wave_sum_f(se);
    }
    // keys, and every lane's two largest
    uint32_t m1 = 0, m2 = 0;
#pragma unroll
    for (int i = 0; i < kTopV; ++i) {
        uint32_t k = okey(__uint_as_float(key[i]));
        if (!FULL && 256 * (i >> 2) + 4 * lane + (i & 3) >= C) k = 0u;
        key[i] = k;
        m2 = max(m2, min(m1, k));
        m1 = max(m1, k);
    }
    uint32_t T = 0;
    for (int b = 31; b >= 0; --b) {
        const uint32_t t = T | (1u << b);
        if (ballot_count(m1 >= t) + ballot_count(m2 >= t) >= 64) T = t;
    }
    uint32_t cl = 0;
#pragma unroll
    for (int i = 0; i < kTopV; ++i) cl += key[i] >= T ? 1u : 0u;
    uint32_t incl = wave_scan_incl(cl);
    int n = __builtin_amdgcn_readlane((int)incl, 63);
    if (T >= 1u && n <= 128) {
        uint32_t pos = incl - cl;
#pragma unroll
        for (int i = 0; i < kTopV; ++i)
            if (key[i] >= T) cand.put(pos++, key[i], ncol0 - (uint32_t)(256 * (i >> 2) + (i & 3)));
    } else {
        // the exact 64th largest key; every threshold tried is at least 1,
        // so absent columns never count
        T = 0;
        for (int b = 31; b >= 0; --b) {
            const uint32_t t = T | (1u << b);
            uint32_t c = 0;
#pragma unroll
            for (int i = 0; i < kTopV; ++i) c += key[i] >= t ? 1u : 0u;
            if (wave_sum_u(c) >= 64u) T = t;
        }
        uint32_t cg = 0;
#pragma unroll
        for (int i = 0; i < kTopV; ++i) cg += key[i] > T ? 1u : 0u;
        incl = wave_scan_incl(cg);
        uint32_t run = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);   // fewer than 64
        uint32_t pos = incl - cg;
#pragma unroll
        for (int i = 0; i < kTopV; ++i)
            if (key[i] > T) cand.put(pos++, key[i], ncol0 - (uint32_t)(256 * (i >> 2) + (i & 3)));
        // keys equal to T by increasing column: block q holds columns
        // [256 q, 256 q + 256) in (lane, e) order
#pragma unroll
        for (int q = 0; q < kTopQ; ++q) {
            if (run < 64u) {
                uint32_t ce = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) ce += (key[4 * q + e] == T && 256 * q + 4 * lane + e < C) ? 1u : 0u;
                const uint32_t ie = wave_scan_incl(ce);
                uint32_t p = run + ie - ce;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (key[4 * q + e] == T && 256 * q + 4 * lane + e < C) {
                        if (p < 64u) cand.put(p, T, ncol0 - (uint32_t)(256 * q + e));
                        ++p;
                    }
                run += (uint32_t)__builtin_amdgcn_readlane((int)ie, 63);
            }
        }
        n = 64;
    }
    __syncthreads();   // one wave: orders the candidate writes before the reads
    const uint64_t a = lane < n ? cand.get(lane) : 0ull;
    const uint64_t b = lane + 64 < n ? cand.get(lane + 64) : 0ull;
    uint32_t ra = 0, rb = 0;
    if (n <= 64) {
        for (int j = 0; j < n; ++j) ra += cand.get(j) > a ? 1u : 0u;
    } else {
        for (int j = 0; j < n; ++j) {
            const uint64_t v = cand.get(j);
            ra += v > a ? 1u : 0u;
            rb += v > b ? 1u : 0u;
        }
    }
    float ssel = 0.f;
    const float off = -mx * kLog2e;
    if (lane < n && ra < 64u) {
        sel[ra] = ~(uint32_t)a;
        ssel += __builtin_amdgcn_exp2f(fmaf(key_value((uint32_t)(a >> 32)), kLog2e, off));
    }
    if (lane + 64 < n && rb < 64u) {
        sel[rb] = ~(uint32_t)b;
        ssel += __builtin_amdgcn_exp2f(fmaf(key_value((uint32_t)(b >> 32)), kLog2e, off));
    }
    __syncthreads();
    idx_out[(size_t)row * 64 + lane] = (int32_t)sel[lane];
    if (mass_out) {
        ssel = wave_sum_f(ssel);
        if (lane == 0) mass_out[row] = sall > 0.f ? ssel / sall : 0.f;
    }
}

// ---------------------------------------------------------------------------
// softmax cross-entropy over rows of fp32 logits with integer labels (-1 =
// ignored row): loss per row (fp32) and d loss / d logits = (p - onehot) *
// scale, written in bf16 (scale = 1 / number of labelled rows).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_softmax_ce(const float *__restrict__ Z, int rows, int C,
                                                    const int32_t *__restrict__ label, float scale,
                                                    float *__restrict__ loss, uint16_t *__restrict__ dZ) {
    __shared__ float red[4];
    const int row = blockIdx.x, t = threadIdx.x;
    const float *z = Z + (size_t)row * C;
    const int y = label[row];
    float mx = -INFINITY;
    for (int c = t; c < C; c += 256) mx = fmaxf(mx, z[c]);
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((t & 63) == 0) red[t >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    float se = 0.f;
    for (int c = t; c < C; c += 256) se += __expf(z[c] - mx);
    for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off);
    if ((t & 63) == 0) red[t >> 6] = se;
    __syncthreads();
    se = red[0] + red[1] + red[2] + red[3];
    const float lse = mx + __logf(se);
    const bool use = y >= 0 && y < C;
    for (int c = t; c < C; c += 256) {
        const float p = __expf(z[c] - lse);
        dZ[(size_t)row * C + c] = f2bf(use ? (p - (c == y ? 1.f : 0.f)) * scale : 0.f);
    }
    if (t == 0) loss[row] = use ? lse - z[y] : 0.f;
}

// column sums of a bf16 matrix [rows][cols] -> fp32 [cols]
__global__ __launch_bounds__(256) void k_colsum(const uint16_t *__restrict__ X, int rows, int cols,
                                                float *__restrict__ out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    float acc = 0.f;
    for (int r = 0; r < rows; ++r) acc += bf2f(X[(size_t)r * cols + c]);
    out[c] = acc;
}

// per-vector path table: the Kl proposed vocabulary entries, then the first
// Kf paths of the subcarrier's fixed (MoP) table.  One thread per table row;
// 16-level rows move as one 16-byte load and store.
__global__ __launch_bounds__(256) void k_learned_table(const uint8_t *__restrict__ vocab, int V, int N,
                                                       const int32_t *__restrict__ top, int Kl,
                                                       const uint8_t *__restrict__ fixed, int Kfix_stride,
                                                       int Kf, int n_sc, int n_sym, uint8_t *__restrict__ table) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    const int Kt = Kl + Kf;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;   // row (vector, path)
    if (e >= n_vec * Kt) return;
    const size_t v = e / Kt;
    const int k = (int)(e % Kt);
    const uint8_t *src;
    if (k < Kl) {
        int id = top[v * Kl + k];
        id = id < 0 ? 0 : (id >= V ? V - 1 : id);
        src = vocab + (size_t)id * N;
    } else {
        const int sc = (int)(v / n_sym);
        src = fixed + (size_t)sc * Kfix_stride * N + (size_t)(k - Kl) * N;
    }
    uint8_t *dst = table + e * N;
    if (N == 16 && ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0) {
        *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
    } else {
        for (int i = 0; i < N; ++i) dst[i] = src[i];
    }
}

}  // namespace

int launch_gemm(int M, int N, int K, const uint16_t *A, long long lda, int transA, const uint16_t *B, long long ldb,
                int transB, float *Cf, uint16_t *Cb, long long ldc, const float *bias, int relu,
                const uint16_t *mask, long long ldm, float alpha, hipStream_t st) {
    if (M == 0 || N == 0) return VP_OK;
    const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM));
    // 16-byte loads need 16-byte aligned rows
    const int va = ((reinterpret_cast<uintptr_t>(A) & 15) == 0) && (lda % 8 == 0);
    const int vb = ((reinterpret_cast<uintptr_t>(B) & 15) == 0) && (ldb % 8 == 0);
#define VP_G(ta, tb)                                                                                              \
    hipLaunchKernelGGL((k_gemm<ta, tb>), grid, dim3(GT), 0, st, M, N, K, A, lda, B, ldb, va, vb, Cf, Cb, ldc, bias, \
                       relu, mask, ldm, alpha)
    if (!transA && !transB) VP_G(false, false);
    else if (!transA && transB) VP_G(false, true);
    else if (transA && !transB) VP_G(true, false);
    else VP_G(true, true);
#undef VP_G
    return launch_status();
}

int launch_features(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym, int N,
                    unsigned kind, uint16_t *feat, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    if (n_vec == 0) return VP_OK;
    const dim3 g((unsigned)((n_vec + 63) / 64));
    switch (N) {
#define VP_CASE(n)                                                                                           \
    case n:                                                                                                  \
        if (kind == VP_FEAT_RANK0_WALK)                                                                      \
            hipLaunchKernelGGL(k_features_walk<n>, dim3((unsigned)((n_vec + kFeatVPB - 1) / kFeatVPB)),        \
                               dim3(kFeatLPV * kFeatVPB), 0, st, W, perm, s, tau, n_sc, n_sym, feat);      \
        else                                                                                                 \
            hipLaunchKernelGGL(k_features<n>, g, dim3(64), 0, st, W, perm, s, tau, n_sc, n_sym, feat);      \
        break;
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: return VP_EUNSUPPORTED;
    }
    return launch_status();
}

int launch_ranks(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym, int N,
                 const int8_t *l, uint8_t *ranks, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    if (n_vec == 0) return VP_OK;
    const dim3 g((unsigned)((n_vec + 63) / 64));
    switch (N) {
#define VP_CASE(n) \
    case n: hipLaunchKernelGGL(k_ranks<n>, g, dim3(64), 0, st, W, perm, s, tau, n_sc, n_sym, l, ranks); break;
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: return VP_EUNSUPPORTED;
    }
    return launch_status();
}

int launch_topk64(const float *S, int rows, int C, int32_t *idx, float *mass, hipStream_t st) {
    if (rows == 0) return VP_OK;
    const bool full = C == 64 * kTopV, vec4 = (C & 3) == 0 && ((uintptr_t)S & 15) == 0;
    auto k = full ? (vec4 ? k_topk64<true, true> : k_topk64<true, false>)
                  : (vec4 ? k_topk64<false, true> : k_topk64<false, false>);
    hipLaunchKernelGGL(k, dim3(rows), dim3(64), 0, st, S, C, idx, mass);
    return launch_status();
}

int launch_softmax_ce(const float *Z, int rows, int C, const int32_t *label, float scale, float *loss,
                      uint16_t *dZ, hipStream_t st) {
    if (rows == 0) return VP_OK;
    hipLaunchKernelGGL(k_softmax_ce, dim3(rows), dim3(256), 0, st, Z, rows, C, label, scale, loss, dZ);
    return launch_status();
}

int launch_colsum(const uint16_t *X, int rows, int cols, float *out, hipStream_t st) {
    if (cols == 0) return VP_OK;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, st, X, rows, cols, out);
    return launch_status();
}

int launch_learned_table(const uint8_t *vocab, int V, int N, const int32_t *top, int Kl, const uint8_t *fixed,
                         int Kfix, int Kf, int n_sc, int n_sym, uint8_t *table, hipStream_t st) {
    const size_t total = (size_t)n_sc * n_sym * (Kl + Kf);   // table rows
    if (total == 0) return VP_OK;
    hipLaunchKernelGGL(k_learned_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, vocab, V, N, top,
                       Kl, fixed, Kfix, Kf, n_sc, n_sym, table);
    return launch_status();
}

}  // namespace vp
