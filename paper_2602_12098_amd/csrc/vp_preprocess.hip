// Per-subcarrier regularised sorted factorisation (Sec. III-A-1, Alg. 1,
// eq:invr) and the RZF precoder G = H^H (H H^H + alpha I)^{-1} (Sec. II-A).
//
// One wave (a 64-thread workgroup) per subcarrier, so that no step needs a
// workgroup barrier: the N x N Gram matrix lives in LDS, each lane updating
// up to four entries, and the channel rows are staged in dynamically sized
// LDS (N rows of an odd stride >= M), which keeps a workgroup at about 9 KiB
// for 16 x 16 and lets a CU hold all its subcarriers at once.  The kernel is a
// chain of dependent steps per wave with every subcarrier's wave resident
// from the start, so its time is that chain's length: LDS accesses are laid
// out free of bank conflicts, the forward substitution runs on all 64 lanes,
// and the pivot search reads registers.  Alg. 1's sorted Gram-Schmidt on the rows of
// [H, lambda I] is carried out in its equivalent Cholesky form: the squared
// row norms that Alg. 1 downdates are exactly the Schur-complement diagonals
// of A = H H^H + lambda^2 I, so the pivot is the smallest remaining one and the
// column entries are the projections R_ji.  W = Lbar^{-1} is then formed by
// forward substitution (eq:invr's implicit inverse Q2/lambda needs the extended
// Q, which this form never builds, and is undefined for lambda = 0).
#include "vp_internal.hpp"

namespace vp {
namespace {

constexpr int kT = 64;                          // one wave per subcarrier
constexpr int kPer = kMaxN * kMaxN / kT;        // Gram entries per lane

// Value of the partner lane within a row of 16 lanes, for the four steps of a
// row reduction: xor 1, xor 2 (quad permutations), then the half-row and the
// row mirror (each pairs the two halves reduced so far).
__device__ __forceinline__ int row_xchg_i(int v, int step) {
    switch (step) {
        case 0: return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
        case 1: return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
        case 2: return __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
        default: return __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);  // row_mirror
    }
}

__device__ __forceinline__ float row_xchg_f(float v, int step) {
    return __int_as_float(row_xchg_i(__float_as_int(v), step));
}

// Row stride (in entries) of the channel staged in LDS: odd, so that the 16
// rows a Gram step reads at once (one column k of every row j) fall in
// distinct LDS banks instead of all in one for M a multiple of 16.
__host__ __device__ constexpr int h_stride(int M) { return M | 1; }

// W = Lbar^{-1} by forward substitution, W_rc = (delta_rc - sum_{c<=k<r}
// Lbar_rk W_kc) / Lbar_rr, row r of Lbar being user perm[r]'s factor row
// Lc[perm[r]][.], with the whole wave: lane c + 16 s holds W_rc for the rows
// r = s + 4 q (q = 0..3) in registers and the steps k = 0..N-1 sweep the
// rows: row k is complete after step k-1, is scaled by 1/Lbar_kk (the
// reciprocal the factorisation formed, which also makes W_kk exactly that
// reciprocal) and is handed to every lane of its column, which subtracts
// Lbar_rk W_kc from its rows r > k.  Each W_rc takes the same operations in
// the same order as a row-by-row substitution (k ascending from c), but the
// chain of dependent steps is N long instead of N(N-1)/2.
template <int NN>
__device__ __forceinline__ void forward_all(const int *sperm, const float2 (*Lc)[kMaxN + 1], const float *linv,
                                            float2 (*Wl)[kMaxN + 1]) {
    static_assert(kMaxN == 16 && kT == 64, "lane c + 16 s holds rows s + 4 q of column c");
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, s = lane >> 4;
    float2 w[4];
    int ur[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = s + 4 * q;
        w[q] = make_float2(r == c ? 1.f : 0.f, 0.f);
        ur[q] = r < NN ? sperm[r] : 0;
    }
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        const int qk = k >> 2, sk = k & 3;
        if (s == sk) {   // row k is complete: W_kc = acc / Lbar_kk (0 above the diagonal)
            const float di = linv[k];
            w[qk] = (k < c) ? make_float2(0.f, 0.f) : make_float2(w[qk].x * di, w[qk].y * di);
        }
        // W_kc from lane c + 16 sk, register qk (the same register in every lane)
        const int src = c + 16 * sk;
        const float2 b = make_float2(__shfl(w[qk].x, src), __shfl(w[qk].y, src));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = s + 4 * q;
            if (r > k && r < NN && k >= c) {   // - Lbar_rk W_kc
                const float2 a = Lc[ur[q]][k];
                w[q].x = fmaf(-a.x, b.x, fmaf(a.y, b.y, w[q].x));
                w[q].y = fmaf(-a.x, b.y, fmaf(-a.y, b.x, w[q].y));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = s + 4 * q;
        if (r < NN && c < NN) Wl[r][c] = w[q];
    }
}

// One subcarrier: Hs its [N][M] channel; Wsc, w2sc, permsc, Gsc (or NULL),
// status_sc its outputs; sH: LDS for N rows of h_stride(M) channel entries.
// sorted = false: no pivoting, users in their own order (the unsorted
// factorisation the sorted one is compared with in Sec. III-B).
__device__ __forceinline__ void preprocess_one(const float2 *__restrict__ Hs, int N, int M, float alpha,
                                               float2 *__restrict__ Wsc, float *__restrict__ w2sc,
                                               uint8_t *__restrict__ permsc, float2 *__restrict__ Gsc,
                                               int32_t *__restrict__ status_sc, float2 *sH, bool sorted = true) {
    __shared__ float2 S[kMaxN][kMaxN + 1];    // Schur complement, user indices; later A^{-1}
    __shared__ float2 Lc[kMaxN][kMaxN + 1];   // Lc[u][k]: user u's entry of factor column k
    __shared__ float2 Wl[kMaxN][kMaxN + 1];   // W = Lbar^{-1}, search order
    __shared__ int sperm[kMaxN];
    __shared__ float slinv[kMaxN];            // 1 / Lbar_kk of step k

    const int t = threadIdx.x;
    const int NM = N * M;
    const int NN = N * N;
    const int HS = h_stride(M);

    int bad = 0;
    for (int idx = t; idx < NM; idx += kT) {
        const float2 h = Hs[idx];
        sH[(idx / M) * HS + idx % M] = h;
        bad |= !(isfinite(h.x) && isfinite(h.y));
    }
    int st = __any(bad) ? VP_STATUS_NONFINITE : VP_STATUS_OK;   // the same in every lane
    __syncthreads();

    // this lane's Gram entries e = t + q kT, (i, j) = (e / N, e % N)
    int ei[kPer], ej[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int e = t + q * kT;
        ei[q] = e < NN ? e / N : kMaxN;
        ej[q] = e < NN ? e % N : 0;
    }
    float2 sv[kPer];   // this lane's entries of S, kept in registers (only this lane writes them)
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int i = ei[q], j = ej[q];
        sv[q] = make_float2(0.f, 0.f);
        if (i < N) {
            float re = 0.f, im = 0.f;
#pragma unroll 8
            for (int k = 0; k < M; ++k) {   // A_ij = sum_k H_ik conj(H_jk)
                const float2 a = sH[i * HS + k], b = sH[j * HS + k];
                re = fmaf(a.x, b.x, fmaf(a.y, b.y, re));
                im = fmaf(a.y, b.x, fmaf(-a.x, b.y, im));
            }
            if (i == j) {
                re += alpha;
                im = 0.f;
            }
            sv[q] = make_float2(re, im);
            S[i][j] = sv[q];
        }
    }
    __syncthreads();
    const bool same_j = (kT % N) == 0;   // then all of a lane's entries share their column j

    // Pivot floor: N * eps32 * max_u A_uu.
    float floor_ = 0.f;
    for (int u = 0; u < N; ++u) floor_ = fmaxf(floor_, S[u][u].x);
    floor_ *= (float)N * 1.1920929e-7f;

    // Column p of S is only read during step p.  The workgroup is one wave,
    // so the barrier that ends a step costs only the wait for its LDS writes.
    uint32_t rem = (N >= 32) ? ~0u : (1u << N) - 1u;   // users not yet pivoted (the same in every lane)
    // lane t < N keeps user t's Schur diagonal in a register, updated with the
    // very operations of the lane that holds S_tt, so that a step's pivot
    // search needs no LDS read
    float dg = t < N ? S[t][t].x : 0.f;
    for (int step = 0; step < N; ++step) {
        // smallest remaining Schur diagonal, ties to the smaller user, over the
        // 16 lanes of row 0 (N <= 16); a NaN diagonal (only from non-finite or
        // overflowing input, which fails the subcarrier) never beats a number
        // (the minimum over the row by four DPP moves -- fminf returns the
        // number when one operand is NaN -- then the smallest candidate lane
        // that holds it; with only NaN left, the first candidate, whose NaN
        // then fails the subcarrier below)
        const bool cand = (t < N) && ((rem >> t) & 1u);
        float d = cand ? dg : __int_as_float(0x7f800000);
#pragma unroll
        for (int s = 0; s < 4; ++s) d = fminf(d, row_xchg_f(d, s));
        d = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(d)));
        const unsigned long long at_min = __ballot(cand && dg == d);
        int p = (int)__builtin_ctzll(at_min ? at_min : __ballot(cand));
        d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dg), p));
        if (!sorted) {   // the next user in order, whatever its Schur diagonal
            p = step;
            d = __shfl(dg, step);
        }
        if (!(d > floor_) && st == VP_STATUS_OK) st = VP_STATUS_NOT_PD;
        if (t == 0) sperm[step] = p;
        rem &= ~(1u << p);
        const float lpp = sqrtf(fmaxf(d, 0.f));
        const float inv = lpp > 0.f ? 1.0f / lpp : 0.f;   // L_up = S_up / L_pp
        if (t == 0) slinv[step] = inv;
        // every read of the step first (rows beyond N read row 0: discarded),
        // so that they overlap, then the arithmetic, then the writes
        const int tr = t < N ? t : 0;
        const float2 st_ = S[tr][p];
        float2 si[kPer], sj[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) si[q] = S[ei[q] < N ? ei[q] : 0][p];
        if (same_j) {
            const float2 x = S[ej[0]][p];
#pragma unroll
            for (int q = 0; q < kPer; ++q) sj[q] = x;
        } else {
#pragma unroll
            for (int q = 0; q < kPer; ++q) sj[q] = S[ej[q]][p];
        }
        if (t < N) {
            if (t == p) {
                Lc[t][step] = make_float2(lpp, 0.f);
            } else if ((rem >> t) & 1u) {
                const float2 a = make_float2(st_.x * inv, st_.y * inv);
                Lc[t][step] = a;
                dg = fmaf(-a.x, a.x, fmaf(-a.y, a.y, dg));   // S_tt -= |L_t|^2, as the update below forms it
            }
        }
        // S_ij -= L_i conj(L_j) on every entry: an entry of a pivoted row or
        // column becomes garbage, but such entries only ever feed others of
        // their kind (column p is read at step p for the rows of the entries
        // it updates), so no remaining entry, L column or pivot sees them
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int i = ei[q], j = ej[q];
            const float2 a = make_float2(si[q].x * inv, si[q].y * inv), b = make_float2(sj[q].x * inv, sj[q].y * inv);
            float2 v = sv[q];
            v.x = fmaf(-a.x, b.x, fmaf(-a.y, b.y, v.x));
            v.y = fmaf(-a.y, b.x, fmaf(a.x, b.y, v.y));
            sv[q] = v;
            if (i < N) S[i][j] = v;
        }
        __syncthreads();
    }

    const int NP = VP_PACKED(N);
    if (st != VP_STATUS_OK) {
        const float qnan = __int_as_float(0x7fc00000);
        for (int idx = t; idx < NP; idx += kT) Wsc[idx] = make_float2(qnan, qnan);
        if (t < N) {
            w2sc[t] = __int_as_float(0x7f800000);
            permsc[t] = (uint8_t)t;
        }
        if (Gsc)
            for (int idx = t; idx < NM; idx += kT) Gsc[idx] = make_float2(qnan, qnan);
        if (t == 0) *status_sc = st;
        return;
    }

    // W = Lbar^{-1} (forward substitution by the whole wave)
    switch (N) {
#define VP_CASE(n) \
    case n: forward_all<n>(sperm, Lc, slinv, Wl); break;
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: break;
    }
    __syncthreads();

    // A^{-1} = P^T W^H W P:  (W^H W)_kl = sum_{r >= max(k,l)} conj(W_rk) W_rl, into S
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int i = ei[q], j = ej[q];
        if (i < N) {
            float re = 0.f, im = 0.f;
#pragma unroll 4
            for (int r = (i > j ? i : j); r < N; ++r) {
                const float2 a = Wl[r][i], b = Wl[r][j];
                re = fmaf(a.x, b.x, fmaf(a.y, b.y, re));
                im = fmaf(a.x, b.y, fmaf(-a.y, b.x, im));
            }
            S[sperm[i]][sperm[j]] = make_float2(re, im);
        }
    }
    __syncthreads();

#pragma unroll
    for (int q = 0; q < kPer; ++q) {   // this lane's entries (i, j) of W, i >= j, packed column-major lower
        const int i = ei[q], j = ej[q];
        if (i < N && i >= j) {
            float2 v = Wl[i][j];
            if (i == j) v.y = 0.f;
            Wsc[j * N - (j * (j - 1)) / 2 + (i - j)] = v;
        }
    }
    if (t < N) {
        const float dg = Wl[t][t].x;
        w2sc[t] = dg * dg;
        permsc[t] = (uint8_t)sperm[t];
    }
    if (Gsc) {   // G[m][u] = sum_v conj(H_vm) Ainv_vu
        // (m, u) of idx = t + kT it, stepped without a division per entry
        const int dm = kT / N, du = kT % N;
        int m = t / N, u = t % N;
        for (int idx = t; idx < NM; idx += kT) {
            float re = 0.f, im = 0.f;
#pragma unroll 8
            for (int v = 0; v < N; ++v) {
                const float2 h = sH[v * HS + m], a = S[v][u];
                re = fmaf(h.x, a.x, fmaf(h.y, a.y, re));
                im = fmaf(h.x, a.y, fmaf(-h.y, a.x, im));
            }
            Gsc[idx] = make_float2(re, im);
            m += dm;
            u += du;
            if (u >= N) {
                u -= N;
                ++m;
            }
        }
    }
    if (t == 0) *status_sc = st;
}

__global__ __launch_bounds__(kT) void k_preprocess(const float2 *__restrict__ H, int N, int M, float alpha,
                                                   float2 *__restrict__ Wout, float *__restrict__ w2out,
                                                   uint8_t *__restrict__ perm_out, float2 *__restrict__ Gout,
                                                   int32_t *__restrict__ status_out, int sorted) {
    extern __shared__ float2 sH[];   // [N][h_stride(M)]
    const size_t sc = blockIdx.x;
    const size_t NM = (size_t)N * M;
    preprocess_one(H + sc * NM, N, M, alpha, Wout + sc * VP_PACKED(N), w2out + sc * N, perm_out + sc * N,
                   Gout ? Gout + sc * NM : nullptr, status_out + sc, sH, sorted != 0);
}

// Batched: one wave per subcarrier of any group.
__global__ __launch_bounds__(kT) void k_batch_preprocess(const BatchGroup *__restrict__ groups,
                                                         const int32_t *__restrict__ sc_group, int M,
                                                         const float2 *__restrict__ H, float2 *__restrict__ W,
                                                         float *__restrict__ w2, uint8_t *__restrict__ perm,
                                                         float2 *__restrict__ G, int32_t *__restrict__ status) {
    extern __shared__ float2 sH[];   // [kMaxN][h_stride(M)]
    const int sc = blockIdx.x;
    const BatchGroup g = groups[sc_group[sc]];
    const long long j = sc - g.sc0;
    const long long UM = (long long)g.U * M;
    preprocess_one(H + g.offH + j * UM, g.U, M, g.alpha, W + g.offW + j * VP_PACKED(g.U), w2 + g.offN + j * g.U,
                   perm + g.offN + j * g.U, G + g.offG + j * UM, status + sc, sH);
}

}  // namespace

int launch_batch_preprocess(const BatchGroup *groups, const int32_t *sc_group, int n_sc_total, int M,
                            const float2 *H, float2 *W, float *w2, uint8_t *perm, float2 *G, int32_t *status,
                            hipStream_t st) {
    if (n_sc_total == 0) return VP_OK;
    hipLaunchKernelGGL(k_batch_preprocess, dim3(n_sc_total), dim3(kT), (size_t)kMaxN * h_stride(M) * sizeof(float2), st, groups,
                       sc_group, M, H, W, w2, perm, G, status);
    return launch_status();
}

int launch_preprocess(const float2 *H, int n_sc, int N, int M, float alpha, float2 *W, float *w2,
                      uint8_t *perm, float2 *G, int32_t *status, hipStream_t st, bool sorted) {
    if (n_sc == 0) return VP_OK;
    hipLaunchKernelGGL(k_preprocess, dim3(n_sc), dim3(kT), (size_t)N * h_stride(M) * sizeof(float2), st, H, N, M, alpha, W, w2,
                       perm, G, status, sorted ? 1 : 0);
    return launch_status();
}

}  // namespace vp
