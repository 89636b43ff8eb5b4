// The path walk in 16-bit fixed point: an emulation of the accelerator's
// number format (Sec. V, "Precision and Numerical Accuracy": signed 16 bits
// with F = 8..13 fractional bits), to measure what the format costs in power.
//
// The walk's state is the level centre c_m = -r_m / (tau W_mm).  The child of
// level i moves every centre below it by V_mi l_i (V_mi = -W_mi / W_mm); the
// PED of level i is proportional to w_i |l_i - c_i|^2 with w_i = W_ii^2 over
// the subcarrier's largest W_jj^2.  Centres, V and w are signed 16-bit
// integers with F fractional bits, rounded to nearest (ties to even) and
// saturated; since l is a box point the step is a sum of +-V entries,
// saturated to 16 bits; squared distances use differences saturated to 16
// bits (< 2^31); the PED sum is exact in 64 bits.  Everything after
// vp_fx_quantize is integer arithmetic, so results are exact and
// reproducible.
//
// k_fx_quantize: one lane per vector (its centres) and per subcarrier entry.
// k_fx_search: one 256-thread workgroup per vector, one path per lane; each
// lane keeps its best (PED, path) key and the chosen offsets packed two bits
// per axis, and the workgroup's minimum key says which lane writes l.
#include "vp_device.hpp"
#include "vp_internal.hpp"

namespace vp {
namespace {

constexpr int kT = 256;
constexpr int kFxMin = -32768, kFxMax = 32767;

__device__ __forceinline__ int fx_sat(int x) { return x < kFxMin ? kFxMin : (x > kFxMax ? kFxMax : x); }

// Round to nearest (ties to even) and saturate; NaN becomes 0.
__device__ __forceinline__ int16_t fx_q(float x, float scale) {
    const float q = rintf(x * scale);
    if (!(q == q)) return 0;
    return (int16_t)(q < (float)kFxMin ? kFxMin : (q > (float)kFxMax ? kFxMax : (int)q));
}

// Index of V_mi (m > i) in the packed strictly-lower layout, row by row.
__device__ __forceinline__ int vidx(int m, int i) { return m * (m - 1) / 2 + i; }

template <int N>
__global__ __launch_bounds__(kT) void k_fx_quantize(const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                                    const float2 *__restrict__ s, const float *__restrict__ taus,
                                                    int n_sc, int n_sym, float scale, int16_t *__restrict__ c0,
                                                    int16_t *__restrict__ Vq, int16_t *__restrict__ wq) {
    constexpr int NP = VP_PACKED(N);
    constexpr int NV = N * (N - 1) / 2;
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t t = (size_t)blockIdx.x * kT + threadIdx.x;
    if (t < n_vec) {   // the vector's start centres
        const size_t v = t;
        const int sc = (int)(v / n_sym);
        const float2 *Wc = W + (size_t)sc * NP;
        const uint8_t *pm = perm + (size_t)sc * N;
        const float tau = taus[sc];
        for (int m = 0; m < N; ++m) {
            float re = 0.f, im = 0.f;
            for (int j = 0; j <= m; ++j) {
                const float2 w = Wc[vp_pidx(N, m, j)];
                const int u = pm[j] < N ? pm[j] : N - 1;
                const float2 x = s[(size_t)u * n_vec + v];
                re = fmaf(w.x, x.x, fmaf(-w.y, x.y, re));
                im = fmaf(w.x, x.y, fmaf(w.y, x.x, im));
            }
            const float d = tau * Wc[vp_pidx(N, m, m)].x;
            c0[(v * N + m) * 2] = fx_q(-re / d, scale);
            c0[(v * N + m) * 2 + 1] = fx_q(-im / d, scale);
        }
    }
    if (t < (size_t)n_sc * (NV + N)) {   // the subcarrier's steps and weights
        const int sc = (int)(t / (NV + N)), e = (int)(t % (NV + N));
        const float2 *Wc = W + (size_t)sc * NP;
        if (e < NV) {
            int m = 1;
            while (vidx(m + 1, 0) <= e) ++m;
            const int i = e - vidx(m, 0);
            const float2 w = Wc[vp_pidx(N, m, i)];
            const float d = Wc[vp_pidx(N, m, m)].x;
            Vq[((size_t)sc * NV + e) * 2] = fx_q(-w.x / d, scale);
            Vq[((size_t)sc * NV + e) * 2 + 1] = fx_q(-w.y / d, scale);
        } else {
            const int i = e - NV;
            float mx = 0.f;
            for (int j = 0; j < N; ++j) {
                const float d = Wc[vp_pidx(N, j, j)].x;
                mx = fmaxf(mx, d * d);
            }
            const float d = Wc[vp_pidx(N, i, i)].x;
            wq[(size_t)sc * N + i] = fx_q(d * d / mx, scale);
        }
    }
}

template <int N>
__global__ __launch_bounds__(kT) void k_fx_search(const int16_t *__restrict__ c0, const int16_t *__restrict__ Vq,
                                                  const int16_t *__restrict__ wq, const uint8_t *__restrict__ perm,
                                                  const uint8_t *__restrict__ paths, int K, long long pstride,
                                                  int n_sym, int one, unsigned flags, int8_t *__restrict__ l_out,
                                                  int64_t *__restrict__ ped_out, int32_t *__restrict__ kidx_out) {
    constexpr int NV = N * (N - 1) / 2;
    __shared__ int s_c0[2 * N];
    __shared__ int s_v[2 * (NV > 0 ? NV : 1)];
    __shared__ int s_w[N];
    __shared__ unsigned long long s_red[kT / 64];
    const size_t v = blockIdx.x;
    const size_t n_vec = gridDim.x;
    const int sc = (int)(v / n_sym);
    const int t = threadIdx.x;
    for (int e = t; e < 2 * N; e += kT) s_c0[e] = c0[v * 2 * N + e];
    for (int e = t; e < 2 * NV; e += kT) s_v[e] = Vq[(size_t)sc * 2 * NV + e];
    if (t < N) s_w[t] = wq[(size_t)sc * N + t];
    __syncthreads();
    const uint8_t *P = paths + (size_t)sc * pstride;
    const int Kc = K + ((flags & VP_INCLUDE_ZERO) ? 1 : 0);   // candidate K: the zero perturbation
    unsigned long long best = ~0ull, best_l = 0ull;
    for (int k = t; k < Kc; k += kT) {
        int cx[N], cy[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            cx[i] = s_c0[2 * i];
            cy[i] = s_c0[2 * i + 1];
        }
        unsigned long long ped = 0ull, lw = 0ull;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            int a = 0, b = 0;
            uint32_t dist;
            if (k < K) {
                // the nine squared distances and the box point of the path's rank
                // in the (distance, j) order, j = 3 (a + 1) + (b + 1)
                const int rank = P[(size_t)k * N + i] < 9 ? P[(size_t)k * N + i] : 8;
                uint32_t d[9];
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    const int ex = fx_sat(cx[i] - (j / 3 - 1) * one), ey = fx_sat(cy[i] - (j % 3 - 1) * one);
                    d[j] = (uint32_t)(ex * ex) + (uint32_t)(ey * ey);
                }
                int pick = 0;
                dist = d[0];
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    int r = 0;
#pragma unroll
                    for (int q = 0; q < 9; ++q) r += (d[q] < d[j]) || (d[q] == d[j] && q < j);
                    if (r == rank) {
                        pick = j;
                        dist = d[j];
                    }
                }
                a = pick / 3 - 1;
                b = pick % 3 - 1;
            } else {
                const int ex = fx_sat(cx[i]), ey = fx_sat(cy[i]);
                dist = (uint32_t)(ex * ex) + (uint32_t)(ey * ey);
            }
            ped += (unsigned long long)s_w[i] * dist;   // weights are >= 0
            lw |= (unsigned long long)(((a + 1) << 2) | (b + 1)) << (4 * i);
#pragma unroll
            for (int m = i + 1; m < N; ++m) {
                const int vx = s_v[2 * vidx(m, i)], vy = s_v[2 * vidx(m, i) + 1];
                cx[m] = fx_sat(cx[m] + a * vx - b * vy);
                cy[m] = fx_sat(cy[m] + a * vy + b * vx);
            }
        }
        // PED < 2^15 * 2^31 * 16 = 2^50 and k < 2^13: one ordered 64-bit key
        const unsigned long long key = (ped << 13) | (unsigned long long)k;
        if (key < best) {
            best = key;
            best_l = lw;
        }
    }
    unsigned long long wbest = best;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(wbest, off);
        wbest = o < wbest ? o : wbest;
    }
    if ((t & 63) == 0) s_red[t >> 6] = wbest;
    __syncthreads();
    unsigned long long gbest = s_red[0];
    for (int w = 1; w < kT / 64; ++w) gbest = s_red[w] < gbest ? s_red[w] : gbest;
    if (best == gbest) {   // the one lane that evaluated the winning path (keys are unique)
        const int k = (int)(gbest & 8191ull);
        const uint8_t *pm = perm + (size_t)sc * N;
        for (int i = 0; i < N; ++i) {
            const int u = pm[i] < N ? pm[i] : N - 1;
            const int code = (int)((best_l >> (4 * i)) & 15ull);
            int8_t *o = l_out + ((size_t)u * n_vec + v) * 2;
            o[0] = (int8_t)((code >> 2) - 1);
            o[1] = (int8_t)((code & 3) - 1);
        }
        ped_out[v] = (int64_t)(gbest >> 13);
        kidx_out[v] = k;
    }
}

template <int N>
int launch_fx_n(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, int n_sc, int n_sym,
                int frac_bits, int16_t *c0, int16_t *Vq, int16_t *wq, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t work = n_vec > (size_t)n_sc * (N * (N - 1) / 2 + N) ? n_vec : (size_t)n_sc * (N * (N - 1) / 2 + N);
    hipLaunchKernelGGL(k_fx_quantize<N>, dim3((unsigned)((work + kT - 1) / kT)), dim3(kT), 0, st, W, perm, s, tau,
                       n_sc, n_sym, (float)(1 << frac_bits), c0, Vq, wq);
    return launch_status();
}

template <int N>
int launch_fx_search_n(const int16_t *c0, const int16_t *Vq, const int16_t *wq, const uint8_t *perm,
                       const uint8_t *paths, int K, int64_t pstride, int n_sc, int n_sym, int frac_bits,
                       uint32_t flags, int8_t *l, int64_t *ped, int32_t *kidx, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    hipLaunchKernelGGL(k_fx_search<N>, dim3((unsigned)n_vec), dim3(kT), 0, st, c0, Vq, wq, perm, paths, K,
                       (long long)pstride, n_sym, 1 << frac_bits, flags, l, ped, kidx);
    return launch_status();
}

}  // namespace

int launch_fx_quantize(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, int n_sc, int n_sym,
                       int N, int frac_bits, int16_t *c0, int16_t *Vq, int16_t *wq, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    switch (N) {
#define VP_CASE(n) \
    case n: return launch_fx_n<n>(W, perm, s, tau, n_sc, n_sym, frac_bits, c0, Vq, wq, st);
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: return VP_EUNSUPPORTED;
    }
}

int launch_fx_search(const int16_t *c0, const int16_t *Vq, const int16_t *wq, const uint8_t *perm,
                     const uint8_t *paths, int K, int64_t pstride, int n_sc, int n_sym, int N, int frac_bits,
                     uint32_t flags, int8_t *l, int64_t *ped, int32_t *kidx, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    switch (N) {
#define VP_CASE(n)                                                                                          \
    case n:                                                                                                 \
        return launch_fx_search_n<n>(c0, Vq, wq, perm, paths, K, pstride, n_sc, n_sym, frac_bits, flags, l, \
                                     ped, kidx, st);
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: return VP_EUNSUPPORTED;
    }
}

}  // namespace vp
