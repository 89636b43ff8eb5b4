// Linear precoding of the perturbed vector (Alg. 2 output; Sec. IV-B
// channel-inverse, gamma and PV blocks): x = G (s + tau l), tau per subcarrier, optionally scaled
// by sqrt(P_T / gamma) with gamma the selected search cost (Sec. II-B).
//
// One workgroup per subcarrier and up to kVB of its vectors: the
// subcarrier's G and the vectors' u = s + tau l are staged in LDS with
// coalesced loads, then one lane per (vector, antenna), antennas fastest,
// forms x = G u, so each vector's output row is written by consecutive lanes.
#include <algorithm>

#include "vp_internal.hpp"

namespace vp {
namespace {

constexpr int kT = 256;
constexpr int kVB = 16;   // vectors per workgroup

__global__ __launch_bounds__(kT) void k_precode(const float2 *__restrict__ G, const float2 *__restrict__ s,
                                                const int8_t *__restrict__ l, const float *__restrict__ taus,
                                                const float *__restrict__ cost, int n_sc, int n_sym, int N,
                                                int M, float P_T, float2 *__restrict__ x) {
    __shared__ float2 sG[kMaxM][kMaxN + 1];   // padded rows: lanes of different antennas hit different banks
    __shared__ float2 sU[kVB][kMaxN + 1];
    const int chunks = (n_sym + kVB - 1) / kVB;
    const int sc = (int)(blockIdx.x / chunks);
    const int v0 = (int)(blockIdx.x % chunks) * kVB;
    const int nv = min(kVB, n_sym - v0);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t vb = (size_t)sc * n_sym + v0;
    const int t = threadIdx.x;
    const float2 *__restrict__ g = G + (size_t)sc * M * N;
    float tau = taus[sc];
    if (!(tau > 0.f) || !isfinite(tau)) tau = __int_as_float(0x7fc00000);   // an invalid tau gives x = NaN
    for (int e = t; e < M * N; e += kT) sG[e / N][e % N] = g[e];
    for (int e = t; e < N * nv; e += kT) {   // consecutive lanes: consecutive vectors of one user
        const int i = e / nv, vl = e % nv;
        const size_t o = (size_t)i * n_vec + vb + vl;
        const float2 si = s[o];
        const int8_t *li = l + o * 2;
        sU[vl][i] = make_float2(fmaf(tau, (float)li[0], si.x), fmaf(tau, (float)li[1], si.y));
    }
    __syncthreads();
    for (int e = t; e < nv * M; e += kT) {
        const int vl = e / M, m = e % M;
        float re = 0.f, im = 0.f;
        for (int i = 0; i < N; ++i) {
            const float2 u = sU[vl][i];
            const float2 gi = sG[m][i];
            re = fmaf(gi.x, u.x, fmaf(-gi.y, u.y, re));
            im = fmaf(gi.x, u.y, fmaf(gi.y, u.x, im));
        }
        if (P_T > 0.f) {
            const float c = cost[vb + vl];
            const float sc_ = (c > 0.f && isfinite(c)) ? sqrtf(P_T / c) : __int_as_float(0x7fc00000);
            re *= sc_;
            im *= sc_;
        }
        x[(vb + vl) * M + m] = make_float2(re, im);
    }
}

// Per-user perturbation intervals (one QAM order per user): W's column i
// times tau of the user at level i, w2 times its square, G's column u times
// tau_u, and s's row u divided by tau_u.  One thread per entry of the largest
// of those arrays for its subcarrier.
__global__ __launch_bounds__(kT) void k_user_tau(const float *__restrict__ tau, const uint8_t *__restrict__ perm,
                                                 int n_sc, int n_sym, int N, int M, float2 *__restrict__ W,
                                                 float *__restrict__ w2, float2 *__restrict__ G,
                                                 const float2 *__restrict__ s, float2 *__restrict__ s_out) {
    const int NP = VP_PACKED(N);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    const size_t per_sc = (size_t)max(max(NP, M * N), N * n_sym);
    if (i >= per_sc * n_sc) return;
    const int sc = (int)(i / per_sc), e = (int)(i % per_sc);
    const float *ts = tau + (size_t)sc * N;
    const uint8_t *pm = perm + (size_t)sc * N;
    if (e < NP) {   // packed column-major lower: entry e lies in column j
        int j = 0, rem = e;
        while (rem >= N - j) {
            rem -= N - j;
            ++j;
        }
        const int u = pm[j] < N ? pm[j] : N - 1;
        float2 w = W[(size_t)sc * NP + e];
        w.x *= ts[u];
        w.y *= ts[u];
        W[(size_t)sc * NP + e] = w;
        if (rem == 0) w2[(size_t)sc * N + j] *= ts[u] * ts[u];
    }
    if (G && e < M * N) {   // G [M][N], user columns
        float2 g = G[(size_t)sc * M * N + e];
        const float t = ts[e % N];
        g.x *= t;
        g.y *= t;
        G[(size_t)sc * M * N + e] = g;
    }
    if (e < N * n_sym) {   // s [N][n_vec]: user row, this subcarrier's symbols
        const int u = e / n_sym, sym = e % n_sym;
        const size_t o = (size_t)u * n_vec + (size_t)sc * n_sym + sym;
        const float2 x = s[o];
        const float r = 1.0f / ts[u];
        s_out[o] = make_float2(x.x * r, x.y * r);
    }
}

}  // namespace

int launch_user_tau(const float *tau, const uint8_t *perm, int n_sc, int n_sym, int N, int M, float2 *W, float *w2,
                    float2 *G, const float2 *s, float2 *s_out, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    const size_t per_sc = (size_t)std::max(std::max(VP_PACKED(N), M * N), N * n_sym);
    const size_t total = per_sc * (size_t)n_sc;
    hipLaunchKernelGGL(k_user_tau, dim3((unsigned)((total + kT - 1) / kT)), dim3(kT), 0, st, tau, perm, n_sc, n_sym,
                       N, M, W, w2, G, s, s_out);
    return launch_status();
}

int launch_precode(const float2 *G, const float2 *s, const int8_t *l, const float *tau, const float *cost, int n_sc,
                   int n_sym, int N, int M, float P_T, float2 *x, hipStream_t st) {
    if ((size_t)n_sc * n_sym * M == 0) return VP_OK;
    const unsigned blocks = (unsigned)n_sc * (unsigned)((n_sym + kVB - 1) / kVB);
    hipLaunchKernelGGL(k_precode, dim3(blocks), dim3(kT), 0, st, G, s, l, tau, cost, n_sc, n_sym, N, M, P_T, x);
    return launch_status();
}

}  // namespace vp
