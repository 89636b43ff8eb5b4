// Linear precoding of the perturbed vector (Alg. 2 output; Sec. IV-B
// channel-inverse, gamma and PV blocks): x = G (s + tau l), tau per subcarrier, optionally scaled
// by sqrt(P_T / gamma) with gamma the selected search cost (Sec. II-B).
//
// One workgroup per subcarrier and up to kVB of its vectors: the
// subcarrier's G and the vectors' u = s + tau l are staged in LDS with
// coalesced loads, then one lane per (vector, antenna), antennas fastest,
// forms x = G u, so each vector's output row is written by consecutive lanes.
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

}  // namespace

int launch_precode(const float2 *G, const float2 *s, const int8_t *l, const float *tau, const float *cost, int n_sc,
                   int n_sym, int N, int M, float P_T, float2 *x, hipStream_t st) {
    if ((size_t)n_sc * n_sym * M == 0) return VP_OK;
    const unsigned blocks = (unsigned)n_sc * (unsigned)((n_sym + kVB - 1) / kVB);
    hipLaunchKernelGGL(k_precode, dim3(blocks), dim3(kT), 0, st, G, s, l, tau, cost, n_sc, n_sym, N, M, P_T, x);
    return launch_status();
}

}  // namespace vp
