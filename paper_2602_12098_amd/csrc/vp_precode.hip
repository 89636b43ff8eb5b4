// Linear precoding of the perturbed vector (Alg. 2 output; Sec. IV-B
// channel-inverse, gamma and PV blocks): x = G (s + tau l), optionally scaled
// by sqrt(P_T / gamma) with gamma the selected search cost (Sec. II-B).
//
// One lane per (vector, antenna), antennas fastest, so each vector's output
// row is written by consecutive lanes; G rows of the subcarrier are shared by
// its n_sym vectors through the cache.
#include "vp_internal.hpp"

namespace vp {
namespace {

constexpr int kT = 256;

__global__ __launch_bounds__(kT) void k_precode(const float2 *__restrict__ G, const float2 *__restrict__ s,
                                                const int8_t *__restrict__ l, float tau,
                                                const float *__restrict__ cost, int n_sc, int n_sym, int N,
                                                int M, float P_T, float2 *__restrict__ x) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t idx = (size_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= n_vec * M) return;
    const size_t v = idx / M;
    const int m = (int)(idx % M);
    const int sc = (int)(v / n_sym);
    const float2 *__restrict__ g = G + ((size_t)sc * M + m) * N;
    float re = 0.f, im = 0.f;
    for (int i = 0; i < N; ++i) {
        const float2 si = s[(size_t)i * n_vec + v];
        const int8_t *li = l + ((size_t)i * n_vec + v) * 2;
        const float ur = fmaf(tau, (float)li[0], si.x);
        const float ui = fmaf(tau, (float)li[1], si.y);
        const float2 gi = g[i];
        re = fmaf(gi.x, ur, fmaf(-gi.y, ui, re));
        im = fmaf(gi.x, ui, fmaf(gi.y, ur, im));
    }
    if (P_T > 0.f) {
        const float c = cost[v];
        const float sc_ = (c > 0.f && isfinite(c)) ? sqrtf(P_T / c) : __int_as_float(0x7fc00000);
        re *= sc_;
        im *= sc_;
    }
    x[idx] = make_float2(re, im);
}

}  // namespace

int launch_precode(const float2 *G, const float2 *s, const int8_t *l, float tau, const float *cost, int n_sc,
                   int n_sym, int N, int M, float P_T, float2 *x, hipStream_t st) {
    const size_t total = (size_t)n_sc * n_sym * M;
    if (total == 0) return VP_OK;
    hipLaunchKernelGGL(k_precode, dim3((unsigned)((total + kT - 1) / kT)), dim3(kT), 0, st, G, s, l, tau, cost,
                       n_sc, n_sym, N, M, P_T, x);
    return launch_status();
}

}  // namespace vp
