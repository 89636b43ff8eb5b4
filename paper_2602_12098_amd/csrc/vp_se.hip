// Exact vector perturbation over the B = 1 box: a depth-first
// Schnorr-Euchner sphere encoder (the exact solution of eq:se / eq_qrse,
// explored with the PED recursion of Sec. II-B), one lane per vector.
//
// Down the tree the level centre is formed lazily,
//   c_i = -(s-tilde_i / tau + sum_{j<i} W_ij l_j) / W_ii,
// so backtracking needs no saved residuals: each level keeps only its centre,
// the PED above it and the rank of the child being tried.  Children are
// tried in increasing squared distance (equal distances in canonical box
// order), so the first child whose PED reaches the best cost ends the level.
// The search radius may be seeded (e.g. with the K-path result), which only
// prunes: the minimum found is the same.  A vector that runs out of its node
// budget keeps the best point found so far (its status says so).
#include "vp_internal.hpp"

#define VP_LUT_STORAGE static __constant__
#include "vp_device.hpp"

namespace vp {
namespace {

constexpr int kT = 64;

template <int N>
__global__ __launch_bounds__(kT) void k_sphere(const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                               const float2 *__restrict__ s, float tau, int n_sc, int n_sym,
                                               const float *__restrict__ radius, int8_t *__restrict__ l_out,
                                               float *__restrict__ cost_out, int64_t *__restrict__ nodes_out,
                                               uint8_t *__restrict__ status_out, long long max_nodes) {
    constexpr int NP = VP_PACKED(N);
    const size_t n_vec = (size_t)n_sc * n_sym;
    const size_t v = (size_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n_vec) return;
    const int sc = (int)(v / n_sym);
    const float2 *__restrict__ Wc = W + (size_t)sc * NP;
    const uint8_t *pm = perm + (size_t)sc * N;
    const float w00 = Wc[0].x;
    float la[N], lb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) la[i] = lb[i] = 0.f;
    float best = radius ? radius[v] : __int_as_float(0x7f800000);
    long long nodes = 0;
    bool found = false, cut = false;
    if (w00 > 0.f && isfinite(w00)) {
        const float inv_tau = 1.0f / tau;
        float st[2 * N];   // s-tilde / tau
        for (int i = 0; i < N; ++i) {
            float re = 0.f, im = 0.f;
            for (int j = 0; j <= i; ++j) {
                const float2 w = Wc[vp_pidx(N, i, j)];
                const int u = pm[j] < N ? pm[j] : N - 1;
                const float2 x = s[(size_t)u * n_vec + v];
                re = fmaf(w.x, x.x, fmaf(-w.y, x.y, re));
                im = fmaf(w.x, x.y, fmaf(w.y, x.x, im));
            }
            st[2 * i] = re * inv_tau;
            st[2 * i + 1] = im * inv_tau;
        }
        float cx[N], cy[N], ped[N + 1], wd[N];
        int rk[N];
        float ca[N], cb[N];   // current path
        for (int i = 0; i < N; ++i) wd[i] = Wc[vp_pidx(N, i, i)].x;
        const float tau2 = tau * tau;
        int i = 0;
        ped[0] = 0.f;
        {
            const float li = 1.0f / wd[0];
            cx[0] = -(st[0] * li);
            cy[0] = -(st[1] * li);
        }
        rk[0] = 0;
        while (true) {
            bool up = false;
            if (rk[i] >= 9) {
                up = true;
            } else {
                float a, b;
                vp_demapN(cx[i] - 0.5f, cy[i] - 0.5f, cx[i], cy[i], rk[i], VP_DEMAP_LUT, a, b);
                // PED increment: tau^2 W_ii^2 |c_i - l_i|^2
                const float dx = cx[i] - a, dy = cy[i] - b;
                const float d = fmaf(dx, dx, dy * dy);
                const float np_ = fmaf(tau2 * wd[i] * wd[i], d, ped[i]);
                if (!(np_ < best)) {
                    up = true;   // later children are no closer
                } else {
                    ++nodes;
                    ca[i] = a;
                    cb[i] = b;
                    if (i == N - 1) {
                        best = np_;
                        found = true;
#pragma unroll
                        for (int q = 0; q < N; ++q) {
                            la[q] = ca[q];
                            lb[q] = cb[q];
                        }
                        up = true;
                    } else {
                        ped[i + 1] = np_;
                        ++i;
                        // lazy centre of the new level
                        float re = st[2 * i], im = st[2 * i + 1];
                        for (int j = 0; j < i; ++j) {
                            const float2 w = Wc[vp_pidx(N, i, j)];
                            re = fmaf(w.x, ca[j], fmaf(-w.y, cb[j], re));
                            im = fmaf(w.x, cb[j], fmaf(w.y, ca[j], im));
                        }
                        const float li = 1.0f / wd[i];
                        cx[i] = -(re * li);
                        cy[i] = -(im * li);
                        rk[i] = 0;
                    }
                }
            }
            if (up) {
                if (i == 0) break;   // the root's children are done: the search is complete
                if (nodes >= max_nodes) {
                    cut = true;
                    break;
                }
                --i;
                ++rk[i];
            }
        }
    }
    const size_t base = v;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const int u = pm[q] < N ? pm[q] : N - 1;
        int8_t *o = l_out + ((size_t)u * n_vec + base) * 2;
        o[0] = found ? (int8_t)la[q] : 0;
        o[1] = found ? (int8_t)lb[q] : 0;
    }
    cost_out[v] = found ? best : __int_as_float(0x7fc00000);
    if (nodes_out) nodes_out[v] = nodes;
    if (status_out)
        status_out[v] = cut ? (uint8_t)VP_SE_EXHAUSTED : (found ? (uint8_t)VP_SE_EXACT : (uint8_t)VP_SE_NONE);
}

template <int N>
int launch_sphere_n(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym,
                    const float *radius, int8_t *l, float *cost, int64_t *nodes, uint8_t *status,
                    long long max_nodes, hipStream_t st) {
    const size_t n_vec = (size_t)n_sc * n_sym;
    hipLaunchKernelGGL(k_sphere<N>, dim3((unsigned)((n_vec + kT - 1) / kT)), dim3(kT), 0, st, W, perm, s, tau, n_sc,
                       n_sym, radius, l, cost, nodes, status, max_nodes);
    return launch_status();
}

}  // namespace

int launch_sphere(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym, int N,
                  const float *radius, int8_t *l, float *cost, int64_t *nodes, uint8_t *status,
                  long long max_nodes, hipStream_t st) {
    if (n_sc == 0) return VP_OK;
    switch (N) {
#define VP_CASE(n) \
    case n: return launch_sphere_n<n>(W, perm, s, tau, n_sc, n_sym, radius, l, cost, nodes, status, max_nodes, st);
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: return VP_EUNSUPPORTED;
    }
}

}  // namespace vp
