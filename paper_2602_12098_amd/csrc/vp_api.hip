// C ABI of the precoding library: host-side argument validation and dispatch
// to the kernel launchers.  No allocation, no synchronisation.
#include <math.h>

#include <atomic>

#include "vp_internal.hpp"

namespace vp {

static std::atomic<int> g_last_hip_error{0};

int launch_status() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_last_hip_error.store((int)e);
        return VP_ELAUNCH;
    }
    return VP_OK;
}

static bool k_exceeds_box(int K, int N) {   // K > 9^N ?
    long long cap = 1;
    for (int i = 0; i < N; ++i) {
        cap *= 9;
        if (cap >= K) return false;
    }
    return cap < K;
}

}  // namespace vp

using namespace vp;

extern "C" {

int vp_preprocess(const vp_c32 *H, int n_sc, int n_r, int n_t, float alpha, vp_c32 *W, float *w2, uint8_t *perm,
                  vp_c32 *G, int32_t *status, void *stream) {
    if (n_sc < 0 || n_r < 1 || n_t < 1 || !(alpha >= 0.f) || !isfinite(alpha)) return VP_EINVAL;
    if (n_r > kMaxN || n_t > kMaxM) return VP_EUNSUPPORTED;
    if (alpha == 0.f && n_r > n_t) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!H || !W || !w2 || !perm || !status) return VP_EINVAL;
    return launch_preprocess((const float2 *)H, n_sc, n_r, n_t, alpha, (float2 *)W, w2, perm, (float2 *)G, status,
                             (hipStream_t)stream);
}

int vp_paths_mop(const float *w2, int n_sc, int n_r, int K, uint8_t *paths, uint16_t *order, void *stream) {
    if (n_sc < 0 || n_r < 1 || K < 1) return VP_EINVAL;
    if (n_r > kMaxN || K > kMaxKMop) return VP_EUNSUPPORTED;
    if (k_exceeds_box(K, n_r)) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!w2 || !paths) return VP_EINVAL;
    return launch_mop(w2, n_sc, n_r, K, paths, order, (hipStream_t)stream);
}

int vp_search(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, const uint8_t *paths,
              const uint16_t *order, int K, int64_t paths_sc_stride, int n_sc, int n_sym, int n_r,
              uint32_t flags, int8_t *l, float *cost, int32_t *kidx, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || K < 1 || !(tau > 0.f) || !isfinite(tau)) return VP_EINVAL;
    if (n_r > kMaxN || K > kMaxKSearch) return VP_EUNSUPPORTED;
    if (paths_sc_stride < 0 || (paths_sc_stride > 0 && paths_sc_stride < (int64_t)K * n_r)) return VP_EINVAL;
    if (order && paths_sc_stride != (int64_t)K * n_r) return VP_EINVAL;   // one order per subcarrier table
    if (flags & ~(uint32_t)VP_INCLUDE_ZERO) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !paths || !l || !cost || !kidx) return VP_EINVAL;
    return launch_search((const float2 *)W, perm, (const float2 *)s, tau, paths, order, K, paths_sc_stride, n_sc,
                         n_sym,
                         n_r, flags, l, cost, kidx, (hipStream_t)stream);
}

int vp_precode(const vp_c32 *G, const vp_c32 *s, const int8_t *l, float tau, const float *cost, int n_sc, int n_sym,
               int n_r, int n_t, float P_T, vp_c32 *x, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || n_t < 1 || !(tau > 0.f) || !isfinite(tau)) return VP_EINVAL;
    if (!(P_T >= 0.f) || !isfinite(P_T)) return VP_EINVAL;
    if (n_r > kMaxN || n_t > kMaxM) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!G || !s || !l || !x || (P_T > 0.f && !cost)) return VP_EINVAL;
    return launch_precode((const float2 *)G, (const float2 *)s, l, tau, cost, n_sc, n_sym, n_r, n_t, P_T,
                          (float2 *)x, (hipStream_t)stream);
}

int vp_sphere_encode(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, int n_sc, int n_sym,
                     int n_r, const float *radius, int64_t max_nodes, int8_t *l, float *cost, int64_t *nodes,
                     void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || !(tau > 0.f) || !isfinite(tau) || max_nodes <= 0) return VP_EINVAL;
    if (n_r > kMaxN) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !l || !cost) return VP_EINVAL;
    return launch_sphere((const float2 *)W, perm, (const float2 *)s, tau, n_sc, n_sym, n_r, radius, l, cost, nodes,
                         (long long)max_nodes, (hipStream_t)stream);
}

const char *vp_strerror(int code) {
    switch (code) {
        case VP_OK: return "ok";
        case VP_EINVAL: return "invalid argument";
        case VP_EUNSUPPORTED: return "unsupported size";
        case VP_ELAUNCH: return "HIP launch failure";
        default: return "unknown error";
    }
}

int vp_last_hip_error(void) { return g_last_hip_error.load(); }

const char *vp_version(void) { return "vipernl-mi355x 0.1 (gfx950)"; }

}  // extern "C"
