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

void record_hip_error(int code) { g_last_hip_error.store(code); }

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

int vp_preprocess_unsorted(const vp_c32 *H, int n_sc, int n_r, int n_t, float alpha, vp_c32 *W, float *w2,
                           uint8_t *perm, vp_c32 *G, int32_t *status, void *stream) {
    if (n_sc < 0 || n_r < 1 || n_t < 1 || !(alpha >= 0.f) || !isfinite(alpha)) return VP_EINVAL;
    if (n_r > kMaxN || n_t > kMaxM) return VP_EUNSUPPORTED;
    if (alpha == 0.f && n_r > n_t) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!H || !W || !w2 || !perm || !status) return VP_EINVAL;
    return launch_preprocess((const float2 *)H, n_sc, n_r, n_t, alpha, (float2 *)W, w2, perm, (float2 *)G, status,
                             (hipStream_t)stream, false);
}

int vp_paths_mop(const float *w2, int n_sc, int n_r, int K, uint8_t *paths, uint16_t *order, void *stream) {
    if (n_sc < 0 || n_r < 1 || K < 1) return VP_EINVAL;
    if (n_r > kMaxN || K > kMaxKMop) return VP_EUNSUPPORTED;
    if (k_exceeds_box(K, n_r)) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!w2 || !paths) return VP_EINVAL;
    return launch_mop(w2, n_sc, n_r, K, paths, order, (hipStream_t)stream);
}

int vp_search(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau, const uint8_t *paths,
              const uint16_t *order, int K, int64_t paths_sc_stride, int n_sc, int n_sym, int n_r,
              uint32_t flags, int8_t *l, float *cost, int32_t *kidx, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || K < 1) return VP_EINVAL;
    if (n_r > kMaxN || K > kMaxKSearch) return VP_EUNSUPPORTED;
    if (paths_sc_stride < 0 || (paths_sc_stride > 0 && paths_sc_stride < (int64_t)K * n_r)) return VP_EINVAL;
    if (order && paths_sc_stride != (int64_t)K * n_r) return VP_EINVAL;   // one order per subcarrier table
    if (flags & ~(uint32_t)(VP_INCLUDE_ZERO | VP_PATHS_PER_VECTOR | VP_DEMAP_REGION)) return VP_EINVAL;
    if ((flags & VP_PATHS_PER_VECTOR) && (order || paths_sc_stride != (int64_t)K * n_r)) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !tau || !paths || !l || !cost || !kidx) return VP_EINVAL;
    return launch_search((const float2 *)W, perm, (const float2 *)s, tau, paths, order, K, paths_sc_stride, n_sc,
                         n_sym,
                         n_r, flags, l, cost, kidx, (hipStream_t)stream);
}

int vp_search_fallback(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau, const uint8_t *paths,
                       const uint16_t *order, int K, int64_t paths_sc_stride, int n_sc, int n_sym, int n_r,
                       uint32_t flags, const float *mass, float theta, int32_t kidx_base, int8_t *l, float *cost,
                       int32_t *kidx, void *work, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || K < 1) return VP_EINVAL;
    if (n_r > kMaxN || K > kMaxKSearch) return VP_EUNSUPPORTED;
    if (paths_sc_stride < 0 || (paths_sc_stride > 0 && paths_sc_stride < (int64_t)K * n_r)) return VP_EINVAL;
    if (order && paths_sc_stride != (int64_t)K * n_r) return VP_EINVAL;
    if (flags & ~(uint32_t)VP_INCLUDE_ZERO) return VP_EINVAL;
    if (isnan(theta) || kidx_base < 0) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !tau || !paths || !mass || !l || !cost || !kidx || !work) return VP_EINVAL;
    if (reinterpret_cast<uintptr_t>(work) & 3) return VP_EINVAL;
    return launch_search_fallback((const float2 *)W, perm, (const float2 *)s, tau, paths, order, K, paths_sc_stride,
                                  n_sc, n_sym, n_r, flags, mass, theta, kidx_base, l, cost, kidx, work,
                                  (hipStream_t)stream);
}

int vp_search_fallback_noalloc(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau,
                               const uint8_t *paths, const uint16_t *order, int K, int64_t paths_sc_stride, int n_sc,
                               int n_sym, int n_r, uint32_t flags, const float *mass, float theta, int32_t kidx_base,
                               int8_t *l, float *cost, int32_t *kidx, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || K < 1) return VP_EINVAL;
    if (n_r > kMaxN || K > kMaxKSearch) return VP_EUNSUPPORTED;
    if ((int64_t)n_sc * n_sym > (int64_t)kNoAllocVectors) return VP_EUNSUPPORTED;   // beyond the fixed workspace
    if (paths_sc_stride < 0 || (paths_sc_stride > 0 && paths_sc_stride < (int64_t)K * n_r)) return VP_EINVAL;
    if (order && paths_sc_stride != (int64_t)K * n_r) return VP_EINVAL;
    if (flags & ~(uint32_t)VP_INCLUDE_ZERO) return VP_EINVAL;
    if (isnan(theta) || kidx_base < 0) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !tau || !paths || !mass || !l || !cost || !kidx) return VP_EINVAL;
    return launch_search_fallback_noalloc((const float2 *)W, perm, (const float2 *)s, tau, paths, order, K,
                                          paths_sc_stride, n_sc, n_sym, n_r, flags, mass, theta, kidx_base, l, cost,
                                          kidx, (hipStream_t)stream);
}

int vp_precode(const vp_c32 *G, const vp_c32 *s, const int8_t *l, const float *tau, const float *cost, int n_sc,
               int n_sym, int n_r, int n_t, float P_T, vp_c32 *x, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || n_t < 1) return VP_EINVAL;
    if (!(P_T >= 0.f) || !isfinite(P_T)) return VP_EINVAL;
    if (n_r > kMaxN || n_t > kMaxM) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!G || !s || !l || !tau || !x || (P_T > 0.f && !cost)) return VP_EINVAL;
    return launch_precode((const float2 *)G, (const float2 *)s, l, tau, cost, n_sc, n_sym, n_r, n_t, P_T,
                          (float2 *)x, (hipStream_t)stream);
}

int vp_apply_user_tau(const float *tau_user, const uint8_t *perm, int n_sc, int n_sym, int n_r, int n_t, vp_c32 *W,
                      float *w2, vp_c32 *G, const vp_c32 *s, vp_c32 *s_out, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || n_t < 1) return VP_EINVAL;
    if (n_r > kMaxN || n_t > kMaxM) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!tau_user || !perm || !W || !w2 || !s || !s_out) return VP_EINVAL;
    return launch_user_tau(tau_user, perm, n_sc, n_sym, n_r, n_t, (float2 *)W, w2, (float2 *)G, (const float2 *)s,
                           (float2 *)s_out, (hipStream_t)stream);
}

int vp_sphere_encode(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, int n_sc, int n_sym,
                     int n_r, const float *radius, int64_t max_nodes, int8_t *l, float *cost, int64_t *nodes,
                     uint8_t *status, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || !(tau > 0.f) || !isfinite(tau) || max_nodes <= 0) return VP_EINVAL;
    if (n_r > kMaxN) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !l || !cost) return VP_EINVAL;
    return launch_sphere((const float2 *)W, perm, (const float2 *)s, tau, n_sc, n_sym, n_r, radius, l, cost, nodes,
                         status, (long long)max_nodes, (hipStream_t)stream);
}

int vp_fx_quantize(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau, int n_sc, int n_sym,
                   int n_r, int frac_bits, int16_t *c0, int16_t *V, int16_t *w, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || frac_bits < 8 || frac_bits > 13) return VP_EINVAL;
    if (n_r > kMaxN) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !tau || !c0 || !w || (n_r > 1 && !V)) return VP_EINVAL;
    return launch_fx_quantize((const float2 *)W, perm, (const float2 *)s, tau, n_sc, n_sym, n_r, frac_bits, c0, V, w,
                              (hipStream_t)stream);
}

int vp_fx_search(const int16_t *c0, const int16_t *V, const int16_t *w, const uint8_t *perm, const uint8_t *paths,
                 int K, int64_t paths_sc_stride, int n_sc, int n_sym, int n_r, int frac_bits, uint32_t flags,
                 int8_t *l, int64_t *ped, int32_t *kidx, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || K < 1 || frac_bits < 8 || frac_bits > 13) return VP_EINVAL;
    if (n_r > kMaxN || K > kMaxKSearch) return VP_EUNSUPPORTED;
    if (paths_sc_stride < 0 || (paths_sc_stride > 0 && paths_sc_stride < (int64_t)K * n_r)) return VP_EINVAL;
    if (flags & ~(uint32_t)VP_INCLUDE_ZERO) return VP_EINVAL;
    if (n_sc == 0) return VP_OK;
    if ((int64_t)n_sc * n_sym > 0x7fffffffLL) return VP_EUNSUPPORTED;   // one workgroup per vector
    if (!c0 || !w || (n_r > 1 && !V) || !perm || !paths || !l || !ped || !kidx) return VP_EINVAL;
    return launch_fx_search(c0, V, w, perm, paths, K, paths_sc_stride, n_sc, n_sym, n_r, frac_bits, flags, l, ped,
                            kidx, (hipStream_t)stream);
}

int vp_mlp_features(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, int n_sc, int n_sym, int n_r,
                    uint32_t kind, uint16_t *feat, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || !(tau > 0.f) || !isfinite(tau)) return VP_EINVAL;
    if (kind != VP_FEAT_ZERO_CENTRES && kind != VP_FEAT_RANK0_WALK) return VP_EINVAL;
    if (n_r > kMaxN) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !feat) return VP_EINVAL;
    return launch_features((const float2 *)W, perm, (const float2 *)s, tau, n_sc, n_sym, n_r, kind, feat,
                           (hipStream_t)stream);
}

int vp_path_ranks(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, const int8_t *l, int n_sc,
                  int n_sym, int n_r, uint8_t *ranks, void *stream) {
    if (n_sc < 0 || n_sym < 1 || n_r < 1 || !(tau > 0.f) || !isfinite(tau)) return VP_EINVAL;
    if (n_r > kMaxN) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!W || !perm || !s || !l || !ranks) return VP_EINVAL;
    return launch_ranks((const float2 *)W, perm, (const float2 *)s, tau, n_sc, n_sym, n_r, l, ranks,
                        (hipStream_t)stream);
}

int vp_gemm_bf16(int m, int n, int k, const uint16_t *A, int64_t lda, int trans_a, const uint16_t *B, int64_t ldb,
                 int trans_b, const float *bias, uint32_t epilogue, const uint16_t *mask, int64_t ldm, float alpha,
                 float *C, uint16_t *C_bf16, int64_t ldc, void *stream) {
    if (m < 0 || n < 0 || k < 0 || (epilogue & ~(uint32_t)VP_EPI_RELU) || !isfinite(alpha)) return VP_EINVAL;
    if (!C && !C_bf16) return VP_EINVAL;
    if (m == 0 || n == 0) return VP_OK;
    if (k > 0 && (!A || !B)) return VP_EINVAL;
    if (k > 0 && lda < (int64_t)(trans_a ? m : k)) return VP_EINVAL;
    if (k > 0 && ldb < (int64_t)(trans_b ? k : n)) return VP_EINVAL;
    if (ldc < n || (mask && ldm < n)) return VP_EINVAL;
    return launch_gemm(m, n, k, A, (long long)lda, trans_a != 0, B, (long long)ldb, trans_b != 0, C, C_bf16,
                       (long long)ldc, bias, (int)(epilogue & VP_EPI_RELU), mask, (long long)ldm, alpha,
                       (hipStream_t)stream);
}

int vp_logits_top64(const uint16_t *X, int rows, const uint16_t *Wt, const float *bias, int V, int32_t *idx,
                    float *mass, void *work, void *stream) {
    if (rows < 0) return VP_EINVAL;
    if (V < 256 || V > VP_MAX_VOCAB || V % 128 != 0) return VP_EUNSUPPORTED;
    if (rows == 0) return VP_OK;
    if (!X || !Wt || !bias || !idx || !work) return VP_EINVAL;
    if ((reinterpret_cast<uintptr_t>(X) & 15) || (reinterpret_cast<uintptr_t>(Wt) & 15) ||
        (reinterpret_cast<uintptr_t>(work) & 255))
        return VP_EINVAL;
    return launch_logits_top64(X, rows, Wt, bias, V, idx, mass, work, (hipStream_t)stream);
}

int64_t vp_logits_top64_work_bytes(int rows) { return (int64_t)logits_top64_work_bytes(rows); }

int vp_topk64(const float *scores, int rows, int C, int32_t *idx, float *mass, void *stream) {
    if (rows < 0 || C < VP_TOPK) return VP_EINVAL;
    if (C > VP_MAX_VOCAB) return VP_EUNSUPPORTED;
    if (rows == 0) return VP_OK;
    if (!scores || !idx) return VP_EINVAL;
    return launch_topk64(scores, rows, C, idx, mass, (hipStream_t)stream);
}

int vp_softmax_xent(const float *logits, int rows, int C, const int32_t *label, float scale, float *loss,
                    uint16_t *dlogits, void *stream) {
    if (rows < 0 || C < 1 || !isfinite(scale)) return VP_EINVAL;
    if (rows == 0) return VP_OK;
    if (!logits || !label || !loss || !dlogits) return VP_EINVAL;
    return launch_softmax_ce(logits, rows, C, label, scale, loss, dlogits, (hipStream_t)stream);
}

int vp_colsum_bf16(const uint16_t *X, int rows, int cols, float *out, void *stream) {
    if (rows < 0 || cols < 0) return VP_EINVAL;
    if (cols == 0) return VP_OK;
    if (!out || (rows > 0 && !X)) return VP_EINVAL;
    return launch_colsum(X, rows, cols, out, (hipStream_t)stream);
}

int vp_learned_paths(const uint8_t *vocab, int V, int n_r, const int32_t *top, int K_learned, const uint8_t *fixed,
                     int K_fixed_table, int K_fixed, int n_sc, int n_sym, uint8_t *table, void *stream) {
    if (n_r < 1 || n_sc < 0 || n_sym < 1 || K_learned < 0 || K_fixed < 0 || K_fixed_table < 0) return VP_EINVAL;
    if (K_fixed > K_fixed_table || K_learned + K_fixed < 1 || (K_learned > 0 && V < 1)) return VP_EINVAL;
    if (n_r > kMaxN || K_learned + K_fixed > kMaxKSearch) return VP_EUNSUPPORTED;
    if (n_sc == 0) return VP_OK;
    if (!table || (K_learned > 0 && (!vocab || !top)) || (K_fixed > 0 && !fixed)) return VP_EINVAL;
    return launch_learned_table(vocab, V, n_r, top, K_learned, fixed, K_fixed_table, K_fixed, n_sc, n_sym, table,
                                (hipStream_t)stream);
}

const char *vp_strerror(int code) {
    switch (code) {
        case VP_OK: return "ok";
        case VP_EINVAL: return "invalid argument";
        case VP_EUNSUPPORTED: return "unsupported size (or beyond the fixed workspace of an allocation-free call)";
        case VP_ELAUNCH: return "HIP launch failure";
        default: return "unknown error";
    }
}

int vp_last_hip_error(void) { return g_last_hip_error.load(); }

const char *vp_version(void) { return "vipernl-mi355x 0.1 (gfx950)"; }

}  // extern "C"
