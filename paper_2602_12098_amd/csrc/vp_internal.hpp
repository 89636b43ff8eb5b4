// Internal launch helpers of the precoding library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vp.h"
#include "../../include/vp_learn.h"

namespace vp {

// Records the first HIP error of a launch sequence; VP_ELAUNCH on failure.
int launch_status();
// Keeps a HIP error code for vp_last_hip_error().
void record_hip_error(int code);

constexpr int kMaxN = 16;
constexpr int kMaxM = 64;
constexpr int kMaxKSearch = 4096;
constexpr int kMaxKMop = 1024;
constexpr int kNoAllocVectors = VP_NOALLOC_MAX_VECTORS;   // vectors per call of the allocation-free fallback
constexpr int kMaxDevices = 64;

// Inclusive scan over the 64 lanes of a wave by DPP moves: shifts by 1 and 2
// within each row of 16 lanes, by 4 and 8 into the upper banks of a row, then
// the last lane of row 0 (of rows 0-1) added to row 1 (to rows 2-3) and that
// of row 2 to row 3.  Lanes without a source add 0.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x) {
    const int v = (int)x;
    int s = v;
    s += __builtin_amdgcn_update_dpp(0, s, 0x111, 0xF, 0xF, true);   // row_shr:1
    s += __builtin_amdgcn_update_dpp(0, s, 0x112, 0xF, 0xF, true);   // row_shr:2
    s += __builtin_amdgcn_update_dpp(0, s, 0x114, 0xF, 0xE, true);   // row_shr:4, banks 1-3
    s += __builtin_amdgcn_update_dpp(0, s, 0x118, 0xF, 0xC, true);   // row_shr:8, banks 2-3
    s += __builtin_amdgcn_update_dpp(0, s, 0x142, 0xA, 0xF, true);   // row_bcast:15 into rows 1, 3
    s += __builtin_amdgcn_update_dpp(0, s, 0x143, 0xC, 0xF, true);   // row_bcast:31 into rows 2, 3
    return (uint32_t)s;
}

// Reductions over the 64 lanes of a wave by the same DPP pattern (lanes
// without a source contribute the identity); every lane gets the result.
template <int CTRL, int ROWS, int BANKS, class T, class Op>
__device__ __forceinline__ T dpp_combine(T x, int ident, Op op) {
    return op(x, __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(ident, __builtin_bit_cast(int, x), CTRL, ROWS,
                                                                   BANKS, false)));
}

template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T x, T ident, Op op) {
    const int id = __builtin_bit_cast(int, ident);
    x = dpp_combine<0x111, 0xF, 0xF>(x, id, op);   // row_shr:1
    x = dpp_combine<0x112, 0xF, 0xF>(x, id, op);   // row_shr:2
    x = dpp_combine<0x114, 0xF, 0xE>(x, id, op);   // row_shr:4, banks 1-3
    x = dpp_combine<0x118, 0xF, 0xC>(x, id, op);   // row_shr:8, banks 2-3
    x = dpp_combine<0x142, 0xA, 0xF>(x, id, op);   // row_bcast:15 into rows 1, 3
    x = dpp_combine<0x143, 0xC, 0xF>(x, id, op);   // row_bcast:31 into rows 2, 3
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}

__device__ __forceinline__ float wave_max_f(float x) {
    return wave_reduce(x, -INFINITY, [](float a, float b) { return fmaxf(a, b); });
}
__device__ __forceinline__ float wave_sum_f(float x) {
    return wave_reduce(x, 0.0f, [](float a, float b) { return a + b; });
}
__device__ __forceinline__ uint32_t wave_min_u(uint32_t x) {
    return wave_reduce(x, 0xffffffffu, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
}

// Raises a kernel's dynamic LDS limit (once per process at the call site); a
// failure surfaces as that kernel's launch error.
template <class K>
inline bool allow_dynamic_lds(K *kernel, size_t bytes) {
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
           hipSuccess;
}

// Launchers, one per kernel family (defined next to their kernels).
int launch_preprocess(const float2 *H, int n_sc, int N, int M, float alpha, float2 *W, float *w2,
                      uint8_t *perm, float2 *G, int32_t *status, hipStream_t st, bool sorted = true);
int launch_mop(const float *w2, int n_sc, int N, int K, uint8_t *paths, uint16_t *order, hipStream_t st);
int launch_mop_kbest(const float *w2, int n_sc, int N, int K, uint8_t *paths, uint16_t *order, hipStream_t st);
int launch_search(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, const uint8_t *paths,
                  const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, int N, uint32_t flags,
                  int8_t *l, float *cost, int32_t *kidx, hipStream_t st);
int launch_search_fallback(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau,
                           const uint8_t *paths,
                           const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, int N, uint32_t flags,
                           const float *mass, float theta, int32_t kidx_base, int8_t *l, float *cost, int32_t *kidx,
                           void *work, hipStream_t st);
int launch_search_fallback_noalloc(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau,
                                   const uint8_t *paths, const uint16_t *order, int K, int64_t pstride, int n_sc,
                                   int n_sym, int N, uint32_t flags, const float *mass, float theta,
                                   int32_t kidx_base, int8_t *l, float *cost, int32_t *kidx, hipStream_t st);
int launch_user_tau(const float *tau, const uint8_t *perm, int n_sc, int n_sym, int N, int M, float2 *W, float *w2,
                    float2 *G, const float2 *s, float2 *s_out, hipStream_t st);
int launch_fx_quantize(const float2 *W, const uint8_t *perm, const float2 *s, const float *tau, int n_sc, int n_sym,
                       int N, int frac_bits, int16_t *c0, int16_t *Vq, int16_t *wq, hipStream_t st);
int launch_fx_search(const int16_t *c0, const int16_t *Vq, const int16_t *wq, const uint8_t *perm,
                     const uint8_t *paths, int K, int64_t pstride, int n_sc, int n_sym, int N, int frac_bits,
                     uint32_t flags, int8_t *l, int64_t *ped, int32_t *kidx, hipStream_t st);
size_t logits_top64_work_bytes(int rows);
int launch_logits_top64(const uint16_t *X, int rows, const uint16_t *Wt, const float *bias, int V, int32_t *idx,
                        float *mass, void *work, hipStream_t st);
int launch_precode(const float2 *G, const float2 *s, const int8_t *l, const float *tau, const float *cost,
                   int n_sc, int n_sym, int N, int M, float P_T, float2 *x, hipStream_t st);

int launch_sphere(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym, int N,
                  const float *radius, int8_t *l, float *cost, int64_t *nodes, uint8_t *status,
                  long long max_nodes, hipStream_t st);

// Batched workload: one descriptor per group of subcarriers that share the
// number of users, perturbation interval, regularisation and path count.
// Arrays are concatenated group after group; offsets are in elements.
struct BatchGroup {
    int U;           // users = tree levels (1..16)
    int K;           // paths
    int n_sc;        // subcarriers
    int n_vec;       // n_sc * n_sym
    int vt;          // search tile: vectors per wave (1, 2, 4)
    int pl;          // search tile: paths per lane
    float tau, alpha;
    int sc0;         // first subcarrier (over all groups)
    int v0;          // first vector (over all groups)
    long long offH;  // H  [n_sc][U][M]
    long long offW;  // W  [n_sc][U(U+1)/2]
    long long offN;  // w2 / perm [n_sc][U]
    long long offG;  // G  [n_sc][M][U]
    long long offP;  // paths [n_sc][K][U]
    long long offS;  // s [U][n_vec] (and l [U][n_vec][2] at twice this offset)
};

int launch_batch_preprocess(const BatchGroup *groups, const int32_t *sc_group, int n_sc_total, int M,
                            const float2 *H, float2 *W, float *w2, uint8_t *perm, float2 *G, int32_t *status,
                            hipStream_t st);
void prepare_batch_kernels();   // kernel attributes, set once before a graph capture
int launch_batch_mop(const BatchGroup *groups, const int32_t *sc_group, int n_sc_total, int max_K, const float *w2,
                     uint8_t *paths, hipStream_t st);   // max_K: the largest K of the groups

// Learned path proposal (vp_learn.hip).
int launch_gemm(int M, int N, int K, const uint16_t *A, long long lda, int transA, const uint16_t *B, long long ldb,
                int transB, float *Cf, uint16_t *Cb, long long ldc, const float *bias, int relu,
                const uint16_t *mask, long long ldm, float alpha, hipStream_t st);
int launch_features(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym, int N,
                    unsigned kind, uint16_t *feat, hipStream_t st);
int launch_ranks(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym, int N,
                 const int8_t *l, uint8_t *ranks, hipStream_t st);
int launch_topk64(const float *S, int rows, int C, int32_t *idx, float *mass, hipStream_t st);
int launch_softmax_ce(const float *Z, int rows, int C, const int32_t *label, float scale, float *loss,
                      uint16_t *dZ, hipStream_t st);
int launch_colsum(const uint16_t *X, int rows, int cols, float *out, hipStream_t st);
int launch_learned_table(const uint8_t *vocab, int V, int N, const int32_t *top, int Kl, const uint8_t *fixed,
                         int Kfix, int Kf, int n_sc, int n_sym, uint8_t *table, hipStream_t st);

}  // namespace vp
