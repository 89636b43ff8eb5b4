// Internal launch helpers of the precoding library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vp.h"

namespace vp {

// Records the first HIP error of a launch sequence; VP_ELAUNCH on failure.
int launch_status();

constexpr int kMaxN = 16;
constexpr int kMaxM = 64;
constexpr int kMaxKSearch = 4096;
constexpr int kMaxKMop = 1024;

// Launchers, one per kernel family (defined next to their kernels).
int launch_preprocess(const float2 *H, int n_sc, int N, int M, float alpha, float2 *W, float *w2,
                      uint8_t *perm, float2 *G, int32_t *status, hipStream_t st);
int launch_mop(const float *w2, int n_sc, int N, int K, uint8_t *paths, uint16_t *order, hipStream_t st);
int launch_mop_kbest(const float *w2, int n_sc, int N, int K, uint8_t *paths, uint16_t *order, hipStream_t st);
int launch_search(const float2 *W, const uint8_t *perm, const float2 *s, float tau, const uint8_t *paths,
                  const uint16_t *order, int K, int64_t pstride, int n_sc, int n_sym, int N, uint32_t flags,
                  int8_t *l, float *cost, int32_t *kidx, hipStream_t st);
int launch_precode(const float2 *G, const float2 *s, const int8_t *l, float tau, const float *cost,
                   int n_sc, int n_sym, int N, int M, float P_T, float2 *x, hipStream_t st);

int launch_sphere(const float2 *W, const uint8_t *perm, const float2 *s, float tau, int n_sc, int n_sym, int N,
                  const float *radius, int8_t *l, float *cost, int64_t *nodes, long long max_nodes,
                  hipStream_t st);

}  // namespace vp
