/*
 * vp_learn.h -- C ABI of the learned path proposal (gfx950).
 *
 * The paper selects the K candidate paths of a subcarrier from the channel
 * alone, by the Metric of Promise (Sec. III-A-2, eq. for M(r)).  The entry
 * points below let a small network propose a short per-vector path list
 * instead, scored over a fixed vocabulary of position vectors r (one rank
 * 0..8 per level); the proposal is evaluated by the unchanged path search of
 * vp.h (vp_search with VP_PATHS_PER_VECTOR), so the perturbation l is still an
 * exact Gaussian integer and its cost the exact PED sum of Sec. II-B.  The
 * paper itself has no learned component: this is an extension, and every
 * choice below (features, network shape, labels) is a stated design choice.
 *
 * Network: features (64) -> Linear 64x256 -> ReLU -> Linear 256x256 -> ReLU
 * -> Linear 256xV (logits over the vocabulary) -> 64 best entries.
 *
 * Conventions are those of vp.h (device pointers owned by the caller, calls
 * only enqueue on `stream`, VP_OK or a negative code).  bf16 values are passed
 * as their uint16_t bit patterns (the upper half of an IEEE float32).
 * Matrices are row-major with an explicit leading dimension (elements between
 * consecutive rows of the STORED matrix).
 */
#ifndef VP_LEARN_H
#define VP_LEARN_H

#include <stdint.h>

#include "vp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define VP_MLP_FEATURES 64 /* features per vector */
#define VP_TOPK 64         /* entries kept per vector by vp_topk64 */
#define VP_MAX_VOCAB 4096  /* largest vocabulary vp_topk64 accepts */

/* epilogue flags of vp_gemm_bf16 */
enum {
    VP_EPI_RELU = 1 /* C = max(C, 0) after the bias */
};

/* feature kinds of vp_mlp_features */
enum {
    VP_FEAT_ZERO_CENTRES = 0, /* centres of the zero perturbation */
    VP_FEAT_RANK0_WALK = 1    /* centres along the rank-0 (nearest point) walk */
};

/*
 * vp_mlp_features -- the network input of every vector (bf16 [n_vec][64]).
 *
 * W, perm from vp_preprocess.  For levels i < N (slots of levels >= N are 0),
 * with the level centres c_i of Sec. III-A-2:
 *   [i]       W_ii / mean_j W_jj      (the MoP weights of the subcarrier)
 * and, for kind VP_FEAT_ZERO_CENTRES, the centres of the zero perturbation,
 * c0_i = -(W s_pi)_i / (tau W_ii):
 *   [16 + i]  Re c0_i,  [32 + i]  Im c0_i
 *   [48 + i]  W_ii^2 |c0_i - b0(c0_i)|^2 / mean_j W_jj^2, b0 = nearest box point
 * or, for kind VP_FEAT_RANK0_WALK, the centres c_i of the path that takes the
 * nearest box point b_i at every level (float32, the search's own walk):
 *   [16 + i]  Re (c_i - b_i),  [32 + i]  Im (c_i - b_i)
 *   [48 + i]  W_ii^2 (d1_i - d0_i) / mean_j W_jj^2, d0_i / d1_i the squared
 *             distances of c_i to its nearest / second-nearest box point
 * A failed subcarrier (W_00 not finite and > 0) gets all-zero features.
 * Computed in float32 and rounded once to bf16 (round to nearest even).
 *
 * Errors: VP_EINVAL for NULL pointers, n_sc < 0, n_sym < 1, n_r < 1, tau <= 0
 * or not finite, an unknown kind; VP_EUNSUPPORTED for n_r > 16.
 */
int vp_mlp_features(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, int n_sc, int n_sym,
                    int n_r, uint32_t kind, uint16_t *feat, void *stream);

/*
 * vp_path_ranks -- the position vector of a given perturbation (labels).
 *
 * Walks the tree of vector v with the given l (user order, [N][n_vec][2] as
 * written by vp_search / vp_sphere_encode) and writes, per level i, the rank
 * of l_{perm[i]} among the 9 box points ordered by distance to the level's
 * centre c_i (ties in canonical order; the same float32 arithmetic as
 * vp_search), so that vp_search on that position vector reproduces l.  A
 * symbol outside the box is rank 15.  ranks: uint8 [n_vec][N].
 *
 * Errors: as vp_mlp_features, plus NULL l or ranks.
 */
int vp_path_ranks(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, const int8_t *l, int n_sc,
                  int n_sym, int n_r, uint8_t *ranks, void *stream);

/*
 * vp_gemm_bf16 -- C = epilogue(alpha * op(A) op(B) + bias) on the matrix cores.
 *
 * op(A) is m x k: A stored [m][lda] (trans_a = 0) or [k][lda] (trans_a = 1);
 * op(B) is k x n: B stored [k][ldb] (trans_b = 0) or [n][ldb] (trans_b = 1)
 * -- a torch Linear weight [out][in] is op(B) with trans_b = 1.  bf16
 * operands, float32 accumulation (v_mfma_f32_32x32x16_bf16).  Epilogue, in
 * order: bias[n] (float32, or NULL), VP_EPI_RELU, then if mask is non-NULL
 * every element whose mask entry (bf16 [m][ldm]) is not > 0 becomes 0 (the
 * ReLU derivative in a backward pass).  Output to C (float32 [m][ldc]) and/or
 * C_bf16 (bf16 [m][ldc], rounded to nearest even); at least one non-NULL.
 * k = 0 gives C = epilogue(bias).
 *
 * Errors: VP_EINVAL for m, n or k < 0, a leading dimension smaller than the
 * stored row length, NULL operands (when m, n > 0), both outputs NULL, or
 * unknown epilogue flags.
 */
int vp_gemm_bf16(int m, int n, int k, const uint16_t *A, int64_t lda, int trans_a, const uint16_t *B, int64_t ldb,
                 int trans_b, const float *bias, uint32_t epilogue, const uint16_t *mask, int64_t ldm, float alpha,
                 float *C, uint16_t *C_bf16, int64_t ldc, void *stream);

/*
 * vp_topk64 -- the 64 largest of each row of scores (float32 [rows][C]).
 *
 * idx (int32 [rows][64]) lists the selected columns by decreasing score,
 * equal scores by increasing column (a total order, so the result is unique;
 * -0.0 ranks below +0.0, a NaN with the sign bit clear above +inf and one
 * with it set below -inf).  mass (float32 [rows], or
 * NULL) receives the softmax probability mass of the selected columns,
 * sum_sel exp(x - max) / sum_all exp(x - max).
 *
 * Errors: VP_EINVAL for rows < 0, C < 64, NULL pointers; VP_EUNSUPPORTED for
 * C > 4096.
 */
int vp_topk64(const float *scores, int rows, int C, int32_t *idx, float *mass, void *stream);

/*
 * vp_logits_top64 -- the network's last layer fused with vp_topk64.
 *
 * idx and mass are what vp_topk64 gives for the logits
 * z = X Wt^T + bias (float32, as vp_gemm_bf16 computes them with trans_b:
 * bf16 products summed on the matrix cores in increasing k, then the bias),
 * but z is never written to memory: a first pass over the vocabulary bounds
 * each row's 64th largest logit from below, a second keeps the logits at or
 * above that bound, which are then ranked exactly.
 *
 *  X     bf16 [rows][256], 16-byte aligned (the second hidden layer)
 *  Wt    bf16 [V][256], 16-byte aligned;  bias float32 [V]
 *  V     a multiple of 128, 256 <= V <= VP_MAX_VOCAB
 *  idx   int32 [rows][64];  mass float32 [rows] or NULL
 *  work  device memory of vp_logits_top64_work_bytes(rows) bytes owned by
 *        the caller, 256-byte aligned (bounds, candidate lists, partial sums)
 *
 * Errors: VP_EINVAL for rows < 0 or NULL / misaligned pointers;
 * VP_EUNSUPPORTED for a V outside the range above.
 */
int vp_logits_top64(const uint16_t *X, int rows, const uint16_t *Wt, const float *bias, int V, int32_t *idx,
                    float *mass, void *work, void *stream);

/* Workspace bytes vp_logits_top64 needs for `rows` rows (about 2.1 KB each). */
int64_t vp_logits_top64_work_bytes(int rows);

/*
 * vp_softmax_xent -- softmax cross-entropy and its gradient (training).
 *
 * Per row: loss = logsumexp(z) - z[label]; dz = (softmax(z) - onehot(label))
 * * scale, written as bf16 [rows][C].  A row with label outside [0, C) (e.g.
 * -1: no label) has loss 0 and dz 0.  logits float32 [rows][C], label int32
 * [rows], loss float32 [rows].
 *
 * Errors: VP_EINVAL for rows < 0, C < 1, NULL pointers, scale not finite.
 */
int vp_softmax_xent(const float *logits, int rows, int C, const int32_t *label, float scale, float *loss,
                    uint16_t *dlogits, void *stream);

/*
 * vp_colsum_bf16 -- out[j] = sum_i X[i][j] over a bf16 [rows][cols] matrix,
 * accumulated in float32 in row order (the bias gradient).
 *
 * Errors: VP_EINVAL for rows < 0, cols < 0, NULL pointers.
 */
int vp_colsum_bf16(const uint16_t *X, int rows, int cols, float *out, void *stream);

/*
 * vp_learned_paths -- per-vector path tables for vp_search.
 *
 * table (uint8 [n_vec][K_learned + K_fixed][N]) holds, for vector v, the
 * vocabulary rows top[v][0..K_learned) (vocab: uint8 [V][N] rank vectors;
 * an index outside [0, V) is clamped), then the first K_fixed paths of the
 * subcarrier's fixed table (fixed: uint8 [n_sc][K_fixed_table][N], e.g. from
 * vp_paths_mop).  Use with vp_search(..., K_learned + K_fixed, stride
 * (K_learned + K_fixed) * N, flags | VP_PATHS_PER_VECTOR).
 *
 * Errors: VP_EINVAL for NULL pointers (where the sizes use them), negative
 * sizes, K_fixed > K_fixed_table, K_learned + K_fixed < 1, V < 1 with
 * K_learned > 0; VP_EUNSUPPORTED for n_r > 16 or K_learned + K_fixed > 4096.
 */
int vp_learned_paths(const uint8_t *vocab, int V, int n_r, const int32_t *top, int K_learned, const uint8_t *fixed,
                     int K_fixed_table, int K_fixed, int n_sc, int n_sym, uint8_t *table, void *stream);

/*
 * vp_search_fallback -- the fixed path set for the vectors whose proposal is
 * not confident (the fallback of the learned proposal; the paper has no
 * learned part, the search itself is that of vp_search: Sec. II-B PED
 * recursion, Sec. III-A-2 centres and DEMAP, Alg. 2 argmin).
 *
 * l, cost, kidx are in/out and hold on entry the proposal's search result
 * (vp_search with VP_PATHS_PER_VECTOR on the tables of vp_learned_paths).
 * Every vector v with !(mass[v] >= theta) -- a NaN mass counts as not
 * confident; mass from vp_topk64 -- is searched again over the subcarrier's
 * fixed table (tau [n_sc], paths, order, K, paths_sc_stride and VP_INCLUDE_ZERO as for
 * vp_search, e.g. the K = 512 MoP set of vp_paths_mop).  Where that cost is
 * below cost[v], v takes the fixed result: l from the winning fixed path,
 * its cost, and kidx = kidx_base + k (k = the fixed table's path index, K =
 * the zero perturbation).  Equal costs keep the proposal's result, so the
 * fixed set decides only where it is strictly better.  Vectors with
 * mass[v] >= theta are not touched.  theta = +inf sends every vector to the
 * fixed set, theta <= 0 none with a finite mass.
 *
 * work: device memory of 8 * n_sc * n_sym bytes owned by the caller (the
 * fixed search's cost and index per vector), 4-byte aligned.
 *
 * Errors: as vp_search (VP_PATHS_PER_VECTOR is not accepted: the fixed set is
 * one table per subcarrier), plus VP_EINVAL for NULL mass or work, theta NaN
 * or kidx_base < 0.
 */
int vp_search_fallback(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau, const uint8_t *paths,
                       const uint16_t *order, int K, int64_t paths_sc_stride, int n_sc, int n_sym, int n_r,
                       uint32_t flags, const float *mass, float theta, int32_t kidx_base, int8_t *l, float *cost,
                       int32_t *kidx, void *work, void *stream);

/* Most vectors one call of vp_search_fallback_noalloc may serve. */
#define VP_NOALLOC_MAX_VECTORS 65536

/*
 * vp_search_fallback_noalloc -- vp_search_fallback without the caller's
 * workspace, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Same arguments, results and errors as vp_search_fallback, minus `work`:
 * the fixed search's per-vector cost and index live in a workspace the
 * library holds in static device memory, one copy per GPU (512 KiB, held
 * until the process ends; its address is looked up on the first call on
 * each device).  The call allocates and frees nothing.  Limit: n_sc * n_sym
 * <= VP_NOALLOC_MAX_VECTORS (a 100 MHz, 14-symbol slot of 3276 subcarriers
 * fits), else VP_EUNSUPPORTED.  Every call on one GPU uses that GPU's one
 * workspace, so calls that overlap in time on the same GPU (on different
 * streams, or from several host threads) race and must be serialised by the
 * caller; calls on one stream are ordered and safe.  A failed look-up of the
 * workspace returns VP_ELAUNCH (see vp_last_hip_error()).
 */
int vp_search_fallback_noalloc(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau,
                               const uint8_t *paths, const uint16_t *order, int K, int64_t paths_sc_stride, int n_sc,
                               int n_sym, int n_r, uint32_t flags, const float *mass, float theta, int32_t kidx_base,
                               int8_t *l, float *cost, int32_t *kidx, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VP_LEARN_H */
