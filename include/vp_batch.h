/*
 * vp_batch.h -- C ABI of the batched, uneven precoding workload (gfx950).
 *
 * A slot of a multi-user system serves groups of subcarriers (resource-block
 * groups) with different numbers of users N, QAM orders (perturbation
 * intervals tau) and regularisations.  A batch plan runs the whole hot path
 * of vp.h -- preprocessing (Sec. III-A-1, Alg. 1), the MoP path set
 * (Sec. III-A-2), the path search with its argmin (Sec. II-B, Alg. 2) and the
 * precoding x = G (s + tau l) -- for every group of the slot as ONE captured
 * HIP graph: one kernel per stage over all groups, and a persistent search
 * kernel whose waves take (vector block, path chunk) tiles from an atomic
 * queue.  Results are those of the per-call entry points on each group (the
 * same float32 arithmetic path for path).  The paper builds one datapath per
 * size; this batching is an extension of it.
 *
 * Layout (all device arrays, concatenated group after group in the order of
 * `groups`; n_vec_g = n_sc_g * n_sym):
 *   H     vp_c32 [n_sc_g][N_g][n_t]        user-major rows, as vp_preprocess
 *   s     vp_c32 [N_g][n_vec_g]            structure of arrays per group
 *   l     int8   [N_g][n_vec_g][2]         output, per group like s
 *   cost  float  [sum n_vec_g]             output, gamma of each vector
 *   x     vp_c32 [sum n_vec_g][n_t]        output, precoded vectors
 * The plan binds these pointers at creation (a serving loop refills H and s in
 * place and calls vp_batch_run once per slot).  Vector v of group g is
 * subcarrier v / n_sym of the group, symbol v % n_sym.
 *
 * Ownership: vp_batch_create allocates the plan's device memory (factors,
 * path tables, tile queue; about 20 * sum_g n_sc_g * (N_g^2 + K_g N_g) bytes)
 * and its graph; vp_batch_destroy frees them.  A plan runs on the device that
 * was current at creation.  Calls on one plan must not overlap.
 */
#ifndef VP_BATCH_H
#define VP_BATCH_H

#include <stdint.h>

#include "vp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vp_batch vp_batch;

typedef struct {
    int32_t n_users; /* N of every subcarrier of the group, 1..16 */
    int32_t n_sc;    /* subcarriers in the group, >= 1 */
    int32_t K;       /* MoP paths per subcarrier, 1..512 and <= 9^N */
    float tau;       /* perturbation interval (2 sqrt(Q)), > 0 */
    float alpha;     /* regularisation, >= 0; 0 needs N <= n_t */
} vp_group;

#define VP_BATCH_MAX_CLASSES 8 /* distinct K values in one plan */

typedef struct {
    int32_t n_groups, n_sc, n_vec;
    int32_t n_tiles;                /* search tiles of the current tile shapes */
    int32_t persistent_workgroups;  /* one wave each */
    int32_t n_classes;              /* distinct K values */
    int32_t class_K[VP_BATCH_MAX_CLASSES];
    int32_t class_vt[VP_BATCH_MAX_CLASSES];  /* vectors per tile */
    int32_t class_pl[VP_BATCH_MAX_CLASSES];  /* paths per lane per tile */
    int32_t lpt_order;              /* 1: tiles queued by decreasing work */
    float default_ms;               /* slot time with the default shapes (vp_batch_tune), else 0 */
    float tuned_ms;                 /* slot time with the chosen shapes (vp_batch_tune), else 0 */
} vp_batch_info;

/*
 * vp_batch_create -- validate the groups, lay out and allocate the plan,
 * choose default tile shapes and capture the slot's kernels into a graph.
 * P_T > 0 scales each x by sqrt(P_T / cost) (Sec. II-B normalisation);
 * flags: VP_INCLUDE_ZERO (vp.h).  Nothing runs until vp_batch_run.
 *
 * Errors: VP_EINVAL for NULL pointers, n_groups < 1, n_sym < 1, a group with
 * n_sc < 1, K < 1, K > 9^N, tau <= 0, alpha < 0, alpha = 0 with N > n_t,
 * n_sc * n_sym > 65535, non-finite values or unknown flags;
 * VP_EUNSUPPORTED for N > 16, n_t > 64, K > 512, more than 65535 groups or
 * more than VP_BATCH_MAX_CLASSES distinct K; VP_ELAUNCH if an allocation or
 * the capture fails (nothing is left allocated).
 */
int vp_batch_create(const vp_group *groups, int n_groups, int n_t, int n_sym, float P_T, uint32_t flags,
                    const vp_c32 *H, const vp_c32 *s, vp_c32 *x, int8_t *l, float *cost, vp_batch **plan);

/* vp_batch_run -- enqueue one slot (the captured graph) on `stream`. */
int vp_batch_run(vp_batch *plan, void *stream);

/*
 * vp_batch_tune -- the autotuner: for each class of groups with equal K it
 * times the slot with every candidate tile shape (vectors per tile 1, 2, 4 x
 * paths per lane 1, 2, 4, 8, within 1/8 .. 2 K paths per tile), keeping the
 * others fixed, then both queue orders; keeps the fastest and records the
 * times.  Runs the slot about reps * (number of candidates) times and
 * synchronises `stream`; outputs hold the last run's results.
 */
int vp_batch_tune(vp_batch *plan, int reps, void *stream);

/* vp_batch_get_info -- sizes, tile shapes and tuning record. */
int vp_batch_get_info(const vp_batch *plan, vp_batch_info *info);

/*
 * vp_batch_buffers -- the plan's intermediate arrays (device, read-only for
 * the caller, valid until vp_batch_destroy), concatenated per group like the
 * inputs: W [n_sc_g][N_g(N_g+1)/2], w2 and perm [n_sc_g][N_g], G
 * [n_sc_g][n_t][N_g], status [sum n_sc_g], paths [n_sc_g][K_g][N_g].  Any
 * output pointer may be NULL.
 */
int vp_batch_buffers(const vp_batch *plan, const vp_c32 **W, const float **w2, const uint8_t **perm,
                     const vp_c32 **G, const int32_t **status, const uint8_t **paths);

/* vp_batch_destroy -- free the plan (NULL is allowed). */
int vp_batch_destroy(vp_batch *plan);

#ifdef __cplusplus
}
#endif

#endif /* VP_BATCH_H */
