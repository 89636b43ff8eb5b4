/*
 * vp.h -- C ABI of the MI355X (gfx950) vector-perturbation precoding library.
 *
 * ViPer NL-COMM vector perturbation (Thomas, Katsaros, Jayawardena,
 * Nikitopoulos, arXiv 2602.12098): per-subcarrier sorted regularised-ZF
 * preprocessing, channel-only selection of the K most promising tree paths
 * by the Metric of Promise, and per-vector evaluation of those K paths with
 * an argmin, followed by the linear precoding x = G (s + tau l).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller.  Nothing is
 *    allocated, freed or synchronised by these calls: each one validates its
 *    scalar arguments on the host and enqueues kernels on `stream` (a
 *    hipStream_t; NULL is the default stream), then returns.
 *  - Complex numbers are vp_c32 {re, im} (interleaved float32, 8 bytes).
 *  - N = n_r = users/streams = tree levels (1..16); M = n_t = AP antennas
 *    (1..64).  Row i of H is user i (Sec. II).
 *  - Vector index v = sc * n_sym + sym, n_vec = n_sc * n_sym.
 *  - "Search order" is the level order of the tree (level 0 is the root);
 *    perm[sc][i] is the user served at level i.
 *  - The perturbation is l = -t relative to the paper's v - tau t
 *    (Sec. II-B), so u = s + tau l and both are Gaussian integers with
 *    |Re l|, |Im l| <= 1 (the B = 1 box of Sec. III-A-2).
 *  - Return value: VP_OK, or a negative code for an argument / launch error
 *    (then nothing, or not everything, was enqueued).  Data-dependent
 *    failures are reported per subcarrier in `status` instead.
 *  - Calls on one stream run in order; calls are reentrant and thread-safe
 *    (the library keeps no mutable state besides the last HIP error code).
 */
#ifndef VP_H
#define VP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float re, im;
} vp_c32;

enum {
    VP_OK = 0,
    VP_EINVAL = -1,       /* null pointer, bad size, tau <= 0, K > 9^N, alpha = 0 with N > M, ... */
    VP_EUNSUPPORTED = -2, /* N > 16, M > 64, K > 4096 */
    VP_ELAUNCH = -3       /* a HIP launch failed; see vp_last_hip_error() */
};

/* per-subcarrier status written by vp_preprocess */
enum {
    VP_STATUS_OK = 0,
    VP_STATUS_NOT_PD = 1,    /* a pivot <= N * eps32 * max_u A_uu: A not positive definite */
    VP_STATUS_NONFINITE = 2  /* H or alpha not finite */
};

/* flags for vp_search */
enum {
    VP_INCLUDE_ZERO = 1,     /* also evaluate l = 0 (plain RZF) as candidate index K */
    VP_PATHS_PER_VECTOR = 2, /* one [K][N] table per vector (paths + v * paths_sc_stride) */
    VP_DEMAP_REGION = 4      /* children of rank >= 1 from the paper's region table (Sec. III-A-2 DEMAP),
                                an approximation of the exact order; rank 0 is the same */
};

/* per-vector status written by vp_sphere_encode */
enum {
    VP_SE_EXACT = 0,      /* the search completed: l is the exact minimiser over the box */
    VP_SE_EXHAUSTED = 1,  /* the node budget ran out: l and cost are the best point found so far
                             (cost NaN, l = 0 if none was found inside the radius) */
    VP_SE_NONE = 2        /* the search completed and no point lies inside the radius: l = 0, cost NaN */
};

/* Size (in vp_c32) of one packed lower-triangular N x N matrix. */
#define VP_PACKED(N) ((N) * ((N) + 1) / 2)

/*
 * vp_preprocess -- regularised sorted factorisation (Sec. III-A-1, Alg. 1,
 * eq:invr; Alg. 2 "regularise & factorise").
 *
 * For every subcarrier: A = H H^H + alpha I (alpha = lambda^2; alpha = 0 is
 * zero forcing, Sec. II-A).  A is factorised as A[pi][:,pi] = Lbar Lbar^H,
 * choosing at each step the remaining user with the smallest Schur-complement
 * diagonal (ties -> smaller user index): this is the sorted RQ of
 * [H, lambda I] computed by Alg. 1 (Lbar = Rbar).  W = Lbar^{-1} is the
 * R-tilde of Sec. III-A-2.
 *
 *  H      [n_sc][N][M]   input channel, row-major
 *  alpha  >= 0 (finite)
 *  W      [n_sc][VP_PACKED(N)]  output, lower triangle of W in LAPACK
 *         column-major packed order: element (i, j), i >= j, lives at
 *         j*N - j*(j-1)/2 + (i - j).  The diagonal is real and positive.
 *  w2     [n_sc][N]  output, |W_ii|^2, the Metric-of-Promise weights (eq_mop)
 *  perm   [n_sc][N]  output, level -> user
 *  G      [n_sc][M][N] output or NULL: G = H^H A^{-1}, the RZF precoder
 *         (x = G u, Sec. II-A; equal to the Tikhonov pseudo-inverse of
 *         Sec. III-A-1)
 *  status [n_sc]     output, VP_STATUS_*; on failure W and G are filled with
 *         NaN and w2 with +inf, so later calls see the failure.
 *
 * Errors: VP_EINVAL for NULL H/W/w2/perm/status, n_sc < 0, N < 1, M < 1,
 * alpha < 0 or not finite, or alpha == 0 with N > M (rank-deficient A);
 * VP_EUNSUPPORTED for N > 16 or M > 64.  n_sc == 0 is a no-op.
 */
int vp_preprocess(const vp_c32 *H, int n_sc, int n_r, int n_t, float alpha, vp_c32 *W, float *w2,
                  uint8_t *perm, vp_c32 *G, int32_t *status, void *stream);

/*
 * vp_preprocess_unsorted -- vp_preprocess without the sorting of Alg. 1: the
 * plain Cholesky factorisation A = Lbar Lbar^H in the users' own order
 * (perm = identity).  It is the unsorted reference against which Sec. III-B
 * measures the gain of the improved sorted QR decomposition; the search,
 * precoding and sphere encoder accept its outputs unchanged.  Arguments,
 * outputs and errors as vp_preprocess.
 */
int vp_preprocess_unsorted(const vp_c32 *H, int n_sc, int n_r, int n_t, float alpha, vp_c32 *W, float *w2,
                           uint8_t *perm, vp_c32 *G, int32_t *status, void *stream);

/*
 * vp_paths_mop -- most promising paths (Sec. III-A-2, eq_mop; Alg. 2
 * "MoP-Search").
 *
 * For every subcarrier, the K position vectors r in {0..8}^N (r = p - 1,
 * 0-based ranks; rank 0 is the closest child) with the smallest Metric of
 * Promise M(r) = sum_i w2_i r_i -- the result of the paper's breadth-first
 * K-best search over the partial metrics.  Partial sums are formed in
 * float64 in level order; ties in M are broken by the lexicographic order of
 * r (level 0 most significant), which makes the K-best result equal to the
 * exact K smallest.  Output order is (M, lexicographic r): path k = 0 is the
 * zero-rank (Babai) path.  (The kernel finds the same set by enumerating
 * all r below a counted threshold; see the design notes.)
 *
 *  w2       [n_sc][N]     input (from vp_preprocess), finite and > 0; a
 *                         subcarrier with any other weight gets all-zero ranks
 *  paths    [n_sc][K][N]  output ranks 0..8, uint8
 *  order    [n_sc][2][K]  output or NULL: order[sc][0][j] is the path index k
 *                         of the j-th path in lexicographic order (level 0
 *                         most significant); order[sc][1][j] the same with
 *                         the deepest level most significant.  vp_search uses
 *                         the first to share the work of common path prefixes
 *                         and the second to batch paths whose deep levels need
 *                         the same kind of DEMAP work.
 *
 * Errors: VP_EINVAL for NULL pointers, n_sc < 0, N < 1, K < 1, K > 9^N;
 * VP_EUNSUPPORTED for N > 16 or K > 1024.
 */
int vp_paths_mop(const float *w2, int n_sc, int n_r, int K, uint8_t *paths, uint16_t *order, void *stream);

/*
 * vp_search -- per-vector evaluation of K paths and argmin (Sec. II-B PED
 * recursion, Sec. III-A-2 centres and DEMAP, Alg. 2 parallel post-processing).
 *
 * For every vector v of subcarrier sc and every path k: s_pi = s[perm] (user
 * -> level order), s-tilde = W s_pi, and down the levels i = 0..N-1 the centre
 * c_i = -(s-tilde_i + tau sum_{j<i} W_ij l_j) / (tau W_ii); l_i is the box
 * point of rank paths[k][i] in the order of increasing |c_i - b|^2 (equal
 * distances in canonical order j = 3(bx+1) + (by+1)).  cost_k =
 * || W (s_pi + tau l) ||^2.  The result is the k with the smallest cost (ties
 * -> smaller k); with VP_INCLUDE_ZERO the zero perturbation competes as index
 * K.  cost is gamma_VP of Alg. 2 (the squared norm that sets the transmit
 * normalisation).  With VP_DEMAP_REGION the child of rank >= 1 comes instead
 * from the paper's region-indexed table: the centre relative to its nearest
 * box point, folded by the square's symmetries, selects one of 78 cells of a
 * 1/8 grid, each holding the offset order of its representative point; rank
 * p > 0 is the p-th stored offset that stays inside the box.
 *
 *  W, perm  from vp_preprocess (W's diagonal must be real and > 0)
 *  s        [N][n_vec]  symbols, structure of arrays (user-major), user order
 *  tau      [n_sc] perturbation interval of each subcarrier, 2 sqrt(Q) for
 *           its Q-QAM constellation (Sec. II-B), so that one call may mix
 *           modulation orders across subcarriers
 *  paths    ranks uint8; subcarrier sc uses paths + sc * paths_sc_stride,
 *           a [K][N] table (stride 0 = one table for every subcarrier).
 *           With VP_PATHS_PER_VECTOR vector v uses paths + v * paths_sc_stride
 *           (stride must be K*N; e.g. the tables of vp_learned_paths).
 *  order    [n_sc][2][K] or NULL: the tables' two orders as written by
 *           vp_paths_mop (requires paths_sc_stride == K*N).  With them, the
 *           work of each distinct prefix of the first N/4 levels is done once
 *           per vector instead of once per path; results are identical.  A
 *           table whose prefix-sharing state (about 14 K bytes plus 24 KiB at
 *           N = 16) exceeds the LDS one workgroup may hold is searched per
 *           path instead, with the same results.
 *  l        [N][n_vec][2] output int8 (re, im) in {-1, 0, 1}, user order
 *  cost     [n_vec] output
 *  kidx     [n_vec] output, selected path (K = zero perturbation)
 *
 * A subcarrier whose W_00 is not finite and > 0 (a failed vp_preprocess), or
 * whose tau is not finite and > 0, gets l = 0, cost = NaN, kidx = -1.
 *
 * Errors: VP_EINVAL for NULL pointers, n_sc < 0, n_sym < 1, N < 1, K < 1,
 * paths_sc_stride < 0 (or 0 < stride < K*N), order
 * given with paths_sc_stride != K*N, unknown flags, VP_PATHS_PER_VECTOR with
 * an order or with paths_sc_stride != K*N; VP_EUNSUPPORTED for N > 16 or
 * K > 4096.
 */
int vp_search(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau,
              const uint8_t *paths, const uint16_t *order, int K, int64_t paths_sc_stride, int n_sc,
              int n_sym, int n_r, uint32_t flags, int8_t *l, float *cost, int32_t *kidx, void *stream);

/*
 * vp_precode -- precoded vector (Alg. 2 output; Sec. IV-B channel-inverse,
 * gamma and PV blocks).
 *
 * x_v = G (s_v + tau_sc l_v); with P_T > 0 also scaled by sqrt(P_T / cost_v),
 * the transmit-power normalisation of Sec. II-B.  A vector whose cost is not
 * finite and > 0 is written as NaN when P_T > 0, and so is every vector of a
 * subcarrier whose tau is not finite and > 0.
 *
 *  G     [n_sc][M][N]  from vp_preprocess
 *  s     [N][n_vec], l [N][n_vec][2], tau [n_sc] as in vp_search
 *  cost  [n_vec] (may be NULL when P_T == 0)
 *  x     [n_vec][M] output
 *
 * Errors: VP_EINVAL for NULL pointers, bad sizes, P_T < 0, or cost == NULL
 * with P_T > 0; VP_EUNSUPPORTED for N > 16 or M > 64.
 */
int vp_precode(const vp_c32 *G, const vp_c32 *s, const int8_t *l, const float *tau, const float *cost,
               int n_sc, int n_sym, int n_r, int n_t, float P_T, vp_c32 *x, void *stream);

/*
 * vp_apply_user_tau -- one perturbation interval per user (Sec. II-B with a
 * QAM order per user; the paper's tau is one system constant).
 *
 * The search objective || W (s_pi + D l) ||^2 with D = diag(tau of the user
 * at each level) equals || W' (s'_pi + l) ||^2 with W' = W D and s' = s / tau
 * per user, so after this call the other entry points run unchanged with
 * tau = 1 on every subcarrier: the per-level tau enters the walk through W'
 * (centres c_i = -r_i / (tau_i W_ii), residual steps tau_i W_mi l_i) and the
 * Metric-of-Promise weights become |W'_ii|^2 = tau_i^2 w2_i.  G' = G diag(tau)
 * gives x = G' (s' + l) = G (s + tau l).  For QAM, tau = 2 sqrt(Q) is a power of
 * two and every scaling here is exact in float32.
 *
 *  tau_user [n_sc][N]  per-user intervals (user order), finite and > 0
 *  perm     [n_sc][N]  from vp_preprocess
 *  W, w2    in/out: scaled in place (vp_preprocess outputs)
 *  G        in/out or NULL: scaled in place
 *  s        [N][n_vec] input symbols;  s_out [N][n_vec] output s' (may equal s)
 *
 * Errors: VP_EINVAL for NULL pointers or bad sizes; VP_EUNSUPPORTED for
 * N > 16 or M > 64.  Run it once per slot, after vp_preprocess and before
 * vp_paths_mop.
 */
int vp_apply_user_tau(const float *tau_user, const uint8_t *perm, int n_sc, int n_sym, int n_r, int n_t, vp_c32 *W,
                      float *w2, vp_c32 *G, const vp_c32 *s, vp_c32 *s_out, void *stream);

/*
 * vp_sphere_encode -- exact vector perturbation over the B = 1 box (eq:se,
 * solved as the tree search of eq_qrse with the PED recursion of Sec. II-B).
 *
 * For every vector, the l in {-1,0,1}^2N minimising || W (s_pi + tau l) ||^2,
 * found by a depth-first Schnorr-Euchner search (children in increasing
 * distance to the level centre, equal distances in canonical box order).
 * This is the reference the power gap of the K-path method is measured
 * against, and the label generator of the learned path proposal.
 *
 *  W, perm, s, n_sc, n_sym, n_r  as in vp_search
 *  tau       one perturbation interval for every subcarrier, > 0
 *  radius    [n_vec] initial squared radius, or NULL for none; a radius at or
 *            slightly above a known solution's cost (e.g. vp_search's cost)
 *            only prunes
 *  max_nodes per-vector node budget (> 0); a vector that exhausts it keeps the
 *            best point found so far (status VP_SE_EXHAUSTED); a vector with
 *            no point inside its radius gets l = 0 and cost = NaN
 *  l         [N][n_vec][2] output, user order;  cost [n_vec] output
 *  nodes     [n_vec] output (int64) or NULL: tree nodes visited
 *  status    [n_vec] output (uint8, VP_SE_*) or NULL
 *
 * Errors: as vp_search (no K / paths), plus max_nodes <= 0 -> VP_EINVAL.
 */
int vp_sphere_encode(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, float tau, int n_sc, int n_sym,
                     int n_r, const float *radius, int64_t max_nodes, int8_t *l, float *cost, int64_t *nodes,
                     uint8_t *status, void *stream);

/*
 * vp_fx_quantize -- the walk's inputs in signed 16-bit fixed point with
 * frac_bits fractional bits (the number format of the accelerator, Sec. V
 * precision study: 16-bit words, F = 8..13 fractional bits).
 *
 * The fixed-point walk follows the level centres c_m = -r_m / (tau W_mm)
 * instead of the residuals: the child l_i of level i moves every centre below
 * it by V_mi l_i with V_mi = -W_mi / W_mm, and adds w_i |l_i - c_i|^2 to the
 * PED, w_i = W_ii^2 / max_j W_jj^2 (the PED of the float walk divided by
 * tau^2 max_j W_jj^2, which orders paths the same way).  Every value is
 * rounded to nearest (ties to even) after scaling by 2^frac_bits and
 * saturated to [-32768, 32767]; the arithmetic before rounding is float32.
 *
 *  W, perm, s, tau, n_sc, n_sym, n_r  as in vp_search; tau finite and > 0
 *  c0  [n_vec][N][2] output int16: start centres (re, im) in level order
 *  V   [n_sc][N(N-1)/2][2] output int16: V_mi for m > i, entry m(m-1)/2 + i
 *  w   [n_sc][N] output int16
 *
 * Non-finite values (a failed vp_preprocess) quantise to 0 (NaN) or
 * saturate (infinities).  Errors: VP_EINVAL for NULL pointers, bad sizes or
 * frac_bits outside 8..13; VP_EUNSUPPORTED for N > 16.
 */
int vp_fx_quantize(const vp_c32 *W, const uint8_t *perm, const vp_c32 *s, const float *tau, int n_sc, int n_sym,
                   int n_r, int frac_bits, int16_t *c0, int16_t *V, int16_t *w, void *stream);

/*
 * vp_fx_search -- the same-path-set search (Alg. 2) walked in 16-bit fixed
 * point on the outputs of vp_fx_quantize.
 *
 * Every path's walk is integer arithmetic: the nine squared distances to the
 * box points come from differences saturated to 16 bits (each < 2^31), the
 * path's rank picks the box point in (distance, box index) order with box
 * index 3 (re + 1) + (im + 1), the PED sum_i w_i d_i is exact in 64 bits, and
 * each centre step c_m + V_mi l_i is saturated to 16 bits.  With
 * VP_INCLUDE_ZERO the zero perturbation is candidate K.  The chosen path has
 * the smallest (PED, path index).
 *
 *  c0, V, w   from vp_fx_quantize (same n_sc, n_sym, n_r, frac_bits)
 *  perm       [n_sc][N] from vp_preprocess (writes l in user order)
 *  paths, K, paths_sc_stride  as in vp_search (no order, no per-vector paths)
 *  flags      0 or VP_INCLUDE_ZERO
 *  l          [N][n_vec][2] output int8, user order
 *  ped        [n_vec] output int64: the chosen path's fixed-point PED
 *  kidx       [n_vec] output: chosen path (K = zero perturbation)
 *
 * Errors: VP_EINVAL for NULL pointers, bad sizes or strides, unknown flags,
 * frac_bits outside 8..13; VP_EUNSUPPORTED for N > 16 or K > 4096.
 */
int vp_fx_search(const int16_t *c0, const int16_t *V, const int16_t *w, const uint8_t *perm, const uint8_t *paths,
                 int K, int64_t paths_sc_stride, int n_sc, int n_sym, int n_r, int frac_bits, uint32_t flags,
                 int8_t *l, int64_t *ped, int32_t *kidx, void *stream);

/* Human-readable text for a return code. */
const char *vp_strerror(int code);

/* The hipError_t value of the last failed launch (0 if none). */
int vp_last_hip_error(void);

/* Library version string. */
const char *vp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */
