/*
 * Exact vector perturbation over the B = 1 box by a depth-first
 * Schnorr-Euchner sphere encoder, in float64.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  The product library never
 * links, loads or calls this file; it shares no code with the HIP path.
 *
 * It minimises || W (s_pi + tau l) ||^2 over l in {-1,0,1}^2 per level (eq:se
 * after the triangular step of eq_qrse, with l = -t).  The tree is walked from
 * level 0 (the root of the lower-triangular W); the children of a node are
 * visited in increasing squared distance to the level centre
 * c_i = -r_i / (tau W_ii), equal distances in canonical box order
 * j = 3 (bx + 1) + (by + 1) (Sec. III-A-2), and a subtree is cut as soon as its
 * partial Euclidean distance (the PED recursion of Sec. II-B) is not below the
 * best full cost found so far.
 *
 * Layout: W is [n][n] complex (interleaved re, im), row-major, lower
 * triangular, search order.  st is [nvec][n] complex = W s_pi per vector.
 * wsel [nvec] (may be NULL) picks, per vector, which of several stacked W
 * matrices to use (one per subcarrier).
 * Outputs: jcode [nvec][n] box index per level, cost [nvec], nodes [nvec].
 * radius [nvec] (may be NULL) is the initial bound; +inf means none.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define NMAX 16

static const double BX[9] = {-1, -1, -1, 0, 0, 0, 1, 1, 1};
static const double BY[9] = {-1, 0, 1, -1, 0, 1, -1, 0, 1};

typedef struct {
    int n;
    double tau;
    const double *W; /* [n][n][2] */
    double best;
    int best_j[NMAX];
    int cur_j[NMAX];
    int64_t nodes;
} se_ctx;

static void order9(double cx, double cy, int ord[9], double d[9]) {
    for (int j = 0; j < 9; ++j) {
        double dx = cx - BX[j], dy = cy - BY[j];
        d[j] = dx * dx + dy * dy;
        ord[j] = j;
    }
    /* insertion sort on (d, j): stable, so equal distances keep j order */
    for (int a = 1; a < 9; ++a) {
        int v = ord[a];
        int b = a - 1;
        while (b >= 0 && d[ord[b]] > d[v]) {
            ord[b + 1] = ord[b];
            --b;
        }
        ord[b + 1] = v;
    }
}

static void rec(se_ctx *c, int i, const double *resid /* [n][2] */, double ped) {
    const int n = c->n;
    const double *W = c->W;
    double wre = W[2 * (i * n + i)], wim = W[2 * (i * n + i) + 1];
    double den = c->tau * (wre * wre + wim * wim);
    /* c_i = -r_i / (tau W_ii) */
    double rre = resid[2 * i], rim = resid[2 * i + 1];
    double cx = -(rre * wre + rim * wim) / den;
    double cy = -(rim * wre - rre * wim) / den;
    double d[9];
    int ord[9];
    order9(cx, cy, ord, d);
    double wabs2 = wre * wre + wim * wim;
    for (int a = 0; a < 9; ++a) {
        int j = ord[a];
        double nped = ped + c->tau * c->tau * wabs2 * d[j];
        if (nped >= c->best) break;
        c->nodes++;
        c->cur_j[i] = j;
        if (i + 1 == n) {
            c->best = nped;
            memcpy(c->best_j, c->cur_j, sizeof(int) * n);
        } else {
            double nres[2 * NMAX];
            memcpy(nres, resid, sizeof(double) * 2 * n);
            double lre = BX[j], lim = BY[j];
            for (int m = i + 1; m < n; ++m) {
                double are = W[2 * (m * n + i)], aim = W[2 * (m * n + i) + 1];
                nres[2 * m] += c->tau * (are * lre - aim * lim);
                nres[2 * m + 1] += c->tau * (are * lim + aim * lre);
            }
            rec(c, i + 1, nres, nped);
        }
    }
}

int oracle_se(int n, int nvec, const double *W, const int32_t *wsel, const double *st,
              double tau, const double *radius, int32_t *jcode, double *cost, int64_t *nodes) {
    if (n < 1 || n > NMAX) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < nvec; ++v) {
        se_ctx c;
        c.n = n;
        c.tau = tau;
        c.W = W + (wsel ? (size_t)2 * n * n * wsel[v] : 0);
        c.best = radius ? radius[v] : INFINITY;
        c.nodes = 0;
        for (int i = 0; i < n; ++i) c.best_j[i] = -1;
        rec(&c, 0, st + (size_t)2 * n * v, 0.0);
        for (int i = 0; i < n; ++i) jcode[(size_t)v * n + i] = c.best_j[i];
        cost[v] = c.best;
        nodes[v] = c.nodes;
    }
    return 0;
}
