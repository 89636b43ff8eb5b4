// Device building blocks shared by the precoding kernels: the exact child
// order of the B = 1 box (DEMAP, Sec. III-A-2) and packed-triangle indexing.
//
// The functions are plain float32 code with every fused multiply-add written
// out, so that each kernel that walks a path (the search and its re-walk that
// materialises l) performs bit-identical arithmetic.  They also compile for
// the host, which lets the CPU test-suite check them exhaustively.
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define VP_HD __host__ __device__ __forceinline__
#else
#define VP_HD static inline
#endif

#include "demap_lut.h"
#include "region_lut.h"

// Offset of element (i, j), i >= j, in LAPACK column-major lower packed storage.
VP_HD constexpr int vp_pidx(int n, int i, int j) { return j * n - (j * (j - 1)) / 2 + (i - j); }

// The DEMAP routines take the level centre c twice: as cp = c - 1/2, because
// ceil(cp) is the integer nearest to c with a half-way c going to the smaller
// integer (the canonical index order of equal distances) in one instruction,
// and, for ranks above 0, as c itself, from which the per-axis gaps are
// formed: gaps taken from cp would lose the low bits of c and break the exact
// ties of symmetric centres (|c_x| = |c_y|) differently on the two axes.  The
// walk forms cp with one fused multiply-add from the residual and c only
// where a rank above 0 is asked for.

// Nearest box offset to c = cp + 1/2 (half-way: the smaller offset).
VP_HD float vp_o0(float cp) { return fminf(fmaxf(ceilf(cp), -1.0f), 1.0f); }

// Per-axis order of the three box offsets {-1, 0, 1} by squared distance to
// c: o0 nearest, o2 farthest, with gaps A = (c-o1)^2 - (c-o0)^2 and
// B = (c-o2)^2 - (c-o0)^2.  With t = |2c|: A = |1 - t|, and B = 1 + t when the
// nearest offset is 0, else 2t.  The side s of c (c = 0 counts as negative:
// then -1 comes before +1) gives o2 = -s and o1 = s - o0.  Whatever rounding
// did to cp and c, (o0, o1, o2) is a permutation of the box offsets with
// 0 <= A <= B, so every variant below makes the same, consistent choice.
struct vp_axis {
    float o0, o1, o2, A, B;
};

VP_HD vp_axis vp_axis_order(float cp, float c) {
    vp_axis r;
    const float o0 = vp_o0(cp);
    const float s = (c > 0.0f) ? 1.0f : -1.0f;
    const float t = fabsf(c + c);
    r.o0 = o0;
    r.o1 = s - o0;
    r.o2 = -s;
    r.A = fabsf(1.0f - t);
    r.B = (o0 == 0.0f) ? 1.0f + t : t + t;
    return r;
}

// Rank-0 child: the box point nearest to c.
VP_HD void vp_demap0(float cpx, float cpy, float &a, float &b) {
    a = vp_o0(cpx);
    b = vp_o0(cpy);
}

// Cell (0,1) -- y moved to its second offset -- precedes (1,0) when C < A, or
// on a tie when its x offset (o0 of x) is the smaller one (canonical order).
VP_HD bool vp_q1(const vp_axis &X, const vp_axis &Y) { return (Y.A < X.A) | ((Y.A == X.A) & (X.o0 < X.o1)); }

// Children of rank 0 or 1.  Non-short-circuit logic and selects, so that no
// lane-divergent branch is made.
VP_HD void vp_demap1(float cpx, float cpy, float cx, float cy, int rank, float &a, float &b) {
    const vp_axis X = vp_axis_order(cpx, cx);
    const vp_axis Y = vp_axis_order(cpy, cy);
    const bool q1 = vp_q1(X, Y);
    const bool r1 = (rank == 1);
    a = (r1 & !q1) ? X.o1 : X.o0;
    b = (r1 & q1) ? Y.o1 : Y.o0;
}

// Any rank 0..8: eight cell comparisons form the signature of the box order,
// a 256 x 9 table gives the cell (p, q) of the requested rank.
// Bit pattern of a non-negative float: increasing in the value, so that
// a < b  <=>  bits(a) < bits(b), and "a <= b" is bits(a) < bits(b) + 1.
VP_HD int32_t vp_fbits(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __float_as_int(x);
#else
    int32_t i;
    memcpy(&i, &x, sizeof i);
    return i;
#endif
}

VP_HD int vp_demap_signature(const vp_axis &X, const vp_axis &Y) {
    // each bit: the first cell comes first in the (distance, j) order; the two
    // cells always differ in x offset, which decides equal distances -- the
    // first cell then wins when its x offset is the smaller one, i.e. the
    // comparison is "<=" instead of "<".  All gaps are >= +0, so the
    // comparisons run on their bit patterns and the tie rule is a +1.
    const float A = X.A, B = X.B, C = Y.A, D = Y.B;
    const int32_t a = vp_fbits(A), b = vp_fbits(B), c = vp_fbits(C), d = vp_fbits(D);
    const int32_t ac = vp_fbits(A + C), bc = vp_fbits(B + C), ad = vp_fbits(A + D);
    const int32_t x01 = X.o0 < X.o1, x02 = X.o0 < X.o2, x12 = X.o1 < X.o2;
    const int32_t a1 = a + x01, b2 = b + x02, b12 = b + x12;
    int sig = (int)(c < a1);                      // (0,1) before (1,0)
    sig |= (int)(c < b2) << 1;                    // (0,1) before (2,0)
    sig |= (int)(d < a1) << 2;                    // (0,2) before (1,0)
    sig |= (int)(d < ac + x01) << 3;              // (0,2) before (1,1)
    sig |= (int)(d < b2) << 4;                    // (0,2) before (2,0)
    sig |= (int)(d < bc + x02) << 5;              // (0,2) before (2,1)
    sig |= (int)(ac < b12) << 6;                  // (1,1) before (2,0)
    sig |= (int)(ad < b12) << 7;                  // (1,2) before (2,0)
    return sig;
}

// Offset of per-axis rank p.  The three offsets are taken by value: a select
// over fields of one struct lets the compiler turn the choice into an
// indexed load from a stack copy (private memory).
VP_HD float vp_pick_offset(float o0, float o1, float o2, int p) {
    float v = (p == 1) ? o1 : o0;
    v = (p == 2) ? o2 : v;
    return v;
}

// Children of rank 0, 1 or 2.  In the box order a cell follows every cell
// that is nearer on both axes, so the rank-2 cell is, after a rank-1 cell
// (0,1), the first of (1,0) and (0,2), and after a rank-1 cell (1,0), the
// first of (0,1) and (2,0).  The three comparisons are bits 0, 2 and 1 of the
// signature above with the same tie rule (float compares of the same gaps),
// so the result is that of the table for every rank up to 2.
VP_HD void vp_demap2(float cpx, float cpy, float cx, float cy, int rank, float &a, float &b) {
    const vp_axis X = vp_axis_order(cpx, cx);
    const vp_axis Y = vp_axis_order(cpy, cy);
    const bool q1 = vp_q1(X, Y);                                                // (0,1) before (1,0)
    const bool y2 = (Y.B < X.A) | ((Y.B == X.A) & (X.o0 < X.o1));               // (0,2) before (1,0)
    const bool y1 = (Y.A < X.B) | ((Y.A == X.B) & (X.o0 < X.o2));               // (0,1) before (2,0)
    const bool r1 = (rank == 1), r2 = (rank == 2);
    // cell (p, q) of the requested rank, as per-axis ranks
    const bool p1 = (r1 & !q1) | (r2 & q1 & !y2);
    const bool p2 = r2 & !q1 & !y1;
    const bool s1 = (r1 & q1) | (r2 & !q1 & y1);
    const bool s2 = r2 & q1 & y2;
    a = p2 ? X.o2 : (p1 ? X.o1 : X.o0);
    b = s2 ? Y.o2 : (s1 ? Y.o1 : Y.o0);
}

VP_HD void vp_demapN(float cpx, float cpy, float cx, float cy, int rank, const uint8_t *lut, float &a, float &b) {
    const vp_axis X = vp_axis_order(cpx, cx);
    const vp_axis Y = vp_axis_order(cpy, cy);
    const int sig = vp_demap_signature(X, Y);
    const int cell = lut[sig * 9 + (rank < 8 ? rank : 8)];   // a rank beyond the box must not leave the table
    a = vp_pick_offset(X.o0, X.o1, X.o2, cell & 3);
    b = vp_pick_offset(Y.o0, Y.o1, Y.o2, cell >> 2);
}

// The paper's DEMAP (Sec. III-A-2, Alg. 2 "Demap", after FlexCore): the
// centre c is taken relative to its anchor n, the box point nearest to it
// (the rank-0 child, from cp); delta = c - n is folded by the symmetries of
// the square lattice (sign flips, then the swap that makes |dx| >= |dy|) and
// its cell on a grid of step 1/8 (12 cells along the larger coordinate)
// selects a stored order of the lattice offsets, the order of the cell's
// representative point (region_lut.h, generated by gen_region_lut.py).  Rank
// p is the anchor for p = 0, else the p-th stored offset that keeps the point
// inside the box.  An approximation of the exact order, exact at rank 0.
VP_HD void vp_demap_region(float cpx, float cpy, float cx, float cy, int rank, const uint8_t *rlut, float &a,
                           float &b) {
    const float nx = vp_o0(cpx), ny = vp_o0(cpy);
    const float dx = cx - nx, dy = cy - ny;
    const bool fx = dx < 0.0f, fy = dy < 0.0f;
    const float ax = fabsf(dx), ay = fabsf(dy);
    const bool sw = ay > ax;
    const float u = sw ? ay : ax, w = sw ? ax : ay;
    const int iu = (int)fminf(u * (float)VP_REGION_STEP_INV, (float)(VP_REGION_UCELLS - 1));
    const int iw0 = (int)(w * (float)VP_REGION_STEP_INV);
    const int iw = iw0 < iu ? iw0 : iu;
    const int reg = iu * (iu + 1) / 2 + iw;
    // the anchor under the same fold
    const float mx0 = fx ? -nx : nx, my0 = fy ? -ny : ny;
    const float mx = sw ? my0 : mx0, my = sw ? mx0 : my0;
    const int an = 3 * ((int)mx + 1) + ((int)my + 1);
    const int r = rank < 8 ? rank : 8;
    const int e = rlut[(reg * 9 + an) * 9 + r];
    const float ox = (float)((e & 15) - 2), oy = (float)((e >> 4) - 2);   // folded offset
    const float ux = sw ? oy : ox, uy = sw ? ox : oy;                     // unswap, then unflip
    a = nx + (fx ? -ux : ux);
    b = ny + (fy ? -uy : uy);
}

// Box code of a perturbation symbol: j = 3 (a + 1) + (b + 1).
VP_HD int vp_box_code(float a, float b) { return 3 * ((int)a + 1) + ((int)b + 1); }
