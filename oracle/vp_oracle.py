"""FP64 CPU oracle for ViPer NL-COMM vector-perturbation precoding.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything in this directory; only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark do.  It shares no code,
tables or constants with the HIP path.

Every function is a plain, slow, obviously-correct restatement of the paper
(Thomas, Katsaros, Jayawardena, Nikitopoulos, "ViPer NL-COMM: Making Vector
Perturbation Precoding Practical", arXiv 2602.12098), in complex128 / float64.
Citations name the section, equation label or algorithm.

Notation (search order = level order of the tree; level 0 is the root):
  A       = H H^H + alpha I                        (RZF Gram matrix, Sec. II-A / III-A-1)
  pi      : level -> user permutation              (the sorting P-bar of Alg. 1)
  Lbar    : lower-triangular, A[pi][:,pi] = Lbar Lbar^H   (Rbar of Alg. 1)
  W       = Lbar^{-1} (lower-triangular)           (R-tilde = Rbar^{-1}, Sec. III-A-2)
  w_i     = |W_ii|^2                               (MoP weights, eq_mop)
  u       = s + tau * l    (l = -t: the paper writes v - tau t, Sec. II-B)
  cost(l) = || W u_pi ||^2 = u^H A^{-1} u          (eq:se after the unitary step, eq_qrse)

Readings of the paper that this file fixes (each is also listed in the
design notes):
  * Alg. 1 is read as sorted modified Gram-Schmidt on the rows of
    [H, lambda I]: the argmin runs over the rows not yet processed, each new
    basis row is normalised by Rbar_ii, and the projection uses q_j (the
    printed listing drops the index).  This equals a Cholesky factorisation
    of A with the smallest remaining Schur-complement diagonal as pivot.
  * With sorting, the implicit inverse of eq:invr becomes
    Rbar^{-1} = Q2[:, pi] / lambda (columns permuted).
  * The child order at each level is the exact order of the nine points of
    the B=1 box by squared distance to the level centre (Sec. III-A-2,
    "position vector ... ordered according to increasing PEDs"); equal
    distances are ordered by the canonical box index j = 3(bx+1) + (by+1).
  * Ties elsewhere: pivots -> smaller user index; MoP -> lexicographic
    position vector (level 0 most significant); path costs -> smaller path
    index k (the zero perturbation, when included, has index K).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass
from fractions import Fraction
from functools import lru_cache
from typing import Optional

import numpy as np

# The B = 1 perturbation box (Sec. III-A-2: |Re t|, |Im t| <= 1, |B| = 9),
# in canonical index order j = 3 (bx + 1) + (by + 1).
BOX = np.array([complex(bx, by) for bx in (-1, 0, 1) for by in (-1, 0, 1)], dtype=np.complex128)
NBOX = 9

def sqabs(z):
    """|z|^2 as Re^2 + Im^2: no square root, so two equal distances compare
    equal whenever their operands are exact (the tie rule of the box order
    needs exact ties to be seen as ties)."""
    z = np.asarray(z)
    return z.real ** 2 + z.imag ** 2


STATUS_OK = 0
STATUS_NOT_PD = 1
STATUS_NONFINITE = 2


# ---------------------------------------------------------------------------
# Preprocessing (Sec. III-A-1, Alg. 1, eq:invr)
# ---------------------------------------------------------------------------

def gram(H: np.ndarray, alpha: float) -> np.ndarray:
    """A = H H^H + alpha I (the regularised Gram matrix of Sec. II-A and Sec. III-A-1)."""
    H = np.asarray(H, dtype=np.complex128)
    return H @ H.conj().T + alpha * np.eye(H.shape[0])


@dataclass
class Prep:
    L: np.ndarray        # Lbar, lower, search order
    W: np.ndarray        # Lbar^{-1}
    perm: np.ndarray     # level -> user
    w2: np.ndarray       # |W_ii|^2
    G: Optional[np.ndarray]   # H^H A^{-1}   [M][N]
    status: int
    pivots: np.ndarray   # Schur-complement diagonal chosen at each step
    pivot_margin: np.ndarray  # gap to the runner-up pivot at each step (inf if none)


def cholesky_minpivot(A: np.ndarray):
    """Pivoted Cholesky A[pi][:,pi] = L L^H choosing, at each step, the remaining
    user whose Schur-complement diagonal is smallest (ties -> smaller user index).

    This is the factorisation that Alg. 1 (ISRQD) produces: its squared row norms
    after each Gram-Schmidt sweep are exactly these Schur-complement diagonals.
    Returns (L, perm, pivots, margins, status)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    C = np.zeros((n, n), dtype=np.complex128)   # C[u, k]: user u's entry in column k
    remaining = list(range(n))
    perm = []
    pivots = np.zeros(n)
    margins = np.full(n, np.inf)
    status = STATUS_OK
    # A pivot at or below n * eps * max_u A_uu is treated as zero: A is then not
    # numerically positive definite (e.g. alpha = 0 with more users than antennas).
    floor = n * np.finfo(np.float64).eps * float(np.max(np.real(np.diag(A))))
    for i in range(n):
        schur = np.array([A[u, u].real - np.sum(np.abs(C[u, :i]) ** 2) for u in remaining])
        order = np.argsort(schur, kind="stable")       # stable: ties keep ascending user index
        p_pos = int(order[0])
        p = remaining[p_pos]
        if len(remaining) > 1:
            margins[i] = schur[order[1]] - schur[order[0]]
        piv = schur[p_pos]
        pivots[i] = piv
        if not np.isfinite(piv) or piv <= floor:
            status = STATUS_NOT_PD
            piv = max(piv, 0.0) if np.isfinite(piv) else 0.0
        lii = math.sqrt(piv)
        C[p, i] = lii
        for u in remaining:
            if u == p:
                continue
            num = A[u, p] - np.sum(C[u, :i] * np.conj(C[p, :i]))
            C[u, i] = num / lii if lii > 0 else 0.0
        perm.append(p)
        remaining.pop(p_pos)
    perm = np.array(perm, dtype=np.int64)
    L = C[perm, :]
    return L, perm, pivots, margins, status


def forward_inverse(L: np.ndarray) -> np.ndarray:
    """W = L^{-1} for lower-triangular L by forward substitution, column by column."""
    n = L.shape[0]
    W = np.zeros_like(L, dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        x = np.zeros(n, dtype=np.complex128)
        for i in range(n):
            x[i] = (e[i] - np.dot(L[i, :i], x[:i])) / L[i, i]
        W[:, j] = x
    return W


def cholesky_unsorted(A: np.ndarray):
    """A = L L^H without pivoting (users in their own order): the unsorted
    factorisation that Sec. III-B compares the sorted one (Alg. 1) with.
    Same returns as cholesky_minpivot; the margins are all inf (no choice)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    try:
        L = np.linalg.cholesky(A)
        status = STATUS_OK
    except np.linalg.LinAlgError:
        L = np.zeros((n, n), dtype=np.complex128)
        status = STATUS_NOT_PD
    pivots = np.abs(np.diag(L)) ** 2
    floor = n * np.finfo(np.float64).eps * float(np.max(np.real(np.diag(A))))
    if status == STATUS_OK and np.min(pivots) <= floor:
        status = STATUS_NOT_PD
    return L, np.arange(n), pivots, np.full(n, np.inf), status


def preprocess(H: np.ndarray, alpha: float, want_G: bool = True, sort: bool = True) -> Prep:
    """Per-subcarrier preprocessing of Alg. 2's "regularise and factorise" step:
    A = H H^H + alpha I, sorted factorisation (Alg. 1 via its Cholesky form;
    with sort=False the plain one in user order), W = Rbar^{-1}, MoP weights
    w_i = |W_ii|^2 (eq_mop) and the RZF matrix G = H^H A^{-1} (Sec. II-A;
    equal to the Tikhonov pseudo-inverse of Sec. III-A-1)."""
    H = np.asarray(H, dtype=np.complex128)
    if not np.all(np.isfinite(H.view(np.float64))) or not math.isfinite(alpha):
        n = H.shape[0]
        return Prep(np.zeros((n, n), complex), np.zeros((n, n), complex), np.arange(n),
                    np.zeros(n), None, STATUS_NONFINITE, np.zeros(n), np.full(n, np.inf))
    A = gram(H, alpha)
    L, perm, pivots, margins, status = cholesky_minpivot(A) if sort else cholesky_unsorted(A)
    if status != STATUS_OK:
        n = H.shape[0]
        return Prep(L, np.zeros((n, n), complex), perm, np.zeros(n), None, status, pivots, margins)
    W = forward_inverse(L)
    w2 = np.abs(np.diag(W)) ** 2
    G = np.linalg.solve(A, H).conj().T if want_G else None   # H^H A^{-1} = (A^{-1} H)^H
    return Prep(L, W, perm, w2, G, status, pivots, margins)


def isrqd(H: np.ndarray, lam: float):
    """Alg. 1 (improved sorted RQ decomposition) of Hbar = [H, lambda I].

    Sorted modified Gram-Schmidt on the rows: the remaining row of smallest
    squared norm is processed next (ties -> smaller user index), it becomes
    q_i = row / Rbar_ii, and every later row j loses its projection
    Rbar_ji = <row_j, q_i>, with its squared norm downdated by |Rbar_ji|^2.
    Returns (Rbar lower-triangular, Qbar with orthonormal rows, perm) such that
    Hbar[perm] = Rbar Qbar."""
    H = np.asarray(H, dtype=np.complex128)
    n, m = H.shape
    Qb = np.concatenate([H, lam * np.eye(n)], axis=1)
    norms = np.sum(np.abs(Qb) ** 2, axis=1)
    perm = np.arange(n)
    R = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        rest = np.arange(i, n)
        best = min(rest, key=lambda j: (norms[j], perm[j]))
        for arr in (Qb, norms, perm):
            arr[[i, best]] = arr[[best, i]]
        R[[i, best], :i] = R[[best, i], :i]
        R[i, i] = math.sqrt(norms[i])
        Qb[i] = Qb[i] / R[i, i]
        for j in range(i + 1, n):
            R[j, i] = np.dot(Qb[j], np.conj(Qb[i]))
            Qb[j] = Qb[j] - R[j, i] * Qb[i]
            norms[j] = norms[j] - abs(R[j, i]) ** 2
    return R, Qb, perm


# ---------------------------------------------------------------------------
# Metric of Promise and the path set (Sec. III-A-2, eq_mop)
# ---------------------------------------------------------------------------

def mop_value(w2: np.ndarray, r) -> float:
    """M(p) = sum_l |Rtilde_ll|^2 (p_l - 1) with r = p - 1, summed in level order."""
    acc = 0.0
    for wi, ri in zip(np.asarray(w2, dtype=np.float64), r):
        acc = acc + float(wi) * float(ri)
    return acc


def mop_paths_bruteforce(w2: np.ndarray, K: int) -> np.ndarray:
    """The K position vectors of smallest MoP over all 9^N candidates, ordered by
    (MoP, lexicographic r with level 0 most significant).  Tiny N only."""
    n = len(w2)
    cands = list(itertools.product(range(NBOX), repeat=n))
    cands.sort(key=lambda r: (mop_value(w2, r), r))
    return np.array(cands[:K], dtype=np.int64).reshape(K, n)


def mop_paths_kbest(w2: np.ndarray, K: int) -> np.ndarray:
    """Breadth-first K-best over the MoP tree (Sec. III-A-2): from level 0, expand
    every survivor to its 9 children, keep the K smallest partial MoPs
    (ties -> lexicographic prefix), repeat to depth N.  Partial sums are
    accumulated in level order, as in mop_value."""
    w2 = np.asarray(w2, dtype=np.float64)
    n = len(w2)
    surv_m = np.zeros(1)
    surv_r = np.zeros((1, 0), dtype=np.int64)
    for lvl in range(n):
        cm = (surv_m[:, None] + w2[lvl] * np.arange(NBOX)[None, :]).reshape(-1)
        cr = np.concatenate([np.repeat(surv_r, NBOX, axis=0),
                             np.tile(np.arange(NBOX), len(surv_r))[:, None]], axis=1)
        keys = [cr[:, c] for c in range(lvl, -1, -1)] + [cm]   # lexsort: last key primary
        order = np.lexsort(keys)[:K]
        surv_m, surv_r = cm[order], cr[order]
    return surv_r


# ---------------------------------------------------------------------------
# Same-path-set search (Sec. II-B PED recursion, Sec. III-A-2 centres and DEMAP,
# Alg. 2 parallel evaluation + argmin)
# ---------------------------------------------------------------------------

@dataclass
class SearchResult:
    l: np.ndarray          # complex [n_vec][N], user order, exact Gaussian integers
    cost: np.ndarray       # [n_vec] selected cost (gamma of Alg. 2)
    kidx: np.ndarray       # [n_vec] selected path (K = the zero perturbation)
    path_cost: np.ndarray  # [n_vec][K(+1)] every candidate's cost
    path_l: np.ndarray     # [n_vec][K][N] every candidate's l, level order
    margin: np.ndarray     # [n_vec][K] smallest order margin met along each path


# ---------------------------------------------------------------------------
# The paper's region-table DEMAP (Sec. III-A-2 DEMAP paragraph; Alg. 2 "Demap")
# ---------------------------------------------------------------------------
# Reading (the FlexCore construction the paper defers to is not available):
# the centre c is taken relative to its anchor n, the box point nearest to it
# (the rank-0 child of the exact order); delta = c - n is folded by the
# symmetries of the square lattice -- sign flips of both axes, then the swap
# that makes |dx| >= |dy| -- into 0 <= w <= u; the cell (iu, iw) of that point
# on a grid of step 1/8 (iu capped at 11, iw at iu) is the region; its order
# of the 25 lattice offsets of [-2, 2]^2 is the distance order from the cell's
# representative point (the cell centre, or the centroid of the lower triangle
# for diagonal cells), equal distances by the folded index 5 (dx+2) + (dy+2).
# Rank 0 is the anchor; rank p > 0 is the p-th offset of that order, other
# than (0, 0), whose point lies in the box once unfolded.

REGION_STEP = Fraction(1, 8)
REGION_UCELLS = 12
_OFFSETS25 = [(dx, dy) for dx in range(-2, 3) for dy in range(-2, 3)]


def region_representative(iu: int, iw: int):
    """Representative point (u, w) of region (iu, iw), exact rationals."""
    if iw < iu:
        return (iu + Fraction(1, 2)) * REGION_STEP, (iw + Fraction(1, 2)) * REGION_STEP
    return (iu + Fraction(2, 3)) * REGION_STEP, (iu + Fraction(1, 3)) * REGION_STEP


@lru_cache(maxsize=None)
def region_ranks(iu: int, iw: int, mx: int, my: int):
    """Folded offsets of ranks 0..8 in region (iu, iw) for the folded anchor
    (mx, my): (0, 0) first, then the region's distance order restricted to
    the offsets that keep the anchor inside the box."""
    u, w = region_representative(iu, iw)
    dist = [((u - dx) ** 2 + (w - dy) ** 2, 5 * (dx + 2) + (dy + 2)) for dx, dy in _OFFSETS25]
    order = sorted(range(25), key=lambda j: dist[j])
    out = [(0, 0)]
    for j in order:
        dx, dy = _OFFSETS25[j]
        if (dx, dy) != (0, 0) and abs(mx + dx) <= 1 and abs(my + dy) <= 1:
            out.append((dx, dy))
    return tuple(out)


def fold_region(delta: complex):
    """Region (iu, iw) and fold (flip x, flip y, swap) of an offset from the anchor."""
    fx, fy = delta.real < 0, delta.imag < 0
    ax, ay = abs(delta.real), abs(delta.imag)
    sw = ay > ax
    u, w = (ay, ax) if sw else (ax, ay)
    iu = min(int(math.floor(u / float(REGION_STEP))), REGION_UCELLS - 1)
    iw = min(int(math.floor(w / float(REGION_STEP))), iu)
    return iu, iw, fx, fy, sw


def folded_ranks_at(u: float, w: float, mx: int, my: int):
    """As region_ranks, with the order taken at the folded point (u, w) itself:
    the table a region-table DEMAP would hold if its regions were points."""
    dist = [((u - dx) ** 2 + (w - dy) ** 2, 5 * (dx + 2) + (dy + 2)) for dx, dy in _OFFSETS25]
    out = [(0, 0)]
    for j in sorted(range(25), key=lambda j: dist[j]):
        dx, dy = _OFFSETS25[j]
        if (dx, dy) != (0, 0) and abs(mx + dx) <= 1 and abs(my + dy) <= 1:
            out.append((dx, dy))
    return tuple(out)


def demap_region(c: complex, rank: int, exact_point: bool = False) -> complex:
    """The box point of the given rank for centre c under the region-table
    DEMAP (exact_point: the order of the folded point itself instead of its
    region's representative)."""
    d = sqabs(c - BOX)
    n = BOX[int(np.argsort(d, kind="stable")[0])]      # anchor: the exact rank-0 child
    if rank == 0:
        return n
    iu, iw, fx, fy, sw = fold_region(c - n)
    mx, my = int(-n.real if fx else n.real), int(-n.imag if fy else n.imag)
    if sw:
        mx, my = my, mx
    if exact_point:
        ax, ay = abs((c - n).real), abs((c - n).imag)
        ranks = folded_ranks_at(max(ax, ay), min(ax, ay), mx, my)
    else:
        ranks = region_ranks(iu, iw, mx, my)
    ox, oy = ranks[rank]
    ux, uy = (oy, ox) if sw else (ox, oy)             # unswap, then unflip
    return n + complex(-ux if fx else ux, -uy if fy else uy)


def level_tau(tau, perm):
    """tau per tree level: a scalar (the paper's one system constant, Sec. II-B)
    or one value per user (a QAM order per user), taken in level order."""
    t = np.asarray(tau, dtype=np.float64)
    n = len(perm)
    return np.full(n, float(t)) if t.ndim == 0 else t[np.asarray(perm)]


def demap_walk(W, st, tau, ranks, demap: str = "exact"):
    """Walk the tree along position vectors for many (vector, path) pairs at once.

    st: complex [V][N] = W s_pi (s-tilde of the PED recursion); ranks: int
    [P][N]; tau: a scalar or one value per level.  Returns (l [V][P][N],
    cost [V][P], margin [V][P]).  At level i the centre is
    c_i = -r_i / (tau_i W_ii) where r_i is the running residual
    s-tilde_i + sum_{j<i} tau_j W_ij l_j (the s-hat of Sec. III-A-2 with l = -t);
    the child of rank p_i is the p_i-th box point in the (distance, j) order;
    the PED grows by tau_i^2 |W_ii|^2 |c_i - l_i|^2 (Sec. II-B)."""
    V, n = st.shape
    P = ranks.shape[0]
    taul = np.broadcast_to(np.asarray(tau, dtype=np.float64), (n,))
    resid = np.broadcast_to(st[:, None, :], (V, P, n)).copy()
    l = np.zeros((V, P, n), dtype=np.complex128)
    cost = np.zeros((V, P))
    margin = np.full((V, P), np.inf)
    for i in range(n):
        wii = W[i, i]
        ti = taul[i]
        c = -resid[:, :, i] / (ti * wii)
        d = sqabs(c[:, :, None] - BOX[None, None, :])                    # [V][P][9]
        order = np.argsort(d, axis=2, kind="stable")                      # (d, j) order
        dsorted = np.take_along_axis(d, order, axis=2)
        r = np.broadcast_to(ranks[None, :, i], (V, P))[:, :, None]
        j = np.take_along_axis(order, r, axis=2)[:, :, 0]
        dch = np.take_along_axis(dsorted, r, axis=2)[:, :, 0]
        dlo = np.take_along_axis(dsorted, np.maximum(r - 1, 0), axis=2)[:, :, 0]
        dhi = np.take_along_axis(dsorted, np.minimum(r + 1, NBOX - 1), axis=2)[:, :, 0]
        lo = np.where(r[:, :, 0] > 0, dch - dlo, np.inf)
        hi = np.where(r[:, :, 0] < NBOX - 1, dhi - dch, np.inf)
        margin = np.minimum(margin, np.minimum(lo, hi))
        if demap in ("region", "region-exact-point"):   # the paper's region-table DEMAP instead of the exact order
            ep = demap == "region-exact-point"
            li = BOX[j].copy()                             # rank 0: the nearest box point, as the exact order
            for b in np.nonzero(ranks[:, i] > 0)[0]:
                for a in range(V):
                    li[a, b] = demap_region(complex(c[a, b]), int(ranks[b, i]), ep)
            dch = sqabs(c - li)
        else:
            li = BOX[j]
        l[:, :, i] = li
        cost += (ti ** 2) * (abs(wii) ** 2) * dch
        if i + 1 < n:
            resid[:, :, i + 1:] += ti * W[None, None, i + 1:, i] * li[:, :, None]
    return l, cost, margin


def search_paths(W, perm, s, tau, paths, include_zero: bool = True, demap: str = "exact") -> SearchResult:
    """Alg. 2's data-dependent part for one subcarrier: for every vector (columns
    of s, user order) evaluate every path of the set, then take the argmin.

    W: complex [N][N] lower (search order); perm: level -> user; s: complex
    [N][V] (user order); tau: a scalar or one value per user; paths: int
    [K][N] ranks 0..8.  With include_zero, the zero perturbation (plain RZF)
    is candidate index K.  demap = "region" walks with the paper's region-table
    DEMAP (demap_region) instead of the exact child order."""
    W = np.asarray(W, dtype=np.complex128)
    perm = np.asarray(perm, dtype=np.int64)
    s = np.asarray(s, dtype=np.complex128)
    if s.ndim == 1:
        s = s[:, None]
    paths = np.asarray(paths, dtype=np.int64)
    K, n = paths.shape
    s_pi = s[perm, :].T                     # [V][N] level order
    st = s_pi @ W.T                         # s-tilde = W s_pi, per vector
    l, cost, margin = demap_walk(W, st, level_tau(tau, perm), paths, demap=demap)
    if include_zero:
        c0 = np.sum(np.abs(st) ** 2, axis=1)
        cost_all = np.concatenate([cost, c0[:, None]], axis=1)
    else:
        cost_all = cost
    k = np.argmin(cost_all, axis=1)         # first minimum -> smaller k on ties
    V = st.shape[0]
    l_sel = np.zeros((V, n), dtype=np.complex128)
    for v in range(V):
        if k[v] < K:
            l_sel[v, perm] = l[v, k[v]]
    return SearchResult(l_sel, cost_all[np.arange(V), k], k, cost_all, l, margin)


def cost_closed_form(A: np.ndarray, s: np.ndarray, l: np.ndarray, tau) -> float:
    """u^H A^{-1} u with u = s + tau l (user order; tau a scalar or one value per
    user): the quantity eq:se minimises, written with the RZF inverse
    (Sec. III-A-1)."""
    u = np.asarray(s, np.complex128) + tau * np.asarray(l, np.complex128)
    return float(np.real(np.vdot(u, np.linalg.solve(A, u))))


def cost_tri(W, perm, s, l, tau) -> float:
    """|| W (s + tau l)_pi ||^2 (eq_qrse with l = -t; tau a scalar or per user)."""
    u = np.asarray(s, np.complex128) + tau * np.asarray(l, np.complex128)
    return float(np.sum(np.abs(np.asarray(W, np.complex128) @ u[np.asarray(perm)]) ** 2))


# ---------------------------------------------------------------------------
# Exact VP over the box: brute force and a depth-first sphere encoder
# ---------------------------------------------------------------------------

def brute_force(W, perm, s, tau):
    """Exact minimiser of eq:se over the whole box B^N (9^N candidates): the
    smallest || W (s_pi + tau l) ||^2 (tau a scalar or one per user); ties ->
    lexicographically smallest box index vector in level order.  Returns
    (l user order, cost)."""
    W = np.asarray(W, np.complex128)
    n = W.shape[0]
    s_pi = np.asarray(s, np.complex128)[np.asarray(perm)]
    J = np.array(list(itertools.product(range(NBOX), repeat=n)), dtype=np.int64)   # lexicographic
    U = s_pi[None, :] + level_tau(tau, perm)[None, :] * BOX[J]
    costs = np.sum(np.abs(U @ W.T) ** 2, axis=1)
    b = int(np.argmin(costs))
    l = np.zeros(n, dtype=np.complex128)
    l[np.asarray(perm)] = BOX[J[b]]
    return l, float(costs[b])


def sphere_encode(W, perm, s, tau, radius: float = math.inf):
    """Depth-first Schnorr-Euchner sphere encoder over the box (the exact VP of
    eq:se restricted to |Re|,|Im| <= 1).  Children of a node are visited in
    (distance, j) order; a subtree is pruned when its PED is not below the best
    cost found so far.  Returns (l user order, cost, nodes visited)."""
    W = np.asarray(W, np.complex128)
    n = W.shape[0]
    s_pi = np.asarray(s, np.complex128)[np.asarray(perm)]
    st = W @ s_pi
    taul = level_tau(tau, perm)
    best = [radius, None]
    nodes = [0]
    lvl_l = np.zeros(n, dtype=np.complex128)

    def rec(i, resid, ped):
        wii = W[i, i]
        c = -resid[i] / (taul[i] * wii)
        d = sqabs(c - BOX)
        for j in np.argsort(d, kind="stable"):
            nped = ped + taul[i] ** 2 * abs(wii) ** 2 * d[j]
            if nped >= best[0]:
                break
            nodes[0] += 1
            lvl_l[i] = BOX[j]
            if i + 1 == n:
                best[0] = nped
                best[1] = lvl_l.copy()
            else:
                rec(i + 1, resid + taul[i] * W[:, i] * BOX[j] * (np.arange(n) > i), nped)

    rec(0, st.copy(), 0.0)
    if best[1] is None:
        return None, math.inf, nodes[0]
    l = np.zeros(n, dtype=np.complex128)
    l[np.asarray(perm)] = best[1]
    return l, float(best[0]), nodes[0]


# ---------------------------------------------------------------------------
# The path walk in 16-bit fixed point (the accelerator's number format,
# Sec. V "Precision and Numerical Accuracy": signed 16 bits, F = 8..13
# fractional bits)
# ---------------------------------------------------------------------------
# Reading (the paper fixes only the word width and the fractional bits): the
# walk's state is the level centre c_m = -r_m / (tau W_mm); a level's child
# moves the centres below it by V_mi l_i with V_mi = -W_mi / W_mm, and its PED
# is tau^2 W_ii^2 |l_i - c_i|^2.  Centres, V and the weights
# w_i = W_ii^2 / max_j W_jj^2 are signed 16-bit numbers with F fractional bits
# (round to nearest, ties to even, saturating); squared distances are formed
# from differences saturated to 16 bits, and the PED sum sum_i w_i d_i is kept
# exactly (64 bits), as a DSP accumulator would.

FX_MIN, FX_MAX = -32768, 32767


def fx_quantize(x, frac_bits: int):
    """Real values to signed 16-bit integers with frac_bits fractional bits."""
    return np.clip(np.rint(np.asarray(x, dtype=np.float64) * 2.0 ** frac_bits), FX_MIN, FX_MAX).astype(np.int64)


def fx_inputs(W, perm, s, tau, frac_bits: int):
    """The fixed-point inputs of the walk for one subcarrier: start centres
    c0 [V][N] (complex as [..., 2] int), step coefficients V [N][N] (lower, [..., 2])
    and weights w [N], from float64 W, perm, symbols s [N][V] (user order)."""
    W = np.asarray(W, np.complex128)
    n = W.shape[0]
    st = (np.asarray(s, np.complex128)[np.asarray(perm), :]).T @ W.T        # [V][N] = (W s_pi)^T
    d = np.real(np.diag(W))
    c0 = -st / (tau * d[None, :])
    Vm = -W / d[:, None]                                                     # V_mi = -W_mi / W_mm
    w = d ** 2 / np.max(d ** 2)
    def q(z):
        return np.stack([fx_quantize(np.real(z), frac_bits), fx_quantize(np.imag(z), frac_bits)], axis=-1)

    Vq = q(Vm)
    Vq[np.triu_indices(n)] = 0          # only the strictly lower part (m > i) is used
    return q(c0), Vq, fx_quantize(w, frac_bits)


def fx_sat(x):
    return np.clip(x, FX_MIN, FX_MAX)


def fx_demap(cx: int, cy: int, rank: int, frac_bits: int):
    """Box point of the given rank for a fixed-point centre: the nine squared
    distances from differences saturated to 16 bits, ordered by (distance, j)."""
    one = 1 << frac_bits
    d = []
    for j, b in enumerate(BOX):
        ex = int(fx_sat(cx - int(b.real) * one))
        ey = int(fx_sat(cy - int(b.imag) * one))
        d.append((ex * ex + ey * ey, j))
    d.sort()
    dist, j = d[rank]
    return int(BOX[j].real), int(BOX[j].imag), dist


def fx_search(c0, Vq, wq, paths, frac_bits: int, include_zero: bool = True):
    """The same-path-set search in fixed point for one subcarrier.  c0 [V][N][2],
    Vq [N][N][2] (lower), wq [N] from fx_inputs; paths [K][N].  Returns
    (l level order [V][N] complex, ped [V] int, kidx [V]); the zero perturbation,
    with include_zero, is candidate K with PED sum_i w_i |c0_i|^2."""
    c0 = np.asarray(c0, np.int64)
    n = c0.shape[1]
    K = len(paths)
    Vn = c0.shape[0]
    l_out = np.zeros((Vn, n), dtype=np.complex128)
    ped_out = np.zeros(Vn, dtype=object)
    k_out = np.zeros(Vn, dtype=np.int64)
    for v in range(Vn):
        best = None
        for k in range(K + (1 if include_zero else 0)):
            c = c0[v].copy()
            ped = 0
            l = np.zeros(n, dtype=np.complex128)
            for i in range(n):
                if k == K:
                    a, b = 0, 0
                    ex, ey = int(fx_sat(c[i, 0])), int(fx_sat(c[i, 1]))
                    dist = ex * ex + ey * ey
                else:
                    a, b, dist = fx_demap(int(c[i, 0]), int(c[i, 1]), int(paths[k][i]), frac_bits)
                l[i] = complex(a, b)
                ped += int(wq[i]) * dist
                for m in range(i + 1, n):   # c_m += V_mi l_i, l_i in the box: additions
                    vx, vy = int(Vq[m, i, 0]), int(Vq[m, i, 1])
                    c[m, 0] = fx_sat(c[m, 0] + a * vx - b * vy)
                    c[m, 1] = fx_sat(c[m, 1] + a * vy + b * vx)
            if best is None or ped < best[0]:
                best = (ped, k, l)
        ped_out[v], k_out[v], l_out[v] = best
    return l_out, ped_out, k_out


# ---------------------------------------------------------------------------
# Precoding, receiver modulo, power gap (Alg. 2 output, eq:postproc)
# ---------------------------------------------------------------------------

def precode(G, s, l, tau, gamma=None, P_T: float = 0.0):
    """x = G (s + tau l) (Alg. 2 / Sec. IV-B: the precoded vector before and,
    with P_T > 0, after the sqrt(P_T / gamma) normalisation)."""
    u = np.asarray(s, np.complex128) + tau * np.asarray(l, np.complex128)
    x = np.asarray(G, np.complex128) @ u
    if P_T > 0.0:
        x = x * math.sqrt(P_T / gamma)
    return x


def mod_tau(a, tau):
    """Receiver modulo of eq:postproc, applied to both rails:
    mod(a) = a - tau * floor((a + tau/2) / tau)."""
    a = np.asarray(a, np.complex128)
    f = lambda v: v - tau * np.floor((v + tau / 2.0) / tau)
    return f(a.real) + 1j * f(a.imag)


def gap_db(gamma_method, gamma_exact) -> float:
    """Transmit-power gap 10 log10(sum gamma_method / sum gamma_exact)."""
    return 10.0 * math.log10(float(np.sum(gamma_method)) / float(np.sum(gamma_exact)))


def complexity_cm(n_r: int, n_t: int, K: int) -> int:
    """Per-vector complex multiplications of ViPer (Sec. III-B complexity paragraph):
    N_r N_t + N_t^2 + K N_t (1 + (N_t + 1) / 2)."""
    return n_r * n_t + n_t * n_t + (K * n_t * (2 + n_t + 1)) // 2
