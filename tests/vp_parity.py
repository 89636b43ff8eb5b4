"""Parity rules between the HIP path and the FP64 oracle (test infrastructure).

Selected perturbation l: bit-exact, except where float32 cannot decide what
float64 decides:
  * cost tie  - the two choices' float64 costs agree to 1e-5 relative;
  * order tie - a DEMAP decision on the GPU's (or the oracle's) winning path
    had two box points within TIE_EPS of each other in squared distance, so
    float32 may order them either way.  Then l_gpu must be reachable by
    re-walking the GPU's path with every such near-tied choice allowed, and
    its float64 cost must not exceed any path's (tie-relaxed) cost by more
    than 1e-5 relative.
Reported cost: within 1e-5 relative of the float64 cost of l_gpu.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from oracle import vp_oracle as O

COST_RTOL = 1e-5
TIE_EPS = 1e-4        # squared-distance units of the normalised level centre

# Totals over every parity check of a test session, printed at the end of the
# run (tests/conftest.py) so that tie and mismatch counts appear in the log.
TOTALS: dict = {}


def record(kind: str, rep: "ParityReport") -> None:
    """Add one report to the session totals under `kind`."""
    t = TOTALS.setdefault(kind, {"n": 0, "exact": 0, "cost_ties": 0, "order_ties": 0, "failures": 0,
                                 "max_cost_rel_err": 0.0})
    t["n"] += rep.n
    t["exact"] += rep.exact
    t["cost_ties"] += rep.cost_ties
    t["order_ties"] += rep.order_ties
    t["failures"] += len(rep.failures)
    t["max_cost_rel_err"] = max(t["max_cost_rel_err"], rep.max_cost_rel_err)


def count(kind: str, key: str, k: int = 1) -> None:
    """Add k to a named counter of the session totals (e.g. flagged pivot ties)."""
    TOTALS.setdefault(kind, {}).setdefault(key, 0)
    TOTALS[kind][key] += k


def unpack_W(Wp: np.ndarray, N: int) -> np.ndarray:
    """Packed column-major lower [..., N(N+1)/2] -> dense lower [..., N, N]."""
    Wp = np.asarray(Wp)
    out = np.zeros(Wp.shape[:-1] + (N, N), dtype=np.complex128)
    idx = 0
    for j in range(N):
        for i in range(j, N):
            out[..., i, j] = Wp[..., idx]
            idx += 1
    return out


def l_from_gpu(l_i8: np.ndarray) -> np.ndarray:
    """int8 [N][n_vec][2] -> complex [n_vec][N]."""
    return (l_i8[..., 0].astype(np.float64) + 1j * l_i8[..., 1].astype(np.float64)).T


def relaxed_walks(W, st, tau, ranks, eps=TIE_EPS, limit=64):
    """Every l (level order) the walk of `ranks` can produce when each near-tied
    DEMAP decision may go either way (tau a scalar or one value per level).
    Returns a list of (l, cost)."""
    n = W.shape[0]
    taul = np.broadcast_to(np.asarray(tau, dtype=np.float64), (n,))
    out = []

    def rec(i, resid, l, cost):
        if len(out) >= limit:
            return
        if i == n:
            out.append((l.copy(), cost))
            return
        c = -resid[i] / (taul[i] * W[i, i])
        d = O.sqabs(c - O.BOX)
        order = np.argsort(d, kind="stable")
        dr = d[order[ranks[i]]]
        for p in range(9):
            j = order[p]
            if abs(d[j] - dr) <= eps * (1.0 + abs(c)) ** 2:
                l[i] = O.BOX[j]
                nres = resid.copy()
                nres[i + 1:] += taul[i] * W[i + 1:, i] * O.BOX[j]
                rec(i + 1, nres, l, cost + taul[i] ** 2 * abs(W[i, i]) ** 2 * d[j])
        l[i] = 0

    rec(0, st.copy(), np.zeros(n, dtype=np.complex128), 0.0)
    return out


@dataclass
class ParityReport:
    n: int = 0
    exact: int = 0
    cost_ties: int = 0
    order_ties: int = 0
    max_cost_rel_err: float = 0.0
    failures: list = field(default_factory=list)

    def ok(self):
        return not self.failures

    def __str__(self):
        return (f"n={self.n} exact={self.exact} cost_ties={self.cost_ties} order_ties={self.order_ties} "
                f"max_cost_rel_err={self.max_cost_rel_err:.2e} failures={len(self.failures)}")


def check_search_subcarrier(rep: ParityReport, W, perm, s_user, tau, paths, include_zero,
                            l_gpu, cost_gpu, kidx_gpu, cost_rtol: float = COST_RTOL):
    """Compare one subcarrier's GPU results (l_gpu complex [V][N], cost [V], kidx [V])
    with the oracle's same-path-set search on the same (upcast) inputs.

    cost_rtol bounds the reported cost against the float64 cost of l_gpu; it
    is 1e-5 for same-input parity and larger only where W itself comes from a
    different (float64) factorisation of H (end-to-end parity)."""
    W = np.asarray(W, np.complex128)
    perm = np.asarray(perm, np.int64)
    paths = np.asarray(paths, np.int64)
    K, n = paths.shape
    res = O.search_paths(W, perm, s_user, tau, paths, include_zero=include_zero)
    s_user = np.asarray(s_user, np.complex128)
    for v in range(s_user.shape[1]):
        rep.n += 1
        lg = l_gpu[v]
        c64_g = O.cost_tri(W, perm, s_user[:, v], lg, tau)
        rel = abs(float(cost_gpu[v]) - c64_g) / max(c64_g, 1e-30)
        rep.max_cost_rel_err = max(rep.max_cost_rel_err, rel)
        if not rel <= cost_rtol:
            rep.failures.append((v, "cost", float(cost_gpu[v]), c64_g))
            continue
        c_orc = float(res.cost[v])
        if np.array_equal(lg, res.l[v]):
            rep.exact += 1
            continue
        if abs(c64_g - c_orc) <= COST_RTOL * c_orc:
            rep.cost_ties += 1
            continue
        # order tie: l_gpu must come from relaxing near ties on the GPU's path,
        # and be no worse than every path's best tie-relaxed outcome
        kg = int(kidx_gpu[v])
        st = W @ s_user[perm, v]
        lg_level = lg[perm]
        ok = False
        if 0 <= kg < K:
            walks = relaxed_walks(W, st, O.level_tau(tau, perm), paths[kg])
            ok = any(np.array_equal(w[0], lg_level) for w in walks)
        elif kg == K and include_zero:
            ok = not np.any(lg)
        if ok:
            bound = math.inf
            for k in range(K):
                ws = (relaxed_walks(W, st, O.level_tau(tau, perm), paths[k])
                      if res.margin[v, k] <= 100 * TIE_EPS else None)
                if ws is None:
                    bound = min(bound, float(res.path_cost[v, k]))
                else:
                    bound = min(bound, max(w[1] for w in ws))
            if include_zero:
                bound = min(bound, float(np.sum(np.abs(st) ** 2)))
            ok = c64_g <= bound * (1 + COST_RTOL)
        if ok:
            rep.order_ties += 1
        else:
            rep.failures.append((v, "l", lg.tolist(), res.l[v].tolist(), kg, int(res.kidx[v]), c64_g, c_orc))
    return res


def region_relaxed_walks(W, st, tau, ranks, eps=1e-5, limit=64):
    """Every l (level order) the region-table DEMAP walk of `ranks` can produce
    when float32 may put a centre on either side of a boundary within eps
    (relative) of it -- the anchor's rounding, the fold or a cell edge: the
    region DEMAP is evaluated at the centre and at eight points around it.
    Returns a list of (l, cost)."""
    n = W.shape[0]
    taul = np.broadcast_to(np.asarray(tau, dtype=np.float64), (n,))
    around = [0, 1, -1, 1j, -1j, 1 + 1j, 1 - 1j, -1 + 1j, -1 - 1j]
    out = []

    def rec(i, resid, l, cost):
        if len(out) >= limit:
            return
        if i == n:
            out.append((l.copy(), cost))
            return
        c = -resid[i] / (taul[i] * W[i, i])
        e = eps * (1.0 + abs(c))
        seen = []
        for z in around:
            t = O.demap_region(c + e * z, int(ranks[i]))
            if t not in seen:
                seen.append(t)
        for t in seen:
            l[i] = t
            nres = resid.copy()
            nres[i + 1:] += taul[i] * W[i + 1:, i] * t
            rec(i + 1, nres, l, cost + taul[i] ** 2 * abs(W[i, i]) ** 2 * O.sqabs(c - t))
        l[i] = 0

    rec(0, st.copy(), np.zeros(n, dtype=np.complex128), 0.0)
    return out


def check_search_subcarrier_region(rep: ParityReport, W, perm, s_user, tau, paths, include_zero,
                                   l_gpu, cost_gpu, kidx_gpu):
    """As check_search_subcarrier, for the region-table DEMAP: the oracle walks
    with it too; a differing l must be a cost tie, or a boundary tie -- the
    GPU's path, re-walked with boundary decisions relaxed, reaches l_gpu, and
    l_gpu costs no more than every path's relaxed outcomes."""
    W = np.asarray(W, np.complex128)
    perm = np.asarray(perm, np.int64)
    paths = np.asarray(paths, np.int64)
    K, n = paths.shape
    res = O.search_paths(W, perm, s_user, tau, paths, include_zero=include_zero, demap="region")
    s_user = np.asarray(s_user, np.complex128)
    taul = O.level_tau(tau, perm)
    for v in range(s_user.shape[1]):
        rep.n += 1
        lg = l_gpu[v]
        c64_g = O.cost_tri(W, perm, s_user[:, v], lg, tau)
        rel = abs(float(cost_gpu[v]) - c64_g) / max(c64_g, 1e-30)
        rep.max_cost_rel_err = max(rep.max_cost_rel_err, rel)
        if not rel <= COST_RTOL:
            rep.failures.append((v, "cost", float(cost_gpu[v]), c64_g))
            continue
        c_orc = float(res.cost[v])
        if np.array_equal(lg, res.l[v]):
            rep.exact += 1
            continue
        if abs(c64_g - c_orc) <= COST_RTOL * c_orc:
            rep.cost_ties += 1
            continue
        kg = int(kidx_gpu[v])
        st = W @ s_user[perm, v]
        ok = False
        if 0 <= kg < K:
            ok = any(np.array_equal(w[0], lg[perm]) for w in region_relaxed_walks(W, st, taul, paths[kg]))
        elif kg == K and include_zero:
            ok = not np.any(lg)
        if ok:
            bound = min(max(w[1] for w in region_relaxed_walks(W, st, taul, paths[k])) for k in range(K))
            if include_zero:
                bound = min(bound, float(np.sum(np.abs(st) ** 2)))
            ok = c64_g <= bound * (1 + COST_RTOL)
        if ok:
            rep.order_ties += 1
        else:
            rep.failures.append((v, "l", lg.tolist(), res.l[v].tolist(), kg, int(res.kidx[v]), c64_g, c_orc))
    return res
