"""Pins for the Metric of Promise and the path set (Sec. III-A-2, eq_mop).

The K-best procedure of the paper is checked against exhaustive enumeration,
against a hand-worked tie case, and against a closed-form count; the MoP
value itself against eq_mop evaluated from W's diagonal."""
import itertools

import numpy as np
import pytest

from oracle import vp_oracle as O


def test_worked_equal_weights():
    # w = [1/2, 1/2]: M(r) = (r0 + r1) / 2.  Order by (M, lexicographic r):
    # (0,0) | (0,1) (1,0) | (0,2) (1,1) (2,0) | ...
    p = O.mop_paths_kbest(np.array([0.5, 0.5]), 5)
    assert p.tolist() == [[0, 0], [0, 1], [1, 0], [0, 2], [1, 1]]


@pytest.mark.parametrize("N,K", [(1, 9), (2, 7), (3, 40), (4, 32), (4, 200), (3, 729)])
def test_kbest_equals_exhaustive(N, K):
    rng = np.random.default_rng(N * 1000 + K)
    for trial in range(4):
        w = rng.uniform(0.05, 1.0, N)
        if trial == 3:
            w[:] = w[0]                     # all ties: order falls back to lexicographic
        a = O.mop_paths_kbest(w, K)
        b = O.mop_paths_bruteforce(w, K)
        assert a.tolist() == b.tolist()


def test_exhaustive_order_is_by_metric_then_lex():
    rng = np.random.default_rng(3)
    w = rng.uniform(0.1, 0.6, 3)
    allp = O.mop_paths_bruteforce(w, 9 ** 3)
    assert sorted(map(tuple, allp.tolist())) == list(itertools.product(range(9), repeat=3))
    m = np.array([float(np.dot(w, r)) for r in allp])
    assert np.all(np.diff(m) >= -1e-12)


def test_mop_value_is_eq_mop_from_W():
    # eq_mop: M(p) = sum_l |Rtilde_ll|^2 (p_l - 1), Rtilde = W
    rng = np.random.default_rng(9)
    h = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    p = O.preprocess(h, 0.1)
    r = [3, 0, 1, 8]
    direct = sum(abs(p.W[i, i]) ** 2 * ((r[i] + 1) - 1) for i in range(4))
    assert np.isclose(O.mop_value(p.w2, r), direct, rtol=1e-14)


def test_count_closed_form_equal_weights():
    # With equal weights the first K paths are exactly all r with sum(r) <= t for
    # the t where the cumulative count reaches K (when K falls on a boundary).
    N = 3
    counts = [sum(1 for r in itertools.product(range(9), repeat=N) if sum(r) == t) for t in range(25)]
    K = counts[0] + counts[1] + counts[2] + counts[3]      # 1 + 3 + 6 + 10 = 20
    p = O.mop_paths_kbest(np.full(N, 0.3), K)
    assert K == 20
    assert sorted(map(sum, p.tolist())) == sorted([s for s in range(4) for _ in range(counts[s])])


def test_paths_are_a_down_set():
    # Every path's component-wise predecessors are in the set (w > 0 makes M strictly
    # monotone), so the set is closed downwards.
    rng = np.random.default_rng(21)
    w = rng.uniform(0.1, 0.5, 6)
    P = O.mop_paths_kbest(w, 300)
    S = set(map(tuple, P.tolist()))
    for r in S:
        for i in range(6):
            if r[i] > 0:
                q = list(r)
                q[i] -= 1
                assert tuple(q) in S
