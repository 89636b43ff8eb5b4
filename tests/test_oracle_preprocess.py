"""Pins for the oracle's preprocessing (Sec. III-A-1, Alg. 1, eq:invr).

Each test checks the oracle against something other than itself: a
hand-worked example, an independent library factorisation, the ISRQD
Gram-Schmidt form of Alg. 1, the implicit-inverse identity of eq:invr, the
brute-force pivot rule, and closed forms of the RZF matrix."""
import math

import numpy as np
import pytest

import vpgen
from oracle import vp_oracle as O


def test_worked_2x2_zf():
    # H = [[2,0],[1,1]], alpha = 0: A = H H^T = [[4,2],[2,2]].  The smallest
    # diagonal is user 1 (2 < 4), so pi = [1,0]; Lbar_00 = sqrt(2); user 0's
    # column entry is A_01 / sqrt(2) = sqrt(2); its Schur diagonal is 4 - 2 = 2.
    # Lbar = sqrt(2) [[1,0],[1,1]] -> W = [[1,0],[-1,1]] / sqrt(2); w = [1/2,1/2].
    # G = H^T A^{-1} = [[0.5,0],[-0.5,1]], and H G = I (zero forcing).
    H = np.array([[2, 0], [1, 1]], dtype=np.complex64)
    p = O.preprocess(H, 0.0)
    r2 = math.sqrt(2.0)
    assert list(p.perm) == [1, 0]
    np.testing.assert_allclose(p.L, [[r2, 0], [r2, r2]], atol=1e-14)
    np.testing.assert_allclose(p.W, [[1 / r2, 0], [-1 / r2, 1 / r2]], atol=1e-14)
    np.testing.assert_allclose(p.w2, [0.5, 0.5], atol=1e-14)
    np.testing.assert_allclose(p.G, [[0.5, 0], [-0.5, 1]], atol=1e-14)
    assert p.status == O.STATUS_OK


@pytest.mark.parametrize("N,M,alpha,rho", [(4, 4, 0.0, 0.0), (8, 8, 0.08, 0.0), (16, 16, 0.16, 0.5),
                                           (6, 4, 0.3, 0.0), (3, 7, 0.0, 0.0)])
def test_factor_against_library_and_isrqd(N, M, alpha, rho):
    rng = np.random.default_rng(100 + N * 10 + M)
    H = (vpgen.draw_correlated(rng, 3, N, M, rho) if rho else vpgen.draw_rayleigh(rng, 3, N, M))
    for h in H:
        p = O.preprocess(h, alpha)
        assert p.status == O.STATUS_OK
        A = O.gram(h, alpha)
        Ap = A[np.ix_(p.perm, p.perm)]
        # library Cholesky of the permuted Gram matrix is the same factor
        np.testing.assert_allclose(p.L, np.linalg.cholesky(Ap), rtol=0, atol=1e-10 * np.abs(Ap).max())
        # W is the inverse and w are its squared diagonal
        np.testing.assert_allclose(p.W @ p.L, np.eye(N), atol=1e-10)
        np.testing.assert_allclose(p.w2, 1.0 / np.diag(p.L).real ** 2, rtol=1e-12)
        # determinant: prod Lbar_ii^2 = det A
        assert np.isclose(np.prod(np.diag(p.L).real ** 2), np.linalg.det(A).real, rtol=1e-9)
        # Alg. 1 (Gram-Schmidt on rows of [H, lambda I]) gives the same Rbar and order
        if alpha > 0:
            lam = math.sqrt(alpha)
            R, Qb, perm = O.isrqd(h, lam)
            assert list(perm) == list(p.perm)
            np.testing.assert_allclose(R, p.L, atol=1e-10)
            np.testing.assert_allclose(Qb @ Qb.conj().T, np.eye(N), atol=1e-10)
            Hbar = np.concatenate([h.astype(np.complex128), lam * np.eye(N)], axis=1)
            np.testing.assert_allclose(R @ Qb, Hbar[perm], atol=1e-10)
            # eq:invr with the sort: Rbar^{-1} = Q2[:, pi] / lambda
            np.testing.assert_allclose(np.linalg.inv(R), Qb[:, M:][:, perm] / lam, atol=1e-10)


def test_pivot_rule_by_brute_force():
    # At step i the chosen user must have the smallest Schur-complement diagonal
    # of A given the users already chosen; Schur complements computed directly
    # with a linear solve, independent of the factorisation.
    rng = np.random.default_rng(7)
    for trial in range(6):
        N = 6
        h = vpgen.draw_rayleigh(rng, 1, N, N)[0].astype(np.complex128)
        A = O.gram(h, 0.05)
        p = O.preprocess(h, 0.05)
        chosen = []
        for i in range(N):
            rest = [u for u in range(N) if u not in chosen]
            if chosen:
                S = A[np.ix_(rest, rest)] - A[np.ix_(rest, chosen)] @ np.linalg.solve(
                    A[np.ix_(chosen, chosen)], A[np.ix_(chosen, rest)])
            else:
                S = A[np.ix_(rest, rest)]
            diag = np.real(np.diag(S))
            best = rest[int(np.argmin(diag))]
            assert best == p.perm[i]
            assert math.isclose(p.pivots[i], diag.min(), rel_tol=1e-10)
            chosen.append(best)


def test_pivot_ties_pick_smaller_user():
    # H = I: every Schur diagonal equals 1 + alpha at every step -> pi = identity.
    p = O.preprocess(np.eye(5, dtype=np.complex64), 0.1)
    assert list(p.perm) == [0, 1, 2, 3, 4]
    np.testing.assert_allclose(p.w2, np.full(5, 1 / 1.1))


@pytest.mark.parametrize("alpha", [0.0, 0.1, 2.0])
def test_rzf_matrix_closed_forms(alpha):
    rng = np.random.default_rng(11)
    N, M = 5, 7
    h = vpgen.draw_rayleigh(rng, 1, N, M)[0].astype(np.complex128)
    p = O.preprocess(h, alpha)
    if alpha > 0.0:
        # push-through identity: H^H (H H^H + a I)^{-1} = (H^H H + a I)^{-1} H^H
        G2 = np.linalg.solve(h.conj().T @ h + alpha * np.eye(M), h.conj().T)
        np.testing.assert_allclose(p.G, G2, atol=1e-10)
    # and through the triangular factor: A^{-1} = P^T W^H W P
    Pm = np.eye(N)[p.perm]
    np.testing.assert_allclose(p.G, h.conj().T @ Pm.T @ p.W.conj().T @ p.W @ Pm, atol=1e-10)
    if alpha == 0.0:
        np.testing.assert_allclose(h @ p.G, np.eye(N), atol=1e-10)


def test_overloaded_needs_regularisation():
    # N > M: H H^H is rank deficient; with alpha = 0 the factorisation fails,
    # with alpha > 0 it succeeds (Sec. III-A-1, the overloaded case).
    rng = np.random.default_rng(5)
    h = vpgen.draw_rayleigh(rng, 1, 6, 3)[0]
    assert O.preprocess(h, 0.0).status == O.STATUS_NOT_PD
    assert O.preprocess(h, 0.2).status == O.STATUS_OK


def test_nonfinite_input_flagged():
    h = np.eye(3, dtype=np.complex64)
    h[1, 2] = np.nan
    assert O.preprocess(h, 0.1).status == O.STATUS_NONFINITE


def test_unsorted_factorisation_pins():
    """sort=False: A = L L^H with L lower and a positive real diagonal, the
    identity order, W L = I; G does not depend on the ordering (it is
    H^H A^{-1} either way); the exact VP optimum over the box -- a property of
    u^H A^{-1} u alone -- is the same for both factorisations."""
    import vpgen
    wl = vpgen.cfg1(n_sc=3)
    for sc in range(wl.n_sc):
        H = wl.H[sc].astype(np.complex128)
        alpha = 0.05
        u = O.preprocess(H, alpha, sort=False)
        srt = O.preprocess(H, alpha)
        A = O.gram(H, alpha)
        assert u.status == O.STATUS_OK
        assert np.array_equal(u.perm, np.arange(wl.N))
        assert np.allclose(u.L @ u.L.conj().T, A, atol=1e-12)
        assert np.allclose(np.triu(u.L, 1), 0) and np.all(np.diag(u.L).real > 0)
        assert np.allclose(u.W @ u.L, np.eye(wl.N), atol=1e-12)
        assert np.allclose(u.G, srt.G, atol=1e-12)
        for v in range(3):
            s = wl.s[:, sc * wl.n_sym + v]
            lu, cu = O.brute_force(u.W, u.perm, s, wl.tau)
            ls, cs = O.brute_force(srt.W, srt.perm, s, wl.tau)
            assert abs(cu - cs) <= 1e-9 * cs
            assert abs(O.cost_closed_form(A, s, lu, wl.tau) - cu) <= 1e-9 * cu


def test_unsorted_factorisation_flags_singular():
    # two equal user rows under zero forcing: not positive definite
    H = np.array([[1, 2j], [1, 2j]], dtype=np.complex128)
    assert O.preprocess(H, 0.0, sort=False).status == O.STATUS_NOT_PD
