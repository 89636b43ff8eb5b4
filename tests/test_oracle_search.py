"""Pins for the oracle's same-path-set search, exact VP and precoding
(Sec. II-B PED recursion and eq:se / eq_qrse, Sec. III-A-2 DEMAP and
MoP paths, Alg. 2, eq:postproc).

Independent references used here: exhaustive enumeration of the box,
per-coordinate rounding (the rank-0 / Babai point), the RZF closed form
u^H A^{-1} u, hand-worked examples, the receiver modulo and the zero-forcing
identity H x = u."""
import itertools
import os
import math

import numpy as np
import pytest

import vpgen
from oracle import se_c
from oracle import vp_oracle as O


def _worked():
    H = np.array([[2, 0], [1, 1]], dtype=np.complex64)
    s = np.array([1 + 1j, -1 + 3j])
    paths = np.array([[0, 0], [0, 1], [1, 0], [0, 2], [1, 1]])
    return H, s, paths


def test_worked_2x2_search():
    # W = [[1,0],[-1,1]]/sqrt2, pi = [1,0], tau = 8.  s_pi = [-1+3i, 1+i].
    # Level 0: centre -s_pi0/tau = (0.125,-0.375); d(0)=0.15625 -> PED 64*0.5*0.15625 = 5.
    #   rank 1 is (0,-1) with d = 0.40625 -> PED 13.
    # Level 1 after l0 = 0: centre (-0.25, 0.25); rank 0 = 0, d = 0.125 -> +4  => 9.
    #   rank 1: (-1,0) and (0,1) tie at 0.625 -> j order picks (-1,0); +20 => 25.
    #   rank 2 is then (0,1), also +20 => 25.
    # Level 1 after l0 = -i: centre (-0.25,-0.75); rank 0 = (0,-1), d=0.125 -> 13 + 4 = 17;
    #   rank 1: (-1,-1) and (0,0) tie at 0.625 -> j picks (-1,-1); 13 + 20 = 33.
    H, s, paths = _worked()
    p = O.preprocess(H, 0.0)
    res = O.search_paths(p.W, p.perm, s[:, None], 8.0, paths, include_zero=True)
    np.testing.assert_allclose(res.path_cost[0], [9, 25, 17, 25, 33, 9], rtol=1e-12)
    assert res.kidx[0] == 0 and math.isclose(res.cost[0], 9.0)
    lv = res.path_l[0]
    assert lv[2].tolist() == [-1j, -1j]
    assert lv[3].tolist() == [0, 1j]
    # closed form for path 2: l (user order) = [-i, -i], u = [1-7i, -1-5i], cost 17
    A = O.gram(H, 0.0)
    l2 = np.zeros(2, complex)
    l2[p.perm] = lv[2]
    assert math.isclose(O.cost_closed_form(A, s, l2, 8.0), 17.0, rel_tol=1e-12)


def test_child_order_tie_rule():
    # Level-0 centre of the 256-QAM point 3+3i is (-3/32, -3/32).  Squared
    # distances: (0,0) .017578 | (-1,0),(0,-1) .830078 | (0,1),(1,0) 1.205078 |
    # (-1,-1) 1.642578 | (-1,1),(1,-1) 2.017578 | (1,1) 2.392578; equal ones in
    # canonical j order.  A 1x1 channel makes every rank's point observable.
    order = [(0, 0), (-1, 0), (0, -1), (0, 1), (1, 0), (-1, -1), (-1, 1), (1, -1), (1, 1)]
    W = np.array([[1.0 + 0j]])
    paths = np.arange(9)[:, None]
    res = O.search_paths(W, [0], np.array([[3 + 3j]]), 32.0, paths, include_zero=False)
    got = [(int(z.real), int(z.imag)) for z in res.path_l[0, :, 0]]
    assert got == order


@pytest.mark.parametrize("N,alpha", [(2, 0.0), (3, 0.2)])
def test_all_paths_equals_brute_force(N, alpha):
    # With all 9^N position vectors the rank walk is a bijection onto the box,
    # so the search must return the exhaustive optimum (eq:se over B^N).
    rng = np.random.default_rng(40 + N)
    allp = np.array(list(itertools.product(range(9), repeat=N)))
    H = vpgen.draw_rayleigh(rng, 3, N, N)
    s = vpgen.draw_symbols(rng, N, 9, 16)
    for sc in range(3):
        p = O.preprocess(H[sc], alpha)
        ss = s[:, sc * 3:(sc + 1) * 3]
        res = O.search_paths(p.W, p.perm, ss, 8.0, allp, include_zero=False)
        for v in range(3):
            lb, cb = O.brute_force(p.W, p.perm, ss[:, v], 8.0)
            assert math.isclose(res.cost[v], cb, rel_tol=1e-12)
            np.testing.assert_array_equal(res.l[v], lb)
            # every candidate distinct: the walk is a bijection
            assert len({tuple(x) for x in res.path_l[v].tolist()}) == 9 ** N


def test_cfg1_all_paths_few_vectors():
    wl = vpgen.cfg1(n_sc=2)
    allp = np.array(list(itertools.product(range(9), repeat=4)))
    p = O.preprocess(wl.H[0], 0.0)
    ss = wl.s[:, :3]
    res = O.search_paths(p.W, p.perm, ss, wl.tau, allp, include_zero=False)
    for v in range(3):
        lb, cb = O.brute_force(p.W, p.perm, ss[:, v], wl.tau)
        assert math.isclose(res.cost[v], cb, rel_tol=1e-12)


def test_rank0_is_rounding_in_box_and_cost_closed_form():
    # Rank 0 at every level = successive per-coordinate rounding clipped to the box.
    wl = vpgen.cfg3(n_sc=2)
    p = O.preprocess(wl.H[0], wl.alpha)
    A = O.gram(wl.H[0], wl.alpha)
    ss = wl.s[:, :6].astype(np.complex128)
    res = O.search_paths(p.W, p.perm, ss, wl.tau, np.zeros((1, 16), int), include_zero=False)
    for v in range(6):
        st = p.W @ ss[p.perm, v]
        lv = np.zeros(16, complex)
        for i in range(16):
            r = st[i] + wl.tau * np.dot(p.W[i, :i], lv[:i])
            c = -r / (wl.tau * p.W[i, i])
            lv[i] = np.clip(np.round(c.real), -1, 1) + 1j * np.clip(np.round(c.imag), -1, 1)
        np.testing.assert_array_equal(res.path_l[v, 0], lv)
        lu = res.l[v]
        assert math.isclose(res.cost[v], O.cost_closed_form(A, ss[:, v], lu, wl.tau), rel_tol=1e-10)
        assert math.isclose(res.cost[v], O.cost_tri(p.W, p.perm, ss[:, v], lu, wl.tau), rel_tol=1e-10)


def test_nested_path_sets_monotone_and_zero_bound():
    wl = vpgen.cfg2(20, n_sc=3)
    p = O.preprocess(wl.H[1], wl.alpha)
    ss = wl.s[:, 14:28]
    prev = None
    for K in (1, 8, 64, 256):
        paths = O.mop_paths_kbest(p.w2, K)
        res = O.search_paths(p.W, p.perm, ss, wl.tau, paths, include_zero=True)
        st = (p.W @ ss[p.perm, :].astype(np.complex128))
        assert np.all(res.cost <= np.sum(np.abs(st) ** 2, axis=0) * (1 + 1e-12))
        if prev is not None:
            assert np.all(res.cost <= prev * (1 + 1e-12))
        prev = res.cost


def test_single_user_and_diagonal_channel_need_no_perturbation():
    # N = 1 or a diagonal channel under ZF: the problem separates per user and
    # |s| < tau/2 on both rails, so the zero perturbation is optimal.
    rng = np.random.default_rng(2)
    for Q in (4, 16, 64, 256):
        tau = vpgen.qam_tau(Q)
        s = vpgen.draw_symbols(rng, 3, 20, Q)
        h = np.diag([1.3, 0.4, 2.2]).astype(np.complex64)
        p = O.preprocess(h, 0.0)
        paths = O.mop_paths_kbest(p.w2, 50)
        res = O.search_paths(p.W, p.perm, s, tau, paths)
        assert np.all(res.l == 0)
        p1 = O.preprocess(np.array([[0.7 - 0.2j]]), 0.0)
        r1 = O.search_paths(p1.W, p1.perm, s[:1], tau, np.arange(9)[:, None])
        assert np.all(r1.l == 0)


def test_sphere_encoder_equals_brute_force():
    rng = np.random.default_rng(13)
    for N, Q, alpha in ((3, 16, 0.0), (4, 16, 0.0), (4, 64, 0.1)):
        tau = vpgen.qam_tau(Q)
        H = vpgen.draw_rayleigh(rng, 2, N, N)
        s = vpgen.draw_symbols(rng, N, 12, Q)
        for sc in range(2):
            p = O.preprocess(H[sc], alpha)
            ss = s[:, sc * 6:(sc + 1) * 6]
            lc, cc, _ = se_c.sphere_encode_batch(p.W, p.perm, ss, tau)
            for v in range(6):
                lb, cb = O.brute_force(p.W, p.perm, ss[:, v], tau)
                lp, cp, _ = O.sphere_encode(p.W, p.perm, ss[:, v], tau)
                assert math.isclose(cb, cc[v], rel_tol=1e-12) and math.isclose(cb, cp, rel_tol=1e-12)
                np.testing.assert_array_equal(lc[v], lb)
                np.testing.assert_array_equal(lp, lb)


def test_sphere_encoder_bounds_the_path_search():
    wl = vpgen.cfg3(n_sc=2)
    p = O.preprocess(wl.H[1], wl.alpha)
    ss = wl.s[:, 14:28]
    paths = O.mop_paths_kbest(p.w2, 64)
    res = O.search_paths(p.W, p.perm, ss, wl.tau, paths)
    l, c, nodes = se_c.sphere_encode_batch(p.W, p.perm, ss, wl.tau, radius=res.cost * (1 + 1e-12))
    assert np.all(c <= res.cost * (1 + 1e-12))
    assert O.gap_db(res.cost, c) >= 0.0
    A = O.gram(wl.H[1], wl.alpha)
    for v in range(3):
        assert math.isclose(c[v], O.cost_closed_form(A, ss[:, v], l[v], wl.tau), rel_tol=1e-9)


@pytest.mark.parametrize("alpha", [0.0, 0.16])
def test_precode_invariants(alpha):
    wl = vpgen.cfg1(n_sc=2)
    H = wl.H[0]
    p = O.preprocess(H, alpha)
    paths = O.mop_paths_kbest(p.w2, 32)
    ss = wl.s[:, :14].astype(np.complex128)
    res = O.search_paths(p.W, p.perm, ss, wl.tau, paths)
    A = O.gram(H, alpha)
    for v in range(14):
        u = ss[:, v] + wl.tau * res.l[v]
        # eq:postproc: the receiver's modulo removes the perturbation exactly
        np.testing.assert_allclose(O.mod_tau(u, wl.tau), ss[:, v], atol=1e-12)
        x = O.precode(p.G, ss[:, v], res.l[v], wl.tau)
        if alpha == 0.0:
            np.testing.assert_allclose(H.astype(np.complex128) @ x, u, atol=1e-9)
        # gamma (the search cost) splits into radiated power plus the regulariser part
        z = np.linalg.solve(A, u)
        assert math.isclose(np.vdot(x, x).real + alpha * np.vdot(z, z).real, res.cost[v], rel_tol=1e-9)
        xn = O.precode(p.G, ss[:, v], res.l[v], wl.tau, gamma=res.cost[v], P_T=2.0)
        assert math.isclose(np.vdot(xn, xn).real, 2.0 * np.vdot(x, x).real / res.cost[v], rel_tol=1e-12)


def test_complexity_count():
    # Sec. III-B: N_r N_t + N_t^2 + K N_t (1 + (N_t + 1)/2) complex multiplications.
    assert O.complexity_cm(16, 16, 512) == 256 + 256 + 512 * 16 * 19 // 2 == 78336
    assert O.complexity_cm(4, 4, 32) == 16 + 16 + 32 * 4 * 7 // 2


def test_per_user_tau_pins():
    """One perturbation interval per user (a QAM order per user).  Pinned by:
    equal intervals reproduce the scalar-tau results; the search over all 9^N
    paths and the sphere encoder both equal the brute-force optimum of
    || W (s_pi + tau l) ||^2 with per-user tau; the reported cost is the closed
    form u^H A^{-1} u with u = s + tau l; the receiver modulo of each user's
    own tau recovers s; and the walk with per-level tau equals the plain walk
    on the rescaled problem W diag(tau_pi), s / tau, tau = 1 (a different
    route to the same objective)."""
    import itertools
    rng = np.random.default_rng(77)
    N = 3
    Qs = np.array([4, 64, 16])
    tau = np.array([2 * np.sqrt(q) for q in Qs])
    H = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(2)
    p = O.preprocess(H, 0.05)
    A = O.gram(H, 0.05)
    allp = np.array(list(itertools.product(range(9), repeat=N)))
    for v in range(6):
        s = np.array([(rng.integers(0, int(np.sqrt(q))) * 2 - (np.sqrt(q) - 1)) +
                      1j * (rng.integers(0, int(np.sqrt(q))) * 2 - (np.sqrt(q) - 1)) for q in Qs])
        lb, cb = O.brute_force(p.W, p.perm, s, tau)
        res = O.search_paths(p.W, p.perm, s[:, None], tau, allp, include_zero=False)
        assert abs(res.cost[0] - cb) <= 1e-9 * cb
        lse, cse, _ = O.sphere_encode(p.W, p.perm, s, tau)
        assert abs(cse - cb) <= 1e-9 * cb
        assert abs(O.cost_closed_form(A, s, res.l[0], tau) - res.cost[0]) <= 1e-9 * cb
        np.testing.assert_allclose(O.mod_tau(s + tau * res.l[0], tau), s, atol=1e-9)
        # rescaled problem: W' = W diag(tau_pi), s' = s / tau, tau = 1
        Wr = p.W * tau[p.perm][None, :]
        paths = O.mop_paths_kbest(np.abs(np.diag(Wr)) ** 2, 40)
        a = O.search_paths(p.W, p.perm, s[:, None], tau, paths)
        b = O.search_paths(Wr, p.perm, (s / tau)[:, None], 1.0, paths)
        assert np.array_equal(a.l, b.l) and abs(a.cost[0] - b.cost[0]) <= 1e-9 * a.cost[0]
    # equal intervals reproduce the scalar results
    s = rng.integers(-3, 4, size=(N, 5)) * 2 + 1 + 1j * (rng.integers(-3, 4, size=(N, 5)) * 2 + 1)
    paths = O.mop_paths_kbest(p.w2, 30)
    a = O.search_paths(p.W, p.perm, s, 16.0, paths)
    b = O.search_paths(p.W, p.perm, s, np.full(N, 16.0), paths)
    assert np.array_equal(a.l, b.l) and np.array_equal(a.cost, b.cost)


def _golden_region_cases():
    path = os.path.join(os.path.dirname(__file__), "golden", "region_demap_cases.txt")
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = line.split()
        c = complex(float(f[0]), float(f[1]))
        pts = [complex(*map(float, t.split(","))) for t in f[2:]]
        yield c, pts


def test_region_demap_worked_cases():
    """The region-table DEMAP against cases worked by hand (tests/golden)."""
    n = 0
    for c, pts in _golden_region_cases():
        got = [O.demap_region(c, r) for r in range(9)]
        assert got == pts, (c, got)
        n += 1
    assert n == 3


def test_region_demap_properties():
    """Rank 0 is the exact nearest box point; ranks 0..8 are nine distinct box
    points; with the order taken at the folded point itself (a table whose
    regions are points) the region DEMAP is the exact (distance, j) order at
    every rank; at a region's representative point the stored order is the
    exact one."""
    rng = np.random.default_rng(8)
    cs = rng.uniform(-2.5, 2.5, 3000) + 1j * rng.uniform(-2.5, 2.5, 3000)
    for c in cs:
        d = O.sqabs(c - O.BOX)
        exact = O.BOX[np.argsort(d, kind="stable")]
        got = [O.demap_region(c, r) for r in range(9)]
        assert got[0] == exact[0]
        assert len(set(got)) == 9 and all(abs(g.real) <= 1 and abs(g.imag) <= 1 for g in got)
        assert [O.demap_region(c, r, exact_point=True) for r in range(9)] == list(exact)
    for iu in range(4):
        for iw in range(iu + 1):
            u, w = O.region_representative(iu, iw)
            for fx in (1, -1):
                for fy in (1, -1):
                    for sw in (False, True):
                        x, y = (float(w), float(u)) if sw else (float(u), float(w))
                        c = complex(fx * x, fy * y)
                        d = O.sqabs(c - O.BOX)
                        srt = np.sort(d)
                        got = [O.demap_region(c, r) for r in range(9)]
                        # equal to the exact order wherever that order has no tie
                        for r in range(9):
                            tie = (r > 0 and srt[r] - srt[r - 1] < 1e-12) or (r < 8 and srt[r + 1] - srt[r] < 1e-12)
                            if not tie:
                                assert got[r] == O.BOX[np.argsort(d, kind="stable")[r]], (iu, iw, r)


def test_region_demap_search_with_point_orders_is_the_exact_search():
    """A region table filled with exact orders (demap 'region-exact-point')
    reproduces the exact same-path-set search bit for bit."""
    wl = vpgen.cfg2(20, n_sc=2)
    for sc in range(2):
        p = O.preprocess(wl.H[sc], wl.alpha)
        paths = O.mop_paths_kbest(p.w2, 24)
        sl = slice(sc * wl.n_sym, sc * wl.n_sym + 4)
        a = O.search_paths(p.W, p.perm, wl.s[:, sl], wl.tau, paths)
        b = O.search_paths(p.W, p.perm, wl.s[:, sl], wl.tau, paths, demap="region-exact-point")
        assert np.array_equal(a.l, b.l) and np.array_equal(a.kidx, b.kidx)
        np.testing.assert_allclose(a.path_cost, b.path_cost, rtol=1e-12)


def test_fixed_point_walk_pins():
    """The 16-bit fixed-point walk (Sec. V precision study).  Pinned by: on
    the same quantised inputs it picks what the float64 walk (demap_walk, an
    independent code path) picks on the problem those integers represent --
    W~ with W~_mm = sqrt(w_m), W~_mj = -V_mj W~_mm and s~_m = -c0_m tau W~_mm --
    except at near ties, with a PED equal to that walk's cost scaled by
    2^(3F) / tau^2; saturation of a centre beyond the 16-bit range; and a
    quantisation error that shrinks with the fractional bits."""
    wl = vpgen.cfg2(20, n_sc=3)
    for F in (8, 13):
        for sc in range(3):
            p = O.preprocess(wl.H[sc], wl.alpha)
            paths = O.mop_paths_kbest(p.w2, 16)
            sl = slice(sc * wl.n_sym, sc * wl.n_sym + 5)
            c0, Vq, wq = O.fx_inputs(p.W, p.perm, wl.s[:, sl], wl.tau, F)
            lf, ped, kf = O.fx_search(c0, Vq, wq, paths, F, include_zero=False)
            one = 2.0 ** F
            Wt = np.zeros((wl.N, wl.N), complex)
            d = np.sqrt(wq / one)
            for m in range(wl.N):
                Wt[m, m] = d[m]
                for j in range(m):
                    Wt[m, j] = -(Vq[m, j, 0] + 1j * Vq[m, j, 1]) / one * d[m]
            st = -((c0[..., 0] + 1j * c0[..., 1]) / one) * wl.tau * d[None, :]      # [V][N]
            l64, cost64, margin = O.demap_walk(Wt, st, wl.tau, paths)
            for v in range(st.shape[0]):
                k = int(np.argmin(cost64[v]))
                if np.min(margin[v]) < 1e-6:
                    continue                         # a near tie: float64 and the integers may part
                assert k == kf[v] and np.array_equal(l64[v, k], lf[v]), (F, sc, v)
                assert abs(float(ped[v]) / one ** 3 - cost64[v, k] / wl.tau ** 2) <= 1e-9 * float(ped[v]) / one ** 3
    # saturation: a centre of 5 at 13 fractional bits is held at the largest value
    assert O.fx_quantize(5.0, 13) == 32767 and O.fx_quantize(-5.0, 13) == -32768
    assert O.fx_demap(32767, 0, 0, 13)[:2] == (1, 0)
    # saturated steps and differences, worked by hand at F = 13 (one = 8192):
    # c0 = (32767, 0), (32000, 0); V_10 = 1.0; w = 1.0 each.  Level 0 takes
    # a = 1 (distance 24575^2); the step 32000 + 8192 = 40192 is held at 32767,
    # so level 1 sees the same centre and distance: PED = 8192 * 2 * 24575^2.
    # The zero candidate's distances are 32767^2 and 32000^2.
    c0 = np.array([[[32767, 0], [32000, 0]]])
    Vq = np.zeros((2, 2, 2), dtype=np.int64)
    Vq[1, 0] = (8192, 0)
    wq = np.array([8192, 8192])
    l, ped, k = O.fx_search(c0, Vq, wq, [[0, 0], [1, 0]], 13, include_zero=True)
    assert k[0] == 0 and list(l[0]) == [1, 1] and ped[0] == 8192 * 2 * 24575 ** 2
    # rank 1 at level 0 from a centre of 32767: (1, 1) and (1, -1) tie at
    # 24575^2 + 8192^2; the smaller box index 3 (re + 1) + (im + 1) wins: (1, -1)
    assert O.fx_demap(32767, 0, 1, 13) == (1, -1, 24575 ** 2 + 8192 ** 2)
    # a difference below -32768 saturates: centre -32768, box point +1
    assert O.fx_demap(-32768, 0, 8, 13)[2] == 32768 ** 2 + 8192 ** 2
    # the quantisation error of the inputs halves with every fractional bit
    p = O.preprocess(wl.H[0], wl.alpha)
    errs = []
    for F in (8, 10, 12):
        c0, _, _ = O.fx_inputs(p.W, p.perm, wl.s[:, :14], wl.tau, F)
        st = (wl.s[:, :14][p.perm, :]).T @ p.W.T
        exact = -st / (wl.tau * np.real(np.diag(p.W)))[None, :]
        errs.append(np.max(np.abs(c0[..., 0] / 2.0 ** F - exact.real)))
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 2.0 ** -13
