"""Pins for the learned-proposal oracle (oracle/mlp_oracle.py).

Independent references: hand-worked bfloat16 bit patterns and torch's own
float32 -> bfloat16 conversion; the search oracle's level-0 centre, rank-0
PED and zero-perturbation cost for the features; the search oracle's rank
walk for the labels; central finite differences and torch autograd (float64)
for the hand-derived backward; log C for constant logits; sorting-free
properties for the selection."""
import math

import numpy as np
import pytest
import torch

import vpgen
from oracle import mlp_oracle as L
from oracle import vp_oracle as O


def test_bf16_round_worked_values():
    one = 1.0
    cases = [
        (one, one),
        (one + 2.0 ** -8, one),                      # tie -> even mantissa 0
        (one + 3 * 2.0 ** -8, one + 2.0 ** -6),      # tie between odd 1 and even 2 -> 2
        (one + 2.0 ** -8 + 2.0 ** -20, one + 2.0 ** -7),   # above the tie -> up
        (-(one + 2.0 ** -8), -one),
        (3.0, 3.0),
        (0.0, 0.0),
        (2.0 ** -130, 2.0 ** -130),                  # subnormal that fits in 7 mantissa bits
    ]
    for x, want in cases:
        assert L.bf16_round(x) == want, (x, L.bf16_round(x), want)
    assert math.isnan(float(L.bf16_round(float("nan"))))
    assert L.bf16_round(np.inf) == np.inf


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.standard_normal(1000)]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(L.bf16_round(x), want)


def _subcarrier(n=8, nsym=6, seed=11, Q=64, alpha=0.05):
    wl = vpgen.make("t", N=n, M=n, n_sc=1, n_sym=nsym, Q=Q, alpha=alpha, K=8, seed=seed)
    p = O.preprocess(wl.H[0], alpha)
    s = wl.s[:, :nsym].astype(np.complex128)
    return p, s, wl.tau


def test_features_level0_centre_and_weights():
    p, s, tau = _subcarrier()
    f = L.features(p.W, p.perm, s, tau)
    n = p.W.shape[0]
    c00 = -s[p.perm[0], :] / tau                  # level 0: (W s_pi)_0 = W_00 s_pi0
    np.testing.assert_allclose(f[:, 16], c00.real, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(f[:, 32], c00.imag, rtol=1e-13, atol=1e-15)
    d = np.sqrt(p.w2)
    np.testing.assert_allclose(f[0, :n], d / d.mean(), rtol=1e-13)
    assert np.all(f[:, n:16] == 0) and np.all(f[:, 16 + n:32] == 0) and np.all(f[:, 48 + n:] == 0)


def test_features_zero_perturbation_cost():
    # sum_i tau^2 W_ii^2 |c0_i|^2 = ||W s_pi||^2 = s^H A^-1 s (the l = 0 cost)
    wl = vpgen.make("t", N=6, M=6, n_sc=1, n_sym=5, Q=16, alpha=0.1, K=8, seed=4)
    p = O.preprocess(wl.H[0], 0.1)
    s = wl.s[:, :5].astype(np.complex128)
    f = L.features(p.W, p.perm, s, wl.tau)
    n = 6
    c0 = f[:, 16:16 + n] + 1j * f[:, 32:32 + n]
    cost = (wl.tau ** 2) * np.sum(p.w2[None, :] * np.abs(c0) ** 2, axis=1)
    A = O.gram(wl.H[0], 0.1)
    for v in range(5):
        want = O.cost_closed_form(A, s[:, v], np.zeros(n), wl.tau)
        assert math.isclose(cost[v], want, rel_tol=1e-10)


def test_features_rank0_ped_share():
    # feature 48 + i at level 0 equals the level-0 PED increment of the rank-0
    # path divided by tau^2 mean(W_jj^2); with one level that is the whole cost.
    W = np.array([[0.7 + 0j]])
    s = np.array([[3 + 5j, -7 + 1j, 15 - 15j]])
    tau = 32.0
    f = L.features(W, [0], s, tau)
    res = O.search_paths(W, [0], s, tau, np.zeros((1, 1), int), include_zero=False)
    np.testing.assert_allclose(f[:, 48] * tau ** 2 * 0.49, res.path_cost[:, 0], rtol=1e-12)


def test_features_scale_invariant():
    p, s, tau = _subcarrier(seed=3)
    f1 = L.features(p.W, p.perm, s, tau)
    f2 = L.features(p.W * 3.7, p.perm, s, tau)
    np.testing.assert_allclose(f1, f2, rtol=1e-12, atol=1e-14)


def test_features_walk_reproduce_rank0_path():
    # sum_i tau^2 W_ii^2 |c_i - b_i|^2 along the walk is the cost of the rank-0
    # path; the level-i gap is the extra PED of taking rank 1 at level i alone
    p, s, tau = _subcarrier(n=6, nsym=7, seed=21, Q=64)
    f, gap = L.features_walk(p.W, p.perm, s, tau)
    n = 6
    off = f[:, 16:16 + n] + 1j * f[:, 32:32 + n]
    cost0 = tau ** 2 * np.sum(p.w2[None, :] * np.abs(off) ** 2, axis=1)
    zero = np.zeros((1, n), int)
    res = O.search_paths(p.W, p.perm, s, tau, zero, include_zero=False)
    np.testing.assert_allclose(cost0, res.path_cost[:, 0], rtol=1e-11)
    w2m = np.mean(p.w2)
    for i in range(n):
        path = np.zeros((1, n), int)
        path[0, i] = 1
        r1 = O.search_paths(p.W, p.perm, s, tau, path, include_zero=False)
        # PED of levels <= i: prefix of the rank-0 path, then rank 1 at level i
        pre = tau ** 2 * np.sum(p.w2[None, :i] * np.abs(off[:, :i]) ** 2, axis=1)
        ped_i = tau ** 2 * p.w2[i] * np.abs(off[:, i]) ** 2
        l1 = r1.path_l[:, 0, i]
        c_i = -((p.W @ s[p.perm, :]).T[:, i] + tau * np.sum(p.W[i, :i][None, :] * res.path_l[:, 0, :i], axis=1)) \
            / (tau * p.W[i, i])
        extra = tau ** 2 * p.w2[i] * (np.abs(c_i - l1) ** 2) - ped_i
        np.testing.assert_allclose(f[:, 48 + i] * w2m * tau ** 2, extra, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(pre + ped_i + extra, pre + tau ** 2 * p.w2[i] * np.abs(c_i - l1) ** 2,
                                   rtol=1e-12)
    assert np.all(gap >= 0)


def test_path_ranks_inverts_rank_walk():
    p, s, tau = _subcarrier(n=8, nsym=12, seed=8)
    rng = np.random.default_rng(2)
    ranks = rng.integers(0, 9, size=(12, 8))
    l = L.walk_ranks(p.W, p.perm, s, tau, ranks)
    got, margin = L.path_ranks(p.W, p.perm, s, tau, l)
    ok = margin > 1e-9
    assert ok.mean() > 0.9
    np.testing.assert_array_equal(got[ok], ranks[ok])


def test_path_ranks_outside_box_and_exact_solution():
    p, s, tau = _subcarrier(n=4, nsym=3, seed=9, Q=16)
    l = np.zeros((4, 3), complex)
    l[2, 1] = 2 + 0j
    r, _ = L.path_ranks(p.W, p.perm, s, tau, l)
    lvl = int(np.nonzero(p.perm == 2)[0][0])
    assert r[1, lvl] == 15
    # the exact solution's position vector walks back to the exact solution
    l_bf = np.stack([O.brute_force(p.W, p.perm, s[:, v], tau)[0] for v in range(3)], axis=1)
    rk, _ = L.path_ranks(p.W, p.perm, s, tau, l_bf)
    back = L.walk_ranks(p.W, p.perm, s, tau, rk)
    np.testing.assert_array_equal(back, l_bf)


def _small_net(seed=0, V=40, n_in=64, hidden=256):
    rng = np.random.default_rng(seed)
    p = L.init_params(rng, V, n_in=n_in, hidden=hidden, dtype_round=None)
    x = rng.standard_normal((7, n_in))
    y = rng.integers(-1, V, size=7)
    y[0] = 3
    return p, x, y


def test_backward_matches_finite_differences():
    p, x, y = _small_net(V=12, hidden=16, n_in=8)
    c = L.mlp_forward(x, p)
    loss, g = L.softmax_xent(c.z3, y)
    n = max(int(np.sum(y >= 0)), 1)
    G = L.mlp_backward(c, p, g / n)
    rng = np.random.default_rng(7)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        arr = getattr(p, name)
        ga = getattr(G, "d" + name)
        for _ in range(6):
            idx = tuple(rng.integers(0, d) for d in arr.shape)
            save = arr[idx]
            arr[idx] = save + h
            lp = L.mean_loss(x, y, p)
            arr[idx] = save - h
            lm = L.mean_loss(x, y, p)
            arr[idx] = save
            fd = (lp - lm) / (2 * h)
            assert abs(fd - ga[idx]) <= 1e-6 * (1 + abs(fd)), (name, idx, fd, ga[idx])


def test_backward_matches_torch_autograd():
    p, x, y = _small_net(V=40, hidden=32, n_in=64, seed=4)
    c = L.mlp_forward(x, p)
    _, g = L.softmax_xent(c.z3, y)
    n = max(int(np.sum(y >= 0)), 1)
    G = L.mlp_backward(c, p, g / n)
    T = {k: torch.tensor(getattr(p, k), dtype=torch.float64, requires_grad=True) for k in p._fields}
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    h1 = torch.relu(xt @ T["W1"].T + T["b1"])
    h2 = torch.relu(h1 @ T["W2"].T + T["b2"])
    z = h2 @ T["W3"].T + T["b3"]
    yt = torch.tensor(y)
    lab = yt >= 0
    loss = torch.nn.functional.cross_entropy(z[lab], yt[lab], reduction="sum") / n
    loss.backward()
    for k in p._fields:
        np.testing.assert_allclose(getattr(G, "d" + k), T[k].grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(G.dx, xt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_softmax_xent_constant_logits():
    z = np.full((3, 4096), 2.5)
    loss, g = L.softmax_xent(z, np.array([0, 4095, -1]))
    np.testing.assert_allclose(loss[:2], math.log(4096), rtol=1e-13)
    assert loss[2] == 0 and np.all(g[2] == 0)
    np.testing.assert_allclose(g[0].sum(), 0.0, atol=1e-12)
    assert math.isclose(g[0, 0], 1 / 4096 - 1, rel_tol=1e-12)


def test_topk_properties_and_ties():
    rng = np.random.default_rng(3)
    s = rng.integers(-5, 6, size=(20, 300)).astype(np.float32)   # many ties
    s[0, :5] = [0.0, -0.0, 0.0, -0.0, 0.0]
    sel = L.topk(s, 64)
    for r in range(20):
        chosen = set(sel[r].tolist())
        assert len(chosen) == 64
        rest = [c for c in range(300) if c not in chosen]
        assert s[r, sel[r]].min() >= s[r, rest].max()
        # equal values in column order; boundary ties resolved toward small columns
        vals = s[r, sel[r]]
        assert np.all(np.diff(vals) <= 0)
        for a, b in zip(sel[r][:-1], sel[r][1:]):
            if s[r, a] == s[r, b] and np.signbit(s[r, a]) == np.signbit(s[r, b]):
                assert a < b
        t = vals[-1]
        tied_out = [c for c in rest if s[r, c] == t and np.signbit(s[r, c]) == np.signbit(t)]
        tied_in = [c for c in sel[r] if s[r, c] == t and np.signbit(s[r, c]) == np.signbit(t)]
        if tied_out:
            assert max(tied_in) < min(tied_out)
    # +0 ranks above -0
    z = np.zeros((1, 64), np.float32)
    z[0, :32] = -0.0
    z = np.concatenate([z, np.full((1, 10), -1.0, np.float32)], axis=1)
    sel = L.topk(z, 64)[0]
    assert list(sel[:32]) == list(range(32, 64)) and list(sel[32:]) == list(range(32))


def test_softmax_mass_closed_form():
    z = np.zeros((1, 128))
    assert math.isclose(L.softmax_mass(z, np.arange(64)[None, :])[0], 0.5, rel_tol=1e-14)
    z[0, 0] = math.log(3.0)   # e^z = 3: mass of {0} = 3 / 130
    assert math.isclose(L.softmax_mass(z, np.array([[0]]))[0], 3 / 130, rel_tol=1e-13)
