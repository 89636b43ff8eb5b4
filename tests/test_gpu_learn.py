"""GPU parity of the learned-proposal kernels (include/vp_learn.h) against
the FP64 oracle (oracle/mlp_oracle.py), through the C ABI.

Float results are checked against element-wise error bounds derived from the
float32 / bf16 arithmetic (tests/mlp_bounds.py); selections (top-64, ranks,
path tables) must be bit-exact; per-vector path search follows the search's
parity rule (tests/vp_parity.py)."""
import numpy as np
import pytest

import vpgen
from oracle import mlp_oracle as L
from oracle import vp_oracle as O
from tests import mlp_bounds as MB
from tests.vp_parity import ParityReport, check_search_subcarrier, l_from_gpu, unpack_W, record

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_12098_amd as vp
    import paper_2602_12098_amd.learn as learn
    return vp, learn


def _say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def bf(x):
    """float64 values already representable in bf16 -> bf16 GPU tensor."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV).to(torch.bfloat16)


def host(t):
    if t.dtype == torch.bfloat16:
        t = t.float()
    return t.detach().cpu().numpy()


# --------------------------------------------------------------------------- GEMM

GEMM_CASES = [
    # m, n, k, trans_a, trans_b, bias, relu, mask, alpha
    (1, 1, 1, 0, 1, False, False, False, 1.0),
    (37, 65, 19, 0, 1, True, True, False, 1.0),
    (130, 257, 64, 0, 1, True, False, False, 1.0),
    (300, 129, 300, 0, 0, False, False, True, 1.0),
    (129, 200, 77, 1, 0, False, False, False, 0.5),
    (64, 96, 130, 1, 1, True, True, True, 1.0),
    (256, 256, 256, 0, 1, True, True, False, 1.0),
    (5, 4096, 256, 0, 1, True, False, False, 1.0),
    (33, 17, 0, 0, 1, True, True, False, 1.0),
]


@pytest.mark.parametrize("case", GEMM_CASES)
def test_gemm_bf16_bound(lib, case):
    _, learn = lib
    m, n, k, ta, tb, use_bias, relu, use_mask, alpha = case
    _say("gemm", case)
    rng = np.random.default_rng(m * 1000 + n + k)
    A = L.bf16_round(rng.standard_normal((k, m) if ta else (m, k)))
    B = L.bf16_round(rng.standard_normal((n, k) if tb else (k, n)))
    bias = rng.standard_normal(n).astype(np.float32).astype(np.float64) if use_bias else None
    mask = L.bf16_round(rng.standard_normal((m, n))) if use_mask else None
    Ae = A.T if ta else A
    Be = B.T if tb else B
    C = alpha * (Ae @ Be)
    if bias is not None:
        C = C + bias
    bound = MB.gemm_bound(np.abs(Ae), np.abs(Be), k, np.abs(bias) if bias is not None else None)
    if relu:
        C = np.maximum(C, 0)
    if mask is not None:
        C = np.where(mask > 0, C, 0.0)
        bound = np.where(mask > 0, bound, 0.0)
    Cf, Cb = learn.gemm_bf16(bf(A), bf(B), trans_a=bool(ta), trans_b=bool(tb),
                             bias=dev(bias.astype(np.float32)) if bias is not None else None, relu=relu,
                             mask=bf(mask) if mask is not None else None, alpha=alpha, out_f32=True, out_bf16=True)
    torch.cuda.synchronize()
    gf, gb = host(Cf), host(Cb)
    assert np.all(np.abs(gf - C) <= bound + 1e-30), np.max(np.abs(gf - C) - bound)
    assert np.all(np.abs(gb - C) <= MB.BF * (np.abs(C) + bound) + bound + 1e-30)
    if mask is not None:
        assert np.all(gf[mask <= 0] == 0)


def test_gemm_strided_operands(lib):
    # leading dimensions larger than the row length, and an unaligned start
    _, learn = lib
    rng = np.random.default_rng(9)
    big = L.bf16_round(rng.standard_normal((70, 90)))
    Bm = L.bf16_round(rng.standard_normal((40, 33)))
    Ad = bf(big)[3:60, 1:41]          # 57 x 40 view, ld 90, start not 16-byte aligned
    Bd = bf(Bm)
    C = host(learn.gemm_bf16(Ad, Bd))
    want = big[3:60, 1:41] @ Bm
    bound = MB.gemm_bound(np.abs(big[3:60, 1:41]), np.abs(Bm), 40)
    assert np.all(np.abs(C - want) <= bound + 1e-30)


# --------------------------------------------------------------------------- features / ranks

def _prep(vp, wl):
    Hd = dev(wl.H)
    prep = vp.preprocess(Hd, wl.alpha)
    torch.cuda.synchronize()
    return prep


def _feature_bound(f64, W, perm, s, tau):
    """|gpu - exact| bound of each feature (float32 arithmetic, one bf16 rounding)."""
    n = W.shape[0]
    V = s.shape[1]
    d = np.real(np.diag(W))
    mag = (np.abs(W) @ np.abs(s[perm, :])).T / (tau * d[None, :])       # sum |W_ij||s_j| / (tau W_ii)
    E = np.zeros((V, 64))
    Ec = (4 * n + 8) * U32 * mag + 4 * U32 * np.abs(f64[:, 16:16 + n] + 1j * f64[:, 32:32 + n])
    E[:, :n] = (n + 4) * U32 * np.abs(f64[:, :n])
    E[:, 16:16 + n] = Ec
    E[:, 32:32 + n] = Ec
    c0 = f64[:, 16:16 + n] + 1j * f64[:, 32:32 + n]
    b0 = np.clip(np.round(c0.real), -1, 1) + 1j * np.clip(np.round(c0.imag), -1, 1)
    scale = d[None, :] ** 2 / np.mean(d ** 2)
    E[:, 48:48 + n] = scale * 4 * (np.abs(c0 - b0) + Ec) * Ec + (2 * n + 8) * U32 * np.abs(f64[:, 48:48 + n])
    return MB.BF * (np.abs(f64) + E) + E


def _walk_feature_bound(f64, W, perm, s, tau):
    """Bound for the rank-0-walk features: the float32 residual of level i
    carries the rounding of its level-i sum of W_ij (s_j + tau b_j) terms."""
    n = W.shape[0]
    V = s.shape[1]
    d = np.real(np.diag(W))
    off = f64[:, 16:16 + n] + 1j * f64[:, 32:32 + n]
    smag = np.abs(s[perm, :]).T + tau * 1.5                      # |s_j| + tau |b_j|, |b_j| <= sqrt 2
    mag = (smag @ np.abs(W).T) / (tau * d[None, :])
    Ec = (8 * n + 16) * U32 * mag
    E = np.zeros((V, 64))
    E[:, :n] = (n + 4) * U32 * np.abs(f64[:, :n])
    E[:, 16:16 + n] = Ec + 2 * U32 * np.abs(off)
    E[:, 32:32 + n] = Ec + 2 * U32 * np.abs(off)
    scale = d[None, :] ** 2 / np.mean(d ** 2)
    E[:, 48:48 + n] = scale * 6 * Ec + (2 * n + 8) * U32 * np.abs(f64[:, 48:48 + n])
    return MB.BF * (np.abs(f64) + E) + E


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("N,Q,alpha", [(16, 256, 0.16), (8, 64, 0.08), (5, 16, 0.3), (1, 16, 0.1), (3, 4, 0.05)])
def test_features_vs_oracle(lib, N, Q, alpha, kind):
    vp, learn = lib
    wl = vpgen.make("feat", N=N, M=N, n_sc=9, n_sym=14, Q=Q, alpha=alpha, K=8, seed=100 + N)
    _say("features", N, Q, "kind", kind)
    prep = _prep(vp, wl)
    f = host(learn.mlp_features(prep.W, prep.perm, dev(wl.s), wl.tau, wl.n_sym, kind=kind))
    Wd = unpack_W(host(prep.W), N)
    perm = host(prep.perm).astype(np.int64)
    n_cmp = 0
    for sc in range(wl.n_sc):
        sl = slice(sc * wl.n_sym, (sc + 1) * wl.n_sym)
        s = wl.s[:, sl].astype(np.complex128)
        if kind == 0:
            want = L.features(Wd[sc], perm[sc], s, wl.tau)
            bound = _feature_bound(want, Wd[sc], perm[sc], s, wl.tau)
            use = np.ones(wl.n_sym, bool)
        else:
            # a rank-0 choice within 1e-4 of a tie may go the other way in float32
            want, gap = L.features_walk(Wd[sc], perm[sc], s, wl.tau)
            bound = _walk_feature_bound(want, Wd[sc], perm[sc], s, wl.tau)
            use = gap > 1e-4
        err = np.abs(f[sl] - want)
        assert np.all(err[use] <= bound[use] + 1e-30), (sc, np.max(err[use] - bound[use]))
        n_cmp += int(use.sum())
    assert n_cmp >= 0.9 * wl.n_vec


def test_features_failed_subcarrier_zero(lib):
    vp, learn = lib
    wl = vpgen.make("featbad", N=4, M=4, n_sc=3, n_sym=2, Q=16, alpha=0.1, K=8, seed=5)
    H = wl.H.copy()
    H[1, 0, 0] = np.nan
    prep = vp.preprocess(dev(H), wl.alpha)
    for kind in (0, 1):
        f = host(learn.mlp_features(prep.W, prep.perm, dev(wl.s), wl.tau, wl.n_sym, kind=kind))
        assert np.all(f[2:4] == 0) and np.any(f[0:2] != 0)


@pytest.mark.parametrize("N,Q", [(16, 256), (8, 64), (4, 16), (2, 4)])
def test_path_ranks_vs_oracle(lib, N, Q):
    vp, learn = lib
    wl = vpgen.make("ranks", N=N, M=N, n_sc=6, n_sym=14, Q=Q, alpha=0.1, K=8, seed=200 + N)
    _say("ranks", N)
    prep = _prep(vp, wl)
    Wd = unpack_W(host(prep.W), N)
    perm = host(prep.perm).astype(np.int64)
    rng = np.random.default_rng(N)
    want = rng.integers(0, 9, size=(wl.n_vec, N))
    l = np.zeros((N, wl.n_vec), complex)
    for sc in range(wl.n_sc):
        sl = slice(sc * wl.n_sym, (sc + 1) * wl.n_sym)
        l[:, sl] = L.walk_ranks(Wd[sc], perm[sc], wl.s[:, sl].astype(np.complex128), wl.tau, want[sl])
    l8 = np.stack([l.real, l.imag], axis=-1).astype(np.int8)
    got = host(learn.path_ranks(prep.W, prep.perm, dev(wl.s), wl.tau, dev(l8), wl.n_sym))
    # bit-exact where no DEMAP decision along the walk is within 1e-4 of a tie;
    # elsewhere the GPU's ranks must reach the same l when near ties may go
    # either way (float32 may order near-equal distances differently)
    from tests.vp_parity import relaxed_walks
    n_exact = 0
    for sc in range(wl.n_sc):
        sl = slice(sc * wl.n_sym, (sc + 1) * wl.n_sym)
        s_sc = wl.s[:, sl].astype(np.complex128)
        _, margin = L.path_ranks(Wd[sc], perm[sc], s_sc, wl.tau, l[:, sl])
        for j in range(wl.n_sym):
            v = sc * wl.n_sym + j
            if margin[j] > 1e-4:
                assert np.array_equal(got[v], want[v]), (v, got[v], want[v])
                n_exact += 1
            else:
                st = Wd[sc] @ s_sc[perm[sc], j]
                walks = relaxed_walks(Wd[sc], st, wl.tau, got[v].astype(np.int64))
                assert any(np.array_equal(w[0], l[perm[sc], v]) for w in walks), (v, got[v], want[v])
    _say("ranks exact", n_exact, "of", wl.n_vec)
    # a symbol outside the box has rank 15
    l8[0, 0, 0] = 2
    got = host(learn.path_ranks(prep.W, prep.perm, dev(wl.s), wl.tau, dev(l8), wl.n_sym))
    assert got[0, int(np.nonzero(perm[0] == 0)[0][0])] == 15


# --------------------------------------------------------------------------- selection / loss

@pytest.mark.parametrize("rows,C,kind", [(1, 64, "normal"), (37, 65, "ties"), (200, 4096, "normal"),
                                         (50, 1000, "ties"), (8, 4096, "zeros"), (3, 4096, "const"),
                                         (300, 4096, "coarse"), (40, 4096, "skewed"), (33, 4095, "normal"),
                                         (21, 4096, "unaligned"), (64, 130, "coarse")])
def test_topk64_vs_oracle(lib, rows, C, kind):
    """Every selection route of the kernel: candidates above the bound from the
    lanes' two largest (normal, coarse = ties at the boundary), the exact
    search (short rows, ties over many columns, skewed = the 128 largest in
    two lanes' columns), rows of C = 4095 (no float4 loads) and rows at an
    address that is not 16-byte aligned."""
    _, learn = lib
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(rows + C)
    if kind in ("normal", "unaligned"):
        s = (rng.standard_normal((rows, C)) * 3).astype(np.float32)
    elif kind == "coarse":
        s = (np.round(rng.standard_normal((rows, C)) * 48) / 16).astype(np.float32)
    elif kind == "skewed":
        s = rng.standard_normal((rows, C)).astype(np.float32)
        c = np.arange(C)
        s[:, ((c % 256) // 4) < 2] += 10.0
    elif kind == "ties":
        s = rng.integers(-3, 4, size=(rows, C)).astype(np.float32)
    elif kind == "zeros":
        s = np.where(rng.random((rows, C)) < 0.5, np.float32(0.0), np.float32(-0.0)).astype(np.float32)
        s[:, ::7] = -1.0
    else:
        s = np.full((rows, C), 1.25, np.float32)
    if kind == "unaligned":
        buf = torch.zeros(rows * C + 1, dtype=torch.float32, device="cuda")
        scores = buf[1:].view(rows, C)
        scores.copy_(torch.from_numpy(s))
    else:
        scores = dev(s)
    idx, mass = learn.topk64(scores)
    idx, mass = host(idx), host(mass)
    want = L.topk(s, 64)
    np.testing.assert_array_equal(idx, want)
    wm = L.softmax_mass(s.astype(np.float64), want)
    assert np.all(np.abs(mass - wm) <= 1e-4 * (1 + wm))
    idx2, mass2 = learn.topk64(scores, with_mass=False)
    assert mass2 is None
    np.testing.assert_array_equal(host(idx2), want)



def test_topk64_on_trained_logits_at_the_benchmark_launch(lib):
    """The committed network's logits for all 45,864 vectors of the benchmark's
    slot, selected on the GPU in one launch; 400 sampled rows against the
    oracle (selection bit-exact, mass within 1e-4)."""
    import os
    _, learn = lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(root, "paper_2602_12098_amd", "weights", "proposer_16x16_256qam_res64.safetensors")
    if not os.path.exists(path):
        pytest.skip("no committed proposer")
    import paper_2602_12098_amd as vp
    prop = learn.load_proposer(path)
    wl = vpgen.cfg3(512)
    prep = vp.preprocess(dev(wl.H), wl.alpha)
    with torch.no_grad():
        x = learn.mlp_features(prep.W, prep.perm, dev(wl.s), wl.tau, wl.n_sym, kind=prop.kind)
        z = learn.mlp_logits(x, prop.p)
    assert z.dtype == torch.float32 and tuple(z.shape) == (wl.n_vec, 4096)
    idx, mass = learn.topk64(z)
    rows = np.random.default_rng(3).choice(wl.n_vec, 400, replace=False)
    zs = host(z[torch.from_numpy(rows).to(DEV)])
    want = L.topk(zs, 64)
    np.testing.assert_array_equal(host(idx)[rows], want)
    wm = L.softmax_mass(zs.astype(np.float64), want)
    assert np.all(np.abs(host(mass)[rows] - wm) <= 1e-4 * (1 + wm))

def test_softmax_xent_vs_oracle(lib):
    _, learn = lib
    rng = np.random.default_rng(17)
    rows, C = 70, 4096
    z = (rng.standard_normal((rows, C)) * 4).astype(np.float32)
    y = rng.integers(-1, C, size=rows).astype(np.int32)
    loss, dz = learn.softmax_xent(dev(z), dev(y), 1.0 / 50)
    loss, dz = host(loss), host(dz)
    wl, wg = L.softmax_xent(z.astype(np.float64), y)
    wg = wg / 50
    assert np.all(np.abs(loss - wl) <= 1e-5 * (1 + np.abs(wl)))
    assert np.all(np.abs(dz - wg) <= MB.BF * np.abs(wg) + 1e-6 * (np.abs(wg) + 1e-3 / 50))


def test_colsum_vs_oracle(lib):
    _, learn = lib
    rng = np.random.default_rng(2)
    X = L.bf16_round(rng.standard_normal((1000, 300)))
    got = host(learn.colsum_bf16(bf(X)))
    want = X.sum(axis=0)
    assert np.all(np.abs(got - want) <= MB.gam(1000) * np.abs(X).sum(axis=0))


def test_learned_paths_table(lib):
    _, learn = lib
    rng = np.random.default_rng(4)
    V, N, n_sc, n_sym, Kft, Kf = 100, 12, 5, 3, 20, 6
    vocab = rng.integers(0, 9, size=(V, N)).astype(np.uint8)
    top = rng.integers(0, V, size=(n_sc * n_sym, 64)).astype(np.int32)
    top[0, 0], top[1, 5] = -5, V + 3            # clamped
    fixed = rng.integers(0, 9, size=(n_sc, Kft, N)).astype(np.uint8)
    t = host(learn.learned_paths(dev(vocab), dev(top), dev(fixed), Kf, n_sc, n_sym))
    want = np.concatenate([vocab[np.clip(top, 0, V - 1)], np.repeat(fixed[:, :Kf], n_sym, axis=0)], axis=1)
    np.testing.assert_array_equal(t, want)


# --------------------------------------------------------------------------- per-vector search

@pytest.mark.parametrize("N,Q,K", [(16, 256, 72), (16, 256, 300), (8, 64, 9), (5, 16, 64), (3, 4, 200)])
def test_search_per_vector_tables(lib, N, Q, K):
    vp, learn = lib
    wl = vpgen.make("pv", N=N, M=N, n_sc=5, n_sym=14, Q=Q, alpha=0.1, K=K, seed=300 + N + K)
    _say("per-vector search", N, K)
    prep = _prep(vp, wl)
    rng = np.random.default_rng(K)
    tables = rng.integers(0, 4, size=(wl.n_vec, K, N)).astype(np.uint8)
    tables[:, 0] = 0
    out = vp.search(prep.W, prep.perm, dev(wl.s), wl.tau, dev(tables), wl.n_sym,
                    flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
    torch.cuda.synchronize()
    Wd = unpack_W(host(prep.W), N)
    perm = host(prep.perm).astype(np.int64)
    l = l_from_gpu(host(out.l))
    cost, kidx = host(out.cost), host(out.kidx)
    rep = ParityReport()
    for v in range(wl.n_vec):
        sc = v // wl.n_sym
        sl = slice(v, v + 1)
        check_search_subcarrier(rep, Wd[sc], perm[sc], wl.s[:, sl].astype(np.complex128), wl.tau, tables[v], True,
                                l[sl], cost[sl], kidx[sl])
    _say(rep)
    record("learned-tables", rep)
    assert rep.ok(), rep.failures[:4]
    assert rep.exact >= 0.98 * rep.n


def test_search_per_vector_rejects_bad_args(lib):
    vp, _ = lib
    from paper_2602_12098_amd import _lib
    wl = vpgen.make("pvbad", N=4, M=4, n_sc=2, n_sym=2, Q=16, alpha=0.1, K=8, seed=1)
    prep = _prep(vp, wl)
    tables = torch.zeros((4, 8, 4), dtype=torch.uint8, device=DEV)
    with pytest.raises(ValueError):   # first dimension must be n_vec
        vp.search(prep.W, prep.perm, dev(wl.s), wl.tau, tables[:2], wl.n_sym, flags=vp.VP_PATHS_PER_VECTOR)
    lib_ = _lib.load()
    out = vp.search(prep.W, prep.perm, dev(wl.s), wl.tau, tables, wl.n_sym, flags=vp.VP_PATHS_PER_VECTOR)
    taus = vp.tau_array(wl.tau, wl.n_sc, DEV)
    rc = lib_.vp_search(prep.W.data_ptr(), prep.perm.data_ptr(), dev(wl.s).data_ptr(), taus.data_ptr(),
                        tables.data_ptr(),
                        None, 8, 0, 2, 2, 4, vp.VP_PATHS_PER_VECTOR, out.l.data_ptr(), out.cost.data_ptr(),
                        out.kidx.data_ptr(), None)
    assert rc == _lib.VP_EINVAL


# --------------------------------------------------------------------------- network forward / backward

def _net(V, seed):
    rng = np.random.default_rng(seed)
    p = L.init_params(rng, V)
    return p, rng


def _params_dev(learn, p):
    return learn.MLPParams(bf(p.W1), dev(p.b1.astype(np.float32)), bf(p.W2), dev(p.b2.astype(np.float32)),
                           bf(p.W3), dev(p.b3.astype(np.float32)))


@pytest.mark.parametrize("rows,V", [(300, 4096), (129, 1000), (1, 64)])
def test_mlp_forward_bound(lib, rows, V):
    _, learn = lib
    p, rng = _net(V, rows)
    x = L.bf16_round(rng.standard_normal((rows, 64)))
    z = host(learn.mlp_logits(bf(x), _params_dev(learn, p)))
    c = L.mlp_forward(x, p)
    fb = MB.forward_bounds(c, p)
    err = np.abs(z - c.z3)
    assert np.all(err <= fb["e_z3"] + 1e-30), np.max(err - fb["e_z3"])
    _say("forward max err / bound", float(np.max(err / (fb["e_z3"] + 1e-30))))


def test_mlp_backward_bound(lib):
    _, learn = lib
    rows, V = 200, 1000
    p, rng = _net(V, 77)
    x = L.bf16_round(rng.standard_normal((rows, 64)))
    dz3 = L.bf16_round(rng.standard_normal((rows, V)) * 1e-2)
    P = _params_dev(learn, p)
    params = [t.float().clone().requires_grad_(True) for t in P]   # float32 masters holding bf16 values
    z = learn.MLPFunction.apply(bf(x), *params)
    z.backward(dev(dz3.astype(np.float32)))
    c = L.mlp_forward(x, p)
    fb = MB.forward_bounds(c, p)
    g = L.mlp_backward(c, p, dz3)
    eb = MB.backward_bounds(c, p, dz3, fb)
    for name, t in zip(("W1", "b1", "W2", "b2", "W3", "b3"), params):
        got = host(t.grad)
        want = getattr(g, "d" + name)
        err = np.abs(got - want)
        assert np.all(err <= eb["d" + name] + 1e-30), (name, np.max(err - eb["d" + name]))


def test_mlp_backward_vs_torch_autograd(lib):
    # a plain PyTorch float32 network with the same bf16 roundings, differentiated
    # by autograd: the gradients agree norm-wise to a few bf16 ulps
    _, learn = lib
    rows, V = 256, 4096
    p, rng = _net(V, 5)
    x = L.bf16_round(rng.standard_normal((rows, 64)))
    y = rng.integers(0, V, size=rows).astype(np.int64)
    P = _params_dev(learn, p)
    params = [t.float().clone().requires_grad_(True) for t in P]
    z = learn.MLPFunction.apply(bf(x), *params)
    loss = torch.nn.functional.cross_entropy(z, dev(y))
    loss.backward()
    T = [t.detach().float().clone().requires_grad_(True) for t in P]
    xf = bf(x).float()
    h1 = torch.relu(xf @ T[0].T + T[1]).to(torch.bfloat16).float()
    h2 = torch.relu(h1 @ T[2].T + T[3]).to(torch.bfloat16).float()
    zr = h2 @ T[4].T + T[5]
    lr = torch.nn.functional.cross_entropy(zr, dev(y))
    lr.backward()
    assert abs(loss.item() - lr.item()) <= 1e-3 * (1 + abs(lr.item()))
    for a, b in zip(params, T):
        assert a.grad.dtype == torch.float32
        ga, gb = a.grad, b.grad
        rel = (ga - gb).norm() / gb.norm().clamp_min(1e-30)
        assert rel.item() <= 2.0 ** -5, rel.item()
