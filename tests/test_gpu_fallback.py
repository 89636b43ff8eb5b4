"""GPU tests of vp_search_fallback: the fixed path set for the vectors whose
proposal is not confident.

The fallback must equal, bit for bit, the plain vp_search over the fixed table
restricted to the flagged vectors (that search is itself held to the FP64
oracle by the parity tests), merged with the proposal's result where the
fixed cost is strictly lower.  A direct oracle check covers a few flagged
vectors as well.  Every search kernel is reached: prefix sharing (orders),
one wave per vector (K <= 192) and one workgroup per vector (K > 192), with
an odd symbol count so that the last workgroup of the prefix-sharing kernel
holds one live vector."""
import numpy as np
import pytest

import vpgen
from oracle import vp_oracle as O
from tests.vp_parity import l_from_gpu, unpack_W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_12098_amd as vp
    import paper_2602_12098_amd.learn as learn
    return vp, learn


def _proposal_tables(rng, n_vec, K, N):
    """Per-vector tables of small random ranks (a stand-in for a proposal)."""
    t = rng.integers(0, 3, size=(n_vec, K, N)).astype(np.uint8)
    t[:, 0, :] = 0
    return t


@pytest.mark.parametrize("K_fix,use_order,theta,n_sc,n_sym", [(128, True, 0.5, 10, 5), (128, False, 0.5, 10, 5),
                                                               (300, False, 0.3, 10, 5), (512, True, 0.7, 10, 5),
                                                               (512, True, float("inf"), 10, 5),
                                                               (512, True, 0.5, 10, 14), (512, True, 0.5, 2, 71)])
def test_fallback_matches_restricted_fixed_search(lib, K_fix, use_order, theta, n_sc, n_sym):
    # with orders, a workgroup of the prefix-sharing kernel takes the j-th pair
    # of its subcarrier's flagged vectors (up to 64 symbols per subcarrier;
    # beyond, the symbols 2 j and 2 j + 1 with those not flagged skipped)
    vp, learn = lib
    wl = vpgen.make("16x16-rzf-256qam-rho0.5", 16, 16, n_sc, n_sym, 256, 0.16, K_fix, seed=41, rho=0.5)
    N, n_sym, n_vec = wl.N, wl.n_sym, wl.n_vec
    rng = np.random.default_rng(K_fix)
    print(f"fallback case K={K_fix} order={use_order} theta={theta} n_sc={n_sc} n_sym={n_sym}", flush=True)
    H = torch.from_numpy(wl.H).to(DEV)
    s = torch.from_numpy(wl.s).to(DEV)
    prep = vp.preprocess(H, wl.alpha)
    order = torch.empty((wl.n_sc, 2, K_fix), dtype=torch.int16, device=DEV)
    fixed = vp.paths_mop(prep.w2, K_fix, order=order)
    Kp = 24
    prop = torch.from_numpy(_proposal_tables(rng, n_vec, Kp, N)).to(DEV)
    flags_pv = vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR
    lr = vp.search(prep.W, prep.perm, s, wl.tau, prop, n_sym, flags=flags_pv)
    mass_np = rng.random(n_vec).astype(np.float32)
    mass_np[::7] = np.nan
    mass = torch.from_numpy(mass_np).to(DEV)
    out = vp.SearchOut(lr.l.clone(), lr.cost.clone(), lr.kidx.clone())
    base = Kp + 1
    learn.search_fallback(prep.W, prep.perm, s, wl.tau, fixed, n_sym, mass, theta, out, base,
                          order=order if use_order else None)
    fx = vp.search(prep.W, prep.perm, s, wl.tau, fixed, n_sym, order=order if use_order else None)
    torch.cuda.synchronize()
    l_p, c_p, k_p = (t.cpu().numpy() for t in (lr.l, lr.cost, lr.kidx))
    l_f, c_f, k_f = (t.cpu().numpy() for t in (fx.l, fx.cost, fx.kidx))
    l_o, c_o, k_o = (t.cpu().numpy() for t in (out.l, out.cost, out.kidx))
    flagged = ~(mass_np >= theta)
    take = flagged & (c_f < c_p)
    want_c = np.where(take, c_f, c_p)
    want_k = np.where(take, base + k_f, k_p)
    want_l = np.where(take[None, :, None], l_f, l_p)
    assert np.array_equal(c_o.view(np.uint32), want_c.view(np.uint32))
    assert np.array_equal(k_o, want_k)
    assert np.array_equal(l_o, want_l)
    assert take.sum() > 0
    print(f"flagged {int(flagged.sum())} of {n_vec}, fixed set better for {int(take.sum())}", flush=True)
    # oracle: the flagged vectors of two subcarriers, searched over the fixed table in FP64
    W = prep.W.cpu().numpy()
    perm = prep.perm.cpu().numpy()
    tables = fixed.cpu().numpy()
    l_user = l_from_gpu(l_o)   # [n_vec][N] user order
    for sc in (0, wl.n_sc - 1):
        sl = slice(sc * n_sym, (sc + 1) * n_sym)
        ref = O.search_paths(unpack_W(W[sc], N), perm[sc], wl.s[:, sl], wl.tau, tables[sc])
        for j in range(n_sym):
            v = sc * n_sym + j
            if not take[v]:
                continue
            assert abs(c_o[v] - ref.cost[j]) <= 1e-5 * ref.cost[j], (v, c_o[v], ref.cost[j])
            got = np.linalg.norm(unpack_W(W[sc], N) @ (wl.s[perm[sc], v] + wl.tau * l_user[v][perm[sc]])) ** 2
            assert abs(got - c_o[v]) <= 1e-5 * got, (v, got, c_o[v])


def test_fallback_theta_nothing_flagged(lib):
    """theta = -inf flags only the vectors with a NaN mass; the others keep
    every byte of the proposal's result."""
    vp, learn = lib
    wl = vpgen.make("16x16-rzf-256qam-rho0.5", 16, 16, 4, 14, 256, 0.16, 64, seed=43, rho=0.5)
    H = torch.from_numpy(wl.H).to(DEV)
    s = torch.from_numpy(wl.s).to(DEV)
    prep = vp.preprocess(H, wl.alpha)
    order = torch.empty((wl.n_sc, 2, 64), dtype=torch.int16, device=DEV)
    fixed = vp.paths_mop(prep.w2, 64, order=order)
    prop = torch.from_numpy(_proposal_tables(np.random.default_rng(1), wl.n_vec, 8, wl.N)).to(DEV)
    lr = vp.search(prep.W, prep.perm, s, wl.tau, prop, wl.n_sym, flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
    mass = torch.full((wl.n_vec,), 0.25, dtype=torch.float32, device=DEV)
    mass[3] = float("nan")
    out = vp.SearchOut(lr.l.clone(), lr.cost.clone(), lr.kidx.clone())
    learn.search_fallback(prep.W, prep.perm, s, wl.tau, fixed, wl.n_sym, mass, float("-inf"), out, 9, order=order)
    fx = vp.search(prep.W, prep.perm, s, wl.tau, fixed, wl.n_sym, order=order)
    keep = np.ones(wl.n_vec, bool)
    keep[3] = False
    for a, b in ((out.l, lr.l), (out.cost, lr.cost), (out.kidx, lr.kidx)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        if a.ndim == 3:
            assert np.array_equal(a[:, keep], b[:, keep])
        else:
            assert np.array_equal(a[keep], b[keep])
    c3, cp3, cf3 = float(out.cost[3]), float(lr.cost[3]), float(fx.cost[3])
    assert c3 == (cf3 if cf3 < cp3 else cp3)


def test_fallback_at_the_benchmark_launch(lib):
    """The benchmark's launch: 3276 subcarriers x 14 symbols, the committed
    proposer's tables and masses, theta = 0.3 over the K = 512 MoP set with its
    orders.  Every vector is checked against the plain search restricted to
    the flagged ones (bit-exact)."""
    import os
    vp, learn = lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(root, "paper_2602_12098_amd", "weights", "proposer_16x16_256qam_res64.safetensors")
    if not os.path.exists(path):
        pytest.skip("no committed proposer")
    prop = learn.load_proposer(path)
    wl = vpgen.cfg3(512)
    print("fallback at the benchmark launch", flush=True)
    H = torch.from_numpy(wl.H).to(DEV)
    s = torch.from_numpy(wl.s).to(DEV)
    prep = vp.preprocess(H, wl.alpha)
    order = torch.empty((wl.n_sc, 2, 512), dtype=torch.int16, device=DEV)
    fixed = vp.paths_mop(prep.w2, 512, order=order)
    table, mass = prop.propose(prep.W, prep.perm, s, wl.tau, wl.n_sym, fixed_paths=fixed, K_fixed=64)
    lr = vp.search(prep.W, prep.perm, s, wl.tau, table, wl.n_sym,
                   flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
    out = vp.SearchOut(lr.l.clone(), lr.cost.clone(), lr.kidx.clone())
    base = table.shape[1] + 1
    learn.search_fallback(prep.W, prep.perm, s, wl.tau, fixed, wl.n_sym, mass, 0.3, out, base, order=order)
    fx = vp.search(prep.W, prep.perm, s, wl.tau, fixed, wl.n_sym, order=order)
    flagged = ~(mass >= 0.3)
    take = flagged & (fx.cost < lr.cost)
    assert torch.equal(out.cost, torch.where(take, fx.cost, lr.cost))
    assert torch.equal(out.kidx, torch.where(take, fx.kidx + base, lr.kidx))
    assert torch.equal(out.l, torch.where(take[None, :, None], fx.l, lr.l))
    frac = float(flagged.float().mean())
    print(f"flagged {frac:.3f}, fixed set better for {int(take.sum())} vectors", flush=True)
    assert 0.05 < frac < 0.95 and int(take.sum()) > 0
