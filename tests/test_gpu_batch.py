"""GPU tests of the batched uneven workload (include/vp_batch.h).

The plan runs preprocessing, MoP paths, search and precoding for groups of
different user counts, QAM orders and path counts in one captured graph.
Checked: its search results against the FP64 oracle on the plan's own
factors and path tables (same-input parity, sampled subcarriers of every
group); its every intermediate and output against the per-call entry points
on each group alone (bit-identical: the same float32 arithmetic); results
independent of the autotuned tile shapes; repeated graph replays with eager
work in between; failed subcarriers; argument errors."""
import math

import numpy as np
import pytest

import vpgen
from oracle import vp_oracle as O
from tests.vp_parity import ParityReport, check_search_subcarrier, l_from_gpu, unpack_W, record

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
K_BY_U = {4: 16, 5: 32, 6: 32, 7: 64, 8: 64, 9: 64, 10: 128, 11: 128, 12: 128, 13: 256, 14: 256, 15: 256, 16: 256}


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_12098_amd as vp
    from paper_2602_12098_amd import batch
    return vp, batch


def _say(*a):
    print(*a, flush=True)


def host(t):
    return t.detach().cpu().numpy()


def make_batch(batch_mod, wl, P_T=1.0, kmap=K_BY_U):
    groups = [batch_mod.GroupSpec(int(u), wl.sc_per_rbg, kmap[int(u)], float(vpgen.qam_tau(int(q))), float(a))
              for u, q, a in zip(wl.U, wl.Q, wl.alpha)]
    b = batch_mod.Batch(groups, wl.M, wl.n_sym, P_T=P_T)
    b.set_inputs(wl.H, wl.s)
    return b


def per_call(vp, wl, gi, K, P_T):
    H = torch.from_numpy(wl.H[gi]).to(DEV)
    s = torch.from_numpy(wl.s[gi]).to(DEV)
    tau = float(vpgen.qam_tau(int(wl.Q[gi])))
    prep = vp.preprocess(H, float(wl.alpha[gi]))
    paths = vp.paths_mop(prep.w2, K)
    out = vp.search(prep.W, prep.perm, s, tau, paths, wl.n_sym)
    x = vp.precode(prep.G, s, out.l, tau, out.cost, wl.n_sym, P_T=P_T)
    return prep, paths, out, x


def eq_nan(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if np.iscomplexobj(a):
        return eq_nan(a.real, b.real) and eq_nan(a.imag, b.imag)
    return np.array_equal(a, b) or bool(np.all((a == b) | (np.isnan(a) & np.isnan(b))))


def check_against_per_call(vp, b, wl, P_T):
    bufs = b.buffers()
    for gi in range(wl.n_rbg):
        K = b.groups[gi].K
        prep, paths, out, x = per_call(vp, wl, gi, K, P_T)
        gb = b.group_buffers(gi, bufs)
        l, cost, xb = b.group_outputs(gi)
        assert eq_nan(host(gb["W"]), host(prep.W)), gi
        assert np.array_equal(host(gb["perm"]), host(prep.perm)), gi
        assert eq_nan(host(gb["w2"]), host(prep.w2)), gi
        assert eq_nan(host(gb["G"]), host(prep.G)), gi
        assert np.array_equal(host(gb["status"]), host(prep.status)), gi
        assert np.array_equal(host(gb["paths"]), host(paths)), gi
        assert np.array_equal(host(l), host(out.l)), gi
        assert eq_nan(host(cost), host(out.cost)), gi
        assert eq_nan(host(xb), host(x)), gi
    return bufs


def test_batch_matches_oracle_and_per_call(mods):
    vp, bm = mods
    wl = vpgen.cfg4(n_rbg=39, seed=11, users=np.arange(4, 17))   # every user count at least once
    _say("batch groups", wl.n_rbg, "users", wl.U.tolist())
    b = make_batch(bm, wl)
    b.run()
    torch.cuda.synchronize()
    bufs = check_against_per_call(vp, b, wl, 1.0)
    # same-input parity against the oracle: two subcarriers of every group
    rep = ParityReport()
    for gi in range(wl.n_rbg):
        U, K = int(wl.U[gi]), b.groups[gi].K
        gb = b.group_buffers(gi, bufs)
        Wd = unpack_W(host(gb["W"]), U)
        perm = host(gb["perm"]).astype(np.int64)
        P = host(gb["paths"])
        l, cost, _ = b.group_outputs(gi)
        lg = l_from_gpu(host(l))
        cg = host(cost)
        # the per-call search gives the winning indices (identical results, checked above)
        H = torch.from_numpy(wl.H[gi]).to(DEV)
        prep = vp.preprocess(H, float(wl.alpha[gi]))
        kidx = host(vp.search(prep.W, prep.perm, torch.from_numpy(wl.s[gi]).to(DEV), b.groups[gi].tau,
                              vp.paths_mop(prep.w2, K), wl.n_sym).kidx)
        for sc in (0, wl.sc_per_rbg - 1):
            sl = slice(sc * wl.n_sym, (sc + 1) * wl.n_sym)
            check_search_subcarrier(rep, Wd[sc], perm[sc], wl.s[gi][:, sl].astype(np.complex128), b.groups[gi].tau,
                                    P[sc], True, lg[sl], cg[sl], kidx[sl])
    _say(rep)
    record("batched-groups", rep)
    assert rep.ok(), rep.failures[:4]
    assert rep.exact >= 0.98 * rep.n
    info = b.info()
    _say(info)
    assert info["n_vec"] == wl.n_rbg * wl.sc_per_rbg * wl.n_sym
    b.close()


def test_batch_tuning_keeps_results(mods):
    vp, bm = mods
    wl = vpgen.cfg4(n_rbg=64, seed=5)
    b = make_batch(bm, wl, P_T=0.0)
    b.run()
    torch.cuda.synchronize()
    ref = [tuple(host(t).copy() for t in b.group_outputs(gi)) for gi in range(wl.n_rbg)]
    info = b.tune(reps=2)
    _say(info)
    assert info["tuned_ms"] > 0 and info["default_ms"] > 0 and info["tuned_ms"] <= info["default_ms"] * 1.0001
    for rep_i in range(3):   # graph replays with eager work between them
        junk = torch.randn(1000, device=DEV).sum()
        b.H.mul_(1.0)
        b.run()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for gi in range(wl.n_rbg):
            got = [host(t) for t in b.group_outputs(gi)]
            for a, r in zip(got, ref[gi]):
                assert eq_nan(a, r), (rep_i, gi)
    check_against_per_call(vp, b, wl, 0.0)
    b.close()


def test_batch_failed_subcarrier(mods):
    vp, bm = mods
    wl = vpgen.cfg4(n_rbg=4, seed=2)
    wl.H[1][3, 0, 0] = np.nan
    b = make_batch(bm, wl)
    b.run()
    torch.cuda.synchronize()
    l, cost, x = b.group_outputs(1)
    c = host(cost)
    bad = slice(3 * wl.n_sym, 4 * wl.n_sym)
    assert np.all(np.isnan(c[bad])) and np.all(np.isfinite(np.delete(c, np.arange(3 * wl.n_sym, 4 * wl.n_sym))))
    assert not np.any(host(l)[:, bad])
    check_against_per_call(vp, b, wl, 1.0)
    b.close()


def test_batch_rejects_bad_groups(mods):
    _, bm = mods
    from paper_2602_12098_amd._lib import VPError
    G = bm.GroupSpec
    with pytest.raises(VPError):
        bm.Batch([G(4, 12, 0, 8.0, 0.04)], 16, 14)              # K < 1
    with pytest.raises(VPError):
        bm.Batch([G(2, 12, 82, 8.0, 0.04)], 16, 14)             # K > 9^N
    with pytest.raises(VPError):
        bm.Batch([G(17, 12, 8, 8.0, 0.04)], 16, 14)             # N > 16
    with pytest.raises(VPError):
        bm.Batch([G(4, 12, 1024, 8.0, 0.04)], 16, 14)           # K > 512
    with pytest.raises(VPError):
        bm.Batch([G(8, 12, 8, 8.0, 0.0)], 4, 14)                # alpha = 0 with N > n_t
    with pytest.raises(VPError):
        bm.Batch([G(4, 12, 8, -1.0, 0.04)], 16, 14)             # tau <= 0
    with pytest.raises(VPError):
        bm.Batch([G(4, 5000, 8, 8.0, 0.04)], 16, 14)            # n_sc * n_sym > 65535
    with pytest.raises(VPError):
        bm.Batch([G(4, 1, k, 8.0, 0.04) for k in range(1, 10)], 16, 14)   # 9 distinct K


def test_batch_kbest_fallback(mods):
    # orthogonal users of equal gain give equal MoP weights: the threshold
    # pass overflows its frontier and the K-best kernel redoes those tables
    vp, bm = mods
    wl = vpgen.cfg4(n_rbg=5, seed=21, users=[16, 9, 16, 5, 13])
    for gi in (0, 2):
        U = int(wl.U[gi])
        H = np.zeros((wl.sc_per_rbg, U, wl.M), np.complex64)
        for sc in range(wl.sc_per_rbg):
            H[sc, :, :U] = np.eye(U, dtype=np.complex64) * (1.0 + 0.25 * sc)
        wl.H[gi] = H
    b = make_batch(bm, wl)
    b.run()
    torch.cuda.synchronize()
    bufs = check_against_per_call(vp, b, wl, 1.0)
    # the redone tables are the exact K smallest (MoP, lexicographic) of the oracle
    for gi in (0, 2):
        gb = b.group_buffers(gi, bufs)
        w2 = host(gb["w2"])
        P = host(gb["paths"])
        assert np.all(w2 == w2[:, :1])   # equal weights within each subcarrier
        for sc in (0, wl.sc_per_rbg - 1):
            ref = O.mop_paths_kbest(w2[sc].astype(np.float64), b.groups[gi].K)
            assert np.array_equal(P[sc].astype(np.int64), ref), (gi, sc)
    b.close()
