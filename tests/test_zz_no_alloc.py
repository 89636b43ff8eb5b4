"""GPU test of vp_search_fallback_noalloc, the allocation-free variant of
vp_search_fallback (its workspace is the library's static per-GPU array).

Called through the C ABI, it must give, bit for bit, what vp_search_fallback
gives with a caller-owned workspace on the same inputs -- on two calls in a
row, the second with a smaller input, so that the workspace left behind by
the first call cannot leak into the second.  Both calls share the kernels, so
the comparison is exact; vp_search_fallback itself is held to the FP64
oracle by tests/test_gpu_fallback.py."""
import ctypes

import numpy as np
import pytest

import vpgen

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


def _case(vp, n_sc, n_sym, K_fix, seed):
    wl = vpgen.make("16x16-rzf-256qam-rho0.5", 16, 16, n_sc, n_sym, 256, 0.16, K_fix, seed=seed, rho=0.5)
    rng = np.random.default_rng(seed)
    H = torch.from_numpy(wl.H).to(DEV)
    s = torch.from_numpy(wl.s).to(DEV)
    tau = vp.tau_array(wl.tau, wl.n_sc, DEV)
    prep = vp.preprocess(H, wl.alpha)
    order = torch.empty((wl.n_sc, 2, K_fix), dtype=torch.int16, device=DEV)
    fixed = vp.paths_mop(prep.w2, K_fix, order=order)
    prop = rng.integers(0, 3, size=(wl.n_vec, 24, wl.N)).astype(np.uint8)
    prop[:, 0, :] = 0
    lr = vp.search(prep.W, prep.perm, s, tau, torch.from_numpy(prop).to(DEV), n_sym,
                   flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
    mass_np = rng.random(wl.n_vec).astype(np.float32)
    mass_np[::5] = np.nan
    mass = torch.from_numpy(mass_np).to(DEV)
    return wl, prep, s, tau, fixed, order, lr, mass


@pytest.mark.parametrize("first,second", [((120, 14), (37, 9)), ((3276, 14), (5, 3))])
def test_noalloc_equals_workspace_variant_twice(lib, first, second):
    vp, learn = lib
    for (n_sc, n_sym), seed in ((first, 61), (second, 62)):
        print(f"no-alloc fallback n_sc={n_sc} n_sym={n_sym} seed={seed}", flush=True)
        wl, prep, s, tau, fixed, order, lr, mass = _case(vp, n_sc, n_sym, 512, seed)
        a = vp.SearchOut(lr.l.clone(), lr.cost.clone(), lr.kidx.clone())
        b = vp.SearchOut(lr.l.clone(), lr.cost.clone(), lr.kidx.clone())
        learn.search_fallback(prep.W, prep.perm, s, tau, fixed, n_sym, mass, 0.5, a, 25, order=order)
        learn.search_fallback_noalloc(prep.W, prep.perm, s, tau, fixed, n_sym, mass, 0.5, b, 25, order=order)
        torch.cuda.synchronize()
        assert torch.equal(a.cost.view(torch.int32), b.cost.view(torch.int32))
        assert torch.equal(a.kidx, b.kidx) and torch.equal(a.l, b.l)
        changed = int((a.kidx != lr.kidx).sum())
        print(f"  fixed set took over {changed} of {wl.n_vec} vectors", flush=True)
        assert changed > 0


def test_noalloc_rejects_more_vectors_than_its_workspace(lib):
    vp, learn = lib
    from paper_2602_12098_amd import _lib
    lib_ = _lib.load()
    P = ctypes.c_void_p(16)   # never dereferenced: the size check fails first
    n_sym = 14
    n_sc = _lib.VP_NOALLOC_MAX_VECTORS // n_sym + 1
    rc = lib_.vp_search_fallback_noalloc(P, P, P, P, P, None, 512, 512 * 16, n_sc, n_sym, 16, 1, P, 0.5, 0,
                                         P, P, P, None)
    assert rc == _lib.VP_EUNSUPPORTED
