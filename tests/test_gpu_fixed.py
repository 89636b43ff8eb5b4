"""GPU parity of the 16-bit fixed-point walk (vp_fx_quantize, vp_fx_search)
against the oracle's fixed-point section, through the C ABI.

The search is integer arithmetic after quantisation, so it is checked
bit-exactly (chosen l, PED, path index) on the GPU's own quantised inputs.
The quantiser rounds float32 values, the oracle float64 ones: they may differ
by one unit in the last place where the value sits next to a rounding
boundary, and nowhere by more."""
import numpy as np
import pytest

import vpgen
from oracle import vp_oracle as O
from tests.vp_parity import l_from_gpu, unpack_W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def vp():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_12098_amd as vp
    return vp


def _to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def _workload(name, K, n_sc):
    if name == "cfg1":
        return vpgen.cfg1(n_sc=n_sc)
    if name == "cfg2":
        return vpgen.cfg2(20, n_sc=n_sc)
    if name == "cfg3":
        return vpgen.cfg3(K, n_sc=n_sc)
    N, M = {"n5": (5, 5), "n1": (1, 2), "n12": (12, 12)}[name]
    return vpgen.make(f"ragged-{N}x{M}", N, M, n_sc, 7, 64, 0.05, K, seed=40 + N)


def _V_dense(Vp, N):
    """Packed strictly-lower [N(N-1)/2][2] -> [N][N][2] (m > i)."""
    out = np.zeros((N, N, 2), dtype=np.int64)
    for m in range(1, N):
        for i in range(m):
            out[m, i] = Vp[m * (m - 1) // 2 + i]
    return out


@pytest.mark.parametrize("frac_bits,tau_scale", [(8, 1), (10, 1), (13, 1), (13, 1 / 16)])
def test_fx_quantize_matches_oracle(vp, frac_bits, tau_scale):
    wl = vpgen.cfg3(512, n_sc=24)
    N = wl.N
    tau = wl.tau * tau_scale
    prep = vp.preprocess(_to_dev(wl.H), wl.alpha)
    q = vp.fx_quantize(prep.W, prep.perm, _to_dev(wl.s), tau, wl.n_sym, frac_bits)
    torch.cuda.synchronize()
    Wd = unpack_W(host(prep.W), N)
    perm = host(prep.perm).astype(np.int64)
    c0, Vp, w = host(q.c0).astype(np.int64), host(q.V).astype(np.int64), host(q.w).astype(np.int64)
    n_el = n_off = 0
    for sc in range(wl.n_sc):
        sl = slice(sc * wl.n_sym, (sc + 1) * wl.n_sym)
        rc0, rV, rw = O.fx_inputs(Wd[sc], perm[sc], wl.s[:, sl].astype(np.complex128), tau, frac_bits)
        gV = _V_dense(Vp[sc], N)
        for g, r in ((c0[sl], rc0), (gV, rV), (w[sc], rw)):
            d = np.abs(g - r)
            assert d.max() <= 1, (sc, d.max())
            n_el += d.size
            n_off += int((d == 1).sum())
    # float32 against float64 rounding: a flip needs the value within the
    # float32 error of the inputs' dot products (a few 1e-7 relative) of a
    # half-integer, i.e. well under 1 % of the elements at 13 fractional bits
    print(f"fx_quantize F={frac_bits}: {n_off} of {n_el} elements one unit off", flush=True)
    assert n_off <= 0.01 * n_el


@pytest.mark.parametrize("name,K,n_sc,frac_bits,include_zero,shared,sample,tau_scale", [
    ("cfg3", 512, 4, 13, True, False, 12, 1),
    ("cfg3", 512, 4, 10, True, False, 12, 1),
    ("cfg2", 64, 4, 8, True, False, None, 1),
    ("cfg2", 64, 4, 12, False, False, None, 1),
    ("cfg1", 32, 8, 11, True, True, None, 1),
    ("n5", 300, 3, 9, True, False, None, 1),
    ("n1", 9, 5, 13, True, True, None, 1),
    ("n12", 257, 2, 11, False, True, 8, 1),
    # an interval 16 times too small: centres up to about 8 leave the 16-bit
    # range at 13 and 12 fractional bits, so the walk saturates
    ("cfg2", 64, 3, 13, True, False, None, 1 / 16),
    ("cfg3", 300, 2, 12, True, False, 10, 1 / 16),
])
def test_fx_search_bit_exact(vp, name, K, n_sc, frac_bits, include_zero, shared, sample, tau_scale):
    wl = _workload(name, K, n_sc)
    N, n_sym = wl.N, wl.n_sym
    tau = wl.tau * tau_scale
    print("fx search", wl.name, "K", K, "F", frac_bits, "zero", include_zero, "shared", shared, "tau", tau,
          flush=True)
    prep = vp.preprocess(_to_dev(wl.H), wl.alpha)
    paths = vp.paths_mop(prep.w2, K)
    if shared:
        paths = paths[0].contiguous()
    q = vp.fx_quantize(prep.W, prep.perm, _to_dev(wl.s), tau, n_sym, frac_bits)
    out = vp.fx_search(q, prep.perm, paths, n_sym, flags=vp.VP_INCLUDE_ZERO if include_zero else 0)
    torch.cuda.synchronize()
    perm = host(prep.perm).astype(np.int64)
    P = host(paths)
    c0, Vp, w = host(q.c0).astype(np.int64), host(q.V).astype(np.int64), host(q.w).astype(np.int64)
    l = l_from_gpu(host(out.l))
    ped, kidx = host(out.ped), host(out.kidx)
    rng = np.random.default_rng(7)
    n_sat = 0
    checked = 0
    for sc in range(wl.n_sc):
        vs = np.arange(sc * n_sym, (sc + 1) * n_sym)
        if sample is not None:
            vs = np.sort(rng.choice(vs, size=min(sample // wl.n_sc + 1, n_sym), replace=False))
        Psc = P if shared else P[sc]
        rl, rped, rk = O.fx_search(c0[vs], _V_dense(Vp[sc], N), w[sc], Psc, frac_bits, include_zero)
        n_sat += int(((c0[vs] >= 32767) | (c0[vs] <= -32768)).sum())
        for j, v in enumerate(vs):
            lu = np.zeros(N, dtype=np.complex128)
            lu[perm[sc]] = rl[j]
            assert int(kidx[v]) == int(rk[j]), (sc, v, kidx[v], rk[j])
            assert int(ped[v]) == int(rped[j]), (sc, v, ped[v], rped[j])
            assert np.array_equal(l[v], lu), (sc, v)
            checked += 1
    print(f"  {checked} vectors bit-exact ({n_sat} saturated start centres)", flush=True)
    if tau_scale < 1:
        assert n_sat > 0


def test_fx_search_errors(vp):
    wl = vpgen.cfg1(n_sc=2)
    prep = vp.preprocess(_to_dev(wl.H), wl.alpha)
    from paper_2602_12098_amd._lib import VP_EINVAL, VPError
    with pytest.raises(VPError) as e:
        vp.fx_quantize(prep.W, prep.perm, _to_dev(wl.s), wl.tau, wl.n_sym, 14)
    q = vp.fx_quantize(prep.W, prep.perm, _to_dev(wl.s), wl.tau, wl.n_sym, 12)
    assert e.value.code == VP_EINVAL
    paths = vp.paths_mop(prep.w2, 16)
    for bad in (dict(q=q._replace(frac_bits=7)), dict(flags=vp.VP_DEMAP_REGION)):
        with pytest.raises(VPError) as e:
            vp.fx_search(bad.get("q", q), prep.perm, paths, wl.n_sym, flags=bad.get("flags", vp.VP_INCLUDE_ZERO))
        assert e.value.code == VP_EINVAL
