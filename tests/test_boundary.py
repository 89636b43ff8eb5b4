"""CPU-side checks of the C ABI boundary and of the host build of the DEMAP code.

No compute call reaches the GPU here: argument validation returns before any
HIP call, and the DEMAP routines are exercised through their host build."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from oracle import vp_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]
PKG = os.path.join(ROOT, "paper_2602_12098_amd")


@pytest.fixture(scope="module")
def lib():
    from paper_2602_12098_amd import _lib
    return _lib.load()


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(vp_[a-z0-9_]+)\(", text, flags=re.M)))


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert {"vp_preprocess", "vp_paths_mop", "vp_search", "vp_precode", "vp_strerror", "vp_sphere_encode",
            "vp_mlp_features", "vp_path_ranks", "vp_gemm_bf16", "vp_topk64", "vp_softmax_xent", "vp_colsum_bf16",
            "vp_learned_paths", "vp_search_fallback", "vp_fx_quantize", "vp_fx_search"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(PKG, "libvp.so")],
                         capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_argument_validation(lib):
    from paper_2602_12098_amd._lib import VP_EINVAL, VP_EUNSUPPORTED, VP_OK
    F = 0
    # vp_preprocess
    assert lib.vp_preprocess(None, 1, 4, 4, 0.1, None, None, None, None, None, None) == VP_EINVAL
    assert lib.vp_preprocess(None, 1, 17, 17, 0.1, None, None, None, None, None, None) == VP_EUNSUPPORTED
    assert lib.vp_preprocess(None, 1, 4, 65, 0.1, None, None, None, None, None, None) == VP_EUNSUPPORTED
    assert lib.vp_preprocess(None, 1, 6, 4, 0.0, None, None, None, None, None, None) == VP_EINVAL
    assert lib.vp_preprocess(None, 1, 4, 4, -1.0, None, None, None, None, None, None) == VP_EINVAL
    assert lib.vp_preprocess(None, 1, 4, 4, float("nan"), None, None, None, None, None, None) == VP_EINVAL
    assert lib.vp_preprocess(None, 0, 4, 4, 0.1, None, None, None, None, None, None) == VP_OK
    assert lib.vp_preprocess(None, -1, 4, 4, 0.1, None, None, None, None, None, None) == VP_EINVAL
    # vp_paths_mop
    assert lib.vp_paths_mop(None, 1, 2, 82, None, None, None) == VP_EINVAL          # K > 9^2
    assert lib.vp_paths_mop(None, 1, 16, 1025, None, None, None) == VP_EUNSUPPORTED
    assert lib.vp_paths_mop(None, 1, 16, 0, None, None, None) == VP_EINVAL
    assert lib.vp_paths_mop(None, 0, 4, 32, None, None, None) == VP_OK
    assert lib.vp_paths_mop(None, 3, 4, 32, None, None, None) == VP_EINVAL          # null pointers
    # vp_search (tau is a per-subcarrier device array: a NULL tau is an
    # argument error, its values are data, checked per subcarrier on the GPU)
    P = ctypes.c_void_p(16)   # non-NULL, never dereferenced (every call below fails its checks or has n_sc = 0)
    args = dict(tau=P, K=32, stride=0, n_sc=1, n_sym=14, N=4, flags=1)

    def search(Q=None, **kw):
        a = dict(args, **kw)
        return lib.vp_search(Q, Q, Q, a["tau"], Q, a.get("lex"), a["K"], a["stride"], a["n_sc"],
                             a["n_sym"], a["N"], a["flags"], Q, Q, Q, None)
    assert search() == VP_EINVAL
    assert search(n_sc=0) == VP_OK
    assert search(P, tau=None) == VP_EINVAL
    assert search(N=17, n_sc=0) == VP_EUNSUPPORTED
    assert search(K=4097, n_sc=0) == VP_EUNSUPPORTED
    assert search(stride=5, n_sc=0) == VP_EINVAL      # 0 < stride < K*N
    assert search(stride=-1, n_sc=0) == VP_EINVAL
    assert search(flags=2, n_sc=0) == VP_EINVAL
    assert search(n_sym=0, n_sc=0) == VP_EINVAL
    assert search(lex=1, stride=0, n_sc=0) == VP_EINVAL       # lexorder needs a per-subcarrier table
    # vp_search_fallback: the checks of vp_search, plus mass, theta, kidx_base and work
    fargs = dict(tau=P, K=32, stride=0, n_sc=1, n_sym=14, N=4, flags=1, theta=0.5, base=72)

    def fallback(P=None, **kw):
        a = dict(fargs, **kw)
        return lib.vp_search_fallback(P, P, P, a["tau"], P, a.get("lex"), a["K"], a["stride"], a["n_sc"],
                                      a["n_sym"], a["N"], a["flags"], a.get("mass", P), a["theta"], a["base"],
                                      P, P, P, a.get("work", P), None)
    assert fallback() == VP_EINVAL
    assert fallback(n_sc=0) == VP_OK
    assert fallback(P, mass=None) == VP_EINVAL
    assert fallback(P, work=None) == VP_EINVAL
    assert fallback(P, work=ctypes.c_void_p(18)) == VP_EINVAL             # work not 4-byte aligned
    assert fallback(P, theta=float("nan")) == VP_EINVAL
    assert fallback(P, base=-1) == VP_EINVAL
    assert fallback(P, flags=2) == VP_EINVAL                               # VP_PATHS_PER_VECTOR
    assert fallback(P, tau=None) == VP_EINVAL
    assert fallback(P, N=17) == VP_EUNSUPPORTED
    assert fallback(P, K=4097) == VP_EUNSUPPORTED
    assert fallback(P, stride=5) == VP_EINVAL
    assert fallback(P, lex=P, stride=0) == VP_EINVAL
    assert fallback(theta=float("inf"), n_sc=0) == VP_OK
    # vp_precode
    assert lib.vp_precode(None, None, None, P, None, 0, 14, 4, 4, 0.0, None, None) == VP_OK
    assert lib.vp_precode(None, None, None, P, None, 1, 14, 4, 4, 1.0, None, None) == VP_EINVAL
    assert lib.vp_precode(P, P, P, None, P, 1, 14, 4, 4, 1.0, P, None) == VP_EINVAL       # NULL tau
    assert lib.vp_precode(None, None, None, P, None, 1, 14, 4, 4, -1.0, None, None) == VP_EINVAL
    assert lib.vp_precode(None, None, None, P, None, 1, 14, 17, 4, 0.0, None, None) == VP_EUNSUPPORTED
    # vp_fx_quantize / vp_fx_search: frac_bits in 8..13, the vp_search checks
    assert lib.vp_fx_quantize(None, None, None, P, 0, 14, 4, 12, None, None, None, None) == VP_OK
    assert lib.vp_fx_quantize(P, P, P, P, 1, 14, 4, 14, P, P, P, None) == VP_EINVAL
    assert lib.vp_fx_quantize(P, P, P, P, 1, 14, 4, 7, P, P, P, None) == VP_EINVAL
    assert lib.vp_fx_quantize(P, P, P, None, 1, 14, 4, 12, P, P, P, None) == VP_EINVAL      # NULL tau
    assert lib.vp_fx_quantize(P, P, P, P, 1, 14, 4, 12, P, None, P, None) == VP_EINVAL      # NULL V, N > 1
    assert lib.vp_fx_quantize(P, P, P, P, 1, 14, 17, 12, P, P, P, None) == VP_EUNSUPPORTED

    def fx(Q=P, **kw):
        a = dict(dict(K=32, stride=0, n_sc=1, n_sym=14, N=4, F=12, flags=1), **kw)
        return lib.vp_fx_search(Q, Q, Q, Q, Q, a["K"], a["stride"], a["n_sc"], a["n_sym"], a["N"], a["F"],
                                a["flags"], Q, Q, Q, None)
    assert fx(None) == VP_EINVAL
    assert fx(None, n_sc=0) == VP_OK
    assert fx(F=14) == VP_EINVAL
    assert fx(flags=4) == VP_EINVAL                 # no region DEMAP in fixed point
    assert fx(flags=2) == VP_EINVAL                 # no per-vector paths
    assert fx(stride=5) == VP_EINVAL
    assert fx(K=0) == VP_EINVAL
    assert fx(K=4097) == VP_EUNSUPPORTED
    assert fx(N=17) == VP_EUNSUPPORTED
    assert lib.vp_strerror(VP_EINVAL) == b"invalid argument"
    assert lib.vp_last_hip_error() == 0
    _ = F


def _host_demap():
    path = os.path.join(PKG, "libvphost.so")
    h = ctypes.CDLL(path)
    h.vp_host_demap.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int] * 2 + [ctypes.c_void_p] * 2
    h.vp_host_demap.restype = ctypes.c_int

    def run(cx, cy, r, tier):
        n = len(cx)
        a = np.zeros(n, np.float32)
        b = np.zeros(n, np.float32)
        cx = np.ascontiguousarray(cx, np.float32)
        cy = np.ascontiguousarray(cy, np.float32)
        r = np.ascontiguousarray(r, np.int32)
        assert h.vp_host_demap(cx.ctypes.data, cy.ctypes.data, r.ctypes.data, n, tier,
                               a.ctypes.data, b.ctypes.data) == 0
        return a, b
    return run


def test_demap_exact_ties_follow_canonical_order():
    """Centres on a grid of eighths give exact distance ties (also at
    half-integers, where two offsets of one axis are equally far): every rank
    of every tier must follow the (distance, j) order exactly."""
    run = _host_demap()
    g = np.arange(-20, 21) / 8.0
    gx, gy = np.meshgrid(g, g)
    cx, cy = gx.ravel().astype(np.float32), gy.ravel().astype(np.float32)
    c = cx.astype(np.float64) + 1j * cy.astype(np.float64)
    order = np.argsort(O.sqabs(c[:, None] - O.BOX[None, :]), axis=1, kind="stable")
    for r in range(9):
        ref = O.BOX[order[:, r]]
        for tier in (0, 1, 2, 3):
            if r > tier and tier < 3:
                continue
            a, b = run(cx, cy, np.full(len(cx), r), tier)
            bad = np.nonzero((a != ref.real) | (b != ref.imag))[0]
            assert bad.size == 0, (r, tier, [(cx[i], cy[i]) for i in bad[:4]])


def test_demap_matches_oracle_order():
    """The GPU's DEMAP (host build) picks the same box point as the oracle's
    (distance, j) order for every rank, except where two distances are within
    1e-5 (float32 cannot order them); its three variants agree exactly."""
    run = _host_demap()
    rng = np.random.default_rng(0)
    cx = rng.uniform(-4, 4, 60000).astype(np.float32)
    cy = rng.uniform(-4, 4, 60000).astype(np.float32)
    q = (np.arange(-15, 16, 2) / 32.0).astype(np.float32)      # 256-QAM level-0 centres, exact ties
    gx, gy = np.meshgrid(q, q)
    cx = np.concatenate([cx, gx.ravel(), cx[:5000]])
    cy = np.concatenate([cy, gy.ravel(), -cx[:5000]])
    c = cx.astype(np.float64) + 1j * cy.astype(np.float64)
    d = O.sqabs(c[:, None] - O.BOX[None, :])
    order = np.argsort(d, axis=1, kind="stable")
    ds = np.take_along_axis(d, order, 1)
    for r in range(9):
        a, b = run(cx, cy, np.full(len(cx), r), 3)
        ref = O.BOX[order[:, r]]
        mism = (a != ref.real) | (b != ref.imag)
        lo = ds[:, r] - ds[:, max(r - 1, 0)] if r > 0 else np.full(len(cx), np.inf)
        hi = ds[:, min(r + 1, 8)] - ds[:, r] if r < 8 else np.full(len(cx), np.inf)
        assert not np.any(mism & (np.minimum(lo, hi) > 1e-5)), r
        if r <= 2:
            a2, b2 = run(cx, cy, np.full(len(cx), r), 2)
            assert np.array_equal(a2, a) and np.array_equal(b2, b)
        if r <= 1:
            a1, b1 = run(cx, cy, np.full(len(cx), r), 1)
            assert np.array_equal(a1, a) and np.array_equal(b1, b)
        if r == 0:
            a0, b0 = run(cx, cy, np.full(len(cx), r), 0)
            assert np.array_equal(a0, a) and np.array_equal(b0, b)
    # the exact diagonal ties of QAM centres are resolved by the canonical index
    for tier in (1, 2, 3):
        a, b = run(np.array([-3 / 32.0]), np.array([-3 / 32.0]), np.array([1]), tier)
        assert (a[0], b[0]) == (-1.0, 0.0)
    for tier in (2, 3):
        a, b = run(np.array([-3 / 32.0]), np.array([-3 / 32.0]), np.array([2]), tier)
        assert (a[0], b[0]) == (0.0, -1.0)


def test_demap_table_is_generated():
    gen = os.path.join(PKG, "csrc", "gen_demap_lut.py")
    out = subprocess.run([sys.executable, gen], capture_output=True, text=True, check=True).stdout
    assert out == open(os.path.join(PKG, "csrc", "demap_lut.h")).read()


def test_product_never_imports_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text).lower(), f


def test_learned_argument_validation():
    from paper_2602_12098_amd import learn
    from paper_2602_12098_amd._lib import VP_EINVAL, VP_EUNSUPPORTED, VP_OK
    lib = learn._load()
    P = ctypes.c_void_p(16)   # never dereferenced: validation fails or returns before any launch
    assert lib.vp_mlp_features(None, None, None, 8.0, 1, 14, 4, 1, None, None) == VP_EINVAL
    assert lib.vp_mlp_features(P, P, P, 0.0, 1, 14, 4, 1, P, None) == VP_EINVAL
    assert lib.vp_mlp_features(P, P, P, 8.0, 1, 14, 4, 2, P, None) == VP_EINVAL   # unknown kind
    assert lib.vp_mlp_features(P, P, P, 8.0, 1, 14, 17, 0, P, None) == VP_EUNSUPPORTED
    assert lib.vp_mlp_features(None, None, None, 8.0, 0, 14, 4, 0, None, None) == VP_OK
    assert lib.vp_path_ranks(P, P, P, 8.0, None, 1, 14, 4, P, None) == VP_EINVAL
    assert lib.vp_path_ranks(P, P, P, 8.0, P, 1, 0, 4, P, None) == VP_EINVAL
    # gemm: bad sizes, leading dimensions, flags, no output
    assert lib.vp_gemm_bf16(-1, 4, 4, P, 4, 0, P, 4, 0, None, 0, None, 0, 1.0, P, None, 4, None) == VP_EINVAL
    assert lib.vp_gemm_bf16(4, 4, 4, P, 3, 0, P, 4, 0, None, 0, None, 0, 1.0, P, None, 4, None) == VP_EINVAL
    assert lib.vp_gemm_bf16(4, 5, 8, P, 8, 0, P, 4, 0, None, 0, None, 0, 1.0, P, None, 5, None) == VP_EINVAL
    assert lib.vp_gemm_bf16(4, 5, 8, P, 8, 0, P, 8, 1, None, 2, None, 0, 1.0, P, None, 5, None) == VP_EINVAL
    assert lib.vp_gemm_bf16(4, 5, 8, P, 8, 0, P, 8, 1, None, 0, None, 0, 1.0, None, None, 5, None) == VP_EINVAL
    assert lib.vp_gemm_bf16(4, 5, 8, P, 8, 0, P, 8, 1, None, 0, P, 4, 1.0, P, None, 5, None) == VP_EINVAL
    assert lib.vp_gemm_bf16(4, 5, 8, P, 8, 0, P, 8, 1, None, 0, None, 0, 1.0, P, None, 4, None) == VP_EINVAL
    assert lib.vp_gemm_bf16(0, 5, 8, None, 8, 0, None, 8, 1, None, 0, None, 0, 1.0, P, None, 5, None) == VP_OK
    assert lib.vp_gemm_bf16(4, 5, 8, None, 8, 0, P, 8, 1, None, 0, None, 0, 1.0, P, None, 5, None) == VP_EINVAL
    # top-k / loss / colsum / tables
    assert lib.vp_topk64(P, 4, 63, P, None, None) == VP_EINVAL
    assert lib.vp_topk64(P, 4, 4097, P, None, None) == VP_EUNSUPPORTED
    assert lib.vp_topk64(None, 0, 100, None, None, None) == VP_OK
    assert lib.vp_topk64(None, 3, 100, P, None, None) == VP_EINVAL
    assert lib.vp_softmax_xent(P, 3, 0, P, 1.0, P, P, None) == VP_EINVAL
    assert lib.vp_softmax_xent(P, 3, 10, P, float("inf"), P, P, None) == VP_EINVAL
    assert lib.vp_softmax_xent(P, 3, 10, None, 1.0, P, P, None) == VP_EINVAL
    assert lib.vp_colsum_bf16(P, -1, 3, P, None) == VP_EINVAL
    assert lib.vp_colsum_bf16(None, 3, 3, P, None) == VP_EINVAL
    assert lib.vp_learned_paths(P, 10, 4, P, 64, P, 8, 9, 2, 14, P, None) == VP_EINVAL     # K_fixed > table
    assert lib.vp_learned_paths(P, 0, 4, P, 64, P, 8, 8, 2, 14, P, None) == VP_EINVAL     # empty vocabulary
    assert lib.vp_learned_paths(P, 10, 17, P, 64, P, 8, 8, 2, 14, P, None) == VP_EUNSUPPORTED
    assert lib.vp_learned_paths(P, 10, 4, P, 4000, P, 200, 200, 2, 14, P, None) == VP_EUNSUPPORTED
    assert lib.vp_learned_paths(P, 10, 4, P, 0, P, 8, 0, 2, 14, P, None) == VP_EINVAL     # empty table
    assert lib.vp_learned_paths(P, 10, 4, None, 64, P, 8, 8, 2, 14, P, None) == VP_EINVAL
    # fused last layer + top-64: vocabulary a multiple of 128 in 256..4096,
    # 16-byte aligned operands, a 256-byte aligned workspace, a bias
    A = ctypes.c_void_p(4096)
    assert lib.vp_logits_top64(A, 10, A, A, 200, A, None, A, None) == VP_EUNSUPPORTED
    assert lib.vp_logits_top64(A, 10, A, A, 128, A, None, A, None) == VP_EUNSUPPORTED
    assert lib.vp_logits_top64(A, 10, A, A, 4224, A, None, A, None) == VP_EUNSUPPORTED
    assert lib.vp_logits_top64(A, -1, A, A, 4096, A, None, A, None) == VP_EINVAL
    assert lib.vp_logits_top64(None, 0, None, None, 4096, None, None, None, None) == VP_OK
    assert lib.vp_logits_top64(A, 10, A, None, 4096, A, None, A, None) == VP_EINVAL      # no bias
    assert lib.vp_logits_top64(ctypes.c_void_p(4098), 10, A, A, 4096, A, None, A, None) == VP_EINVAL
    assert lib.vp_logits_top64(A, 10, A, A, 4096, A, None, ctypes.c_void_p(4096 + 64), None) == VP_EINVAL
    assert lib.vp_logits_top64_work_bytes(0) >= 0
    assert lib.vp_logits_top64_work_bytes(1000) > 1000 * 2048


def test_region_demap_device_code_matches_oracle_definition():
    """The device region-table DEMAP (host build, with the table generated by
    gen_region_lut.py) against the oracle's own construction of the same
    definition, at every rank: random float32 centres, and a grid of
    sixteenths where the fold, the cells and the anchor meet exact
    boundaries."""
    run = _host_demap()
    rng = np.random.default_rng(11)
    cx = rng.uniform(-3, 3, 4000).astype(np.float32)
    cy = rng.uniform(-3, 3, 4000).astype(np.float32)
    g = (np.arange(-40, 41) / 16.0).astype(np.float32)
    gx, gy = np.meshgrid(g, g)
    cx = np.concatenate([cx, gx.ravel()])
    cy = np.concatenate([cy, gy.ravel()])
    for r in range(9):
        a, b = run(cx, cy, np.full(len(cx), r), 4)
        for k in range(len(cx)):
            want = O.demap_region(complex(float(cx[k]), float(cy[k])), r)
            assert (a[k], b[k]) == (want.real, want.imag), (r, cx[k], cy[k], a[k], b[k], want)


def test_region_table_is_generated():
    gen = os.path.join(PKG, "csrc", "gen_region_lut.py")
    out = subprocess.run([sys.executable, gen], capture_output=True, text=True, check=True).stdout
    assert out == open(os.path.join(PKG, "csrc", "region_lut.h")).read()
