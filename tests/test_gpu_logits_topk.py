"""GPU parity of vp_logits_top64 (the network's last layer fused with its
top-64) through the C ABI.

The reference is the oracle's top-64 and softmax mass (oracle/mlp_oracle.py)
of the logits that the unfused GEMM (vp_gemm_bf16, itself checked against the
FP64 oracle within its derived bound in test_gpu_learn.py) writes for the same
operands: the fused kernels must select exactly what the oracle selects from
those values, and give the mass within 1e-4.  Cases cover ragged row counts,
every accepted vocabulary shape, rows whose candidates overflow into the
exact path (ties over many columns, constant rows), and the committed network
at the benchmark's launch."""
import os

import numpy as np
import pytest

import vpgen
from oracle import mlp_oracle as L

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


def host(t):
    return t.detach().cpu().numpy()


def _operands(rng, rows, V, kind):
    """X (post-ReLU hidden layer), Wt, bias as float32 (rounded to bf16 by the
    caller) for one kind of logit distribution."""
    X = np.maximum(rng.standard_normal((rows, 256)), 0.0).astype(np.float32)
    Wt = (rng.standard_normal((V, 256)) * 0.06).astype(np.float32)
    b = (rng.standard_normal(V) * 0.1).astype(np.float32)
    if kind == "ties":       # few distinct values: ties at the boundary, many candidates
        X = (rng.integers(0, 2, size=(rows, 256))).astype(np.float32)
        Wt = (rng.integers(-1, 2, size=(V, 256)) * 0.25).astype(np.float32)
        b = np.zeros(V, np.float32)
    elif kind == "const":    # every logit equal: all columns are candidates
        Wt[:] = 0.0
        b[:] = 0.5
    elif kind == "mixed":    # zero rows (logits = bias, coarse) among ordinary rows
        X[::3] = 0.0
        b = (np.round(rng.standard_normal(V) * 2) / 4).astype(np.float32)
    elif kind == "skewed":   # the largest logits all in one split
        b[(np.arange(V) // 32) % 4 == 1] += 3.0
    return X, Wt, b


@pytest.mark.parametrize("rows,V,kind", [(300, 4096, "normal"), (1, 256, "normal"), (257, 384, "normal"),
                                         (3000, 4096, "normal"), (513, 4096, "ties"), (100, 4096, "const"),
                                         (600, 1024, "mixed"), (700, 4096, "skewed"), (255, 2048, "ties")])
def test_logits_top64_vs_oracle(lib, rows, V, kind):
    _, learn = lib
    print("logits_top64", rows, V, kind, flush=True)
    rng = np.random.default_rng(rows * 7 + V)
    Xf, Wf, bf = _operands(rng, rows, V, kind)
    X = torch.from_numpy(Xf).to(DEV).to(torch.bfloat16).contiguous()
    Wt = torch.from_numpy(Wf).to(DEV).to(torch.bfloat16).contiguous()
    b = torch.from_numpy(bf).to(DEV)
    z = learn.gemm_bf16(X, Wt, trans_b=True, bias=b)
    idx, mass = learn.logits_top64(X, Wt, b)
    idx2, mass2 = learn.logits_top64(X, Wt, b, with_mass=False)
    torch.cuda.synchronize()
    zs = host(z)
    want = L.topk(zs, 64)
    np.testing.assert_array_equal(host(idx), want)
    np.testing.assert_array_equal(host(idx2), want)
    assert mass2 is None
    wm = L.softmax_mass(zs.astype(np.float64), want)
    assert np.all(np.abs(host(mass) - wm) <= 1e-4 * (1 + wm))


def test_logits_top64_reuses_a_workspace(lib):
    # two calls in a row on one workspace, the second with fewer rows and a
    # smaller vocabulary: nothing of the first call leaks into the second
    _, learn = lib
    rng = np.random.default_rng(11)
    work = learn.logits_top64_work(2000, DEV)
    for rows, V in ((2000, 4096), (700, 512)):
        Xf, Wf, bf = _operands(rng, rows, V, "normal")
        X = torch.from_numpy(Xf).to(DEV).to(torch.bfloat16).contiguous()
        Wt = torch.from_numpy(Wf).to(DEV).to(torch.bfloat16).contiguous()
        b = torch.from_numpy(bf).to(DEV)
        z = host(learn.gemm_bf16(X, Wt, trans_b=True, bias=b))
        idx, _ = learn.logits_top64(X, Wt, b, work=work)
        np.testing.assert_array_equal(host(idx), L.topk(z, 64))


def test_logits_top64_on_the_trained_network_at_the_benchmark_launch(lib):
    """The committed network on all 45,864 vectors of the benchmark's slot:
    the fused selection equals topk64 of the written logits on every row, and
    400 sampled rows equal the oracle's selection (mass within 1e-4)."""
    vp, learn = lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(root, "paper_2602_12098_amd", "weights", "proposer_16x16_256qam_res64.safetensors")
    if not os.path.exists(path):
        pytest.skip("no committed proposer")
    prop = learn.load_proposer(path)
    wl = vpgen.cfg3(512)
    prep = vp.preprocess(torch.from_numpy(wl.H).to(DEV), wl.alpha)
    p = prop.p
    with torch.no_grad():
        x = learn.mlp_features(prep.W, prep.perm, torch.from_numpy(wl.s).to(DEV), wl.tau, wl.n_sym, kind=prop.kind)
        h1 = learn.gemm_bf16(x, p.W1, trans_b=True, bias=p.b1, relu=True, out_f32=False, out_bf16=True)
        h2 = learn.gemm_bf16(h1, p.W2, trans_b=True, bias=p.b2, relu=True, out_f32=False, out_bf16=True)
        z = learn.gemm_bf16(h2, p.W3, trans_b=True, bias=p.b3)
        idx, mass = learn.logits_top64(h2, p.W3, p.b3)
        ref_idx, ref_mass = learn.topk64(z)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(idx), host(ref_idx))
    assert float((mass - ref_mass).abs().max()) <= 1e-4
    rows = np.random.default_rng(5).choice(wl.n_vec, 400, replace=False)
    zs = host(z[torch.from_numpy(rows).to(DEV)])
    want = L.topk(zs, 64)
    np.testing.assert_array_equal(host(idx)[rows], want)
    wm = L.softmax_mass(zs.astype(np.float64), want)
    assert np.all(np.abs(host(mass)[rows] - wm) <= 1e-4 * (1 + wm))


def test_logits_top64_errors(lib):
    _, learn = lib
    from paper_2602_12098_amd._lib import VP_EINVAL, VP_EUNSUPPORTED, VPError
    X = torch.zeros((10, 256), dtype=torch.bfloat16, device=DEV)
    b = torch.zeros((200,), dtype=torch.float32, device=DEV)
    with pytest.raises(VPError) as e:
        learn.logits_top64(X, torch.zeros((200, 256), dtype=torch.bfloat16, device=DEV), b)
    assert e.value.code == VP_EUNSUPPORTED
    Xu = torch.zeros((10 * 256 + 1,), dtype=torch.bfloat16, device=DEV)[1:].view(10, 256)   # 2-byte offset
    W = torch.zeros((256, 256), dtype=torch.bfloat16, device=DEV)
    with pytest.raises(VPError) as e:
        learn.logits_top64(Xu, W, torch.zeros((256,), dtype=torch.float32, device=DEV))
    assert e.value.code == VP_EINVAL
    with pytest.raises(ValueError):
        learn.logits_top64(X, W, torch.zeros((256,), dtype=torch.float32, device=DEV),
                           work=torch.empty((16,), dtype=torch.uint8, device=DEV))
