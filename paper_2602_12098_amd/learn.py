"""Learned path proposal: torch binding of include/vp_learn.h, the network's
autograd.Function (hand-written backward on the HIP kernels) and its use.

The proposal replaces the channel-only path set of the Metric of Promise
(Sec. III-A-2) by a per-vector list: a 64 -> 256 -> 256 -> V network (ReLU)
scores a fixed vocabulary of V position vectors, the 64 best are kept, the
first few MoP paths of the subcarrier are appended, and the unchanged path
search (Sec. II-B PED, Alg. 2 argmin) evaluates the list.  The search result
is an exact Gaussian-integer perturbation whatever the network proposes; the
network only decides which candidates are walked.

Arithmetic runs in the HIP kernels; this module marshals tensors.  Training
(the optimiser step, data shuffling, building the vocabulary from label
counts) uses torch on the GPU as plumbing around those kernels.
"""
from __future__ import annotations

import ctypes
from typing import NamedTuple, Optional

import torch

from . import _lib
from ._lib import check
from .vp import VP_INCLUDE_ZERO, _req, _stream, packed_size, tau_array

__all__ = ["VP_EPI_RELU", "VP_PATHS_PER_VECTOR", "N_FEATURES", "TOPK", "mlp_features", "path_ranks", "gemm_bf16",
           "topk64", "logits_top64", "logits_top64_work", "softmax_xent", "colsum_bf16", "learned_paths", "MLPParams", "MLPFunction", "mlp_logits",
           "pack_ranks", "Proposer", "load_proposer"]

VP_EPI_RELU = 1
VP_PATHS_PER_VECTOR = 2
VP_FEAT_ZERO_CENTRES = 0
VP_FEAT_RANK0_WALK = 1
N_FEATURES = 64
TOPK = 64
HIDDEN = 256

_P = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.c_float
_I64 = ctypes.c_int64

SIGNATURES = {
    "vp_mlp_features": [_P, _P, _P, _F, _I, _I, _I, ctypes.c_uint32, _P, _P],
    "vp_path_ranks": [_P, _P, _P, _F, _P, _I, _I, _I, _P, _P],
    "vp_gemm_bf16": [_I, _I, _I, _P, _I64, _I, _P, _I64, _I, _P, ctypes.c_uint32, _P, _I64, _F, _P, _P, _I64, _P],
    "vp_topk64": [_P, _I, _I, _P, _P, _P],
    "vp_softmax_xent": [_P, _I, _I, _P, _F, _P, _P, _P],
    "vp_colsum_bf16": [_P, _I, _I, _P, _P],
    "vp_learned_paths": [_P, _I, _I, _P, _I, _P, _I, _I, _I, _I, _P, _P],
    "vp_logits_top64": [_P, _I, _P, _P, _I, _P, _P, _P, _P],
    "vp_logits_top64_work_bytes": [_I],
}
_bound = False


def _load():
    global _bound
    lib = _lib.load()
    if not _bound:
        for name, argtypes in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = argtypes
            fn.restype = _I
        lib.vp_logits_top64_work_bytes.restype = _I64
        _bound = True
    return lib


def mlp_features(W: torch.Tensor, perm: torch.Tensor, s: torch.Tensor, tau: float, n_sym: int,
                 kind: int = VP_FEAT_RANK0_WALK, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vp_mlp_features -> bf16 [n_vec][64]."""
    lib = _load()
    n_sc, N = perm.shape
    n_vec = n_sc * n_sym
    if out is None:
        out = torch.empty((n_vec, N_FEATURES), dtype=torch.bfloat16, device=W.device)
    check(lib.vp_mlp_features(_req(W, "W", torch.complex64, (n_sc, packed_size(N))),
                              _req(perm, "perm", torch.uint8, (n_sc, N)),
                              _req(s, "s", torch.complex64, (N, n_vec)), float(tau), n_sc, int(n_sym), N, int(kind),
                              _req(out, "feat", torch.bfloat16, (n_vec, N_FEATURES)), _stream()), "vp_mlp_features")
    return out


def path_ranks(W: torch.Tensor, perm: torch.Tensor, s: torch.Tensor, tau: float, l: torch.Tensor, n_sym: int,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vp_path_ranks -> uint8 [n_vec][N] (rank of each level's l in the DEMAP order)."""
    lib = _load()
    n_sc, N = perm.shape
    n_vec = n_sc * n_sym
    if out is None:
        out = torch.empty((n_vec, N), dtype=torch.uint8, device=W.device)
    check(lib.vp_path_ranks(_req(W, "W", torch.complex64, (n_sc, packed_size(N))),
                            _req(perm, "perm", torch.uint8, (n_sc, N)),
                            _req(s, "s", torch.complex64, (N, n_vec)), float(tau),
                            _req(l, "l", torch.int8, (N, n_vec, 2)), n_sc, int(n_sym), N,
                            _req(out, "ranks", torch.uint8, (n_vec, N)), _stream()), "vp_path_ranks")
    return out


def _bf16_2d(t: torch.Tensor, name: str) -> int:
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    if t.dtype != torch.bfloat16 or not t.is_cuda:
        raise TypeError(f"{name} must be a bf16 GPU tensor")
    return t.data_ptr()


def gemm_bf16(A: torch.Tensor, B: torch.Tensor, trans_a: bool = False, trans_b: bool = False,
              bias: Optional[torch.Tensor] = None, relu: bool = False, mask: Optional[torch.Tensor] = None,
              alpha: float = 1.0, out_f32: bool = True, out_bf16: bool = False):
    """vp_gemm_bf16: alpha op(A) op(B) + bias (ReLU, mask).  Returns the float32
    and/or bf16 result (a tuple when both are requested)."""
    lib = _load()
    m = A.shape[1] if trans_a else A.shape[0]
    k = A.shape[0] if trans_a else A.shape[1]
    kb = B.shape[1] if trans_b else B.shape[0]
    n = B.shape[0] if trans_b else B.shape[1]
    if kb != k:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    pa, pb = _bf16_2d(A, "A"), _bf16_2d(B, "B")
    dev = A.device
    Cf = torch.empty((m, n), dtype=torch.float32, device=dev) if out_f32 else None
    Cb = torch.empty((m, n), dtype=torch.bfloat16, device=dev) if out_bf16 else None
    pbias = _req(bias, "bias", torch.float32, (n,)) if bias is not None else None
    pm = None
    ldm = 0
    if mask is not None:
        pm = _req(mask, "mask", torch.bfloat16, (m, n))
        ldm = n
    check(lib.vp_gemm_bf16(m, n, k, pa, A.stride(0), int(trans_a), pb, B.stride(0), int(trans_b), pbias,
                           VP_EPI_RELU if relu else 0, pm, ldm, float(alpha),
                           Cf.data_ptr() if Cf is not None else None, Cb.data_ptr() if Cb is not None else None,
                           n, _stream()), "vp_gemm_bf16")
    if out_f32 and out_bf16:
        return Cf, Cb
    return Cf if out_f32 else Cb


def topk64(scores: torch.Tensor, with_mass: bool = True):
    """vp_topk64: (idx int32 [rows][64], mass float32 [rows] or None)."""
    lib = _load()
    rows, C = scores.shape
    idx = torch.empty((rows, TOPK), dtype=torch.int32, device=scores.device)
    mass = torch.empty((rows,), dtype=torch.float32, device=scores.device) if with_mass else None
    check(lib.vp_topk64(_req(scores, "scores", torch.float32), rows, C, idx.data_ptr(),
                        mass.data_ptr() if mass is not None else None, _stream()), "vp_topk64")
    return idx, mass


def logits_top64_work(rows: int, device) -> torch.Tensor:
    """Workspace for logits_top64 on `rows` rows (uint8, 256-byte aligned)."""
    n = int(_load().vp_logits_top64_work_bytes(int(rows)))
    return torch.empty((n,), dtype=torch.uint8, device=device)


def logits_top64(X: torch.Tensor, Wt: torch.Tensor, bias: torch.Tensor, with_mass: bool = True,
                 work: Optional[torch.Tensor] = None):
    """vp_logits_top64: the top-64 (idx int32 [rows][64]) and softmax mass of
    X Wt^T + bias without writing the logits; X bf16 [rows][256], Wt bf16
    [V][256], bias float32 [V]."""
    lib = _load()
    rows = X.shape[0]
    V = Wt.shape[0]
    _req(X, "X", torch.bfloat16, (rows, HIDDEN))
    _req(Wt, "Wt", torch.bfloat16, (V, HIDDEN))
    _req(bias, "bias", torch.float32, (V,))
    idx = torch.empty((rows, TOPK), dtype=torch.int32, device=X.device)
    mass = torch.empty((rows,), dtype=torch.float32, device=X.device) if with_mass else None
    need = int(lib.vp_logits_top64_work_bytes(rows))
    if work is None:
        work = torch.empty((need,), dtype=torch.uint8, device=X.device)
    elif work.numel() * work.element_size() < need:
        raise ValueError(f"work: need {need} bytes")
    check(lib.vp_logits_top64(X.data_ptr(), rows, Wt.data_ptr(), bias.data_ptr(), V, idx.data_ptr(),
                              mass.data_ptr() if mass is not None else None, _req(work, "work", work.dtype),
                              _stream()), "vp_logits_top64")
    return idx, mass


def softmax_xent(logits: torch.Tensor, labels: torch.Tensor, scale: float):
    """vp_softmax_xent: (loss float32 [rows], dlogits bf16 [rows][C])."""
    lib = _load()
    rows, C = logits.shape
    loss = torch.empty((rows,), dtype=torch.float32, device=logits.device)
    dz = torch.empty((rows, C), dtype=torch.bfloat16, device=logits.device)
    check(lib.vp_softmax_xent(_req(logits, "logits", torch.float32), rows, C,
                              _req(labels, "labels", torch.int32, (rows,)), float(scale), loss.data_ptr(),
                              dz.data_ptr(), _stream()), "vp_softmax_xent")
    return loss, dz


def colsum_bf16(X: torch.Tensor) -> torch.Tensor:
    lib = _load()
    rows, cols = X.shape
    out = torch.empty((cols,), dtype=torch.float32, device=X.device)
    check(lib.vp_colsum_bf16(_req(X, "X", torch.bfloat16), rows, cols, out.data_ptr(), _stream()),
          "vp_colsum_bf16")
    return out


def learned_paths(vocab: torch.Tensor, top: torch.Tensor, fixed: Optional[torch.Tensor], K_fixed: int, n_sc: int,
                  n_sym: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vp_learned_paths -> uint8 [n_vec][K_learned + K_fixed][N]."""
    lib = _load()
    V, N = vocab.shape
    n_vec = n_sc * n_sym
    Kl = top.shape[1]
    Kft = fixed.shape[1] if fixed is not None else 0
    Kt = Kl + K_fixed
    if out is None:
        out = torch.empty((n_vec, Kt, N), dtype=torch.uint8, device=vocab.device)
    check(lib.vp_learned_paths(_req(vocab, "vocab", torch.uint8), V, N, _req(top, "top", torch.int32, (n_vec, Kl)),
                               Kl, _req(fixed, "fixed", torch.uint8, (n_sc, Kft, N)) if fixed is not None else None,
                               Kft, int(K_fixed), n_sc, int(n_sym), _req(out, "table", torch.uint8, (n_vec, Kt, N)),
                               _stream()), "vp_learned_paths")
    return out


def search_fallback(W: torch.Tensor, perm: torch.Tensor, s: torch.Tensor, tau, paths: torch.Tensor,
                    n_sym: int, mass: torch.Tensor, theta: float, out, kidx_base: int,
                    order: Optional[torch.Tensor] = None, flags: int = VP_INCLUDE_ZERO,
                    work: Optional[torch.Tensor] = None):
    """vp_search_fallback: vectors with mass < theta (or NaN mass) are searched
    over the fixed per-subcarrier table paths [n_sc][K][N]; out (a SearchOut
    holding the proposal's search result) takes the fixed result where it is
    strictly cheaper, with kidx = kidx_base + k.  Returns out."""
    lib = _load()
    n_sc, K, N = paths.shape
    n_vec = n_sc * n_sym
    if work is None:
        work = torch.empty((2 * n_vec,), dtype=torch.int32, device=W.device)
    pw = _req(work, "work", torch.int32)
    if work.numel() < 2 * n_vec:
        raise ValueError(f"work: needs {2 * n_vec} int32 elements")
    check(lib.vp_search_fallback(_req(W, "W", torch.complex64, (n_sc, packed_size(N))),
                                 _req(perm, "perm", torch.uint8, (n_sc, N)),
                                 _req(s, "s", torch.complex64, (N, n_vec)),
                                 tau_array(tau, n_sc, W.device).data_ptr(),
                                 _req(paths, "paths", torch.uint8, (n_sc, K, N)),
                                 _req(order, "order", torch.int16, (n_sc, 2, K)) if order is not None else None,
                                 int(K), int(K * N), n_sc, int(n_sym), N, int(flags),
                                 _req(mass, "mass", torch.float32, (n_vec,)), float(theta), int(kidx_base),
                                 _req(out.l, "l", torch.int8, (N, n_vec, 2)),
                                 _req(out.cost, "cost", torch.float32, (n_vec,)),
                                 _req(out.kidx, "kidx", torch.int32, (n_vec,)), pw, _stream()),
          "vp_search_fallback")
    return out


def search_fallback_noalloc(W: torch.Tensor, perm: torch.Tensor, s: torch.Tensor, tau: torch.Tensor,
                            paths: torch.Tensor, n_sym: int, mass: torch.Tensor, theta: float, out, kidx_base: int,
                            order: Optional[torch.Tensor] = None, flags: int = VP_INCLUDE_ZERO):
    """vp_search_fallback_noalloc: search_fallback without a workspace (the
    library's static per-GPU one, at most VP_NOALLOC_MAX_VECTORS vectors per
    call).  tau must already be a float32 device tensor [n_sc]: nothing is
    allocated on this path.  Returns out."""
    lib = _lib.load()
    n_sc, K, N = paths.shape
    n_vec = n_sc * n_sym
    check(lib.vp_search_fallback_noalloc(_req(W, "W", torch.complex64, (n_sc, packed_size(N))),
                                         _req(perm, "perm", torch.uint8, (n_sc, N)),
                                         _req(s, "s", torch.complex64, (N, n_vec)),
                                         _req(tau, "tau", torch.float32, (n_sc,)),
                                         _req(paths, "paths", torch.uint8, (n_sc, K, N)),
                                         _req(order, "order", torch.int16, (n_sc, 2, K)) if order is not None
                                         else None,
                                         int(K), int(K * N), n_sc, int(n_sym), N, int(flags),
                                         _req(mass, "mass", torch.float32, (n_vec,)), float(theta), int(kidx_base),
                                         _req(out.l, "l", torch.int8, (N, n_vec, 2)),
                                         _req(out.cost, "cost", torch.float32, (n_vec,)),
                                         _req(out.kidx, "kidx", torch.int32, (n_vec,)), _stream()),
          "vp_search_fallback_noalloc")
    return out


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

class MLPParams(NamedTuple):
    W1: torch.Tensor   # [256][64]   (torch Linear layout [out][in])
    b1: torch.Tensor   # [256] float32
    W2: torch.Tensor   # [256][256]
    b2: torch.Tensor
    W3: torch.Tensor   # [V][256]
    b3: torch.Tensor   # [V]


class MLPFunction(torch.autograd.Function):
    """logits = L3(relu(L2(relu(L1(x))))) with bf16 weights / activations and
    float32 accumulation; forward and backward both run on vp_gemm_bf16.

    Backward (chain rule of the three affine maps and the ReLUs):
      dW3 = dZ3^T H2, db3 = colsum dZ3, dH2 = (dZ3 W3) * [H2 > 0]
      dW2 = dH2^T H1, db2 = colsum dH2, dH1 = (dH2 W2) * [H1 > 0]
      dW1 = dH1^T X,  db1 = colsum dH1
    Weight and bias gradients are float32; the weights' own gradient inputs
    are the bf16 weights the forward used (the float32 master copy lives in
    the optimiser)."""

    @staticmethod
    def forward(ctx, x, W1, b1, W2, b2, W3, b3):
        # weights may be float32 masters (rounded to bf16 here) or bf16 already;
        # the gradients returned are float32 either way
        W1, W2, W3 = (w.to(torch.bfloat16).contiguous() for w in (W1, W2, W3))
        b1, b2, b3 = (b.float().contiguous() for b in (b1, b2, b3))
        h1 = gemm_bf16(x, W1, trans_b=True, bias=b1, relu=True, out_f32=False, out_bf16=True)
        h2 = gemm_bf16(h1, W2, trans_b=True, bias=b2, relu=True, out_f32=False, out_bf16=True)
        z = gemm_bf16(h2, W3, trans_b=True, bias=b3)
        ctx.save_for_backward(x, W1, W2, W3, h1, h2)
        return z

    @staticmethod
    def backward(ctx, dz):
        x, W1, W2, W3, h1, h2 = ctx.saved_tensors
        dz = dz.to(torch.bfloat16).contiguous()
        dW3 = gemm_bf16(dz, h2, trans_a=True)
        db3 = colsum_bf16(dz)
        dh2 = gemm_bf16(dz, W3, mask=h2, out_f32=False, out_bf16=True)
        dW2 = gemm_bf16(dh2, h1, trans_a=True)
        db2 = colsum_bf16(dh2)
        dh1 = gemm_bf16(dh2, W2, mask=h1, out_f32=False, out_bf16=True)
        dW1 = gemm_bf16(dh1, x, trans_a=True)
        db1 = colsum_bf16(dh1)
        dx = gemm_bf16(dh1, W1, out_f32=False, out_bf16=True) if ctx.needs_input_grad[0] else None
        return dx, dW1, db1, dW2, db2, dW3, db3


def mlp_logits(x: torch.Tensor, p: MLPParams) -> torch.Tensor:
    return MLPFunction.apply(x, p.W1, p.b1, p.W2, p.b2, p.W3, p.b3)


class SoftmaxXentFunction(torch.autograd.Function):
    """Mean softmax cross-entropy over the labelled rows (label -1 = unlabelled),
    forward and gradient from vp_softmax_xent."""

    @staticmethod
    def forward(ctx, z, labels):
        n_lab = int((labels >= 0).sum().item())
        scale = 1.0 / max(n_lab, 1)
        loss, dz = softmax_xent(z.contiguous(), labels, scale)
        ctx.save_for_backward(dz)
        return loss.sum() * scale

    @staticmethod
    def backward(ctx, g):
        (dz,) = ctx.saved_tensors
        return dz.float() * g, None


def pack_ranks(ranks: torch.Tensor) -> torch.Tensor:
    """uint8 [n][N] ranks -> int64 [n] words, level i in bits 4i..4i+3 (the
    path-word layout of the search)."""
    n, N = ranks.shape
    sh = (4 * torch.arange(N, device=ranks.device, dtype=torch.int64))
    return (ranks.to(torch.int64) << sh).sum(dim=1)


class Proposer:
    """A trained network plus its vocabulary: proposes per-vector path tables."""

    def __init__(self, params: MLPParams, vocab: torch.Tensor, feature_kind: int = VP_FEAT_RANK0_WALK):
        self.kind = int(feature_kind)
        self.p = MLPParams(*[t.to(torch.bfloat16).contiguous() if t.dim() == 2 else t.float().contiguous()
                             for t in params])
        self.vocab = vocab.contiguous()   # uint8 [V][N]

    @torch.no_grad()
    def propose(self, W, perm, s, tau, n_sym, fixed_paths=None, K_fixed=8, fused=True, work=None,
                with_mass=True):
        """Features -> hidden layers -> top-64 of the logits -> table
        [n_vec][64 + K_fixed][N].  Returns (table, mass).  fused: the last layer
        and the top-64 in one pass that never writes the logits
        (logits_top64); else the logits GEMM and topk64 (same result).
        with_mass=False (fused only): mass is None, and the fused kernels
        leave out the softmax sums."""
        n_sc = perm.shape[0]
        x = mlp_features(W, perm, s, tau, n_sym, kind=self.kind)
        p = self.p
        if fused and self.vocab.shape[0] % 128 == 0 and self.vocab.shape[0] >= 256:
            h1 = gemm_bf16(x, p.W1, trans_b=True, bias=p.b1, relu=True, out_f32=False, out_bf16=True)
            h2 = gemm_bf16(h1, p.W2, trans_b=True, bias=p.b2, relu=True, out_f32=False, out_bf16=True)
            top, mass = logits_top64(h2, p.W3, p.b3, with_mass=with_mass, work=work)
        else:
            z = MLPFunction.forward(_NoCtx(), x, *p)
            top, mass = topk64(z)
        table = learned_paths(self.vocab, top, fixed_paths, K_fixed if fixed_paths is not None else 0, n_sc, n_sym)
        return table, mass


def load_proposer(path: str, device: str = "cuda:0") -> Proposer:
    """A Proposer from a safetensors file written by the training script
    (weights W1..b3, vocabulary; metadata: feature kind).  Safe loader only."""
    from safetensors import safe_open
    from safetensors.torch import load_file
    t = load_file(path, device=device)
    with safe_open(path, framework="pt") as fh:
        meta = fh.metadata() or {}
    p = MLPParams(t["W1"], t["b1"], t["W2"], t["b2"], t["W3"], t["b3"])
    prop = Proposer(p, t["vocab"], feature_kind=int(meta.get("feature_kind", VP_FEAT_RANK0_WALK)))
    prop.meta = meta
    return prop


class _NoCtx:
    def save_for_backward(self, *a):
        pass
