"""Thin torch binding of the C ABI (argument marshalling only).

Every function takes device tensors, checks dtype / shape / contiguity, passes
raw pointers and the current HIP stream to libvp.so and returns the output
tensors.  All arithmetic happens in the HIP kernels.  Names and layouts follow
include/vp.h."""
from __future__ import annotations

from typing import NamedTuple, Optional

import torch

from . import _lib
from ._lib import VP_DEMAP_REGION, VP_INCLUDE_ZERO, VP_PATHS_PER_VECTOR, VP_SE_EXACT, VP_SE_EXHAUSTED, VP_SE_NONE, check

__all__ = ["Prep", "SearchOut", "SEOut", "FxInputs", "FxOut", "fx_quantize", "fx_search", "tau_array", "apply_user_tau", "preprocess", "paths_mop", "search", "precode", "sphere_encode", "packed_size",
           "VP_INCLUDE_ZERO", "VP_PATHS_PER_VECTOR", "VP_DEMAP_REGION", "VP_SE_EXACT", "VP_SE_EXHAUSTED", "VP_SE_NONE", "version"]


def packed_size(n: int) -> int:
    return n * (n + 1) // 2


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _req(t: torch.Tensor, name: str, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def tau_array(tau, n_sc: int, device) -> torch.Tensor:
    """tau as the per-subcarrier float32 device array [n_sc] the C ABI takes:
    a tensor is checked and passed through, a number is expanded."""
    if isinstance(tau, torch.Tensor):
        _req(tau, "tau", torch.float32, (n_sc,))
        return tau
    return torch.full((n_sc,), float(tau), dtype=torch.float32, device=device)


class Prep(NamedTuple):
    W: torch.Tensor       # complex64 [n_sc][N(N+1)/2] packed lower, column-major, search order
    w2: torch.Tensor      # float32 [n_sc][N]
    perm: torch.Tensor    # uint8 [n_sc][N] level -> user
    G: Optional[torch.Tensor]   # complex64 [n_sc][M][N]
    status: torch.Tensor  # int32 [n_sc]


class SearchOut(NamedTuple):
    l: torch.Tensor       # int8 [N][n_vec][2]
    cost: torch.Tensor    # float32 [n_vec]
    kidx: torch.Tensor    # int32 [n_vec]


def preprocess(H: torch.Tensor, alpha: float, want_G: bool = True, out: Optional[Prep] = None,
               sorted: bool = True) -> Prep:
    """vp_preprocess (sorted = False: vp_preprocess_unsorted): H complex64
    [n_sc][N][M] -> W, w2, perm, G, status."""
    lib = _lib.load()
    n_sc, N, M = H.shape
    dev = H.device
    if out is None:
        out = Prep(torch.empty((n_sc, packed_size(N)), dtype=torch.complex64, device=dev),
                   torch.empty((n_sc, N), dtype=torch.float32, device=dev),
                   torch.empty((n_sc, N), dtype=torch.uint8, device=dev),
                   torch.empty((n_sc, M, N), dtype=torch.complex64, device=dev) if want_G else None,
                   torch.empty((n_sc,), dtype=torch.int32, device=dev))
    pH = _req(H, "H", torch.complex64)
    pW = _req(out.W, "W", torch.complex64, (n_sc, packed_size(N)))
    pw = _req(out.w2, "w2", torch.float32, (n_sc, N))
    pp = _req(out.perm, "perm", torch.uint8, (n_sc, N))
    pG = _req(out.G, "G", torch.complex64, (n_sc, M, N)) if out.G is not None else None
    ps = _req(out.status, "status", torch.int32, (n_sc,))
    fn = lib.vp_preprocess if sorted else lib.vp_preprocess_unsorted
    check(fn(pH, n_sc, N, M, float(alpha), pW, pw, pp, pG, ps, _stream()),
          "vp_preprocess" if sorted else "vp_preprocess_unsorted")
    return out


def paths_mop(w2: torch.Tensor, K: int, out: Optional[torch.Tensor] = None,
              order: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vp_paths_mop: w2 float32 [n_sc][N] -> paths uint8 [n_sc][K][N].  If `order`
    (int16 [n_sc][2][K], read as uint16) is given it receives the two path orders."""
    lib = _lib.load()
    n_sc, N = w2.shape
    if out is None:
        out = torch.empty((n_sc, K, N), dtype=torch.uint8, device=w2.device)
    pw = _req(w2, "w2", torch.float32)
    po = _req(out, "paths", torch.uint8, (n_sc, K, N))
    pl = _req(order, "order", torch.int16, (n_sc, 2, K)) if order is not None else None
    check(lib.vp_paths_mop(pw, n_sc, N, int(K), po, pl, _stream()), "vp_paths_mop")
    return out


def search(W: torch.Tensor, perm: torch.Tensor, s: torch.Tensor, tau, paths: torch.Tensor,
           n_sym: int, flags: int = VP_INCLUDE_ZERO, out: Optional[SearchOut] = None,
           order: Optional[torch.Tensor] = None) -> SearchOut:
    """vp_search: tau is a number or a float32 tensor [n_sc]; paths is [K][N]
    (one table for all subcarriers), [n_sc][K][N], or with VP_PATHS_PER_VECTOR
    in flags [n_vec][K][N]; order (int16 [n_sc][2][K] from paths_mop) enables
    prefix sharing."""
    lib = _lib.load()
    n_sc = W.shape[0]
    N = perm.shape[1]
    n_vec = n_sc * n_sym
    if paths.dim() == 2:
        K, stride = paths.shape[0], 0
    else:
        lead = n_vec if (flags & VP_PATHS_PER_VECTOR) else n_sc
        if paths.shape[0] != lead:
            raise ValueError(f"paths: first dimension must be {lead}")
        K, stride = paths.shape[1], paths.shape[1] * paths.shape[2]
    if paths.shape[-1] != N:
        raise ValueError("paths: last dimension must be N")
    dev = W.device
    if out is None:
        out = SearchOut(torch.empty((N, n_vec, 2), dtype=torch.int8, device=dev),
                        torch.empty((n_vec,), dtype=torch.float32, device=dev),
                        torch.empty((n_vec,), dtype=torch.int32, device=dev))
    pW = _req(W, "W", torch.complex64, (n_sc, packed_size(N)))
    pp = _req(perm, "perm", torch.uint8, (n_sc, N))
    ps = _req(s, "s", torch.complex64, (N, n_vec))
    pP = _req(paths, "paths", torch.uint8)
    pl = _req(out.l, "l", torch.int8, (N, n_vec, 2))
    pc = _req(out.cost, "cost", torch.float32, (n_vec,))
    pk = _req(out.kidx, "kidx", torch.int32, (n_vec,))
    plx = _req(order, "order", torch.int16, (n_sc, 2, K)) if order is not None else None
    taus = tau_array(tau, n_sc, dev)
    check(lib.vp_search(pW, pp, ps, taus.data_ptr(), pP, plx, int(K), int(stride), n_sc, int(n_sym), N,
                        int(flags), pl, pc, pk, _stream()), "vp_search")
    return out


def precode(G: torch.Tensor, s: torch.Tensor, l: torch.Tensor, tau, cost: Optional[torch.Tensor],
            n_sym: int, P_T: float = 0.0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vp_precode: x complex64 [n_vec][M] = G (s + tau l) (* sqrt(P_T / cost));
    tau is a number or a float32 tensor [n_sc]."""
    lib = _lib.load()
    n_sc, M, N = G.shape
    n_vec = n_sc * n_sym
    if out is None:
        out = torch.empty((n_vec, M), dtype=torch.complex64, device=G.device)
    pG = _req(G, "G", torch.complex64)
    ps = _req(s, "s", torch.complex64, (N, n_vec))
    pl = _req(l, "l", torch.int8, (N, n_vec, 2))
    pc = _req(cost, "cost", torch.float32, (n_vec,)) if cost is not None else None
    px = _req(out, "x", torch.complex64, (n_vec, M))
    taus = tau_array(tau, n_sc, G.device)
    check(lib.vp_precode(pG, ps, pl, taus.data_ptr(), pc, n_sc, int(n_sym), N, M, float(P_T), px, _stream()),
          "vp_precode")
    return out


def apply_user_tau(prep: Prep, s: torch.Tensor, tau_user: torch.Tensor, n_sym: int,
                   s_out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vp_apply_user_tau: scales prep.W, prep.w2 and prep.G in place for the
    per-user intervals tau_user (float32 [n_sc][N], user order) and returns
    s' = s / tau per user; then search, paths_mop, precode and sphere_encode
    run with tau = 1."""
    lib = _lib.load()
    n_sc, N = prep.perm.shape
    M = prep.G.shape[1] if prep.G is not None else 1
    n_vec = n_sc * n_sym
    if s_out is None:
        s_out = torch.empty_like(s)
    check(lib.vp_apply_user_tau(_req(tau_user, "tau_user", torch.float32, (n_sc, N)),
                                _req(prep.perm, "perm", torch.uint8, (n_sc, N)), n_sc, int(n_sym), N, M,
                                _req(prep.W, "W", torch.complex64, (n_sc, packed_size(N))),
                                _req(prep.w2, "w2", torch.float32, (n_sc, N)),
                                _req(prep.G, "G", torch.complex64, (n_sc, M, N)) if prep.G is not None else None,
                                _req(s, "s", torch.complex64, (N, n_vec)), _req(s_out, "s_out", torch.complex64,
                                                                                (N, n_vec)), _stream()),
          "vp_apply_user_tau")
    return s_out


def version() -> str:
    return _lib.load().vp_version().decode()


class SEOut(NamedTuple):
    l: torch.Tensor       # int8 [N][n_vec][2]
    cost: torch.Tensor    # float32 [n_vec] (NaN: no point found inside the radius)
    nodes: torch.Tensor   # int64 [n_vec]
    status: torch.Tensor  # uint8 [n_vec]: VP_SE_EXACT, VP_SE_EXHAUSTED (best found so far) or VP_SE_NONE


def sphere_encode(W: torch.Tensor, perm: torch.Tensor, s: torch.Tensor, tau: float, n_sym: int,
                  radius: Optional[torch.Tensor] = None, max_nodes: int = 1 << 22,
                  out: Optional[SEOut] = None) -> SEOut:
    """vp_sphere_encode: exact VP over the box (optionally seeded with a radius)."""
    lib = _lib.load()
    n_sc = W.shape[0]
    N = perm.shape[1]
    n_vec = n_sc * n_sym
    dev = W.device
    if out is None:
        out = SEOut(torch.empty((N, n_vec, 2), dtype=torch.int8, device=dev),
                    torch.empty((n_vec,), dtype=torch.float32, device=dev),
                    torch.empty((n_vec,), dtype=torch.int64, device=dev),
                    torch.empty((n_vec,), dtype=torch.uint8, device=dev))
    pW = _req(W, "W", torch.complex64, (n_sc, packed_size(N)))
    pp = _req(perm, "perm", torch.uint8, (n_sc, N))
    ps = _req(s, "s", torch.complex64, (N, n_vec))
    pr = _req(radius, "radius", torch.float32, (n_vec,)) if radius is not None else None
    pl = _req(out.l, "l", torch.int8, (N, n_vec, 2))
    pc = _req(out.cost, "cost", torch.float32, (n_vec,))
    pn = _req(out.nodes, "nodes", torch.int64, (n_vec,))
    pst = _req(out.status, "status", torch.uint8, (n_vec,))
    check(lib.vp_sphere_encode(pW, pp, ps, float(tau), n_sc, int(n_sym), N, pr, int(max_nodes), pl, pc, pn, pst,
                               _stream()), "vp_sphere_encode")
    return out


class FxInputs(NamedTuple):
    c0: torch.Tensor      # int16 [n_vec][N][2] start centres, level order
    V: torch.Tensor       # int16 [n_sc][N(N-1)/2][2] steps V_mi (m > i) at m(m-1)/2 + i
    w: torch.Tensor       # int16 [n_sc][N] PED weights
    frac_bits: int


class FxOut(NamedTuple):
    l: torch.Tensor       # int8 [N][n_vec][2]
    ped: torch.Tensor     # int64 [n_vec] fixed-point PED of the chosen path
    kidx: torch.Tensor    # int32 [n_vec]


def fx_quantize(W: torch.Tensor, perm: torch.Tensor, s: torch.Tensor, tau, n_sym: int, frac_bits: int,
                out: Optional[FxInputs] = None) -> FxInputs:
    """vp_fx_quantize: the walk's inputs in 16-bit fixed point with frac_bits
    fractional bits (8..13)."""
    lib = _lib.load()
    n_sc = W.shape[0]
    N = perm.shape[1]
    n_vec = n_sc * n_sym
    dev = W.device
    nv = N * (N - 1) // 2
    if out is None:
        out = FxInputs(torch.empty((n_vec, N, 2), dtype=torch.int16, device=dev),
                       torch.empty((n_sc, nv, 2), dtype=torch.int16, device=dev),
                       torch.empty((n_sc, N), dtype=torch.int16, device=dev), int(frac_bits))
    taus = tau_array(tau, n_sc, dev)
    check(lib.vp_fx_quantize(_req(W, "W", torch.complex64, (n_sc, packed_size(N))),
                             _req(perm, "perm", torch.uint8, (n_sc, N)),
                             _req(s, "s", torch.complex64, (N, n_vec)), taus.data_ptr(), n_sc, int(n_sym), N,
                             int(frac_bits), _req(out.c0, "c0", torch.int16, (n_vec, N, 2)),
                             _req(out.V, "V", torch.int16, (n_sc, nv, 2)) if nv else None,
                             _req(out.w, "w", torch.int16, (n_sc, N)), _stream()), "vp_fx_quantize")
    return out._replace(frac_bits=int(frac_bits))


def fx_search(q: FxInputs, perm: torch.Tensor, paths: torch.Tensor, n_sym: int, flags: int = VP_INCLUDE_ZERO,
              out: Optional[FxOut] = None) -> FxOut:
    """vp_fx_search: the path walk in 16-bit fixed point; paths is [K][N] (one
    table) or [n_sc][K][N]."""
    lib = _lib.load()
    n_sc, N = perm.shape
    n_vec = n_sc * n_sym
    if paths.dim() == 2:
        K, stride = paths.shape[0], 0
    else:
        if paths.shape[0] != n_sc:
            raise ValueError(f"paths: first dimension must be {n_sc}")
        K, stride = paths.shape[1], paths.shape[1] * paths.shape[2]
    if paths.shape[-1] != N:
        raise ValueError("paths: last dimension must be N")
    dev = perm.device
    nv = N * (N - 1) // 2
    if out is None:
        out = FxOut(torch.empty((N, n_vec, 2), dtype=torch.int8, device=dev),
                    torch.empty((n_vec,), dtype=torch.int64, device=dev),
                    torch.empty((n_vec,), dtype=torch.int32, device=dev))
    check(lib.vp_fx_search(_req(q.c0, "c0", torch.int16, (n_vec, N, 2)),
                           _req(q.V, "V", torch.int16, (n_sc, nv, 2)) if nv else None,
                           _req(q.w, "w", torch.int16, (n_sc, N)), _req(perm, "perm", torch.uint8, (n_sc, N)),
                           _req(paths, "paths", torch.uint8), int(K), int(stride), n_sc, int(n_sym), N,
                           int(q.frac_bits), int(flags), _req(out.l, "l", torch.int8, (N, n_vec, 2)),
                           _req(out.ped, "ped", torch.int64, (n_vec,)), _req(out.kidx, "kidx", torch.int32, (n_vec,)),
                           _stream()), "vp_fx_search")
    return out
