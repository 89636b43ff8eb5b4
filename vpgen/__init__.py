"""Seeded synthetic workloads for ViPer NL-COMM vector-perturbation precoding.

This module only draws random inputs (channels, symbols) and describes the
workload shapes.  It holds none of the precoding method's arithmetic, so both
the FP64 oracle and the HIP path can consume the very same complex64 arrays.

Shapes and value distributions follow the paper's evaluation setup
(Sec. III-B, Table I: 30 kHz SCS, 14-symbol slot, i.i.d. Rayleigh channels,
QPSK..256-QAM) and the correlated-channel stand-in for its CDL-B runs
(exponential Kronecker correlation).  No public dataset is involved: every
array here is synthetic.

Conventions
-----------
* ``H``  complex64 ``[n_sc][N][M]``; row ``i`` is user ``i`` (Sec. II, the
  channel entry between user i and antenna j).
* ``s``  complex64 structure-of-arrays ``[N][n_vec]`` with the vector index
  ``v = sc * n_sym + sym``.  Values are unnormalised odd-integer QAM points
  ``{+-1, +-3, ..., +-(sqrt(Q)-1)}`` on both rails; the perturbation
  interval is ``tau = 2 sqrt(Q)`` (Sec. II-B).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Workload",
    "qam_tau",
    "qam_levels",
    "draw_rayleigh",
    "draw_correlated",
    "draw_symbols",
    "make",
    "cfg1",
    "cfg2",
    "cfg3",
    "cfg4",
    "BatchedWorkload",
    "CONFIGS",
]


def qam_tau(Q: int) -> float:
    """Perturbation interval tau = 2 sqrt(Q) for square Q-QAM with odd-integer points."""
    r = int(round(math.sqrt(Q)))
    if r * r != Q or r < 2:
        raise ValueError(f"Q={Q} is not a square QAM order")
    return float(2 * r)


def qam_levels(Q: int) -> np.ndarray:
    r = int(round(math.sqrt(Q)))
    return np.arange(-(r - 1), r, 2, dtype=np.float64)


@dataclasses.dataclass
class Workload:
    name: str
    N: int            # users / streams (tree levels)
    M: int            # AP antennas
    n_sc: int
    n_sym: int
    Q: int
    alpha: float      # Tikhonov / RZF regulariser (lambda^2)
    K: int            # path-set size
    H: np.ndarray     # complex64 [n_sc][N][M]
    s: np.ndarray     # complex64 [N][n_vec]
    seed: int
    rho: float = 0.0

    @property
    def tau(self) -> float:
        return qam_tau(self.Q)

    @property
    def n_vec(self) -> int:
        return self.n_sc * self.n_sym


def draw_rayleigh(rng: np.random.Generator, n_sc: int, N: int, M: int) -> np.ndarray:
    """i.i.d. CN(0,1): real parts for every subcarrier first, then imaginary parts."""
    re = rng.standard_normal((n_sc, N, M)) * math.sqrt(0.5)
    im = rng.standard_normal((n_sc, N, M)) * math.sqrt(0.5)
    return (re + 1j * im).astype(np.complex64)


def _expcorr_sqrt(n: int, rho: float) -> np.ndarray:
    T = rho ** np.abs(np.subtract.outer(np.arange(n), np.arange(n)))
    return np.linalg.cholesky(T)


def draw_correlated(rng: np.random.Generator, n_sc: int, N: int, M: int, rho: float) -> np.ndarray:
    """Kronecker model H = C_r Hw C_t^T with T[i,j] = rho^|i-j| on both sides."""
    Hw = draw_rayleigh(rng, n_sc, N, M).astype(np.complex128)
    Cr = _expcorr_sqrt(N, rho)
    Ct = _expcorr_sqrt(M, rho)
    return np.einsum("ij,sjk,lk->sil", Cr, Hw, Ct).astype(np.complex64)


def draw_symbols(rng: np.random.Generator, N: int, n_vec: int, Q: int) -> np.ndarray:
    lv = qam_levels(Q)
    ire = rng.integers(0, lv.size, size=(N, n_vec))
    iim = rng.integers(0, lv.size, size=(N, n_vec))
    return (lv[ire] + 1j * lv[iim]).astype(np.complex64)


def make(name: str, N: int, M: int, n_sc: int, n_sym: int, Q: int, alpha: float, K: int,
         seed: int, rho: float = 0.0) -> Workload:
    rng = np.random.default_rng(seed)
    if rho:
        H = draw_correlated(rng, n_sc, N, M, rho)
    else:
        H = draw_rayleigh(rng, n_sc, N, M)
    s = draw_symbols(rng, N, n_sc * n_sym, Q)
    return Workload(name, N, M, n_sc, n_sym, Q, float(alpha), K, H, s, seed, rho)


def cfg1(n_sc: int = 64) -> Workload:
    """4x4 ZF, 16-QAM (tau=8), 64 subcarriers x 14 symbols, 32 paths."""
    return make("4x4-zf-16qam", 4, 4, n_sc, 14, 16, 0.0, 32, seed=1)


def cfg2(snr_db: int = 20, n_sc: int = 1638) -> Workload:
    """8x8 RZF, 64-QAM (tau=16), alpha = N / SNR_lin, 1638 subcarriers x 14 symbols, 64 paths."""
    idx = {10: 0, 20: 1, 30: 2}[snr_db]
    alpha = 8.0 / (10.0 ** (snr_db / 10.0))
    return make(f"8x8-rzf-64qam-snr{snr_db}", 8, 8, n_sc, 14, 64, alpha, 64, seed=20 + idx)


def cfg3(K: int = 512, n_sc: int = 3276) -> Workload:
    """16x16 at 100 MHz, 256-QAM (tau=32), rho=0.5 Kronecker, alpha=0.16, 3276 x 14."""
    return make(f"16x16-rzf-256qam-rho0.5-K{K}", 16, 16, n_sc, 14, 256, 0.16, K, seed=3, rho=0.5)


@dataclasses.dataclass
class BatchedWorkload:
    """Resource-block groups with uneven user counts on a common antenna array."""
    name: str
    M: int
    n_rbg: int
    sc_per_rbg: int
    n_sym: int
    U: np.ndarray        # int32 [n_rbg] users per RBG
    Q: np.ndarray        # int32 [n_rbg] QAM order per RBG
    alpha: np.ndarray    # float32 [n_rbg]
    H: List[np.ndarray]  # per RBG complex64 [sc_per_rbg][U][M]
    s: List[np.ndarray]  # per RBG complex64 [U][sc_per_rbg * n_sym]
    seed: int


def cfg4(n_rbg: int = 2048, seed: int = 4, users=None) -> BatchedWorkload:
    """2048 RBGs x 12 subcarriers x 14 symbols, U ~ Unif{4..16}, Q ~ Unif{4,16,64,256}, M=16.
    `users` (optional) replaces the first len(users) user counts."""
    rng = np.random.default_rng(seed)
    M, spr, n_sym = 16, 12, 14
    U = rng.integers(4, 17, size=n_rbg).astype(np.int32)
    if users is not None:
        U[:len(users)] = np.asarray(users, dtype=np.int32)
    Q = np.array([4, 16, 64, 256], dtype=np.int32)[rng.integers(0, 4, size=n_rbg)]
    alpha = (U / 100.0).astype(np.float32)
    H = [draw_rayleigh(rng, spr, int(u), M) for u in U]
    s = [draw_symbols(rng, int(u), spr * n_sym, int(q)) for u, q in zip(U, Q)]
    return BatchedWorkload("batched-rbg-4to16", M, n_rbg, spr, n_sym, U, Q, alpha, H, s, seed)


CONFIGS = {
    "cfg1": cfg1,
    "cfg2": cfg2,
    "cfg3": cfg3,
    "cfg4": cfg4,
}
