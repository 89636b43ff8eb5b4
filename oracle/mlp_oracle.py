"""FP64 CPU oracle for the learned path proposal (an extension of the paper's
Metric-of-Promise path selection, Sec. III-A-2; the paper has no learned part).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything in this directory; only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark do.  It shares no code with
the HIP path.

Contents, each a plain restatement of its definition in float64:
  bf16_round       IEEE binary32 -> bfloat16, round to nearest even (the format)
  features         the 64 network inputs: MoP weights and zero-perturbation
                   centres of the tree (Sec. III-A-2 centres with l = 0)
  features_walk    the same weights with the centres along the rank-0 walk
  path_ranks       position vector of a given perturbation: the rank of each
                   level's symbol in the (distance, canonical index) box order
  mlp_forward      64 -> 256 -> 256 -> V, ReLU (optionally rounding the hidden
                   activations to bf16 where the GPU does)
  softmax_xent     softmax cross-entropy per row and its gradient
  mlp_backward     the chain rule of the network, derived by hand
  topk             the k largest entries, ties by smaller column
  softmax_mass     probability mass of a selected set

Pins (tests/test_oracle_learn.py): bf16 rounding against hand-worked bit
patterns and torch's own conversion; features against the first-level centre,
the rank-0 PED and the zero-perturbation cost; walk features against the
search oracle's rank-0 path cost and its rank-1 neighbours; ranks as the inverse of the
search's rank walk; the backward against central finite differences and
torch autograd in float64; the loss against log C for constant logits.
"""
from __future__ import annotations

from typing import NamedTuple, Optional

import numpy as np

from .vp_oracle import BOX, demap_walk, sqabs

N_FEATURES = 64
MAXN = 16


# ---------------------------------------------------------------------------
# bfloat16
# ---------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (8 significant bits), nearest even, via binary32:
    the value is first rounded to binary32 (as the GPU holds it), then the low
    16 bits of the binary32 pattern are rounded away.  NaN stays NaN."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ---------------------------------------------------------------------------
# features and labels
# ---------------------------------------------------------------------------

def features(W, perm, s, tau) -> np.ndarray:
    """Network input of every vector of one subcarrier, float64 [V][64].

    W: complex [N][N] lower (search order), perm: level -> user, s: complex
    [N][V] user order.  With s-tilde = W s_pi and the zero-perturbation centres
    c0_i = -s-tilde_i / (tau W_ii) (the level centres of Sec. III-A-2 when
    every earlier level chose l = 0):
      [i]      W_ii / mean_j W_jj
      [16+i]   Re c0_i,   [32+i]  Im c0_i
      [48+i]   W_ii^2 |c0_i - b0_i|^2 / mean_j W_jj^2,  b0_i the box point
               nearest to c0_i (per axis: round, then clip to [-1, 1])
    Slots of levels >= N are zero."""
    W = np.asarray(W, dtype=np.complex128)
    perm = np.asarray(perm, dtype=np.int64)
    s = np.asarray(s, dtype=np.complex128)
    if s.ndim == 1:
        s = s[:, None]
    n = W.shape[0]
    V = s.shape[1]
    d = np.real(np.diag(W))
    st = (W @ s[perm, :]).T                    # [V][N]
    c0 = -st / (tau * d[None, :])
    b0 = np.clip(np.round(c0.real), -1, 1) + 1j * np.clip(np.round(c0.imag), -1, 1)
    f = np.zeros((V, N_FEATURES))
    f[:, :n] = d[None, :] / d.mean()
    f[:, 16:16 + n] = c0.real
    f[:, 32:32 + n] = c0.imag
    f[:, 48:48 + n] = (d[None, :] ** 2) * sqabs(c0 - b0) / np.mean(d ** 2)
    return f


def features_walk(W, perm, s, tau):
    """Network input along the rank-0 walk, float64 [V][64]: the path that
    takes the nearest box point b_i (rank 0 of the box order) at every level
    has centres c_i (Sec. III-A-2, with the earlier levels' choices in the
    residual); with d0_i, d1_i the squared distances of c_i to its nearest and
    second-nearest box points:
      [i]      W_ii / mean_j W_jj
      [16+i]   Re (c_i - b_i),   [32+i]  Im (c_i - b_i)
      [48+i]   W_ii^2 (d1_i - d0_i) / mean_j W_jj^2
    Slots of levels >= N are zero.  Also returns the smallest gap between the
    first and second distances along the walk (near 0: the rank-0 choice is
    close to a tie and float32 may walk another path; d1 itself does not
    depend on which of two equally far points is second)."""
    W = np.asarray(W, dtype=np.complex128)
    perm = np.asarray(perm, dtype=np.int64)
    s = np.asarray(s, dtype=np.complex128)
    if s.ndim == 1:
        s = s[:, None]
    n, V = s.shape
    d = np.real(np.diag(W))
    resid = (W @ s[perm, :]).T
    f = np.zeros((V, N_FEATURES))
    f[:, :n] = d[None, :] / d.mean()
    gap = np.full(V, np.inf)
    for i in range(n):
        c = -resid[:, i] / (tau * W[i, i])
        dist = sqabs(c[:, None] - BOX[None, :])
        order = np.argsort(dist, axis=1, kind="stable")
        ds = np.take_along_axis(dist, order, axis=1)
        b = BOX[order[:, 0]]
        f[:, 16 + i] = (c - b).real
        f[:, 32 + i] = (c - b).imag
        f[:, 48 + i] = d[i] ** 2 * (ds[:, 1] - ds[:, 0]) / np.mean(d ** 2)
        gap = np.minimum(gap, ds[:, 1] - ds[:, 0])
        if i + 1 < n:
            resid[:, i + 1:] += tau * W[None, i + 1:, i] * b[:, None]
    return f, gap


def path_ranks(W, perm, s, tau, l):
    """Position vector of given perturbations (the inverse of the rank walk).

    l: complex [N][V] (user order, entries in the B = 1 box).  Walks each
    vector's tree along l and returns (ranks int [V][N], margin [V]): the rank
    of l_{perm[i]} among the nine box points ordered by distance to the level
    centre c_i (ties by canonical index j), and the smallest gap between the
    chosen point's distance and a neighbouring rank's distance (how close the
    rank is to a tie).  A symbol outside the box gets rank 15."""
    W = np.asarray(W, dtype=np.complex128)
    perm = np.asarray(perm, dtype=np.int64)
    s = np.asarray(s, dtype=np.complex128)
    l = np.asarray(l, dtype=np.complex128)
    if s.ndim == 1:
        s, l = s[:, None], l[:, None]
    n, V = s.shape
    st = (W @ s[perm, :]).T
    lp = l[perm, :].T                           # level order [V][N]
    resid = st.copy()
    ranks = np.zeros((V, n), dtype=np.int64)
    margin = np.full(V, np.inf)
    for i in range(n):
        c = -resid[:, i] / (tau * W[i, i])
        dist = sqabs(c[:, None] - BOX[None, :])
        order = np.argsort(dist, axis=1, kind="stable")
        pos = np.argmax(BOX[order] == lp[:, i:i + 1], axis=1)
        found = np.any(BOX[order] == lp[:, i:i + 1], axis=1)
        ranks[:, i] = np.where(found, pos, 15)
        ds = np.take_along_axis(dist, order, axis=1)
        r = np.minimum(pos, 8)
        lo = np.where(r > 0, ds[np.arange(V), r] - ds[np.arange(V), np.maximum(r - 1, 0)], np.inf)
        hi = np.where(r < 8, ds[np.arange(V), np.minimum(r + 1, 8)] - ds[np.arange(V), r], np.inf)
        margin = np.minimum(margin, np.minimum(lo, hi))
        if i + 1 < n:
            resid[:, i + 1:] += tau * W[None, i + 1:, i] * lp[:, i:i + 1]
    return ranks, margin


def walk_ranks(W, perm, s, tau, ranks):
    """l (complex [N][V], user order) reached by walking each vector's own
    position vector (ranks int [V][N]) -- one path per vector."""
    W = np.asarray(W, dtype=np.complex128)
    perm = np.asarray(perm, dtype=np.int64)
    s = np.asarray(s, dtype=np.complex128)
    n, V = s.shape
    st = (W @ s[perm, :]).T
    out = np.zeros((n, V), dtype=np.complex128)
    for v in range(V):
        lv, _, _ = demap_walk(W, st[v:v + 1], tau, np.asarray(ranks[v:v + 1], dtype=np.int64))
        out[perm, v] = lv[0, 0]
    return out


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

class Params(NamedTuple):
    W1: np.ndarray   # [256][64]  (out, in)
    b1: np.ndarray
    W2: np.ndarray   # [256][256]
    b2: np.ndarray
    W3: np.ndarray   # [V][256]
    b3: np.ndarray


class Cache(NamedTuple):
    x: np.ndarray
    z1: np.ndarray
    h1: np.ndarray
    z2: np.ndarray
    h2: np.ndarray
    z3: np.ndarray


def relu(x):
    return np.maximum(x, 0.0)


def mlp_forward(x, p: Params, round_hidden: bool = False) -> Cache:
    """z1 = x W1^T + b1, h1 = relu(z1), z2 = h1 W2^T + b2, h2 = relu(z2),
    z3 = h2 W3^T + b3 (logits).  round_hidden rounds h1 and h2 to bf16, where
    the GPU stores them in bf16."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p.W1.T + p.b1
    h1 = relu(z1)
    if round_hidden:
        h1 = bf16_round(h1)
    z2 = h1 @ p.W2.T + p.b2
    h2 = relu(z2)
    if round_hidden:
        h2 = bf16_round(h2)
    z3 = h2 @ p.W3.T + p.b3
    return Cache(x, z1, h1, z2, h2, z3)


def softmax_xent(z, labels):
    """Per row: loss = logsumexp(z) - z[y], grad = softmax(z) - onehot(y); a row
    whose label is outside [0, C) has loss 0 and gradient 0."""
    z = np.asarray(z, dtype=np.float64)
    labels = np.asarray(labels, dtype=np.int64)
    rows, C = z.shape
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    lse = m[:, 0] + np.log(e.sum(axis=1))
    p = e / e.sum(axis=1, keepdims=True)
    use = (labels >= 0) & (labels < C)
    yy = np.where(use, labels, 0)
    loss = np.where(use, lse - z[np.arange(rows), yy], 0.0)
    g = p.copy()
    g[np.arange(rows), yy] -= 1.0
    g[~use] = 0.0
    return loss, g


class Grads(NamedTuple):
    dW1: np.ndarray
    db1: np.ndarray
    dW2: np.ndarray
    db2: np.ndarray
    dW3: np.ndarray
    db3: np.ndarray
    dx: np.ndarray


def mlp_backward(c: Cache, p: Params, dz3, round_hidden_grad: bool = False) -> Grads:
    """Reverse pass of mlp_forward for the upstream gradient dz3 = dL/dz3:
      dW3 = dz3^T h2, db3 = sum_rows dz3, dh2 = dz3 W3, dz2 = dh2 [z2 > 0]
      dW2 = dz2^T h1, db2 = sum_rows dz2, dh1 = dz2 W2, dz1 = dh1 [z1 > 0]
      dW1 = dz1^T x,  db1 = sum_rows dz1, dx = dz1 W1
    round_hidden_grad rounds dz2 and dz1 to bf16, where the GPU stores them."""
    dz3 = np.asarray(dz3, dtype=np.float64)
    dW3 = dz3.T @ c.h2
    db3 = dz3.sum(axis=0)
    dz2 = (dz3 @ p.W3) * (c.z2 > 0)
    if round_hidden_grad:
        dz2 = bf16_round(dz2)
    dW2 = dz2.T @ c.h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ p.W2) * (c.z1 > 0)
    if round_hidden_grad:
        dz1 = bf16_round(dz1)
    dW1 = dz1.T @ c.x
    db1 = dz1.sum(axis=0)
    dx = dz1 @ p.W1
    return Grads(dW1, db1, dW2, db2, dW3, db3, dx)


def mean_loss(x, labels, p: Params) -> float:
    loss, _ = softmax_xent(mlp_forward(x, p).z3, labels)
    n = max(int(np.sum((np.asarray(labels) >= 0) & (np.asarray(labels) < p.W3.shape[0]))), 1)
    return float(loss.sum() / n)


# ---------------------------------------------------------------------------
# selection
# ---------------------------------------------------------------------------

def total_order_key(x) -> np.ndarray:
    """Integer key of float32 values that is increasing in the IEEE total order
    (-0 below +0; NaNs beyond the infinities by their sign)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.int64)
    return np.where(u & 0x80000000, 0xFFFFFFFF - u, u | 0x80000000)


def topk(scores, k: int = 64) -> np.ndarray:
    """Columns of the k largest entries of each row, by decreasing value, equal
    values by increasing column."""
    s = np.asarray(scores, dtype=np.float32)
    key = total_order_key(s)
    rows, C = s.shape
    out = np.zeros((rows, k), dtype=np.int64)
    cols = np.arange(C)
    for r in range(rows):
        order = np.lexsort((cols, -key[r]))      # primary: key desc; secondary: column asc
        out[r] = order[:k]
    return out


def softmax_mass(scores, sel) -> np.ndarray:
    """sum_{c in sel} softmax(scores)_c per row."""
    z = np.asarray(scores, dtype=np.float64)
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    return np.take_along_axis(e, np.asarray(sel), axis=1).sum(axis=1) / e.sum(axis=1)


def init_params(rng: np.random.Generator, V: int, n_in: int = N_FEATURES, hidden: int = 256,
                dtype_round: Optional[str] = "bf16") -> Params:
    """Seeded weights of the network's shape (He-uniform), optionally rounded
    to bf16 so that the GPU and this oracle hold the same values."""
    def lin(o, i):
        b = np.sqrt(6.0 / i)
        return rng.uniform(-b, b, size=(o, i)), rng.uniform(-0.1, 0.1, size=o)
    W1, b1 = lin(hidden, n_in)
    W2, b2 = lin(hidden, hidden)
    W3, b3 = lin(V, hidden)
    if dtype_round == "bf16":
        W1, W2, W3 = bf16_round(W1), bf16_round(W2), bf16_round(W3)
        b1, b2, b3 = [np.asarray(b, np.float32).astype(np.float64) for b in (b1, b2, b3)]
    return Params(W1, b1, W2, b2, W3, b3)
