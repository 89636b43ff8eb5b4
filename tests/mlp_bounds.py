"""Element-wise error bounds of the float32 / bf16 network arithmetic against
the exact float64 oracle (test infrastructure).

Model of the GPU arithmetic (vp_gemm_bf16): products of bf16 operands are
exact in float32; a k-term float32 sum, the alpha scaling and the bias add
stay within (k + 2) u sum |a_i b_i| + u |bias| of the exact value (u = 2^-24
per rounding, doubled here for slack); a value stored as bf16 moves by at
most 2^-8 of its magnitude (half an ulp of an 8-bit significand).  A ReLU is
1-Lipschitz; a ReLU mask whose pre-activation lies within its own error bound
of 0 may go either way, so there the bound admits the whole unmasked value.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
BF = 2.0 ** -8


def gam(k: int) -> float:
    return 2.0 * (k + 2) * U32


def gemm_bound(Aabs, Babs, k, bias_abs=None):
    b = gam(k) * (Aabs @ Babs)
    if bias_abs is not None:
        b = b + 2 * U32 * bias_abs
    return b


def forward_bounds(c, p):
    """c: oracle Cache of the exact forward (no rounding); p: Params (bf16
    values).  Returns dict of element-wise bounds |gpu - exact| for h1, h2, z3
    and the masks' certainty (True where the ReLU decision cannot flip)."""
    aW1, aW2, aW3 = np.abs(p.W1), np.abs(p.W2), np.abs(p.W3)
    e_z1 = gam(p.W1.shape[1]) * (np.abs(c.x) @ aW1.T + np.abs(p.b1))
    e_h1 = e_z1 + BF * (np.abs(c.h1) + e_z1)
    H1 = np.abs(c.h1) + e_h1
    e_z2 = e_h1 @ aW2.T + gam(p.W2.shape[1]) * (H1 @ aW2.T + np.abs(p.b2))
    e_h2 = e_z2 + BF * (np.abs(c.h2) + e_z2)
    H2 = np.abs(c.h2) + e_h2
    e_z3 = e_h2 @ aW3.T + gam(p.W3.shape[1]) * (H2 @ aW3.T + np.abs(p.b3))
    sure1 = np.abs(c.z1) > e_z1
    sure2 = np.abs(c.z2) > e_z2
    return dict(e_h1=e_h1, e_h2=e_h2, e_z3=e_z3, H1=H1, H2=H2, sure1=sure1, sure2=sure2)


def backward_bounds(c, p, dz3, fb):
    """Bounds of the GPU gradients against the exact float64 backward of the
    exact forward, for the same bf16 upstream gradient dz3."""
    rows = dz3.shape[0]
    ad3 = np.abs(dz3)
    aW1, aW2, aW3 = np.abs(p.W1), np.abs(p.W2), np.abs(p.W3)
    e_dW3 = ad3.T @ fb["e_h2"] + gam(rows) * (ad3.T @ fb["H2"])
    e_db3 = gam(rows) * ad3.sum(axis=0)
    pre2 = dz3 @ p.W3                               # exact unmasked dh2
    e_pre2 = gam(p.W3.shape[0]) * (ad3 @ aW3)
    dz2 = pre2 * (c.z2 > 0)
    e_dz2 = np.where(fb["sure2"], e_pre2, np.abs(pre2) + e_pre2)
    e_dz2 = e_dz2 + BF * (np.abs(dz2) + e_dz2)
    D2 = np.abs(dz2) + e_dz2
    e_dW2 = e_dz2.T @ fb["H1"] + np.abs(dz2).T @ fb["e_h1"] + gam(rows) * (D2.T @ fb["H1"])
    e_db2 = e_dz2.sum(axis=0) + gam(rows) * D2.sum(axis=0)
    pre1 = dz2 @ p.W2
    e_pre1 = e_dz2 @ aW2 + gam(p.W2.shape[0]) * (D2 @ aW2)
    dz1 = pre1 * (c.z1 > 0)
    e_dz1 = np.where(fb["sure1"], e_pre1, np.abs(pre1) + e_pre1)
    e_dz1 = e_dz1 + BF * (np.abs(dz1) + e_dz1)
    D1 = np.abs(dz1) + e_dz1
    ax = np.abs(c.x)
    e_dW1 = e_dz1.T @ ax + gam(rows) * (D1.T @ ax)
    e_db1 = e_dz1.sum(axis=0) + gam(rows) * D1.sum(axis=0)
    return dict(dW3=e_dW3, db3=e_db3, dW2=e_dW2, db2=e_db2, dW1=e_dW1, db1=e_db1)
