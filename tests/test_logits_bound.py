"""The bound behind vp_logits_top64 (host model of the rule, no GPU): for each
row, the vocabulary is split four ways by 32-row blocks (split q: blocks
b % 4 == q) and each split into 32 groups by the row within the block; the
two largest logits of every group, truncated to the top 16 bits of their
order-preserving key, give a bound -- the value of their 64th largest key --
that at least 64 logits reach, so the logits below it are never among the
64 largest.  Checked against the oracle's top-64 on logits with ties, signed
zeros, NaNs and heavy tails."""
import numpy as np
import pytest

from oracle import mlp_oracle as L


def okey(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return np.where(u & 0x80000000, 0xFFFFFFFF - u, u | 0x80000000).astype(np.uint64)


def key_value(k):
    k = np.asarray(k, np.uint64)
    u = np.where(k & 0x80000000, k & 0x7FFFFFFF, 0xFFFFFFFF - k).astype(np.uint32)
    return u.view(np.float32)


def bound(z):
    """The rule for one row z (float32 [V], V a multiple of 128)."""
    V = z.shape[0]
    blocks = z.reshape(V // 32, 32)
    zs = np.where(np.isnan(blocks), -np.inf, blocks).astype(np.float32)   # NaN counts as -inf in the statistics
    keys = []
    for q in range(4):
        g = np.sort(zs[q::4], axis=0)[::-1][:2]      # the two largest of each group (row within the block)
        keys.append(okey(g).ravel() >> 16)           # truncated 16-bit keys
    keys = np.sort(np.concatenate(keys))[::-1]
    return key_value(keys[63] << 16)


@pytest.mark.parametrize("kind", ["normal", "ties", "zeros", "heavy", "nan", "skewed"])
@pytest.mark.parametrize("V", [256, 1024, 4096])
def test_bound_keeps_the_top64(kind, V):
    rng = np.random.default_rng(V + len(kind))
    rows = 40
    z = rng.standard_normal((rows, V)).astype(np.float32)
    if kind == "ties":
        z = np.round(z * 2).astype(np.float32) / 2
    elif kind == "zeros":
        z = np.where(rng.random((rows, V)) < 0.5, np.float32(0.0), np.float32(-0.0)).astype(np.float32)
        z[:, ::9] = -1.0
    elif kind == "heavy":
        z = (rng.standard_cauchy((rows, V)) * 3).astype(np.float32)
    elif kind == "nan":
        z[:, ::97] = np.nan
    elif kind == "skewed":
        z[:, (np.arange(V) // 32) % 4 == 1] += 4.0
    top = L.topk(z, 64)
    for r in range(rows):
        T = bound(z[r])
        cand = ~(z[r] < T)                 # the pass-2 test (NaN is always a candidate)
        assert not np.isnan(T) and int(np.sum(cand)) >= 64
        assert np.all(cand[top[r]]), (kind, V, r)


def test_truncated_keys_never_exceed_the_value():
    # the validity argument: a truncated key, extended by zeros, is at most the
    # value's own key, and key_value inverts okey
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, -0.0, np.inf, -np.inf, 1e-38, -1e-38])])
    k = okey(x)
    assert np.all(((k >> 16) << 16) <= k)
    np.testing.assert_array_equal(key_value(k).view(np.uint32), x.view(np.uint32))
