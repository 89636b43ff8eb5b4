"""Training and evaluation of the learned path proposal.

Labels.  For every training vector the exact perturbation over the B = 1 box
(the sphere encoder of vp_sphere_encode, seeded with the radius of the fixed
512-path search) is mapped to its position vector by vp_path_ranks; the V
most frequent position vectors form the vocabulary, and a vector's label is
its position vector's vocabulary index (-1 when it is not in the vocabulary:
such vectors are left out of the loss, and the coverage is reported).

Training.  Softmax cross-entropy (vp_softmax_xent) over the network of
learn.MLPFunction, whose forward and backward run on vp_gemm_bf16; torch's
Adam updates float32 master weights, which are rounded to bf16 for every
step.  Input distribution: the 16 x 16, 256-QAM, rho = 0.5 correlated channel
with alpha = 0.16, on its own seeds (disjoint from the evaluation seed).

Usage:  python -m paper_2602_12098_amd.train --out WEIGHTS.safetensors
"""
from __future__ import annotations

import argparse
import json
import math
import time
from typing import Optional

import numpy as np
import torch

import vpgen

from . import learn
from . import vp

DEV = "cuda:0"


def _log(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------
# labelled data
# ---------------------------------------------------------------------------

@torch.no_grad()
def label_chunk(wl, K_fixed: int = 512, max_nodes: int = 1 << 22, kind: int = learn.VP_FEAT_RANK0_WALK,
                residual_k: int = 0):
    """Features, exact position-vector words and costs for one workload chunk.
    With residual_k > 0, vectors whose exact solution is already reached by
    the first residual_k MoP paths get the word -1 (no label): the network is
    then trained on what those paths miss."""
    Hd = torch.from_numpy(wl.H).to(DEV)
    sd = torch.from_numpy(wl.s).to(DEV)
    prep = vp.preprocess(Hd, wl.alpha, want_G=False)
    order = torch.empty((wl.n_sc, 2, K_fixed), dtype=torch.int16, device=DEV)
    paths = vp.paths_mop(prep.w2, K_fixed, order=order)
    fx = vp.search(prep.W, prep.perm, sd, wl.tau, paths, wl.n_sym, order=order)
    se = vp.sphere_encode(prep.W, prep.perm, sd, wl.tau, wl.n_sym, radius=fx.cost * (1 + 1e-6),
                          max_nodes=max_nodes)
    # where the encoder found nothing better inside the radius (or ran out of
    # budget), the fixed-set solution is the label
    bad = ~torch.isfinite(se.cost)
    l = torch.where(bad[None, :, None], fx.l, se.l)
    cost_exact = torch.where(bad, fx.cost, se.cost)
    ranks = learn.path_ranks(prep.W, prep.perm, sd, wl.tau, l, wl.n_sym)
    feats = learn.mlp_features(prep.W, prep.perm, sd, wl.tau, wl.n_sym, kind=kind)
    words = learn.pack_ranks(ranks)
    if residual_k > 0:
        part = vp.search(prep.W, prep.perm, sd, wl.tau, paths[:, :residual_k].contiguous(), wl.n_sym)
        covered = part.cost <= cost_exact * (1 + 1e-6)
        words = torch.where(covered, torch.full_like(words, -1), words)
    return feats, words, fx.cost, cost_exact


def make_dataset(n_vec: int, seed0: int = 50, chunk_sc: int = 4000, kind: int = learn.VP_FEAT_RANK0_WALK,
                 residual_k: int = 0):
    """n_vec labelled vectors of the 16 x 16 256-QAM correlated workload."""
    feats, words = [], []
    done, shard = 0, 0
    t0 = time.time()
    while done < n_vec:
        n_sc = min(chunk_sc, math.ceil((n_vec - done) / 14))
        wl = vpgen.make(f"train{shard}", 16, 16, n_sc, 14, 256, 0.16, 512, seed=seed0 + shard, rho=0.5)
        f, w, _, _ = label_chunk(wl, kind=kind, residual_k=residual_k)
        feats.append(f)
        words.append(w)
        done += wl.n_vec
        shard += 1
        _log(f"labels {done}/{n_vec}  {time.time() - t0:.1f}s")
    return torch.cat(feats)[:n_vec], torch.cat(words)[:n_vec]


def build_vocab(words: torch.Tensor, V: int = 4096, N: int = 16):
    """The V most frequent words (equal counts: smaller word first) as uint8
    rank rows [V][N], and each word's vocabulary index (-1 if absent)."""
    uniq, counts = torch.unique(words[words >= 0], return_counts=True)
    # sort by (count desc, word asc): unique() returns words ascending, a stable sort keeps that
    order = torch.sort(counts, descending=True, stable=True).indices
    top = uniq[order[:V]]
    V = top.numel()
    sh = 4 * torch.arange(N, device=words.device, dtype=torch.int64)
    vocab = ((top[:, None] >> sh[None, :]) & 15).to(torch.uint8).contiguous()
    srt, perm = torch.sort(top)
    pos = torch.searchsorted(srt, words).clamp_max(V - 1)
    hit = (srt[pos] == words) & (words >= 0)
    labels = torch.where(hit, perm[pos], torch.full_like(pos, -1)).to(torch.int32)
    coverage = float(hit.float().sum() / (words >= 0).float().sum().clamp_min(1))
    return vocab, labels, coverage


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------

def init_params(V: int, seed: int = 0):
    g = torch.Generator(device="cpu").manual_seed(seed)

    def lin(o, i):
        b = math.sqrt(6.0 / i)
        W = (torch.rand((o, i), generator=g) * 2 - 1) * b
        bb = (torch.rand((o,), generator=g) * 2 - 1) * 0.01
        return W.to(DEV).requires_grad_(True), bb.to(DEV).requires_grad_(True)

    W1, b1 = lin(learn.HIDDEN, learn.N_FEATURES)
    W2, b2 = lin(learn.HIDDEN, learn.HIDDEN)
    W3, b3 = lin(V, learn.HIDDEN)
    return [W1, b1, W2, b2, W3, b3]


@torch.no_grad()
def mean_loss(params, feats, labels, batch=8192):
    tot, n = 0.0, 0
    for b in range(0, feats.shape[0], batch):
        y = labels[b:b + batch].contiguous()
        z = learn.MLPFunction.forward(learn._NoCtx(), feats[b:b + batch].contiguous(), *params)
        loss, _ = learn.softmax_xent(z, y, 1.0)
        tot += float(loss.sum())
        n += int((y >= 0).sum())
    return tot / max(n, 1)


def train(feats, labels, V, epochs=20, batch=4096, lr=2e-3, seed=0, val_frac=0.02):
    params = init_params(V, seed)
    opt = torch.optim.Adam(params, lr=lr)
    n_val = int(feats.shape[0] * val_frac)
    vf, vl = feats[-n_val:], labels[-n_val:]
    labels = labels[:-n_val] if n_val else labels
    use = torch.nonzero(labels >= 0).squeeze(1)
    n = use.numel()
    steps = epochs * (n // batch)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr, total_steps=max(steps, 1), pct_start=0.05)
    g = torch.Generator(device=DEV).manual_seed(seed)
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = use[torch.randperm(n, device=DEV, generator=g)]
        tot, cnt = 0.0, 0
        for b in range(n // batch):
            idx = perm[b * batch:(b + 1) * batch]
            x = feats[idx].contiguous()
            y = labels[idx].contiguous()
            z = learn.MLPFunction.apply(x, *params)   # float32 masters, rounded to bf16 inside
            loss = learn.SoftmaxXentFunction.apply(z, y)
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            sched.step()
            step += 1
            tot += float(loss.item()) if (b % 20 == 0) else 0.0
            cnt += 1 if (b % 20 == 0) else 0
        vloss = mean_loss(params, vf, vl) if n_val else float("nan")
        _log(f"epoch {ep + 1}/{epochs} loss {tot / max(cnt, 1):.4f} val {vloss:.4f}  {time.time() - t0:.1f}s")
    return learn.MLPParams(*[t.detach() for t in params])


def save(path: str, params: learn.MLPParams, vocab: torch.Tensor, meta: dict):
    from safetensors.torch import save_file
    t = {k: v.detach().to(torch.bfloat16 if v.dim() == 2 else torch.float32).cpu().contiguous()
         for k, v in params._asdict().items()}
    t["vocab"] = vocab.cpu().contiguous()
    save_file(t, path, metadata={k: str(v) for k, v in meta.items()})


def load(path: str, device: str = DEV) -> learn.Proposer:
    return learn.load_proposer(path, device)


# ---------------------------------------------------------------------------
# evaluation
# ---------------------------------------------------------------------------

@torch.no_grad()
def evaluate(prop: learn.Proposer, wl, K_fixed_fallback: int = 512, K_mop: int = 8,
             thetas=(0.0, 0.3, 0.5, 0.7, 0.8, 0.9, 0.95), K_mop_sweep=(0, 8, 32, 64, 128, 192)):
    """Power gaps (dB) to exact VP of: l = 0, fixed K=64 and K=512 MoP sets,
    the learned 64 + K_mop proposal, and the proposal with a fallback to the
    fixed 512 set for vectors whose top-64 softmax mass is below theta."""
    Hd = torch.from_numpy(wl.H).to(DEV)
    sd = torch.from_numpy(wl.s).to(DEV)
    prep = vp.preprocess(Hd, wl.alpha, want_G=False)
    order = torch.empty((wl.n_sc, 2, K_fixed_fallback), dtype=torch.int16, device=DEV)
    paths = vp.paths_mop(prep.w2, K_fixed_fallback, order=order)
    fx = vp.search(prep.W, prep.perm, sd, wl.tau, paths, wl.n_sym, order=order)
    o64 = torch.empty((wl.n_sc, 2, 64), dtype=torch.int16, device=DEV)
    p64 = vp.paths_mop(prep.w2, 64, order=o64)
    f64 = vp.search(prep.W, prep.perm, sd, wl.tau, p64, wl.n_sym, order=o64)
    se = vp.sphere_encode(prep.W, prep.perm, sd, wl.tau, wl.n_sym, radius=fx.cost * (1 + 1e-6))
    exact = torch.where(torch.isfinite(se.cost), se.cost, fx.cost).double()
    table, mass = prop.propose(prep.W, prep.perm, sd, wl.tau, wl.n_sym, fixed_paths=paths, K_fixed=K_mop)
    K = table.shape[1]
    lr = vp.search(prep.W, prep.perm, sd, wl.tau, table, wl.n_sym,
                   flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
    zero = torch.zeros_like(fx.l)
    z0 = vp.search(prep.W, prep.perm, sd, wl.tau, torch.zeros((1, wl.N), dtype=torch.uint8, device=DEV),
                   wl.n_sym)   # rank-0 path + zero perturbation
    del zero
    E = float(exact.sum())

    def gap(c):
        return 10 * math.log10(float(c.double().sum()) / E)

    res = {"n_vec": wl.n_vec, "K_learned_table": K,
           "gap_babai_or_zero_db": gap(z0.cost), "gap_fixed64_db": gap(f64.cost), "gap_fixed512_db": gap(fx.cost),
           "gap_learned_db": gap(lr.cost), "mass_median": float(mass.median())}
    fb = {}
    for th in thetas:
        sel = mass < th
        c = torch.where(sel, torch.minimum(lr.cost, fx.cost), lr.cost)
        fb[str(th)] = {"fallback_frac": float(sel.float().mean()), "gap_db": gap(c)}
    res["fallback"] = fb
    # learned 64 + the first k MoP paths, against fixed MoP sets of equal size
    sweep = {}
    for k in K_mop_sweep:
        t, _ = prop.propose(prep.W, prep.perm, sd, wl.tau, wl.n_sym, fixed_paths=paths, K_fixed=k)
        r = vp.search(prep.W, prep.perm, sd, wl.tau, t, wl.n_sym, flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
        Kt = 64 + k
        ot = torch.empty((wl.n_sc, 2, Kt), dtype=torch.int16, device=DEV)
        pf = vp.paths_mop(prep.w2, Kt, order=ot)
        fr = vp.search(prep.W, prep.perm, sd, wl.tau, pf, wl.n_sym, order=ot)
        sweep[str(k)] = {"paths": Kt, "gap_learned_db": gap(r.cost), "gap_fixed_same_K_db": gap(fr.cost)}
    res["mop_sweep"] = sweep
    return res


def main(argv: Optional[list] = None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=1_000_000)
    ap.add_argument("--vocab", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-sc", type=int, default=3276)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    ap.add_argument("--features", type=int, default=learn.VP_FEAT_RANK0_WALK, choices=(0, 1))
    ap.add_argument("--residual-k", type=int, default=0)
    a = ap.parse_args(argv)
    t0 = time.time()
    feats, words = make_dataset(a.n_train, kind=a.features, residual_k=a.residual_k)
    vocab, labels, cov = build_vocab(words, a.vocab)
    _log(f"vocabulary {vocab.shape[0]} entries, coverage {cov:.4f}, distinct {torch.unique(words).numel()}")
    params = train(feats, labels, vocab.shape[0], epochs=a.epochs, batch=a.batch, lr=a.lr)
    meta = {"feature_kind": a.features, "residual_k": a.residual_k, "n_train": a.n_train, "vocab": int(vocab.shape[0]), "coverage": cov, "epochs": a.epochs,
            "batch": a.batch, "lr": a.lr, "train_seeds": "50..", "workload": "16x16 rho0.5 256QAM alpha0.16"}
    save(a.out, params, vocab, meta)
    prop = load(a.out)
    wl = vpgen.cfg3(512, n_sc=a.eval_sc)
    rep = evaluate(prop, wl)
    rep.update(meta)
    rep["seconds"] = time.time() - t0
    _log(json.dumps(rep, indent=1))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
