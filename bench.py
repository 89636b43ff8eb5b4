#!/usr/bin/env python3
"""Benchmark: precoded vectors/s of the whole ViPer NL-COMM VP hot path on one MI355X.

One step = one slot of the 16x16 256-QAM workload (3276 subcarriers x 14
symbols, correlated rho = 0.5 channels, alpha = 0.16, K = 512 MoP paths):
per-subcarrier preprocessing, MoP path selection, the per-vector search over
the 512 paths with its argmin, and the precoding x = G (s + tau l).  Inputs
are resident in HBM before the timed region; outputs are preallocated.

Prints one JSON line (rank 0).  Extra fields: per-stage times, the roofline of
the dominant kernel (the path search, VALU-bound), and the FP64 CPU oracle
timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "precoded vectors/s at 16×16 256-QAM, 512 paths; power gap to exact VP (dB)"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 VALU lane-ops/s; an FP32
# FMA is 2 flop -> 78.6 TFLOP/s without packed-FP32 instructions (not used here).
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
FLOP_PER_CM = 6   # one complex multiplication: 4 real multiplies + 2 adds


def search_cm_per_vector(n_t, K):
    """Path-search part of the paper's per-vector count (Sec. III-B): K N_t (1 + (N_t+1)/2)."""
    return K * n_t * (n_t + 3) // 2


def _cpu_worker(args):
    sc_list, wl_seed, K = args
    import vpgen
    from oracle import vp_oracle as O
    wl = vpgen.cfg3(K)
    t0 = time.perf_counter()
    nv = 0
    for sc in sc_list:
        p = O.preprocess(wl.H[sc], wl.alpha)
        paths = O.mop_paths_kbest(p.w2, K)
        sl = slice(sc * wl.n_sym, (sc + 1) * wl.n_sym)
        res = O.search_paths(p.W, p.perm, wl.s[:, sl], wl.tau, paths)
        for v in range(wl.n_sym):
            O.precode(p.G, wl.s[:, sl][:, v], res.l[v], wl.tau)
        nv += wl.n_sym
    return nv, time.perf_counter() - t0


def cpu_baseline(K, budget_s=12.0):
    """FP64 oracle (numpy) on a bounded sample of subcarriers, all host cores."""
    import multiprocessing as mp
    cores = os.cpu_count() or 1
    cores = min(cores, 16)
    # calibrate on one subcarrier, then size the sample to ~budget_s of wall time
    nv, dt = _cpu_worker(([0], 3, K))
    per_sc = dt
    n_sc = int(max(cores, min(3276, budget_s * cores / per_sc)))
    n_sc = min(n_sc, 3275)
    scs = list(range(1, 1 + n_sc))
    chunks = [scs[i::cores] for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(c, 3, K) for c in chunks])
    wall = time.perf_counter() - t0
    nvec = sum(r[0] for r in res)
    return {"value": nvec / wall, "unit": "vectors/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_sc} of 3276 subcarriers x 14 symbols (16x16, K={K}), full pipeline "
                      f"(preprocess, K-best MoP, path search, precode) in float64 numpy, "
                      f"{cores} processes, {wall:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--K", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by "
              "subcarrier with no exchange, see the design notes", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_12098_amd as vp
    import vpgen

    dev = "cuda:0"
    wl = vpgen.cfg3(args.K)
    N, M, n_sc, n_sym, K = wl.N, wl.M, wl.n_sc, wl.n_sym, args.K
    n_vec = n_sc * n_sym
    H = torch.from_numpy(wl.H).to(dev)
    s = torch.from_numpy(wl.s).to(dev)
    prep = vp.Prep(torch.empty((n_sc, vp.packed_size(N)), dtype=torch.complex64, device=dev),
                   torch.empty((n_sc, N), dtype=torch.float32, device=dev),
                   torch.empty((n_sc, N), dtype=torch.uint8, device=dev),
                   torch.empty((n_sc, M, N), dtype=torch.complex64, device=dev),
                   torch.empty((n_sc,), dtype=torch.int32, device=dev))
    paths = torch.empty((n_sc, K, N), dtype=torch.uint8, device=dev)
    order = torch.empty((n_sc, 2, K), dtype=torch.int16, device=dev)
    sout = vp.SearchOut(torch.empty((N, n_vec, 2), dtype=torch.int8, device=dev),
                        torch.empty((n_vec,), dtype=torch.float32, device=dev),
                        torch.empty((n_vec,), dtype=torch.int32, device=dev))
    x = torch.empty((n_vec, M), dtype=torch.complex64, device=dev)

    def step(ev=None):
        if ev: ev[0].record()
        vp.preprocess(H, wl.alpha, out=prep)
        if ev: ev[1].record()
        vp.paths_mop(prep.w2, K, out=paths, order=order)
        if ev: ev[2].record()
        vp.search(prep.W, prep.perm, s, wl.tau, paths, n_sym, out=sout, order=order)
        if ev: ev[3].record()
        vp.precode(prep.G, s, sout.l, wl.tau, sout.cost, n_sym, P_T=1.0, out=x)
        if ev: ev[4].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_names = ["preprocess", "paths_mop", "search", "precode"]
    stage = {n: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(args.steps)]))
             for i, n in enumerate(stage_names)}
    ms_step = float(np.mean([evs[k][0].elapsed_time(evs[k][4]) for k in range(args.steps)]))
    value = n_vec * args.steps / wall
    assert bool(torch.all(prep.status == 0)), "preprocessing failed on some subcarrier"

    flops = search_cm_per_vector(M, K) * FLOP_PER_CM * n_vec
    achieved = flops / (stage["search"] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_TFLOPS, "traffic": None,
            "kernel": "vp_search (k_search_trie + k_search_finalize)",
            "work": f"{search_cm_per_vector(M, K)} complex mult/vector x {FLOP_PER_CM} flop x {n_vec} vectors"}

    line = {
        "metric": METRIC, "value": value, "unit": "vectors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "N": N, "M": M, "n_sc": n_sc, "n_sym": n_sym, "K": K, "Q": wl.Q,
                   "alpha": wl.alpha, "rho": wl.rho, "seed": wl.seed},
        "event_ms_per_step": ms_step, "stages_ms": stage, "roofline": roof,
        "gap_db": None,
    }
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(K)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
