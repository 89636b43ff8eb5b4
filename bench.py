#!/usr/bin/env python3
"""Benchmark: precoded vectors/s of the whole ViPer NL-COMM VP hot path on one MI355X.

One step = one slot of the 16x16 256-QAM workload (3276 subcarriers x 14
symbols, correlated rho = 0.5 channels, alpha = 0.16, K = 512 MoP paths):
per-subcarrier preprocessing, MoP path selection, the per-vector search over
the 512 paths with its argmin, and the precoding x = G (s + tau l).  Inputs
are resident in HBM before the timed region; outputs are preallocated.

Prints one JSON line (rank 0).  Extra fields: per-stage times, the power gap
to exact VP (GPU sphere encoder, outside the timed region), the roofline of
the dominant kernel (the path search, VALU-bound) with its HBM traffic from
committed counter profiles, the FP64 CPU oracle timed on a bounded sample of
the same workload on the host cores, and two further measured forms of the
path: the batched uneven RBG slot (one graph, autotuned, against per-size
launches) and the learned per-vector path proposal.
"""
import argparse
import hashlib
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


SEARCH_SOURCES = ["paper_2602_12098_amd/csrc/vp_search.hip", "paper_2602_12098_amd/csrc/vp_walk.hpp",
                  "paper_2602_12098_amd/csrc/vp_device.hpp", "paper_2602_12098_amd/csrc/demap_lut.h"]
TRAFFIC_FILE = "profiles/k_search_trie_16x16_256qam_K512.traffic.json"


def search_traffic(K):
    """HBM bytes per launch of the search kernel from the committed counter
    profile (taken at K = 512), or None when it is missing, K differs or the
    kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None, "no traffic profile"
    if K != 512:
        return None, "the counters were taken at K = 512"
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec.get("source_files", SEARCH_SOURCES):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None, "kernel changed since the counters were taken"
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"], TRAFFIC_FILE


def gap_to_exact(vp, prep, s, tau, n_sym, cost):
    """Power gap (dB) of the selected perturbations to exact VP over the box:
    the sphere encoder seeded with each vector's own cost as radius."""
    import torch
    se = vp.sphere_encode(prep.W, prep.perm, s, tau, n_sym, radius=cost * (1 + 1e-6))
    exact = torch.where(torch.isfinite(se.cost), se.cost, cost).double()
    return 10 * math.log10(float(cost.double().sum()) / float(exact.sum())), exact


def rzf_powers(prep, s, n_sym):
    """gamma of linear RZF (l = 0) per vector: ||W s_pi||^2, from the packed
    lower W (column-major) and the level order, in complex128 (a reported
    reference, outside every timed region)."""
    import torch
    n_sc, N = prep.perm.shape
    cols = [j for j in range(N) for _ in range(j, N)]
    rows = [i for j in range(N) for i in range(j, N)]
    Wd = torch.zeros((n_sc, N, N), dtype=torch.complex128, device=prep.W.device)
    Wd[:, rows, cols] = prep.W.to(torch.complex128)
    S = s.to(torch.complex128).t().reshape(n_sc, n_sym, N)
    Sp = torch.gather(S, 2, prep.perm.long()[:, None, :].expand(n_sc, n_sym, N)).contiguous()
    Y = torch.matmul(Sp, Wd.transpose(1, 2).contiguous())
    return (Y.abs() ** 2).sum(dim=2).reshape(-1)


def bench_batched(vp, steps, warmup):
    """The 2048-RBG uneven slot (U ~ 4..16, mixed QAM, M = 16) with K(U) from the
    calibration table: one captured graph (default and autotuned tile shapes)
    against per-size launches of the per-call API, and its power gap."""
    import torch
    import vpgen
    from paper_2602_12098_amd import batch as B
    kcal = json.load(open(os.path.join(ROOT, "paper_2602_12098_amd", "kcal_rbg_m16.json")))["K_by_U"]
    wl = vpgen.cfg4()
    groups = [B.GroupSpec(int(u), wl.sc_per_rbg, int(kcal[str(int(u))]), float(vpgen.qam_tau(int(q))), float(a))
              for u, q, a in zip(wl.U, wl.Q, wl.alpha)]
    b = B.Batch(groups, wl.M, wl.n_sym, P_T=1.0)
    b.set_inputs(wl.H, wl.s)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_default = timed(b.run)
    info = b.tune(reps=3)
    ms_tuned = timed(b.run)
    # per-size launches: RBGs grouped by (U, QAM order), each group one call per stage
    keys = sorted(set(zip(wl.U.tolist(), wl.Q.tolist())))
    per = []
    for (u, q) in keys:
        idx = [i for i in range(wl.n_rbg) if wl.U[i] == u and wl.Q[i] == q]
        H = torch.from_numpy(np.concatenate([wl.H[i] for i in idx])).to("cuda:0")
        sg = torch.from_numpy(np.concatenate([wl.s[i] for i in idx], axis=1)).to("cuda:0")
        per.append((H, sg, float(vpgen.qam_tau(q)), float(u) / 100.0, int(kcal[str(u)])))

    def per_size(min_K_sharing=None):
        """One call per stage and (U, QAM) group; with min_K_sharing, groups
        with K >= it pass the MoP orders to vp_search (prefix sharing)."""
        outs = []
        for H, sg, tau, alpha, K in per:
            prep = vp.preprocess(H, alpha)
            share = min_K_sharing is not None and K >= min_K_sharing
            order = torch.empty((H.shape[0], 2, K), dtype=torch.int16, device="cuda:0") if share else None
            paths = vp.paths_mop(prep.w2, K, order=order)
            o = vp.search(prep.W, prep.perm, sg, tau, paths, wl.n_sym, order=order)
            vp.precode(prep.G, sg, o.l, tau, o.cost, wl.n_sym, P_T=1.0)
            outs.append((prep, o))
        return outs

    ms_per_size_plain = timed(per_size)
    ms_per_size_shared = timed(lambda: per_size(64))
    ms_per_size = min(ms_per_size_plain, ms_per_size_shared)
    num = den = 0.0
    for (H, sg, tau, alpha, K), (prep, o) in zip(per, per_size()):
        g, exact = gap_to_exact(vp, prep, sg, tau, wl.n_sym, o.cost)
        num += float(o.cost.double().sum())
        den += float(exact.sum())
    n_vec = b.n_vec
    res = {"workload": f"{wl.n_rbg} RBGs x {wl.sc_per_rbg} sc x {wl.n_sym} sym, U 4..16, QAM 4..256, M {wl.M}",
           "n_vec": n_vec, "K_by_U": kcal, "value": n_vec / (ms_tuned * 1e-3), "unit": "vectors/s",
           "ms_graph_default": ms_default, "ms_graph_tuned": ms_tuned, "ms_per_size_launches": ms_per_size,
           "ms_per_size_plain": ms_per_size_plain, "ms_per_size_prefix_sharing_K64": ms_per_size_shared,
           "per_size_launch_groups": len(per), "speedup_vs_per_size": ms_per_size / ms_tuned,
           "gap_db": 10 * math.log10(num / den), "tuning": info}
    b.close()
    return res


def bench_learned(vp, steps, warmup, wl, H, s, K_mop=64):
    """The learned per-vector proposal on the same slot: features, network and
    top-64 (bf16 MFMA), table of 64 proposed + first K_mop MoP paths, search,
    precode; timed per stage, with its power gap."""
    import torch
    from paper_2602_12098_amd import learn
    path = os.path.join(ROOT, "paper_2602_12098_amd", "weights", "proposer_16x16_256qam_res64.safetensors")
    if not os.path.exists(path):
        return None
    prop = learn.load_proposer(path)
    n_sym = wl.n_sym
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    out = {}

    def step(ev=None):
        if ev: ev[0].record()
        prep = vp.preprocess(H, wl.alpha)
        if ev: ev[1].record()
        paths = vp.paths_mop(prep.w2, K_mop)
        if ev: ev[2].record()
        table, mass = prop.propose(prep.W, prep.perm, s, wl.tau, n_sym, fixed_paths=paths, K_fixed=K_mop)
        if ev: ev[3].record()
        o = vp.search(prep.W, prep.perm, s, wl.tau, table, n_sym, flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
        if ev: ev[4].record()
        vp.precode(prep.G, s, o.l, wl.tau, o.cost, n_sym, P_T=1.0)
        if ev: ev[5].record()
        out["prep"], out["o"] = prep, o

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    names = ["preprocess", "paths_mop", "propose", "search", "precode"]
    stages = {n: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
              for i, n in enumerate(names)}
    ms = float(np.mean([evs[k][0].elapsed_time(evs[k][5]) for k in range(steps)]))
    g, _ = gap_to_exact(vp, out["prep"], s, wl.tau, n_sym, out["o"].cost)
    return {"paths_per_vector": 64 + K_mop, "value": wl.n_vec / (ms * 1e-3), "unit": "vectors/s",
            "ms_per_step": ms, "stages_ms": stages, "gap_db": g,
            "model": "64 -> 256 -> 256 -> 4096 (ReLU), bf16 MFMA; vocabulary of 4096 exact position vectors; "
                     "trained on vectors the first 64 MoP paths miss",
            "train_meta": getattr(prop, "meta", {})}



def bench_learned_fallback(vp, steps, warmup, wl, H, s, theta=0.3, K_mop=64, K_fix=512):
    """The learned proposal with its fallback: vectors whose top-64 softmax mass
    is below theta are searched again over the subcarrier's fixed K_fix MoP set
    (vp_search_fallback), which replaces the proposal's result where it is
    cheaper.  The proposal's table holds the 64 proposed paths and the first
    K_mop paths of that same fixed set.  Timed per stage, with its power gap."""
    import torch
    from paper_2602_12098_amd import learn
    path = os.path.join(ROOT, "paper_2602_12098_amd", "weights", "proposer_16x16_256qam_res64.safetensors")
    if not os.path.exists(path):
        return None
    prop = learn.load_proposer(path)
    n_sym = wl.n_sym
    order = torch.empty((wl.n_sc, 2, K_fix), dtype=torch.int16, device="cuda:0")
    work = torch.empty((2 * wl.n_vec,), dtype=torch.int32, device="cuda:0")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(steps)]
    out = {}

    def step(ev=None):
        if ev: ev[0].record()
        prep = vp.preprocess(H, wl.alpha)
        if ev: ev[1].record()
        paths = vp.paths_mop(prep.w2, K_fix, order=order)
        if ev: ev[2].record()
        table, mass = prop.propose(prep.W, prep.perm, s, wl.tau, n_sym, fixed_paths=paths, K_fixed=K_mop)
        if ev: ev[3].record()
        o = vp.search(prep.W, prep.perm, s, wl.tau, table, n_sym, flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
        if ev: ev[4].record()
        learn.search_fallback(prep.W, prep.perm, s, wl.tau, paths, n_sym, mass, theta, o, 64 + K_mop + 1,
                              order=order, work=work)
        if ev: ev[5].record()
        vp.precode(prep.G, s, o.l, wl.tau, o.cost, n_sym, P_T=1.0)
        if ev: ev[6].record()
        out["prep"], out["o"], out["mass"] = prep, o, mass

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    names = ["preprocess", "paths_mop", "propose", "search", "fallback", "precode"]
    stages = {n: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
              for i, n in enumerate(names)}
    ms = float(np.mean([evs[k][0].elapsed_time(evs[k][6]) for k in range(steps)]))
    g, _ = gap_to_exact(vp, out["prep"], s, wl.tau, n_sym, out["o"].cost)
    frac = float((~(out["mass"] >= theta)).float().mean())
    return {"theta": theta, "fallback_fraction": frac, "fixed_paths": K_fix,
            "paths_per_vector": 64 + K_mop, "value": wl.n_vec / (ms * 1e-3), "unit": "vectors/s",
            "ms_per_step": ms, "stages_ms": stages, "gap_db": g}


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
    ap.add_argument("--no-extras", action="store_true", help="skip the gap, batched and learned measurements")
    ap.add_argument("--no-forms", action="store_true", help="keep the gap, skip the batched and learned forms")
    ap.add_argument("--only", choices=("batched", "learned"), default=None,
                    help="run one further form alone (for profiling) and print its record")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); on several GPUs each would "
              "take a contiguous range of subcarriers, with no exchange between them", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_12098_amd as vp
    import vpgen

    dev = "cuda:0"
    if args.only == "batched":
        print(json.dumps({"batched": bench_batched(vp, args.steps, args.warmup)}), flush=True)
        return
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
    if args.only == "learned":
        lr = bench_learned(vp, args.steps, args.warmup, wl, H, s)
        if lr is not None:
            lr["fallback"] = bench_learned_fallback(vp, args.steps, args.warmup, wl, H, s)
        print(json.dumps({"learned": lr}), flush=True)
        return

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
    traffic, traffic_src = search_traffic(K)
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_TFLOPS, "traffic": traffic, "traffic_source": traffic_src,
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
    if not args.no_extras:
        print("gap to exact VP ...", file=sys.stderr, flush=True)
        line["gap_db"], exact = gap_to_exact(vp, prep, s, wl.tau, n_sym, sout.cost)
        # the gain of VP over linear RZF (l = 0) at exact VP, and at the K paths
        g0 = rzf_powers(prep, s, n_sym)
        ok = torch.isfinite(g0) & torch.isfinite(exact)
        line["gain_over_rzf_db"] = {
            "exact": 10 * math.log10(float(g0[ok].sum()) / float(exact[ok].sum())),
            "paths": 10 * math.log10(float(g0[ok].sum()) / float(sout.cost.double()[ok].sum()))}
    if not args.no_extras and not args.no_forms:
        print("batched slot ...", file=sys.stderr, flush=True)
        line["batched"] = bench_batched(vp, args.steps, args.warmup)
        print("learned proposal ...", file=sys.stderr, flush=True)
        line["learned"] = bench_learned(vp, args.steps, args.warmup, wl, H, s)
        if line["learned"] is not None:
            print("learned proposal with fallback ...", file=sys.stderr, flush=True)
            line["learned"]["fallback"] = bench_learned_fallback(vp, args.steps, args.warmup, wl, H, s)
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(K)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
