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

# MI355X's published fp32 vector peak: 256 CUs x 4 SIMDs x 2.4 GHz x 64 flop per clock
# per SIMD = 157.3 TFLOP/s, taken whole: a stream of independent plain v_fmac_f32
# instructions (no packed FP32; paper_2602_12098_amd/valuref.py) sustains 2.8-2.9 SIMD
# clocks per wave64 instruction, under the 4 a 16-lane SIMD would need, so code without
# packed instructions is not held to half of it.
PEAK_VALU_TFLOPS = 256 * 4 * 64 * 2.4e9 / 1e12
FLOP_PER_CM = 6   # one complex multiplication: 4 real multiplies + 2 adds


def search_cm_per_vector(n_t, K):
    """Path-search part of the paper's per-vector count (Sec. III-B): K N_t (1 + (N_t+1)/2)."""
    return K * n_t * (n_t + 3) // 2


SEARCH_SOURCES = ["paper_2602_12098_amd/csrc/vp_search.hip", "paper_2602_12098_amd/csrc/vp_walk.hpp",
                  "paper_2602_12098_amd/csrc/vp_device.hpp", "paper_2602_12098_amd/csrc/demap_lut.h",
                  "paper_2602_12098_amd/csrc/region_lut.h", "paper_2602_12098_amd/build.py"]   # build flags too
TRAFFIC_FILE = "profiles/k_search_trie_16x16_256qam_K512.traffic.json"


def sources_sha256(files):
    """sha256 over the concatenated bytes of the given repository files."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def search_traffic(K, path=None):
    """HBM bytes per launch of the search kernel from the committed counter
    profile (taken at K = 512), or None when it is missing, K differs or the
    kernel sources changed since."""
    path = path or os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None, "no traffic profile"
    if K != 512:
        return None, "the counters were taken at K = 512"
    rec = json.load(open(path))
    if sources_sha256(rec.get("source_files", SEARCH_SOURCES)) != rec.get("source_sha256"):
        return None, "kernel changed since the counters were taken"
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"], os.path.relpath(path, ROOT)


COUNTERS_FILE = "profiles/search_16x16_256qam_K512.valu.json"


def search_counters(K, path=None):
    """Measured clock and VALU issue of the search kernel from the committed
    counter profile (GRBM_GUI_ACTIVE against the kernel's duration gives the
    shader clock; 1024 SIMDs x those clocks over SQ_INSTS_VALU the SIMD clocks
    per VALU instruction, set against those of a plain FMA stream), or {} when
    it is missing, K differs or the sources changed."""
    path = path or os.path.join(ROOT, COUNTERS_FILE)
    if K != 512 or not os.path.exists(path):
        return {}
    rec = json.load(open(path))
    if sources_sha256(rec.get("source_files", SEARCH_SOURCES)) != rec.get("source_sha256"):
        return {}
    if "simd_clocks_per_valu_instr" not in rec:
        return {}
    return {"sclk_ghz_measured": rec["sclk_ghz"], "simd_clocks_per_valu_instr": rec["simd_clocks_per_valu_instr"],
            "fma_stream_clocks_per_valu_instr": rec["fma_stream_clocks_per_valu_instr"],
            "issue_vs_fma_stream": rec["issue_vs_fma_stream"],
            "valu_instr_per_vector": rec["valu_instr_per_vector"], "counters_source": os.path.relpath(path, ROOT)}


def gap_to_exact(vp, prep, s, tau, n_sym, cost, counts=None):
    """Power gap (dB) of the selected perturbations to exact VP over the box:
    the GPU sphere encoder seeded with each vector's own cost as radius.  A
    vector whose encoder ran out of its node budget contributes the best point
    it found (never above the method's cost); one with no point inside the
    radius contributes the method's own cost.  `counts` (a dict) receives how
    many vectors took either way."""
    import torch
    se = vp.sphere_encode(prep.W, prep.perm, s, tau, n_sym, radius=cost * (1 + 1e-6))
    exact = torch.where(torch.isfinite(se.cost), se.cost, cost).double()
    if counts is not None:
        counts["budget_exhausted"] = int((se.status == vp.VP_SE_EXHAUSTED).sum())
        counts["no_point_inside_radius"] = int((se.status == vp.VP_SE_NONE).sum())
        counts["vectors"] = int(cost.numel())
    return 10 * math.log10(float(cost.double().sum()) / float(exact.sum())), exact


def vp_powers(prep, s, n_sym, l=None, tau=0.0):
    """gamma = ||W (s_pi + tau l_pi)||^2 per vector, from the packed lower W
    (column-major), the level order and l (int8 [N][n_vec][2], user order; None
    for l = 0, linear RZF), in complex128 (a reported reference, outside every
    timed region)."""
    import torch
    n_sc, N = prep.perm.shape
    cols = [j for j in range(N) for _ in range(j, N)]
    rows = [i for j in range(N) for i in range(j, N)]
    Wd = torch.zeros((n_sc, N, N), dtype=torch.complex128, device=prep.W.device)
    Wd[:, rows, cols] = prep.W.to(torch.complex128)
    u = s.to(torch.complex128)
    if l is not None:
        u = u + tau * torch.complex(l[..., 0].double(), l[..., 1].double())
    S = u.t().reshape(n_sc, n_sym, N)
    Sp = torch.gather(S, 2, prep.perm.long()[:, None, :].expand(n_sc, n_sym, N)).contiguous()
    Y = torch.matmul(Sp, Wd.transpose(1, 2).contiguous())
    return (Y.abs() ** 2).sum(dim=2).reshape(-1)


def rzf_powers(prep, s, n_sym):
    return vp_powers(prep, s, n_sym)


def bench_fixed_point(vp, dev="cuda:0"):
    """The 16-bit fixed-point walk (vp_fx_quantize + vp_fx_search) against the
    float32 walk, for F = 8..13 fractional bits: power gap to exact VP of the
    perturbations either one chooses, every power evaluated in complex128 from
    the chosen l (outside every timed region), and the fixed-point search's
    kernel time (an emulation, not a tuned path)."""
    import torch
    import vpgen
    res = {}
    for wl in (vpgen.cfg3(512, n_sc=546), vpgen.cfg2(20, n_sc=546)):
        H = torch.from_numpy(wl.H).to(dev)
        s = torch.from_numpy(wl.s).to(dev)
        prep = vp.preprocess(H, wl.alpha)
        order = torch.empty((wl.n_sc, 2, wl.K), dtype=torch.int16, device=dev)
        paths = vp.paths_mop(prep.w2, wl.K, order=order)
        of = vp.search(prep.W, prep.perm, s, wl.tau, paths, wl.n_sym, order=order)
        pf = vp_powers(prep, s, wl.n_sym, of.l, wl.tau)
        rows, fx = {}, {}
        for F in range(8, 14):
            q = vp.fx_quantize(prep.W, prep.perm, s, wl.tau, wl.n_sym, F)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            o = vp.fx_search(q, prep.perm, paths, wl.n_sym)
            e1.record()
            torch.cuda.synchronize()
            fx[F] = (vp_powers(prep, s, wl.n_sym, o.l, wl.tau), o.l, e0.elapsed_time(e1))
        radius = torch.minimum(pf, torch.stack([v[0] for v in fx.values()]).min(dim=0).values)
        se = vp.sphere_encode(prep.W, prep.perm, s, wl.tau, wl.n_sym, radius=(radius * (1 + 1e-6)).float())
        pe = torch.where(torch.isfinite(se.cost), vp_powers(prep, s, wl.n_sym, se.l, wl.tau), radius)
        pe = torch.minimum(pe, radius)
        den = float(pe.sum())
        for F, (p, l, ms) in fx.items():
            rows[str(F)] = {"gap_db": 10 * math.log10(float(p.sum()) / den),
                            "same_l_as_float32": float((l == of.l).all(dim=2).all(dim=0).double().mean()),
                            "search_ms": ms}
        res[wl.name] = {"K": wl.K, "vectors": wl.n_vec, "gap_db_float32": 10 * math.log10(float(pf.sum()) / den),
                        "fixed_point": rows}
    return res


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
        per.append((H, sg, vp.tau_array(float(vpgen.qam_tau(q)), H.shape[0], "cuda:0"), float(u) / 100.0,
                    int(kcal[str(u)]), float(vpgen.qam_tau(q))))

    def per_size(min_K_sharing=None):
        """One call per stage and (U, QAM) group; with min_K_sharing, groups
        with K >= it pass the MoP orders to vp_search (prefix sharing)."""
        outs = []
        for H, sg, tau, alpha, K, _ in per:
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
    ms_per_size_eager = min(ms_per_size_plain, ms_per_size_shared)

    # the same per-size launches without per-call host work: outputs allocated
    # once, the whole sequence captured in one HIP graph and replayed (no
    # library call in it clears memory with a memset)
    def per_size_graph(min_K_sharing):
        bufs = []
        for H, sg, tau, alpha, K, _ in per:
            prep = vp.preprocess(H, alpha)
            share = min_K_sharing is not None and K >= min_K_sharing
            order = torch.empty((H.shape[0], 2, K), dtype=torch.int16, device="cuda:0") if share else None
            paths = vp.paths_mop(prep.w2, K, order=order)
            o = vp.search(prep.W, prep.perm, sg, tau, paths, wl.n_sym, order=order)
            x = vp.precode(prep.G, sg, o.l, tau, o.cost, wl.n_sym, P_T=1.0)
            bufs.append((prep, order, paths, o, x))
        eager_cost = [o.cost.clone() for _, _, _, o, _ in bufs]

        def launches():
            for (H, sg, tau, alpha, K, _), (prep, order, paths, o, x) in zip(per, bufs):
                vp.preprocess(H, alpha, out=prep)
                vp.paths_mop(prep.w2, K, out=paths, order=order)
                vp.search(prep.W, prep.perm, sg, tau, paths, wl.n_sym, out=o, order=order)
                vp.precode(prep.G, sg, o.l, tau, o.cost, wl.n_sym, P_T=1.0, out=x)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            launches()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            launches()
        ms = timed(g.replay)
        same = all(torch.equal(c, o.cost) for c, (_, _, _, o, _) in zip(eager_cost, bufs))
        del g
        return ms, same

    ms_graph_plain, same_plain = per_size_graph(None)
    ms_graph_shared, same_shared = per_size_graph(64)
    ms_per_size = min(ms_graph_plain, ms_graph_shared)
    num = den = 0.0
    for (H, sg, _, alpha, K, tau), (prep, o) in zip(per, per_size()):
        g, exact = gap_to_exact(vp, prep, sg, tau, wl.n_sym, o.cost)
        num += float(o.cost.double().sum())
        den += float(exact.sum())
    n_vec = b.n_vec
    res = {"workload": f"{wl.n_rbg} RBGs x {wl.sc_per_rbg} sc x {wl.n_sym} sym, U 4..16, QAM 4..256, M {wl.M}",
           "n_vec": n_vec, "K_by_U": kcal, "value": n_vec / (ms_tuned * 1e-3), "unit": "vectors/s",
           "ms_graph_default": ms_default, "ms_graph_tuned": ms_tuned,
           "ms_per_size_launches": ms_per_size,
           "per_size_reference": "the per-call API per (U, QAM) group, all launches captured in one HIP graph "
                                 "(outputs preallocated), the faster of plain and prefix sharing for K >= 64",
           "ms_per_size_graph_plain": ms_graph_plain, "ms_per_size_graph_prefix_sharing_K64": ms_graph_shared,
           "per_size_graph_matches_eager": bool(same_plain and same_shared),
           "ms_per_size_eager_python_loop": ms_per_size_eager,
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
    tau = vp.tau_array(wl.tau, wl.n_sc, "cuda:0")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    out = {}

    def step(ev=None):
        if ev: ev[0].record()
        prep = vp.preprocess(H, wl.alpha)
        if ev: ev[1].record()
        paths = vp.paths_mop(prep.w2, K_mop)
        if ev: ev[2].record()
        table, _ = prop.propose(prep.W, prep.perm, s, wl.tau, n_sym, fixed_paths=paths, K_fixed=K_mop,
                                with_mass=False)
        if ev: ev[3].record()
        o = vp.search(prep.W, prep.perm, s, tau, table, n_sym, flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
        if ev: ev[4].record()
        vp.precode(prep.G, s, o.l, tau, o.cost, n_sym, P_T=1.0)
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
    tau = vp.tau_array(wl.tau, wl.n_sc, "cuda:0")
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
        o = vp.search(prep.W, prep.perm, s, tau, table, n_sym, flags=vp.VP_INCLUDE_ZERO | vp.VP_PATHS_PER_VECTOR)
        if ev: ev[4].record()
        learn.search_fallback(prep.W, prep.perm, s, tau, paths, n_sym, mass, theta, o, 64 + K_mop + 1,
                              order=order, work=work)
        if ev: ev[5].record()
        vp.precode(prep.G, s, o.l, tau, o.cost, n_sym, P_T=1.0)
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


def bench_ablations(vp, dev="cuda:0"):
    """Power-gap ablations standing in for the paper's coded-BER figures
    (outside every timed region): sorted (Alg. 1) against unsorted
    preprocessing at the same path count (the improved-SRQD comparison of
    Sec. III-B), on the 16x16 slot (K = 512) and the 8x8 workloads at SNR 10,
    20 and 30 dB (K = 64); and the path count K = 2..8 at 8x8 (the
    most-promising-path count study).  Exact VP comes from the GPU sphere
    encoder on the sorted factorisation (the optimum does not depend on the
    factorisation), seeded with the smaller of the two costs."""
    import torch
    import vpgen

    def run(wl, K, sorted_):
        H = torch.from_numpy(wl.H).to(dev)
        s = torch.from_numpy(wl.s).to(dev)
        prep = vp.preprocess(H, wl.alpha, sorted=sorted_)
        order = torch.empty((wl.n_sc, 2, K), dtype=torch.int16, device=dev)
        paths = vp.paths_mop(prep.w2, K, order=order)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = vp.search(prep.W, prep.perm, s, wl.tau, paths, wl.n_sym, order=order)
        e1.record()
        torch.cuda.synchronize()
        return prep, s, out, e0.elapsed_time(e1)

    def exact(prep, s, tau, n_sym, cost):
        se = vp.sphere_encode(prep.W, prep.perm, s, tau, n_sym, radius=cost * (1 + 1e-6))
        return torch.where(torch.isfinite(se.cost), se.cost, cost).double()

    def gap(c, ex):
        return 10 * math.log10(float(c.double().sum()) / float(ex.sum()))

    res = {"sorted_vs_unsorted": {}, "K_sweep_8x8": {}}
    for wl in (vpgen.cfg3(512), vpgen.cfg2(10), vpgen.cfg2(20), vpgen.cfg2(30)):
        K = wl.K
        ps, s, os_, ts = run(wl, K, True)
        pu, _, ou, tu = run(wl, K, False)
        ex = exact(ps, s, wl.tau, wl.n_sym, torch.minimum(os_.cost, ou.cost))
        res["sorted_vs_unsorted"][wl.name] = {
            "K": K, "gap_db_sorted": gap(os_.cost, ex), "gap_db_unsorted": gap(ou.cost, ex),
            "search_ms_sorted": ts, "search_ms_unsorted": tu, "vectors": wl.n_vec}
    # one QAM order per user (4..256) on the 16x16 correlated workload: the
    # per-user intervals (vp_apply_user_tau) against one common interval, the
    # largest, for every user (also decodable, at more transmit power)
    rng = np.random.default_rng(5)
    wl = vpgen.cfg3(512, n_sc=1092)
    Qu = np.array([4, 16, 64, 256])[rng.integers(0, 4, size=(wl.n_sc, wl.N))]
    tau_u = torch.from_numpy((2 * np.sqrt(Qu)).astype(np.float32)).to(dev)
    s_np = np.zeros_like(wl.s)
    for sc in range(wl.n_sc):
        for u in range(wl.N):
            s_np[u, sc * wl.n_sym:(sc + 1) * wl.n_sym] = vpgen.draw_symbols(rng, 1, wl.n_sym, int(Qu[sc, u]))[0]
    H = torch.from_numpy(wl.H).to(dev)
    s = torch.from_numpy(s_np).to(dev)
    prep = vp.preprocess(H, wl.alpha)
    pc = vp.Prep(prep.W.clone(), prep.w2.clone(), prep.perm.clone(), prep.G.clone(), prep.status.clone())
    sp = vp.apply_user_tau(prep, s, tau_u, wl.n_sym)
    order = torch.empty((wl.n_sc, 2, 512), dtype=torch.int16, device=dev)
    paths = vp.paths_mop(prep.w2, 512, order=order)
    o = vp.search(prep.W, prep.perm, sp, 1.0, paths, wl.n_sym, order=order)
    ex = exact(prep, sp, 1.0, wl.n_sym, o.cost)
    paths_c = vp.paths_mop(pc.w2, 512, order=order)
    oc = vp.search(pc.W, pc.perm, s, 32.0, paths_c, wl.n_sym, order=order)
    res["per_user_tau"] = {
        "workload": f"16x16 rho 0.5, {wl.n_sc} subcarriers x 14, QAM order per user uniform on 4..256, K = 512",
        "gap_db": gap(o.cost, ex),
        "power_common_tau_over_per_user_db": 10 * math.log10(float(oc.cost.double().sum()) /
                                                             float(o.cost.double().sum()))}
    for snr in (10, 20, 30):
        wl = vpgen.cfg2(snr)
        ref = None
        row = {}
        for K in (2, 3, 4, 5, 6, 7, 8, 16, 64):
            p, s, o, _ = run(wl, K, True)
            if ref is None:
                ref = exact(p, s, wl.tau, wl.n_sym, o.cost)
            row[str(K)] = gap(o.cost, ref)
        res["K_sweep_8x8"][f"snr{snr}"] = row
    return res


# The workload the oracle workers read: built once in the parent before the
# pool forks, so that no worker regenerates it inside the timed wall.
_CPU_WL = None


def _cpu_worker(sc_list):
    from oracle import vp_oracle as O
    wl = _CPU_WL
    K = wl.K
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


def host_description():
    """nproc, the CPUs this process may run on, and the CPU model of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": os.cpu_count() or 1, "cpus_available": avail, "cpu_model": model}


# The GPU machines grant 16 host CPUs per GPU, whatever nproc reports there.
HOST_PROCS_CAP = 16


def cpu_baseline(wl, budget_s=12.0):
    """FP64 oracle (numpy) on a bounded sample of subcarriers of the same
    workload, one process per granted host CPU."""
    import multiprocessing as mp
    global _CPU_WL
    _CPU_WL = wl
    host = host_description()
    procs = max(1, min(host["cpus_available"], HOST_PROCS_CAP))
    # calibrate on one subcarrier, then size the sample to ~budget_s of wall time
    _, per_sc = _cpu_worker([0])
    n_sc = int(max(procs, min(wl.n_sc - 1, budget_s * procs / per_sc)))
    scs = list(range(1, 1 + n_sc))
    chunks = [scs[i::procs] for i in range(procs)]
    ctx = mp.get_context("fork")
    with ctx.Pool(procs) as pool:
        pool.map(abs, range(procs))          # processes started before the clock
        t0 = time.perf_counter()
        res = pool.map(_cpu_worker, chunks)
        wall = time.perf_counter() - t0
    nvec = sum(r[0] for r in res)
    return dict({"value": nvec / wall, "unit": "vectors/s", "cores": procs, "kind": "oracle",
                 "sample": f"{n_sc} of {wl.n_sc} subcarriers x {wl.n_sym} symbols ({wl.N}x{wl.M}, K={wl.K}), "
                           f"full pipeline (preprocess, K-best MoP, path search, precode) in float64 numpy, "
                           f"{procs} processes (capped at {HOST_PROCS_CAP}), {wall:.1f} s wall; the workload is "
                           f"generated before the clock starts"}, **host)


def exact_vp_host(wl, l_gpu, n_vec=4096):
    """The oracle's exact VP (its C sphere encoder, float64) on the first n_vec
    vectors of the workload, timed on the host cores, and the power gap of the
    GPU's selected perturbations to it: both costs are formed in float64 from
    the oracle's own factorisation of H.  The encoder is seeded with each
    vector's method cost (which only prunes)."""
    import numpy as np
    from oracle import se_c
    from oracle import vp_oracle as O
    n_sc = (n_vec + wl.n_sym - 1) // wl.n_sym
    preps = [O.preprocess(wl.H[sc], wl.alpha) for sc in range(n_sc)]
    W = np.stack([p.W for p in preps])
    perm = np.stack([p.perm for p in preps])
    wsel = (np.arange(n_vec) // wl.n_sym).astype(np.int32)
    s = wl.s[:, :n_vec].astype(np.complex128)
    l = l_gpu[:n_vec]
    g_method = np.array([O.cost_tri(W[wsel[v]], perm[wsel[v]], s[:, v], l[v], wl.tau) for v in range(n_vec)])
    se_c.build()
    t0 = time.perf_counter()
    _, g_exact, nodes = se_c.sphere_encode_batch(W, perm, s, wl.tau, radius=g_method * (1 + 1e-9), wsel=wsel)
    wall = time.perf_counter() - t0
    found = np.isfinite(g_exact)
    g_exact = np.where(found, g_exact, g_method)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or host_description()["cpus_available"]
    return {"gap_db": 10 * math.log10(float(g_method.sum()) / float(g_exact.sum())),
            "vectors": n_vec, "value": n_vec / wall, "unit": "vectors/s", "threads": threads,
            "kind": "oracle C sphere encoder (float64, OpenMP), seeded with the method's cost",
            "median_nodes": float(np.median(nodes)), "no_point_inside_radius": int(np.sum(~found)),
            "wall_s": wall}


def run_plain(vp, wl, K, steps, warmup, dev="cuda:0", flags=None):
    """Time the plain path (preprocess, MoP paths with their orders, search,
    precode) on workload wl with K paths: inputs resident in HBM, outputs
    preallocated.  Returns the timings and the buffers of the last step."""
    import torch
    N, M, n_sc, n_sym = wl.N, wl.M, wl.n_sc, wl.n_sym
    n_vec = n_sc * n_sym
    H = torch.from_numpy(wl.H).to(dev)
    s = torch.from_numpy(wl.s).to(dev)
    tau = vp.tau_array(wl.tau, n_sc, dev)
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
        vp.search(prep.W, prep.perm, s, tau, paths, n_sym, out=sout, order=order,
                  flags=vp.VP_INCLUDE_ZERO if flags is None else flags)
        if ev: ev[3].record()
        vp.precode(prep.G, s, sout.l, tau, sout.cost, n_sym, P_T=1.0, out=x)
        if ev: ev[4].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    names = ["preprocess", "paths_mop", "search", "precode"]
    stages = {n: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
              for i, n in enumerate(names)}
    ms_event = float(np.mean([evs[k][0].elapsed_time(evs[k][4]) for k in range(steps)]))
    assert bool(torch.all(prep.status == 0)), "preprocessing failed on some subcarrier"
    return {"value": n_vec * steps / wall, "wall_ms_per_step": wall * 1e3 / steps, "event_ms_per_step": ms_event,
            "stages_ms": stages, "prep": prep, "s": s, "tau": tau, "sout": sout, "x": x}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--K", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the gap, K points, batched and learned forms")
    ap.add_argument("--no-forms", action="store_true", help="keep the gap and K points, skip the batched and "
                                                            "learned forms")
    ap.add_argument("--only", choices=("batched", "learned", "fixed"), default=None,
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
    if args.only == "fixed":
        print(json.dumps({"fixed_point_16bit": bench_fixed_point(vp, dev)}), flush=True)
        return
    wl = vpgen.cfg3(args.K)
    N, M, n_sc, n_sym, K = wl.N, wl.M, wl.n_sc, wl.n_sym, args.K
    n_vec = n_sc * n_sym
    if args.only == "learned":
        H = torch.from_numpy(wl.H).to(dev)
        s = torch.from_numpy(wl.s).to(dev)
        lr = bench_learned(vp, args.steps, args.warmup, wl, H, s)
        if lr is not None:
            lr["fallback"] = bench_learned_fallback(vp, args.steps, args.warmup, wl, H, s)
        print(json.dumps({"learned": lr}), flush=True)
        return

    r = run_plain(vp, wl, K, args.steps, args.warmup, dev)
    print(f"timed {args.steps} steps of K = {K}: {r['wall_ms_per_step']:.3f} ms per step", file=sys.stderr,
          flush=True)
    stage = r["stages_ms"]
    prep, s, sout = r["prep"], r["s"], r["sout"]


    flops = search_cm_per_vector(M, K) * FLOP_PER_CM * n_vec
    achieved = flops / (stage["search"] * 1e-3) / 1e12
    traffic, traffic_src = search_traffic(K)
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_TFLOPS, "traffic": traffic, "traffic_source": traffic_src,
            "kernel": "vp_search (the search kernel and its l write-back, timed together by HIP events on "
                      "the launch stream)",
            "work": f"{search_cm_per_vector(M, K)} complex mult/vector x {FLOP_PER_CM} flop x {n_vec} vectors"}
    roof.update(search_counters(K))

    line = {
        "metric": METRIC, "value": r["value"], "unit": "vectors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["wall_ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "N": N, "M": M, "n_sc": n_sc, "n_sym": n_sym, "K": K, "Q": wl.Q,
                   "alpha": wl.alpha, "rho": wl.rho, "seed": wl.seed},
        "event_ms_per_step": r["event_ms_per_step"], "stages_ms": stage, "roofline": roof,
        "gap_db": None,
    }
    if not args.no_extras:
        print("gap to exact VP ...", file=sys.stderr, flush=True)
        counts = {}
        line["gap_db"], exact = gap_to_exact(vp, prep, s, wl.tau, n_sym, sout.cost, counts)
        line["gap_exact_vp"] = dict(counts, encoder="GPU sphere encoder (vp_sphere_encode), every vector")
        # the gain of VP over linear RZF (l = 0) at exact VP, and at the K paths
        g0 = rzf_powers(prep, s, n_sym)
        ok = torch.isfinite(g0) & torch.isfinite(exact)
        line["gain_over_rzf_db"] = {
            "exact": 10 * math.log10(float(g0[ok].sum()) / float(exact[ok].sum())),
            "paths": 10 * math.log10(float(g0[ok].sum()) / float(sout.cost.double()[ok].sum()))}
        line["K_points"] = {}
        for Kp in (128, 256):
            if Kp == K:
                continue
            print(f"K = {Kp} ...", file=sys.stderr, flush=True)
            rp = run_plain(vp, vpgen.cfg3(Kp), Kp, args.steps, args.warmup, dev)
            g, _ = gap_to_exact(vp, rp["prep"], rp["s"], wl.tau, n_sym, rp["sout"].cost)
            line["K_points"][str(Kp)] = {"value": rp["value"], "unit": "vectors/s",
                                         "ms_per_step": rp["wall_ms_per_step"], "stages_ms": rp["stages_ms"],
                                         "gap_db": g}
            del rp
    if not args.no_extras:
        print("ablations ...", file=sys.stderr, flush=True)
        line["ablations"] = bench_ablations(vp, dev)
        print("16-bit fixed-point walk ...", file=sys.stderr, flush=True)
        line["ablations"]["fixed_point_16bit"] = bench_fixed_point(vp, dev)
    if not args.no_extras:
        # the paper's region-table DEMAP against the exact child order, same slot
        print("region-table DEMAP ...", file=sys.stderr, flush=True)
        line["region_demap"] = {}
        for Kp in (K, 256):
            rr = run_plain(vp, vpgen.cfg3(Kp), Kp, args.steps, args.warmup, dev,
                           flags=vp.VP_INCLUDE_ZERO | vp.VP_DEMAP_REGION)
            g, _ = gap_to_exact(vp, rr["prep"], rr["s"], wl.tau, n_sym, rr["sout"].cost)
            line["region_demap"][str(Kp)] = {"value": rr["value"], "unit": "vectors/s",
                                             "ms_per_step": rr["wall_ms_per_step"], "stages_ms": rr["stages_ms"],
                                             "gap_db": g}
            del rr
    l_host = None
    if not args.no_cpu:
        l_i8 = sout.l.cpu().numpy()
        l_host = (l_i8[..., 0].astype(np.float64) + 1j * l_i8[..., 1].astype(np.float64)).T
    if not args.no_extras and not args.no_forms:
        print("batched slot ...", file=sys.stderr, flush=True)
        line["batched"] = bench_batched(vp, args.steps, args.warmup)
        H = torch.from_numpy(wl.H).to(dev)
        print("learned proposal ...", file=sys.stderr, flush=True)
        line["learned"] = bench_learned(vp, args.steps, args.warmup, wl, H, s)
        if line["learned"] is not None:
            print("learned proposal with fallback ...", file=sys.stderr, flush=True)
            line["learned"]["fallback"] = bench_learned_fallback(vp, args.steps, args.warmup, wl, H, s)
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl)
        print("exact VP on the host (oracle sphere encoder) ...", file=sys.stderr, flush=True)
        ev = exact_vp_host(wl, l_host)
        line["cpu_baseline"]["exact_vp"] = ev
        line["gap_db_oracle_first4096"] = ev["gap_db"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
