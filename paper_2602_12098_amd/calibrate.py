"""Path-count calibration for the batched workload: for every user count
U = 4..16 (M = 16 antennas, i.i.d. Rayleigh channels, alpha = U / 100, QAM
order uniform over 4/16/64/256), the smallest power-of-two K whose MoP path
set stays within a power gap of 0.1 dB of exact VP over the B = 1 box
(exact VP: the sphere encoder of vp_sphere_encode seeded with the K = 512
search radius).  Writes a JSON table {U: K} with the measured gaps.

Usage: python -m paper_2602_12098_amd.calibrate --out kcal.json [--n-sc 200]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import torch

import vpgen

from . import vp

DEV = "cuda:0"
KS = (8, 16, 32, 64, 128, 256, 512)
QS = (4, 16, 64, 256)


@torch.no_grad()
def calibrate(n_sc: int = 200, target_db: float = 0.1, users=range(4, 17), seed0: int = 400):
    table, gaps = {}, {}
    for U in users:
        exact_sum = 0.0
        sums = {K: 0.0 for K in KS}
        for qi, Q in enumerate(QS):
            wl = vpgen.make(f"cal{U}q{Q}", U, 16, n_sc, 14, Q, U / 100.0, 512, seed=seed0 + 10 * U + qi)
            Hd = torch.from_numpy(wl.H).to(DEV)
            sd = torch.from_numpy(wl.s).to(DEV)
            prep = vp.preprocess(Hd, wl.alpha, want_G=False)
            costs = {}
            for K in KS:
                if K > 9 ** U:
                    continue
                paths = vp.paths_mop(prep.w2, K)
                costs[K] = vp.search(prep.W, prep.perm, sd, wl.tau, paths, wl.n_sym).cost.double()
            kmax = max(costs)
            se = vp.sphere_encode(prep.W, prep.perm, sd, wl.tau, wl.n_sym, radius=(costs[kmax] * (1 + 1e-6)).float())
            ex = torch.where(torch.isfinite(se.cost), se.cost.double(), costs[kmax])
            exact_sum += float(ex.sum())
            for K, c in costs.items():
                sums[K] += float(c.sum())
        g = {K: 10 * math.log10(sums[K] / exact_sum) for K in KS if sums[K] > 0}
        gaps[U] = g
        ok = [K for K in sorted(g) if g[K] <= target_db]
        table[U] = ok[0] if ok else max(g)
        print(f"U={U}: K={table[U]}  gaps " + " ".join(f"{K}:{g[K]:.3f}" for K in sorted(g)), flush=True)
    return table, gaps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n-sc", type=int, default=200)
    a = ap.parse_args()
    t0 = time.time()
    table, gaps = calibrate(a.n_sc)
    with open(a.out, "w") as f:
        json.dump({"target_gap_db": 0.1, "n_sc_per_U_and_Q": a.n_sc, "n_sym": 14, "M": 16,
                   "K_by_U": {str(u): k for u, k in table.items()},
                   "gap_db": {str(u): {str(k): v for k, v in g.items()} for u, g in gaps.items()},
                   "seconds": time.time() - t0}, f, indent=1)


if __name__ == "__main__":
    main()
