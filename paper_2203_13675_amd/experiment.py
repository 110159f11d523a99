"""The paper's experiment (Section 3: Table 1, Figs. 2-3) on stand-in inputs.

For each of Table 1's eight 4:3 image sizes (160 x 120 up to 1280 x 960) and
each preconditioner, Algorithm 1 runs with the stopping criteria of Section 3
(``binding.paper_options``: inner test eps = 0.005 on the preconditioned
residual, k_max = 500, outer tolerance 1e-6, l_max = 2MN, FP64) from a seeded
random start.  Reported per run: outer and inner iteration counts, the time of
the call, the part of it spent forming U, V, b and the preconditioner (the
share the paper quotes for building M), and the normalized error Q of
Section 3 between the result and the noise-free phase and between the result
and the first preconditioner's result (both with their means removed, since
the solution is defined up to a constant).

The paper's own wrapped map (Fig. 1) is not available.  The stand-in is the
peaks surface scaled to max |phi| = 30 rad, sampled on the image grid (so
every size shows the same field; at most 2.2 rad per pixel at the smallest
size), plus N(0, 0.3^2) noise, wrapped.

Usage:
    python -m paper_2203_13675_amd.experiment [--scales 0.25,0.5,...]
        [--pcs none,jacobi,ilu0,ic0,ssor,dct] [--precision fp64|mixed] [--json FILE]

Every step runs in the HIP library; this module only generates inputs, calls
``Context.solve`` and tabulates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# Table 1: scale, image width (columns N), image height (rows M)
TABLE1 = [(0.25, 160, 120), (0.50, 320, 240), (0.75, 480, 360), (1.00, 640, 480),
          (1.25, 800, 600), (1.50, 960, 720), (1.75, 1120, 840), (2.00, 1280, 960)]
PAPER_PCS = ["none", "jacobi", "ilu0", "ic0", "ssor"]  # the five of Section 2.1


def normalized_error(mu: np.ndarray, nu: np.ndarray) -> float:
    """Q(mu, nu) = ||mu - nu||_2 / (||mu||_2 + ||nu||_2) (Section 3)."""
    den = float(np.linalg.norm(mu) + np.linalg.norm(nu))
    return float(np.linalg.norm(mu - nu)) / den if den > 0 else 0.0


def stand_in(M: int, N: int, seed: int):
    from paper_2203_13675_amd import synth
    psi, truth = synth.peaks_map(M, N, amplitude=30.0, sigma=0.3, seed=seed)
    phi0 = synth.random_phi0(M, N, seed=seed + 1)
    return psi, truth, phi0


def run(scales=None, pcs=None, precision="fp64", log=print):
    import torch
    from paper_2203_13675_amd.binding import Context, paper_options
    pcs = pcs or PAPER_PCS + ["dct", "ilu0_rb", "ssor_rb"]
    rows = []
    ctx = Context(0)
    dev = torch.device("cuda:0")
    for scale, N, M in TABLE1:
        if scales and scale not in scales:
            continue
        psi, truth, phi0 = stand_in(M, N, seed=int(scale * 100))
        psi_d = torch.from_numpy(psi).to(dev)
        truth0 = truth - truth.mean()
        first = None
        for pc in pcs:
            phi = torch.from_numpy(phi0).to(dev)
            opts = paper_options(precision=precision)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve(psi_d, p=0.0, preconditioner=pc, options=opts, phi=phi, check=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            out = res.phi.cpu().numpy()
            out0 = out - out.mean()
            if first is None:
                first = out0
            st = res.stats
            row = {"scale": scale, "width": N, "height": M, "pc": pc, "status": res.status,
                   "outer_iters": st["outer_iters"], "inner_iters": st["inner_iters_total"],
                   "time_s": wall, "setup_ms": st["setup_ms"],
                   "setup_share": st["setup_ms"] / (wall * 1e3) if wall > 0 else 0.0,
                   "Q_truth": normalized_error(out0, truth0),
                   "Q_vs_first": normalized_error(out0, first)}
            rows.append(row)
            log("%5.2f %5dx%-5d %-6s outer %3d inner %7d  %8.3f s  setup %5.1f%%  "
                "Q(truth) %.4f  Q(vs %s) %.2e  status %d" %
                (scale, N, M, pc, row["outer_iters"], row["inner_iters"], wall,
                 100 * row["setup_share"], row["Q_truth"], pcs[0], row["Q_vs_first"],
                 row["status"]))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--scales", default=None, help="comma-separated Table 1 scales (default all)")
    ap.add_argument("--pcs", default=None, help="comma-separated preconditioners")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--json", default=None, help="write the rows to this file")
    a = ap.parse_args(argv)
    scales = [float(s) for s in a.scales.split(",")] if a.scales else None
    pcs = a.pcs.split(",") if a.pcs else None
    rows = run(scales, pcs, a.precision, log=lambda s: print(s, flush=True))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
