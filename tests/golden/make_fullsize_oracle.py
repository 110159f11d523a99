"""Oracle answers for the full-size workloads, cached for the GPU parity tests.

Calls only ``oracle/`` (and the seeded input generators of
``paper_2203_13675_amd/synth.py``, which hold none of the method's
arithmetic).  Nothing here touches the HIP library.

    python tests/golden/make_fullsize_oracle.py [--jobs 6] [--only SUBSTR] [--force] [--list]

writes one ``tests/golden/fullsize_cache/<case>.npz`` per case (skipping cases
already present unless --force).  Every case runs Algorithm 1 in the oracle on
one input with stated settings:

* ``same``      -- the preconditioner and stop rule of the GPU run it is
                   compared with (inner relative residual ``tol``), ``k_max``
                   outer iterations, outer test off;
* ``exact``     -- inner systems solved to relres 1e-12 (1e-11 at 4096^2;
                   DCT-PCG, at most 4000 iterations per solve), the
                   reference for errors of approximate inner solves;
* ``fixed``     -- a fixed number of PCG iterations per inner solve (the paper's
                   stop test with a bound nothing meets), the same work on both
                   sides whatever the rounding;
* ``perturbed`` -- a ``same`` run on psi * (1 + 1e-14 n), n ~ N(0, 1) seeded:
                   how far rounding-level changes move the answer (stores only
                   that distance);
* ``tolerr``    -- a ``same`` DCT run at another inner tolerance; stores only
                   its distance to the ``exact`` answer (how accurate a solve at
                   that tolerance can be).

Stored: phi on a strided sample (``stride``) of the grid, the mean of phi over
the valid (non-isolated) pixels of the whole map, per-outer-iteration inner
counts, outer errors and final inner residuals, and the settings.

Workloads (``synth``): peaks1024 (1024^2 peaks, 60 rad, noise 0.5),
gauss2048_hole (2048^2, 20 Gaussians, noise 0.8, 10 % zero-quality hole),
ramp4096 (4096^2 peaks + 120 rad ramp, noise 0.5), and one square map of each
side length of the 256-map batch and five rectangular ones.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CACHE = os.path.join(HERE, "fullsize_cache")

# one square map of each side length of the benchmark batch (indices into
# synth.batch_maps(256, 3000)): sides 128, 256, 384, 512, 768, 1024
BATCH_REPS = {128: 33, 256: 7, 384: 19, 512: 105, 768: 23, 1024: 22}
# and rectangular maps of the batch (the two DCT stage parities contract
# different lengths; sides 128 and 384 on one axis only)
BATCH_RECT = {(128, 1024): 4, (1024, 128): 52, (384, 768): 1, (768, 384): 119, (1024, 384): 31}
EXACT_TOL = 1e-12      # 1e-11 for the 4096^2 map (FP64 rounding floor of its residual)
EXACT_LMAX = 4000
TOL_SWEEP = (1e-7, 1e-8, 1e-9)


def _case(key, workload, mode, *, p=0.0, pc="dct", tol=1e-6, k_max=10, stride=1, l_max=None,
          seed=None, needs=None):
    return dict(key=key, workload=workload, mode=mode, p=p, pc=pc, tol=tol, k_max=k_max,
                stride=stride, l_max=l_max, seed=seed, needs=needs)


def cases():
    out = []
    # peaks1024: each preconditioner, p in {0, 1}
    for p in (0, 1):
        out.append(_case("peaks1024_exact_p%d" % p, "peaks1024", "exact", p=p))
        for pc in ("dct", "jacobi", "ilu0", "none", "ic0", "ssor"):
            base = "peaks1024_same_%s_p%d" % (pc, p)
            out.append(_case(base, "peaks1024", "same", p=p, pc=pc))
            for s in range(3):
                out.append(_case("%s_perturbed%d" % (base, s), "peaks1024", "perturbed", p=p,
                                 pc=pc, seed=s, needs=base))
        for t in TOL_SWEEP:
            out.append(_case("peaks1024_tolerr_dct_p%d_%g" % (p, t), "peaks1024", "tolerr", p=p,
                             tol=t, needs="peaks1024_exact_p%d" % p))
    for pc in ("none", "jacobi", "ilu0", "ic0", "ssor", "dct"):
        out.append(_case("peaks1024_fixed_%s_p0" % pc, "peaks1024", "fixed", pc=pc, k_max=3,
                         l_max=40, stride=2))
    # gauss2048_hole and ramp4096: first outer iteration and all ten
    for w, st in (("gauss2048_hole", 2), ("ramp4096", 4)):
        for k in (1, 10):
            out.append(_case("%s_exact_k%d" % (w, k), w, "exact", k_max=k, stride=st))
            out.append(_case("%s_same_k%d" % (w, k), w, "same", k_max=k, stride=st))
    # one square map per side length of the batch
    for k in list(BATCH_REPS.values()) + list(BATCH_RECT.values()):
        w = "batch256:%d" % k
        out.append(_case("batch256_map%d_exact" % k, w, "exact"))
        out.append(_case("batch256_map%d_same" % k, w, "same"))
    return out


def load_input(workload):
    sys.path.insert(0, ROOT)
    from paper_2203_13675_amd import synth
    if workload.startswith("batch256:"):
        psi, _ = synth.batch_map(int(workload.split(":")[1]))
        return psi, None
    psi, mask, _ = synth.workload(workload)
    return psi, mask


def valid_pixels(O, psi, mask):
    M, N = psi.shape
    wx, wy = O.edge_quality(mask, M, N)
    return ~O.isolated_pixels(wx, wy)


def run_case(c):
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import lp_oracle as O
    t0 = time.time()
    psi, mask = load_input(c["workload"])
    valid = valid_pixels(O, psi, mask)
    kw = dict(p=c["p"], precond=c["pc"], tol=c["tol"], k_max=c["k_max"], outer_tol=0.0)
    if c["mode"] == "exact":
        tol = EXACT_TOL if psi.size <= 2048 * 2048 else 10 * EXACT_TOL
        kw.update(precond="dct", tol=tol, l_max=EXACT_LMAX)
    elif c["mode"] == "fixed":
        kw.update(stop_rule="paper", eps_cg=1e-30, l_max=c["l_max"])
    elif c["mode"] == "perturbed":
        rng = np.random.default_rng(123 + c["seed"])
        psi = psi * (1.0 + 1e-14 * rng.standard_normal(psi.shape))
    r = O.unwrap(psi, mask, **kw)
    info = dict(case=c, inner_iters=[int(v) for v in r.inner_iters],
                outer_errs=[float(v) for v in r.outer_errs], relres=[float(v) for v in r.relres],
                outer_iters=int(r.outer_iters), seconds=time.time() - t0)
    out = dict(info=json.dumps(info))
    if c["mode"] in ("perturbed", "tolerr"):
        ref = np.load(os.path.join(CACHE, c["needs"] + ".npz"))
        st = int(ref["stride"])
        a = r.phi[::st, ::st] - r.phi[valid].mean()
        b = ref["phi"] - float(ref["mean"])
        v = valid[::st, ::st]
        out["diff"] = float(abs(a[v] - b[v]).max())
    else:
        st = c["stride"]
        out["phi"] = np.ascontiguousarray(r.phi[::st, ::st])
        out["stride"] = st
        out["mean"] = float(r.phi[valid].mean())
        out["valid"] = np.ascontiguousarray(valid[::st, ::st])
    tmp = os.path.join(CACHE, c["key"] + ".tmp.npz")
    np.savez(tmp, **out)
    os.replace(tmp, os.path.join(CACHE, c["key"] + ".npz"))
    return c["key"], time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--only", default="")
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--list", action="store_true")
    a = ap.parse_args()
    os.makedirs(CACHE, exist_ok=True)
    todo = [c for c in cases() if a.only in c["key"]]
    if not a.force:
        todo = [c for c in todo if not os.path.exists(os.path.join(CACHE, c["key"] + ".npz"))]
    if a.list:
        for c in todo:
            print(c["key"])
        return
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    import multiprocessing as mp
    waves = [[c for c in todo if not c["needs"]], [c for c in todo if c["needs"]]]
    # longest first: the 4096^2 and 2048^2 cases, then the rest
    order = {"ramp4096": 0, "gauss2048_hole": 1}
    with mp.get_context("spawn").Pool(a.jobs) as pool:
        for wave in waves:
            wave.sort(key=lambda c: order.get(c["workload"], 2))
            for key, sec in pool.imap_unordered(run_case, wave):
                print("%-40s %8.1f s" % (key, sec), flush=True)


if __name__ == "__main__":
    main()
