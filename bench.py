"""Throughput benchmark: Mpixel/s unwrapped at 1e-6 relative residual.

One step = one lp_unwrap_batch call over the uneven batch workload (256
random-Gaussian maps, sides drawn from {128,256,384,512,768,1024}, noise
sigma ~ U[0.1, 0.8] rad, p = 0, tau = 0.01, 10 outer iterations, DCT
preconditioner, mixed precision with scaled-fp16 MFMA transforms), with every
psi already resident in HBM when the timed region starts.

Prints one JSON line (rank 0) with the metric, the roofline of the dominant
kernel (achieved = algorithmic bytes or flops of its launches / their summed
HIP-event durations, measured on the library's stream in a timing pass over
the same workload right after the timed region), the same batch at FP64 in
one call and map by map, the oracle's CPU rate on a bounded sample of the
batch (all host cores and single-threaded), and the unwrapped phase's distance
to the oracle's answers on that sample.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP16_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6  # vector FMA units: the plain FP64 path's DCT stages run there
# measured HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE passes,
# scaled by a plain copy), valid while the kernel sources hash as recorded
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_batch256_fp16.txt")
_SHARED_SOURCES = ["engine.h", "lpu_finish.h", "lpu_device.h", "lpu_internal.h"]
CLASS_SOURCE = {"dct": ["engine_dct.hip"] + _SHARED_SOURCES,
                "spmv": ["engine_kernels.hip"] + _SHARED_SOURCES,
                "update": ["engine_kernels.hip"] + _SHARED_SOURCES}


def measured_traffic(cls, dct_mode, maps):
    """Bytes per launch of kernel class `cls` from the committed counter summary,
    or None when the summary is missing, was taken on another workload, or the
    kernel's source (its file or a header it includes) has changed since."""
    import hashlib
    if cls not in CLASS_SOURCE or maps != 256 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    fields = {}
    for line in open(TRAFFIC_PROFILE):
        parts = line.split()
        if len(parts) == 3 and parts[0] in ("traffic_bytes_per_launch", "source_sha256"):
            fields[(parts[0], parts[1])] = parts[2]
        elif len(parts) == 2 and parts[0] == "dct_mode":
            fields["dct_mode"] = parts[1]
    for src in CLASS_SOURCE[cls]:
        path = os.path.join(ROOT, "paper_2203_13675_amd", "csrc", src)
        digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
        if fields.get(("source_sha256", src)) != digest:
            return None
    if fields.get("dct_mode") != dct_mode:
        return None
    v = fields.get(("traffic_bytes_per_launch", cls))
    return float(v) if v is not None else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--maps", type=int, default=256)
    ap.add_argument("--workload", default="batch256",
                    choices=["batch256", "peaks64", "peaks1024", "gauss2048_hole", "ramp4096"],
                    help="batch256 (default, the benchmark line) or one of the single-map "
                         "workloads, run through the same path for profiling")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"],
                    help="mixed (default) or the plain FP64 path (the 64x64 case's setting)")
    ap.add_argument("--outer", type=int, default=10)
    ap.add_argument("--dct-mode", default="fp16_scaled")
    ap.add_argument("--fp64-compare", type=int, default=1,
                    help="also time the plain FP64 sequential loop once (0: skip)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--profile", action="store_true", help="fewer steps, no extras (for rocprof)")
    ap.add_argument("--graph", type=int, default=1, help="graph-captured PCG iterations (0: eager)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="run the library's autotuner on the batch first (not timed)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB copied by a plain device copy after the run (counter calibration)")
    return ap.parse_args()


def dct_floor_record(dct_bytes, dct_ms):
    """The DCT preconditioner as four dense contractions moves 24 B/px per
    application on the benchmark path (tables aside); a fast O(n log n)
    transform needs at least one read of r and one write of s, 8 B/px.  The
    time that floor takes at HBM peak, against the stages' measured time
    (dct_bytes: the stages' algorithmic bytes over the step)."""
    floor_ms = dct_bytes * (8.0 / 24.0) / (PEAK_HBM_GBS * 1e9) * 1e3
    return {"floor_ms_per_step": floor_ms, "dct_ms_per_step": dct_ms, "frac": floor_ms / dct_ms,
            "note": "HBM time of 8 B/px per preconditioner application (read r, write s) at "
                    "8 TB/s over the step's applications, against the four contraction stages' "
                    "measured time"}


def iteration_record(shapes, its, n_spmv):
    """How full the PCG launches can be.  Every launch of an iteration covers
    the maps still iterating; the batch needs at least as many iteration
    launches as its slowest map has iterations, however the maps are
    scheduled, so sum(px * iters) / (max iters * total px) bounds the mean
    fraction of the batch's pixels per launch."""
    px_m = [m * n for m, n in shapes]
    total_px = sum(px_m)
    work = sum(p * i for p, i in zip(px_m, its))
    return {
        "per_map": {"min": min(its), "median": float(np.median(its)),
                    "p90": float(np.percentile(its, 90)), "max": max(its)},
        "spmv_launches": n_spmv,
        "launch_fill": work / (n_spmv * total_px) if n_spmv else None,
        "launch_fill_bound": work / (max(its) * total_px) if max(its) > 0 else None,
        "note": "launch_fill: pixel-iterations / (SpMV launches x batch pixels); "
                "launch_fill_bound: the same with the slowest map's iteration count as the "
                "launch count, the best any schedule of these maps reaches"}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: lp_unwrap runs on one GPU; --gpus %d is not supported "
              "(the maps of a batch are independent, so a batch would shard across GPUs "
              "by map)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    # The oracle's worker processes are started before anything touches the
    # GPU (no process that has initialised the GPU starts another program) and
    # stay idle until the GPU work is done.
    pool = None
    if a.cpu_baseline and not a.profile and a.workload == "batch256":
        pool = CpuPool()
    import torch
    from paper_2203_13675_amd import synth
    from paper_2203_13675_amd.binding import Context, default_options, KERNEL_CLASSES

    dev = torch.device("cuda:0")
    masks = None
    if a.workload == "batch256":
        shapes = synth.batch_sizes(a.maps, seed=3000)
        maps = synth.batch_maps(a.maps, seed=3000)
        desc = ("batch of %d uneven random-Gaussian maps (sides in {128..1024}), p=0, tau=0.01, "
                "%d outer iterations, DCT preconditioner, relres 1e-6" % (a.maps, a.outer))
    else:
        psi1, mask1, truth1 = synth.workload(a.workload)
        shapes = [psi1.shape]
        maps = [(psi1, truth1)]
        if mask1 is not None:
            masks = [torch.from_numpy(mask1).to(dev)]
        desc = ("%s: one %dx%d map, p=0, tau=0.01, %d outer iterations, DCT preconditioner, "
                "relres 1e-6" % ((a.workload,) + tuple(psi1.shape) + (a.outer,)))
    total_px = sum(m * n for m, n in shapes)
    psis = [torch.from_numpy(p).to(dev) for p, _ in maps]
    phis = [torch.zeros_like(t) for t in psis]
    opts = dict(p=0.0, eps=0.01, preconditioner="dct", tol=1e-6)
    ctx = Context(0)
    o = default_options(precision=a.precision, dct_mode=a.dct_mode, k_max=a.outer, outer_tol=0.0)
    fp64 = a.precision == "fp64"

    def step():
        return ctx.batch(psis, masks, phis=phis, options=o, **opts)

    tune = None
    if a.autotune:
        best, tune_ms = ctx.autotune(psis, masks, phis=phis, options=o, probe_iters=20,
                                     cache_path=a.tune_cache, **opts)
        tune = {"tuning": best, "autotune_ms": tune_ms}
    ctx.set_tuning(use_graph=a.graph)

    for _ in range(max(1, a.warmup)):
        step()
    torch.cuda.synchronize()
    # timed region: the production path, no instrumentation.  Python's cyclic
    # garbage collector is paused meanwhile (as timeit does): a full collection
    # in a process holding torch takes tens of milliseconds and has nothing to
    # do with the library's work
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    stats = None
    for _ in range(a.steps):
        _, rc, stats = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    gc.enable()
    # kernel timing pass: one more step of the same workload with every kernel
    # class bracketed by HIP events on the library's stream (launch by launch:
    # events cannot be read per replay inside a captured graph)
    ctx.kernel_timing("all")
    tk0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - tk0
    ktimes = ctx.kernel_timing_report()
    ctx.kernel_timing("off")
    warm_split = {k: v["ms"] for k, v in ktimes.items()}
    # every class's algorithmic rate over its launches in the timing pass
    classes = {}
    for k, v in ktimes.items():
        if v["ms"] <= 0 or v["bytes"] <= 0:
            continue
        gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9
        c = {"launches": v["launches"], "avg_launch_us": v["ms"] * 1e3 / max(v["launches"], 1),
             "alg_GBps": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
        if v["flops"] > 0:
            c["TFLOPps"] = v["flops"] / (v["ms"] * 1e-3) / 1e12
        classes[k] = c

    value = total_px / dt / 1e6
    inner = sum(s["inner_iters_total"] for s in stats)
    worst_relres = max(s["final_relres"] for s in stats)

    # dominant kernel class by summed time
    dom = max(ktimes.items(), key=lambda kv: kv[1]["ms"]) if ktimes else None
    roofline = None
    if dom:
        name, kt = dom
        launches = max(kt["launches"], 1)
        per_launch_s = kt["ms"] / 1e3 / launches
        traffic = (measured_traffic(name, a.dct_mode, a.maps)
                   if a.workload == "batch256" and not fp64 else None)
        common = {"kernel": name, "traffic": traffic, "traffic_unit": "bytes per launch",
                  "alg_bytes_per_launch": kt["bytes"] / launches,
                  "alg_flops_per_launch": kt["flops"] / launches,
                  "avg_launch_us": per_launch_s * 1e6, "launches": kt["launches"]}
        # the binding roof is the one whose time at peak is longer: MFMA when
        # the launch's flops per algorithmic byte exceed the ridge point
        # (peak flops / peak bandwidth), HBM otherwise
        # (on the plain FP64 path the DCT stages run on the FP64 FMA units)
        peak_flops = PEAK_FP64_TFLOPS if fp64 else PEAK_FP16_TFLOPS
        ridge = peak_flops * 1e12 / (PEAK_HBM_GBS * 1e9)
        intensity = kt["flops"] / kt["bytes"] if kt["bytes"] > 0 else float("inf")
        common["flops_per_byte"] = intensity
        common["ridge_flops_per_byte"] = ridge
        if kt["flops"] > 0:
            tf = kt["flops"] / launches / per_launch_s / 1e12
            common["fma_achieved_tflops" if fp64 else "mfma_achieved_tflops"] = tf
            common["fma_frac" if fp64 else "mfma_frac"] = tf / peak_flops
        if kt["flops"] > 0 and intensity >= ridge:
            ach = kt["flops"] / launches / per_launch_s / 1e12
            roofline = {"bound": "alu" if fp64 else "mfma", "achieved": ach, "peak": peak_flops,
                        "unit": "TFLOP/s", "frac": ach / peak_flops, **common}
        else:
            ach = kt["bytes"] / launches / per_launch_s / 1e9
            roofline = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, **common}

    out = {
        "metric": "Mpixel/s unwrapped at 1e-6 rel. residual; batched mixed-prec vs plain FP64",
        "value": value, "unit": "Mpixel/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if fp64 else "f32", "data": "synthetic",
        "config": {"workload": desc,
                   "maps": len(shapes), "total_pixels": total_px, "outer_iters": a.outer,
                   "precision": ("fp64: the plain path, FP64 throughout" if fp64 else
                                 "mixed: f32 CG vectors, %s DCT on MFMA, f64 dots and "
                                 "residual refinement" % a.dct_mode)},
        "pcg_iters_per_step": inner, "cg_iters_per_s": inner / dt,
        # iterations are issued in rounds over every map still iterating, so
        # the slowest map's count is the number of rounds
        "us_per_iteration_round": dt * 1e6 / max(1, max(s["inner_iters_total"] for s in stats)),
        "worst_final_relres": worst_relres,
        "kernel_ms_per_step": warm_split,
        "kernel_classes": classes,
        "ms_per_step_timing_pass": t_eager * 1e3,
        "issue": "graph" if a.graph else "eager",
        "roofline": roofline,
    }
    if tune:
        out["autotune"] = tune
    if "dct" in ktimes and ktimes["dct"]["ms"] > 0 and not fp64 and a.dct_mode == "fp16_scaled":
        out["dct_fast_transform_floor"] = dct_floor_record(ktimes["dct"]["bytes"],
                                                           ktimes["dct"]["ms"])
    out["iterations"] = iteration_record(shapes, [s["inner_iters_total"] for s in stats],
                                         ktimes.get("spmv", {}).get("launches", 0))

    gpu_phis = [ph.cpu().numpy() for ph in phis]
    if a.fp64_compare and not a.profile and not fp64:
        o64 = default_options(precision="fp64", k_max=a.outer, outer_tol=0.0)
        # the same batch in one call at FP64: the precision's share of the gain
        ctx.batch(psis, masks, phis=[torch.zeros_like(t) for t in psis], options=o64, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st64 = ctx.batch(psis, masks, phis=[torch.zeros_like(t) for t in psis], options=o64,
                               **opts)
        torch.cuda.synchronize()
        tb64 = time.perf_counter() - t0
        out["fp64_batched"] = {"value": total_px / tb64 / 1e6, "unit": "Mpixel/s",
                               "seconds": tb64,
                               "pcg_iters": sum(x["inner_iters_total"] for x in st64)}
        # plain FP64, map by map; one untimed solve of the largest map first, so
        # the timed loop reuses work buffers sized for it
        big = max(range(len(psis)), key=lambda k: psis[k].numel())
        ctx.solve(psis[big], masks[big] if masks is not None else None,
                  phi=torch.zeros_like(psis[big]), options=o64, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it64 = 0
        for k, (ps, ph) in enumerate(zip(psis, phis)):
            mk = masks[k] if masks is not None else None
            it64 += ctx.solve(ps, mk, phi=ph, options=o64, **opts).stats["inner_iters_total"]
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        out["fp64_sequential"] = {"value": total_px / t64 / 1e6, "unit": "Mpixel/s",
                                  "seconds": t64, "pcg_iters": it64}
        out["speedup_vs_fp64_sequential"] = out["value"] / out["fp64_sequential"]["value"]
        out["speedup_vs_fp64_batched"] = out["value"] / out["fp64_batched"]["value"]

    if a.calib_copy > 0:
        # plain copy of known size, for scaling the HBM byte counters
        n = a.calib_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes_each"] = 2 * n * 4

    ctx.close()
    if pool is not None:
        cpu, err = pool.run(shapes, a.outer, gpu_phis)
        out["cpu_baseline"] = cpu
        out["err_vs_oracle"] = err
    print(json.dumps(out))


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host cores
# ---------------------------------------------------------------------------
CPU_SAMPLE_STRIDE = 16  # every 16th map of the batch (16 of 256)
CPU_WORKERS_MAX = 16    # the host share of one GPU


def _oracle_map(args):
    """One map of the batch through the oracle, single-threaded, at the
    benchmark's settings (FP64, DCT, inner relres `tol`).  Returns
    (k, phi, seconds)."""
    k, n_maps, outer, tol = args
    from oracle import lp_oracle
    from paper_2203_13675_amd import synth
    psi, _ = synth.batch_map(k, n_maps, seed=3000)
    t0 = time.perf_counter()
    r = lp_oracle.unwrap(psi, p=0.0, tau=0.01, precond="dct", tol=tol, k_max=outer,
                         outer_tol=0.0, l_max=4000 if tol < 1e-6 else None)
    return k, r.phi, time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class CpuPool:
    """Single-threaded oracle workers, one per host core available to this
    process (at most 16), started before the GPU is initialised."""

    def __init__(self):
        import multiprocessing as mp
        try:
            avail = len(os.sched_getaffinity(0))
        except AttributeError:
            avail = os.cpu_count() or 1
        self.workers = max(1, min(CPU_WORKERS_MAX, avail))
        self.host_cores = avail
        for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[var] = "1"
        self.pool = mp.get_context("spawn").Pool(self.workers)

    def run(self, shapes, outer, gpu_phis):
        """The oracle on every CPU_SAMPLE_STRIDE-th map of the batch, one map per
        worker at a time, largest first.  Returns the CPU-baseline record (all
        workers: sample pixels / wall time; single-threaded: sample pixels / the
        summed per-map times) and the GPU's distance to the oracle's answers."""
        n = len(shapes)
        sample = list(range(0, n, CPU_SAMPLE_STRIDE))
        sides = {s for k in sample for s in shapes[k]}
        for k in range(n):  # every side length of the batch appears in the sample
            if not set(shapes[k]) <= sides:
                sample.append(k)
                sides |= set(shapes[k])
        order = sorted(sample, key=lambda k: -shapes[k][0] * shapes[k][1])
        t0 = time.perf_counter()
        res = self.pool.map(_oracle_map, [(k, n, outer, 1e-6) for k in order], chunksize=1)
        wall = time.perf_counter() - t0
        # untimed: the same maps with exact inner solves (relres 1e-12)
        exact = dict((k, phi) for k, phi, _ in
                     self.pool.map(_oracle_map, [(k, n, outer, 1e-12) for k in order], chunksize=1))
        self.pool.close()
        self.pool.join()
        px = sum(shapes[k][0] * shapes[k][1] for k in sample)
        busy = sum(r[2] for r in res)
        dm = lambda a: a - a.mean()
        d_same, d_exact, d_orc = [], [], []
        for k, same, _ in res:
            g = dm(gpu_phis[k])
            d_same.append(float(np.abs(g - dm(same)).max()))
            d_exact.append(float(np.abs(g - dm(exact[k])).max()))
            d_orc.append(float(np.abs(dm(same) - dm(exact[k])).max()))
        cpu = {"value": px / wall / 1e6, "unit": "Mpixel/s", "cores": self.workers,
               "kind": "oracle",
               "single_thread_value": px / busy / 1e6,
               "cpu_model": _cpu_model(), "host_cores_available": self.host_cores,
               "sample": "%d maps of the batch (every %dth, every side length present; %.2f Mpx, "
                         "%s), same settings as the GPU step (FP64, DCT, relres 1e-6, %d outer "
                         "iterations); value: %d single-threaded oracle processes, each taking "
                         "the next map (largest first), sample pixels / %.1f s wall; "
                         "single_thread_value: sample pixels / %.1f s summed per-map time"
                         % (len(sample), CPU_SAMPLE_STRIDE, px / 1e6,
                            ",".join("%dx%d" % shapes[k] for k in sorted(sample)), outer,
                            self.workers, wall, busy)}
        stat = lambda v: {"max_abs_rad": max(v), "median_abs_rad": float(np.median(v))}
        err = {"maps": len(res),
               "vs_oracle_same_tolerance": stat(d_same),
               "vs_oracle_exact_inner": stat(d_exact),
               "oracle_same_tolerance_vs_exact_inner": stat(d_orc),
               "per_map_rad": {"%d:%dx%d" % ((k,) + shapes[k]): [round(a, 9), round(b, 9),
                                                                  round(c, 9)]
                               for (k, *_), a, b, c in zip(res, d_same, d_exact, d_orc)},
               "note": "max |phi - oracle| with the mean removed per map, on the CPU-baseline "
                       "sample.  vs_oracle_same_tolerance: the FP64 oracle running Algorithm 1 "
                       "with the GPU's preconditioner and inner tolerance (relres 1e-6); "
                       "vs_oracle_exact_inner: the oracle with exact inner solves (relres "
                       "1e-12); the third entry is how far the oracle's own same-tolerance "
                       "answer is from its exact one.  per_map_rad: these three per map.  With "
                       "p = 0 the outer fixed-point loop can settle on different fixed points "
                       "under rounding-level differences, so a map may differ by radians "
                       "between any two solves at relres 1e-6"}
        return cpu, err


if __name__ == "__main__":
    main()
