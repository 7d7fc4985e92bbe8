"""Benchmark: DDA time-to-solution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ellipsoid51k]

A step is one whole solve of a workload's right-hand sides (an orientation
is two of them, the two polarizations): interaction-tensor sampling and FFT,
polarizabilities, incident field, BiCGSTAB to the tolerance, the true and
normal-equation residual checks and the efficiencies.  Multi-target
workloads go through one batched call.  Inputs are synthetic (seeded lattice
targets); nothing is cached between steps.

Prints one JSON line: the metric value is seconds per orientation; the
``roofline`` object reports the dominant kernel's algorithmic HBM bytes per
launch over its average launch time (HIP events on the library's stream over
the timed steps) against MI355X's 8 TB/s; ``cpu_baseline`` times the CPU
oracle (FFT-BiCGSTAB in FP64) on one polarization of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMING_SAMPLE = 4   # HIP events on every 4th launch of the timed pass
METRIC = "DDA time-to-solution (s/orientation at 1e-5 residual); FFT-matvec HBM GB/s"

WORKLOADS = {
    # name: (description, precision)
    "ellipsoid51k": ("ellipsoid, semi-axes 32/24/16 on a 64x48x32 box (N=51488), m=1.5+0.02i, x=5, LATTDR, "
                     "BiCGSTAB to 1e-5, FFT grid 128x96x64, incidence +x, polarizations y and z", "fp64"),
    "sphere389": ("integer-site sphere r=4.5 (N=389), m=1.33+0.01i, x=1, LATTDR, BiCGSTAB to 1e-8, FFT grid 18^3",
                  "fp64"),
    "au_brick": ("16x32x32 gold brick (N=16384), m=0.9656+1.8628i, x=3.093665, BiCGSTAB to 1e-5, FFT grid 32x64x64",
                 "fp64"),
    "sphere1m": ("sphere of radius 64 in a 128^3 box (N=1099136), m=1.33+0.01i, x=20, LATTDR, BiCGSTAB to 1e-5, "
                 "FFT grid 256^3", "fp64"),
    "brick48": ("48x24x16 brick (N=18432), m=1.6+0.1i, x=4, 64 random orientations x 2 polarizations = 128 "
                "right-hand sides in one solve, BiCGSTAB to 1e-5, FFT grid 96x48x32", "fp64"),
    "config3": ("the 48x24x16 brick at 64 orientations x 2 polarizations plus 32 integer-site spheres with radii "
                "U(6,20) (x=4, m=1.33+0.01i) x 2 polarizations, one batched call, BiCGSTAB to 1e-5", "fp64"),
}


def build_jobs(dda, w, name, seed, prec, solver="bicgstab"):
    """[(target, options, khat, e0)] of a workload, and orientations per step."""
    if name == "config3":
        d = w.workload("brick48", seed)
        kh_s, e0_s = w.along_x_yz()
        jobs = [(dda.Target(d["ijk"], d["m"]),
                 dda.Options.for_size_parameter(d["x"], tol=d["tol"], precision=prec, recompute_green=True,
                                                solver=solver),
                 d["khat"], d["e0"])]
        for s_ijk in w.sphere_batch(seed):
            jobs.append((dda.Target(s_ijk, 1.33 + 0.01j),
                         dda.Options.for_size_parameter(4.0, tol=1e-5, precision=prec, recompute_green=True,
                                                        solver=solver),
                         kh_s, e0_s))
        return jobs, 64 + 32, d
    d = w.workload(name, seed)
    opts = dda.Options.for_size_parameter(d["x"], tol=d["tol"], precision=prec, recompute_green=True,
                                          solver=solver)
    return [(dda.Target(d["ijk"], d["m"]), opts, d["khat"], d["e0"])], len(d["khat"]) / 2.0, d


PASSES = ["scatter_fft_x", "fft_y_fwd", "fft_z_green", "fft_y_inv", "fft_x_gather"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """Digest of the sources that define the FFT pass kernels."""
    h = hashlib.sha256()
    for f in ("dda_device.h", "dda_passes.h", "dda_kernels.h"):
        with open(os.path.join(ROOT, "paper_1202_3424_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pass_bytes(tgt, n_sites: int, csize: int) -> dict:
    """Algorithmic HBM bytes of each matvec pass for one right-hand side
    (one read and one write of exactly the data the pruned pass needs)."""
    nx, ny, nz = tgt.box
    Mx, My, Mz = tgt.grid
    Hx, Hy, Hz = Mx // 2 + 1, My // 2 + 1, Mz // 2 + 1
    g = 3 * csize                       # three components per grid point
    site = 3 * n_sites * 16             # one FP64 site vector
    nbox = nx * ny * nz
    return {
        # write the x-transformed occupied lines; read the box map and on
        # average 2.5 site vectors, write 1 (p = r + beta(p - omega v) / s = r - alpha v)
        "scatter_fft_x": Mx * ny * nz * g + 4 * nbox + 3.5 * site,
        "fft_y_fwd": Mx * ny * nz * g + Mx * My * nz * g,
        "fft_z_green": 2 * Mx * My * nz * g + Hx * Hy * Hz * 6 * csize,
        "fft_y_inv": Mx * My * nz * g + Mx * ny * nz * g,
        # read the x lines, box map, materials, the input and one more site vector, write the output
        "fft_x_gather": Mx * ny * nz * g + 4 * nbox + 4 * n_sites + 3 * site,
    }


SLOT_OF_PASS = {"fft_y_fwd": 0, "fft_z_green": 1, "fft_y_inv": 2}


def load_traffic(kernel: str, workload: str, precision: str, variants):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, if it was taken on the current kernel sources
    and with the variant the autotuner chose in this run."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    slot = SLOT_OF_PASS.get(kernel)
    if slot is not None and (variants is None or rec.get("variant") != variants[slot]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(d: dict, workload: str, gpu_iters: int) -> dict:
    """The oracle (FFT-BiCGSTAB, FP64) on the first right-hand side of the
    workload, scaled to seconds per orientation (two polarizations).  Targets
    above 300k dipoles run a bounded number of iterations instead: two runs of
    2 and 4 iterations give the set-up and per-iteration cost, extrapolated to
    the iteration count the GPU solve needed for the same right-hand side."""
    workers = min(os.cpu_count() or 1, len(os.sched_getaffinity(0)), 16)
    os.environ["DDA_ORACLE_FFT_WORKERS"] = str(workers)
    import importlib

    from oracle import fftsolve
    importlib.reload(fftsolve)

    def run(max_iter):
        t0 = time.perf_counter()
        r = fftsolve.solve_case(d["ijk"], d["m"], d["x"], d["khat"][0], d["e0"][0], tol=d["tol"],
                                max_iter=max_iter)
        return time.perf_counter() - t0, r

    if len(d["ijk"]) <= 300_000:
        dt, r = run(1000)
        return {"value": 2 * dt, "unit": "s/orientation", "cores": workers, "kind": "oracle",
                "sample": f"{workload}: the first right-hand side solved by the CPU oracle (scipy.fft FFT-BiCGSTAB, "
                          f"FP64, tol {d['tol']:g}, {r['iters']} iterations, {r['matvecs']} matvecs) in {dt:.2f} s; "
                          f"value = 2 polarizations x that time",
                "qext": r["qext"], "qabs": r["qabs"]}
    t2, _ = run(2)
    t4, _ = run(4)
    per_iter = (t4 - t2) / 2
    setup = t2 - 2 * per_iter
    est = setup + per_iter * gpu_iters
    return {"value": 2 * est, "unit": "s/orientation", "cores": workers, "kind": "oracle",
            "sample": f"{workload}: CPU oracle (scipy.fft FFT-BiCGSTAB, FP64) on the first right-hand side, run for "
                      f"2 and 4 iterations ({t2:.1f} s, {t4:.1f} s): set-up {setup:.2f} s + {per_iter:.2f} s/iteration "
                      f"x {gpu_iters} iterations (the GPU solve's count at tol {d['tol']:g}); value = 2 polarizations "
                      f"x that estimate"}


def plain_reference(dda, np, torch, jobs, results, ms_per_step):
    """The plain method on the same workload: every right-hand side solved
    alone by BiCGSTAB with the FP64 matvec at the same tolerance, one after
    another, the tensor FFT of each target reused (outside the timed region).  Returns its time, the speedup of the measured step and the
    largest relative difference of each efficiency from it."""
    import dataclasses
    # the tensor FFT is computed once per target and reused by its solves
    opts64 = [dataclasses.replace(o, precision="fp64", recompute_green=False, solver="bicgstab")
              for _, o, _, _ in jobs]
    def run():
        out = []
        for (t, o, kh, e0), o64 in zip(jobs, opts64):
            for q in range(len(kh)):
                out.append(dda.solve(t, o64, kh[q:q + 1], e0[q:q + 1], want_P=False)[1][0])
        return out
    run()   # tensor FFTs and autotuning, as in the measured warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    diff = {}
    for k in ("qext", "qabs", "qsca"):
        diff[k] = max(abs(r[k] - p[k]) / abs(p[k]) for r, p in zip(results, ref))
    return {"ms": ms, "speedup": ms / ms_per_step, "max_rel_diff": diff,
            "note": "each right-hand side solved alone with the FP64 matvec at the same tolerance, tensor FFT "
                    "reused; max_rel_diff compares the measured step's efficiencies with these"}


def copy_probe(mib: int = 1024, reps: int = 4):
    """A plain device-to-device copy of known size (torch's copy kernel), for
    scaling the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "copies": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ellipsoid51k", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32_matvec"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 single-RHS comparison")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--solver", default="bicgstab", choices=["bicgstab", "qmr", "bicgstab2"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding of the "
              "right-hand sides is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1202_3424_amd as dda
    import workloads as w

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    desc, prec = WORKLOADS[args.workload]
    prec = args.precision or prec
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    jobs, orientations, d = build_jobs(dda, w, args.workload, args.seed, prec, args.solver)
    torch.cuda.synchronize()
    target_create_ms = (time.perf_counter() - t_create) * 1e3
    n_rhs = sum(len(j[2]) for j in jobs)
    log(f"workload {args.workload}: {len(jobs)} target(s), {n_rhs} right-hand sides, prec={prec}, "
        f"first target N={jobs[0][0].n_sites} grid={jobs[0][0].grid}")

    def step():
        if len(jobs) == 1:
            t, o, kh, e0 = jobs[0]
            return dda.solve(t, o, kh, e0, want_P=False)[1]
        rt = [i for i, j in enumerate(jobs) for _ in range(len(j[2]))]
        kh = np.vstack([j[2] for j in jobs])
        e0 = np.vstack([j[3] for j in jobs])
        return dda.solve_batched([j[0] for j in jobs], [j[1] for j in jobs], rt, kh, e0, want_P=False)[1]

    def job_units(results):
        """RHS-matvec units each job executed (iteration matvecs + 3 checks per RHS)."""
        out, k = [], 0
        for j in jobs:
            n = len(j[2])
            out.append(sum(r["matvecs"] for r in results[k:k + n]) + 3 * n)
            k += n
        return out

    csize = 8 if prec == "fp32_matvec" else 16
    bpus = [pass_bytes(j[0], j[0].n_sites, csize) for j in jobs]

    def pass_traffic(name, units):
        return sum(b[name] * u for b, u in zip(bpus, units))

    # warmup; the last warmup step times every kernel category to find the
    # dominant matvec pass, which alone is timed during the measured steps
    for i in range(max(args.warmup, 1)):
        if i == max(args.warmup, 1) - 1:
            dda.set_timing(True)
        res = step()
        log(f"warmup {i}: iters={[r['iters'] for r in res][:8]} status={set(r['status'] for r in res)}")
    calib = dda.get_timing()
    dda.set_timing(False)
    cal_units = job_units(res)
    dominant = max(PASSES, key=lambda k: calib[k][0])
    log(f"dominant matvec kernel: {dominant} ({calib[dominant][0]:.3f} ms in the last warmup step)")

    # events on every TIMING_SAMPLE-th launch of the dominant pass only (a
    # systematic sample over the timed steps; the others carry no event cost)
    dda.set_timing([dominant])
    dda.set_timing_sample(TIMING_SAMPLE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units = [0] * len(jobs)
    results = None
    for i in range(args.steps):
        results = step()
        units = [a + b for a, b in zip(units, job_units(results))]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = dda.get_timing()
    dda.set_timing(False)
    dda.set_timing_sample(1)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    s_per_orientation = ms_per_step / 1e3 / orientations
    for r in results:
        if r["status"] != 0:
            raise SystemExit(f"solve did not converge: {r}")
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step; results {results[0]}")

    ms_tot, launches, all_launches = timing[dominant]
    bytes_tot = pass_traffic(dominant, units)
    # algorithmic bytes per launch (all launches) over the sampled average launch time
    avg_s = ms_tot * 1e-3 / launches
    gbs = bytes_tot / all_launches / avg_s / 1e9
    variants = dda.tuned_variants(jobs[0][0], len(jobs[0][2]), prec) if len(jobs) == 1 else None
    traffic = load_traffic(dominant, args.workload, prec, variants) if len(jobs) == 1 else None
    roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": dominant,
                "algorithmic_bytes_per_launch": bytes_tot / all_launches, "avg_launch_us": avg_s * 1e6,
                "launches": all_launches, "timed_launches": launches}
    # every pass, from the calibration step (one warmup step with all categories timed)
    passes = {}
    for name in PASSES:
        ms, nl, _ = calib[name]
        if nl == 0 or ms == 0:
            continue
        g = pass_traffic(name, cal_units) / (ms * 1e-3) / 1e9
        passes[name] = {"ms_per_launch": ms / nl, "launches": nl, "bytes_per_rhs_matvec": bpus[0][name],
                        "GBps": g, "frac": g / HBM_PEAK_GBS}
    matvec_ms = sum(calib[k][0] for k in PASSES)
    matvec_bytes = sum(pass_traffic(k, cal_units) for k in PASSES)
    out = {
        "metric": METRIC,
        "value": s_per_orientation,
        "unit": "s/orientation",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32 matvec / f64 Krylov",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "solver": args.solver, "targets": len(jobs),
                   "n_sites": [j[0].n_sites for j in jobs][:4], "fft_grid": list(jobs[0][0].grid),
                   "rhs_per_step": n_rhs, "orientations_per_step": orientations, "precision": prec,
                   "seed": args.seed},
        "roofline": roofline,
        "autotuned_variants": variants,
        "target_create_ms": target_create_ms,
        "matvec": {"GBps_all_passes": matvec_bytes / (matvec_ms * 1e-3) / 1e9,
                   "units_per_step": sum(units) / args.steps, "passes_calibration_step": passes},
        "kernel_ms_calibration_step": {k: v[0] for k, v in calib.items()},
        "solver": {"iters": [r["iters"] for r in results][:8], "matvecs": [r["matvecs"] for r in results][:8],
                   "qext": [r["qext"] for r in results][:8], "qabs": [r["qabs"] for r in results][:8],
                   "qsca": [r["qsca"] for r in results][:8], "rel_residual": [r["rel_residual"] for r in results][:8],
                   "normal_eq_residual": [r["normal_eq_residual"] for r in results][:8],
                   "refinements": [r["refinements"] for r in results][:8]},
    }
    if not args.no_plain:
        log("timing the plain FP64 single-right-hand-side solves of the same workload ...")
        out["vs_plain_fp64_single_rhs"] = plain_reference(dda, np, torch, jobs, results, ms_per_step)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on one polarization ...")
        out["cpu_baseline"] = cpu_baseline(d, args.workload, results[0]["iters"])
        if args.workload == "config3":
            out["cpu_baseline"]["sample"] += " (the brick's orientations; the spheres are smaller)"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
