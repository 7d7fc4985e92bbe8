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
                 "FFT grid 256^3, incidence +x, polarizations y and z; FP32 FFT matvec with FP64 Krylov "
                 "recurrences, inner products and residual refinement unless --precision fp64", "fp32_matvec"),
    "brick48": ("48x24x16 brick (N=18432), m=1.6+0.1i, x=4, 64 random orientations x 2 polarizations = 128 "
                "right-hand sides in one solve, BiCGSTAB to 1e-5, FFT grid 96x48x32", "fp64"),
    "au_sphere_nf": ("the guide's near-field example: 48^3-box gold pseudosphere (N=59728), m=0.96+1.01i, x=5, "
                     "GKDLDR, BiCGSTAB to 1e-5, FFT grid 96^3; then E on the 96^3 volume grown by half the box on "
                     "every side (FFT grid 192^3), timed separately", "fp64"),
    "twomat40": ("40^3 brick, every site occupied, two materials (m=1.5+0.01i or 2.0+0.5i, each with probability "
                 "1/2), x=6, LATTDR, BiCGSTAB to 1e-5, FFT grid 80^3, incidence +x, polarization y; then the adjoint "
                 "gradient of Q_abs in the per-site permittivity, timed separately", "fp64"),
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
                                          solver=solver, polarizability=d.get("polarizability", "LATTDR"))
    return [(dda.Target(d["ijk"], d["m"]), opts, d["khat"], d["e0"])], len(d["khat"]) / 2.0, d


# the largest single-GPU configuration: its working set (two FP32 grids of
# 403 MB, the 103 MB tensor octant, the FP64 site vectors) exceeds the 256 MB
# Infinity Cache, so its pass bandwidths are HBM bandwidths
DEFAULT_WORKLOAD = "sphere1m"
# measured in the same run as the default line, for context (cache-resident)
EXTRA_WORKLOAD = "ellipsoid51k"

PASSES = ["scatter_fft_x", "fft_y_fwd", "fft_z_green", "fft_y_inv", "fft_x_gather"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """Digest of the sources that define the FFT pass kernels."""
    h = hashlib.sha256()
    for f in ("dda_device.h", "dda_passes.h"):
        with open(os.path.join(ROOT, "paper_1202_3424_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# FP64 site vectors (read + written) per scatter and per gather, averaged
# over the modes one iteration of each solver uses.  BiCGSTAB: the scatter
# of p reads r, p, v, x, t and writes r, p, x (the previous iteration's
# x += alpha p + omega s, r = s - omega t, then p = r + beta(p - omega v));
# the scatter of s = r - alpha v reads r, v, rhat and writes r; each gather
# reads its input and rhat and writes its output.  QMR: the scatter reads r,
# p and the smoothed pair (s, y) and x, and writes p, s, y; the gather reads
# p and writes v.  BiCGstab(2): 3, 6, 6 and 9 vectors in the four scatters,
# 3 in every gather.  The plain product (near field): its input, and input
# plus output.
SITE_VECTORS = {"bicgstab": (6, 3), "qmr": (8, 2), "bicgstab2": (6, 3), "plain": (1, 2)}


def pass_bytes(tgt, n_sites: int, csize: int, solver: str = "bicgstab") -> dict:
    """Algorithmic HBM bytes of each matvec pass: one read and one write of
    exactly the data the pruned pass needs.  Returns {pass: (per right-hand
    side, once per launch)}: the grids and site vectors belong to each
    right-hand side; the tensor octant, the box map and the materials are
    shared by every right-hand side of a launch (the R of the pruned model's
    6M/R term)."""
    nx, ny, nz = tgt.box
    Mx, My, Mz = tgt.grid
    Hx, Hy, Hz = Mx // 2 + 1, My // 2 + 1, Mz // 2 + 1
    g = 3 * csize                       # three components per grid point
    site = 3 * n_sites * 16             # one FP64 site vector
    nbox = nx * ny * nz
    sv_scatter, sv_gather = SITE_VECTORS[solver]
    return {
        # write the x-transformed occupied lines; the solver's site vectors;
        # the box map once
        "scatter_fft_x": (Mx * ny * nz * g + sv_scatter * site, 4 * nbox),
        "fft_y_fwd": (Mx * ny * nz * g + Mx * My * nz * g, 0),
        "fft_z_green": (2 * Mx * My * nz * g, Hx * Hy * Hz * 6 * csize),
        "fft_y_inv": (Mx * My * nz * g + Mx * ny * nz * g, 0),
        # read the x lines and the solver's site vectors; the box map and
        # materials once
        "fft_x_gather": (Mx * ny * nz * g + sv_gather * site, 4 * nbox + 4 * n_sites),
    }


SLOT_OF_PASS = {"fft_y_fwd": 0, "fft_z_green": 1, "fft_y_inv": 2}


def load_traffic(kernel: str, workload: str, precision: str, variants, rhs_matvecs_per_launch: float):
    """Measured HBM bytes per launch of this kernel: the committed rocprofv3
    counter summary's bytes per right-hand-side matvec for the variant the
    autotuner chose in this run, times this run's right-hand-side matvecs
    per launch (launches skip right-hand sides that have converged).  None
    unless the counters were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    slot = SLOT_OF_PASS.get(kernel)
    if slot is None or variants is None:
        return None
    v = rec.get("by_variant", {}).get(str(variants[slot]))
    return None if v is None else v["bytes_per_rhs_matvec"] * rhs_matvecs_per_launch


# kernel-name patterns of each pass's compile-time family (every variant)
PASS_PATTERNS = {
    "scatter_fft_x": r"k_scatter_x<",
    "fft_y_fwd": r"k_strided<(double|float), 3, 0, -1,|k_strided_rf<(double|float), 0, -1,",
    "fft_z_green": r"k_strided<(double|float), 3, 1, -1,|k_strided_rf<(double|float), 1, -1,|k_zfold<|k_zsq<",
    "fft_y_inv": r"k_strided<(double|float), 3, 0, 1,|k_strided_rf<(double|float), 0, 1,",
    "fft_x_gather": r"k_gather_x<",
}
AUTOTUNE_LAUNCHES = 21   # launches of each candidate while the autotuner times it (1 + 20)
# FFT lengths with compile-time kernels, and their autotuned variants per pass
CT_LENGTHS = (32, 48, 64, 80, 96, 128, 160, 192, 256, 384, 512)
CT_VARIANTS = {"fft_y_fwd": 12, "fft_z_green": 28, "fft_y_inv": 12}


def profile_commands(workload: str, prec: str, out: str = "/root/repo/gpurun_out/tr") -> dict:
    """The rocprofv3 runs behind the committed summaries (run from /tmp)."""
    wl = "" if workload == DEFAULT_WORKLOAD else f" --workload {workload}"
    pr = "" if prec == WORKLOADS[workload][1] else f" --precision {prec}"
    b = f"python -u /root/repo/bench.py{wl}{pr}"
    pre = "cd /tmp && export TMPDIR=/tmp && "
    return {
        "trace": pre + f"timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d {out}/kt -o run "
                       f"-- {b} --steps 20 --warmup 3 --no-cpu-baseline --no-plain --no-extra",
        "fetch": pre + f"timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/f -o run "
                       f"-- {b} --steps 2 --warmup 1 --no-cpu-baseline --no-plain --no-extra",
        "write": pre + f"timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/w -o run "
                       f"-- {b} --steps 2 --warmup 1 --no-cpu-baseline --no-plain --no-extra",
        "copy_fetch": pre + f"timeout -s KILL 60 rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/cf -o run "
                            f"-- python -u /root/repo/bench.py --copy-probe",
        "copy_write": pre + f"timeout -s KILL 60 rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/cw -o run "
                            f"-- python -u /root/repo/bench.py --copy-probe",
        "unprofiled": f"{b} --steps 20 --warmup 3 --no-cpu-baseline --no-plain --no-extra",
    }


def summarize_profiles(tr: str, workload: str, prec: str, unprofiled: str) -> None:
    """Write profiles/<pass>_<workload>_<prec>_traffic.json and
    profiles/dda_kernels_<workload>_<prec>_trace.txt from the outputs of
    ``profile_commands`` under ``tr`` (kt/, f/, w/, cf/, cw/ and the copy
    probe's log cf.log) and the unprofiled bench line in ``unprofiled``.

    Traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) times the factor
    that makes the same counter read the known size of a plain device copy.
    Every candidate of the dominant pass runs AUTOTUNE_LAUNCHES times on the
    real grid, in variant order, while the autotuner times it (pass 3's
    behind the forward y pass, as in the solve): those dispatches give each
    variant's bytes per full launch."""
    import csv
    import re
    import statistics

    def rows(p):
        with open(p) as fh:
            return list(csv.DictReader(fh))

    def short(n):
        return re.sub(r"\(.*", "", n.replace("dda::passes::", "").replace("dda::(anonymous namespace)::", "")
                      .replace("void ", ""))

    with open(os.path.join(tr, "cf.log")) as fh:
        nbytes = json.loads([ln for ln in fh if "copy_probe" in ln][0])["copy_probe_bytes_each_way"]
    cf = [float(r["Counter_Value"]) for r in rows(os.path.join(tr, "cf", "run_counter_collection.csv"))
          if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == "FETCH_SIZE"]
    cw = [float(r["Counter_Value"]) for r in rows(os.path.join(tr, "cw", "run_counter_collection.csv"))
          if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == "WRITE_SIZE"]
    fscale = nbytes / (statistics.mean(cf) * 1024)
    wscale = nbytes / (statistics.mean(cw) * 1024)
    with open(unprofiled) as fh:
        ub = json.loads(fh.read().strip().splitlines()[-1])
    with open(os.path.join(tr, "kt.json")) as fh:
        kt = json.loads(fh.read().strip().splitlines()[-1])
    dom = ub["roofline"]["kernel"]
    slot = SLOT_OF_PASS[dom]
    n_rhs = ub["config"]["rhs_per_step"]
    pat = re.compile(PASS_PATTERNS[dom])

    L_dom = ub["config"]["fft_grid"][SLOT_OF_PASS[dom] // 2 + 1]
    n_var = CT_VARIANTS[dom] if L_dom in CT_LENGTHS else 1

    def per_variant(path, counter, scale):
        fam = sorted((r for r in rows(path) if r["Counter_Name"] == counter and pat.search(r["Kernel_Name"])),
                     key=lambda r: int(r["Dispatch_Id"]))
        out = {}
        v = 0
        while v < n_var and (v + 1) * AUTOTUNE_LAUNCHES <= len(fam):
            grp = fam[v * AUTOTUNE_LAUNCHES:(v + 1) * AUTOTUNE_LAUNCHES]
            names = {short(r["Kernel_Name"]) for r in grp}
            if len(names) != 1:
                break
            out[v] = (names.pop(), statistics.mean(float(r["Counter_Value"]) for r in grp) * 1024 * scale)
            v += 1
        return out

    fv = per_variant(os.path.join(tr, "f", "run_counter_collection.csv"), "FETCH_SIZE", fscale)
    wv = per_variant(os.path.join(tr, "w", "run_counter_collection.csv"), "WRITE_SIZE", wscale)
    cal_dom = ub["matvec"]["passes_calibration_step"][dom]
    # a full launch: every right-hand side of the workload plus the shared bytes once
    alg_full = cal_dom["bytes_per_rhs_matvec"] * n_rhs + cal_dom.get("bytes_per_launch_shared", 0.0)
    by_variant = {}
    for v in sorted(set(fv) & set(wv)):
        if fv[v][0] != wv[v][0]:
            continue
        tot = fv[v][1] + wv[v][1]
        by_variant[str(v)] = {"kernel_name": fv[v][0], "fetch_bytes_per_launch": fv[v][1],
                              "write_bytes_per_launch": wv[v][1], "bytes_per_launch": tot,
                              "bytes_per_rhs_matvec": tot / n_rhs, "over_algorithmic": tot / alg_full}
    cmds = profile_commands(workload, prec, os.path.abspath(tr))
    chosen = ub["autotuned_variants"][slot] if ub.get("autotuned_variants") else None
    rec = {"kernel": dom, "workload": workload, "precision": prec, "rhs_per_launch": n_rhs,
           "variant_unprofiled_run": chosen, "algorithmic_bytes_per_full_launch": alg_full,
           "by_variant": by_variant, "fetch_scale": fscale, "write_scale": wscale,
           "source_sha256": kernel_source_digest(), "commands": cmds,
           "note": "bytes of one launch over all right-hand sides of the workload, from the autotuner's timing "
                   "launches of each variant on the real grid (FETCH_SIZE, WRITE_SIZE in KiB per dispatch, "
                   "averaged over those launches, times the copy-probe factors)"}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    ks = sorted(rows(os.path.join(tr, "kt", "run_kernel_stats.csv")), key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel-trace summary: {workload}, {prec}",
             f"# command: {cmds['trace']}",
             "# source: run_kernel_stats.csv (top kernels; the autotuner's timing launches of each variant included)",
             f"{'kernel':72s} {'calls':>6s} {'total_us':>10s} {'avg_us':>8s} {'min_us':>7s} {'max_us':>8s} {'pct':>5s}"]
    for r in ks[:24]:
        lines.append(f"{short(r['Name'])[:72]:72s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e3:10.1f} "
                     f"{float(r['AverageNs']) / 1e3:8.2f} {float(r['MinNs']) / 1e3:7.2f} "
                     f"{float(r['MaxNs']) / 1e3:8.2f} {float(r['Percentage']):5.1f}")
    kv = kt["autotuned_variants"][slot] if kt.get("autotuned_variants") else None
    kname = by_variant.get(str(kv), {}).get("kernel_name")
    krow = next((r for r in ks if kname and short(r["Name"]) == kname), None)
    rf, urf = kt["roofline"], ub["roofline"]
    lines += ["",
              f"# dominant pass {dom}; autotuned variants (y fwd, z, y inv): profiled run {kt.get('autotuned_variants')}, "
              f"unprofiled run {ub.get('autotuned_variants')}",
              f"#   profiled run: variant {kv} = {kname}: rocprofv3 average "
              f"{float(krow['AverageNs']) / 1e3 if krow else float('nan'):.2f} us/launch over {krow['Calls'] if krow else 0} "
              f"launches; the same run's HIP events {rf['avg_launch_us']:.2f} us/launch (profiler overhead included)",
              f"#   unprofiled run ({cmds['unprofiled']}): HIP events {urf['avg_launch_us']:.2f} us/launch over "
              f"{urf['launches']} launches, {urf['achieved']:.0f} GB/s algorithmic, frac {urf['frac']:.3f}; "
              f"ms/step {ub['ms_per_step']:.3f}",
              f"#   algorithmic bytes of a full launch ({n_rhs} right-hand sides, the shared tensor octant once): "
              f"{alg_full / 1e6:.2f} MB",
              f"#   counter scales from the copy probe: FETCH_SIZE x {fscale:.3f}, WRITE_SIZE x {wscale:.3f}",
              "#   measured HBM bytes of a full launch by variant, per right-hand side (fetch + write, x algorithmic):"]
    for v, e in by_variant.items():
        lines.append(f"#     {int(v):2d} {e['kernel_name'][:64]:64s} {e['fetch_bytes_per_launch'] / n_rhs / 1e6:7.2f} + "
                     f"{e['write_bytes_per_launch'] / n_rhs / 1e6:6.2f} MB  x{e['over_algorithmic']:.2f}")
    # every pass: HBM bytes per production launch (the autotuner's timing
    # launches left out) against the algorithmic bytes per launch of the
    # unprofiled run's calibration step, and over that step's launch time
    grid = ub["config"]["fft_grid"]
    frows = rows(os.path.join(tr, "f", "run_counter_collection.csv"))
    wrows = rows(os.path.join(tr, "w", "run_counter_collection.csv"))
    per_pass = {}
    for name, cal in ub["matvec"]["passes_calibration_step"].items():
        pp = re.compile(PASS_PATTERNS[name])
        L = grid[SLOT_OF_PASS[name] // 2 + 1] if name in SLOT_OF_PASS else None
        trials = AUTOTUNE_LAUNCHES * (CT_VARIANTS[name] if L in CT_LENGTHS else 1) if L else 0
        if name == "fft_y_fwd" and grid[2] in CT_LENGTHS:
            # pass 3's candidates are timed behind the chosen forward y pass:
            # one warm-up and twenty launches of it alone, then twenty per
            # candidate
            trials += AUTOTUNE_LAUNCHES + (AUTOTUNE_LAUNCHES - 1) * CT_VARIANTS["fft_z_green"]

        def prod(rs, counter, scale):
            fam = sorted((r for r in rs if r["Counter_Name"] == counter and pp.search(r["Kernel_Name"])),
                         key=lambda r: int(r["Dispatch_Id"]))[trials:]
            if not fam:
                return None, None
            # the kernel the counted run launched most (its autotuner's choice)
            top = statistics.mode(short(r["Kernel_Name"]) for r in fam)
            return statistics.mean(float(r["Counter_Value"]) for r in fam) * 1024 * scale, top
        (fb, kf), (wb, kw) = prod(frows, "FETCH_SIZE", fscale), prod(wrows, "WRITE_SIZE", wscale)
        if fb is None or wb is None or kf != kw:
            # the two counter runs' autotuners chose different variants of a
            # pass that ties: their production counts do not add up to one
            # kernel's.  Both runs make the autotuner's timing launches of
            # every variant (full launches, every right-hand side), which
            # give each of the two kernels' traffic instead.
            def tuned(rs, counter, scale, k):
                fam = sorted((r for r in rs if r["Counter_Name"] == counter and pp.search(r["Kernel_Name"])),
                             key=lambda r: int(r["Dispatch_Id"]))[:trials]
                v = [float(r["Counter_Value"]) for r in fam if short(r["Kernel_Name"]) == k]
                return statistics.mean(v) * 1024 * scale if v else None
            alg_full = cal["bytes_per_rhs_matvec"] * n_rhs + cal.get("bytes_per_launch_shared", 0.0)
            alts = {}
            for k in sorted({kf, kw} - {None}):
                f_, w_ = tuned(frows, "FETCH_SIZE", fscale, k), tuned(wrows, "WRITE_SIZE", wscale, k)
                if f_ is not None and w_ is not None:
                    alts[k] = {"bytes_per_full_launch": f_ + w_, "over_algorithmic": (f_ + w_) / alg_full}
            per_pass[name] = {"kernel_counted": f"{kf} / {kw}", "measured_bytes_per_launch": None,
                              "us_per_launch": cal["ms_per_launch"] * 1e3, "autotune_full_launches": alts}
            continue
        alg = cal["GBps"] * cal["ms_per_launch"] * 1e6
        per_pass[name] = {"kernel_counted": kf if kf == kw else f"{kf} / {kw}",
                          "measured_bytes_per_launch": fb + wb, "algorithmic_bytes_per_launch": alg,
                          "over_algorithmic": (fb + wb) / alg, "us_per_launch": cal["ms_per_launch"] * 1e3,
                          "measured_GBps": (fb + wb) / (cal["ms_per_launch"] * 1e-3) / 1e9,
                          "measured_frac": (fb + wb) / (cal["ms_per_launch"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    rec["passes"] = per_pass
    with open(os.path.join(ROOT, "profiles", f"{dom}_{workload}_{prec}_traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    lines += ["#   every pass, production launches (measured HBM bytes from the counters; time per launch from the",
              "#   unprofiled run's calibration step, whose autotuned variants are given above; the kernel counted",
              "#   is the one the counter runs launched, which may be another variant of a pass that ties):",
              f"#     {'pass':14s} {'us/launch':>9s} {'measured MB':>11s} {'x alg':>6s} {'measured GB/s':>13s} {'frac':>5s}"
              "  kernel counted"]
    for name, e in per_pass.items():
        if e["measured_bytes_per_launch"] is None:
            lines.append(f"#     {name:14s} the FETCH_SIZE and WRITE_SIZE runs launched different variants "
                         f"({e['kernel_counted']}); their autotuning launches (full launches):")
            for k, a in e.get("autotune_full_launches", {}).items():
                lines.append(f"#       {k[:70]:70s} {a['bytes_per_full_launch'] / 1e6:9.2f} MB  x{a['over_algorithmic']:.2f}")
            continue
        lines.append(f"#     {name:14s} {e['us_per_launch']:9.2f} {e['measured_bytes_per_launch'] / 1e6:11.2f} "
                     f"{e['over_algorithmic']:6.2f} {e['measured_GBps']:13.0f} {e['measured_frac']:5.2f}"
                     f"  {e['kernel_counted']}")
    with open(os.path.join(ROOT, "profiles", f"dda_kernels_{workload}_{prec}_trace.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def host_info(workers: int) -> dict:
    """The host the CPU baseline ran on: CPU model, threads used and visible,
    numpy and scipy versions."""
    import platform

    import numpy
    import scipy
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "threads_used": workers, "cpus_visible": len(os.sched_getaffinity(0)),
            "numpy": numpy.__version__, "scipy": scipy.__version__}


# the guide's own whole-run CPU seconds for its sample calculation nearest to
# each workload (context on other hardware, never the target)
GUIDE_CONTEXT = {
    "ellipsoid51k": {"guide_run": "ELLIPSOID sample: N=59,728 sphere in 48^3, m=1.5+0.01i, x=5, 2 polarizations",
                     "cpu_s": 63.0, "section": "Sample calculation in directory examples_exp/ELLIPSOID"},
    "au_brick": {"guide_run": "RCTGLPRSM sample: the 16x32x32 gold brick (this workload), PBCGS2, 2 polarizations",
                 "cpu_s": 10.0, "section": "Sample calculation in directory examples_exp/RCTGLPRSM"},
    "au_sphere_nf": {"guide_run": "ELLIPSOID_NEARFIELD sample (this workload): solve, then E on the 96^3 volume",
                     "cpu_s": 60.0, "nearfield_cpu_s": 9.6,
                     "section": "Sample calculation in directory examples_exp/ELLIPSOID_NEARFIELD"},
    "brick48": {"guide_run": "RCTGLPRSM run of 3 orientations x 2 polarizations on a 131,072-dipole brick",
                "cpu_s": 672.0, "section": "Running DDSCAT Using the Sample ddscat.par File"},
}


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
                                max_iter=max_iter, scheme=d.get("polarizability", "LATTDR"))
        return time.perf_counter() - t0, r

    if len(d["ijk"]) <= 300_000:
        dt, r = run(1000)
        return {"value": 2 * dt, "unit": "s/orientation", "cores": workers, "kind": "oracle",
                "host": host_info(workers),
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
            "host": host_info(workers),
            "sample": f"{workload}: CPU oracle (scipy.fft FFT-BiCGSTAB, FP64) on the first right-hand side, run for "
                      f"2 and 4 iterations ({t2:.1f} s, {t4:.1f} s): set-up {setup:.2f} s + {per_iter:.2f} s/iteration "
                      f"x {gpu_iters} iterations (the GPU solve's count at tol {d['tol']:g}); value = 2 polarizations "
                      f"x that estimate"}


def padded(n: int) -> int:
    """The library's padded FFT extent: the smallest compile-time FFT length
    (32 ... 512) >= 2n - 1 when at most 1.4 times the smooth extent, else the
    smooth extent (2n if 2,3,5-smooth, else the smallest smooth one >= 2n - 1)."""
    def smooth(m):
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        return m == 1
    if smooth(2 * n):
        m = 2 * n
    else:
        m = max(2 * n - 1, 1)
        while not smooth(m):
            m += 1
    for L in (32, 48, 64, 80, 96, 128, 160, 192, 256, 384, 512):
        if L >= 2 * n - 1:
            return L if 5 * L <= 7 * m else m
    return m


def nearfield_measurement(dda, np, torch, job, d, reps: int = 10, cpu: bool = True) -> dict:
    """dda_nearfield on the workload's solution: wall time per call (both
    polarizations, E_inc and E_sca), per-pass kernel times from HIP events
    against the algorithmic bytes of the product on the grown volume, and the
    oracle's direct sum timed on a bounded sample of points."""
    import dataclasses
    t, o, kh, e0 = job
    ext = d["nf_ext"]
    P, _ = dda.solve(t, o, kh, e0)
    org, dims = dda.nearfield_volume(t, ext)
    # the volume's tensor FFT, rebuilt on every call, then kept (one per kd)
    o_new = dataclasses.replace(o, recompute_green=True)
    o_kept = dataclasses.replace(o, recompute_green=False)

    def timed(opts, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            dda.nearfield(t, opts, ext, kh, e0, P)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n
    for _ in range(2):
        dda.nearfield(t, o_new, ext, kh, e0, P)
    ms_new = timed(o_new, reps)
    ms_kept = timed(o_kept, reps)
    dda.set_timing(True)
    timed(o_kept, reps)
    tm = dda.get_timing()
    dda.set_timing(False)
    ms = ms_kept
    npts = int(np.prod(dims))
    n_rhs = len(kh)

    class Vol:   # the grown volume as the product sees it: every point a site
        box = tuple(int(v) for v in dims)
        grid = tuple(padded(int(v)) for v in dims)
    bp = pass_bytes(Vol, npts, 16, "plain")
    passes = {}
    for name in PASSES:
        pms, nl, _ = tm[name]
        if nl:
            gbs = (bp[name][0] * n_rhs + bp[name][1]) * nl / reps / (pms / reps * 1e-3) / 1e9
            passes[name] = {"ms_per_call": pms / reps, "GBps": gbs, "frac": gbs / HBM_PEAK_GBS}
    kern_ms = sum(tm[k][0] for k in PASSES) / reps
    kern_bytes = sum(bp[k][0] * n_rhs + bp[k][1] for k in PASSES)
    out = {"ms_per_call": ms, "ms_per_call_tensor_rebuilt": ms_new, "points": npts,
           "dims": [int(v) for v in dims], "fft_grid": list(Vol.grid),
           "n_rhs": n_rhs, "product_kernels_ms": kern_ms,
           "product_GBps": kern_bytes / (kern_ms * 1e-3) / 1e9, "passes": passes,
           "note": "one call = E_inc and E_sca for both polarizations on every point of the volume, the "
                   "volume's tensor FFT kept from an earlier call (ms_per_call_tensor_rebuilt: built in the "
                   "call); wall time includes placing P and writing both fields"}
    if cpu:
        from oracle import dense as odense
        from oracle import nearfield as onf
        Pn = P.cpu().numpy()
        rng = np.random.default_rng(3)
        pts = rng.integers(0, dims, size=(48, 3)) + np.asarray(org)
        t0 = time.perf_counter()
        onf.scattered_field(d["ijk"], Pn[0], odense.kd_from_size_parameter(d["x"], len(d["ijk"])), pts)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": dt / len(pts) * npts * n_rhs, "unit": "s/call", "cores": 1, "kind": "oracle",
                             "sample": f"the oracle's direct sum (numpy, FP64) at 48 random points of the volume in "
                                       f"{dt:.2f} s, scaled to {npts} points x {n_rhs} polarizations"}
    return out


def adjoint_measurement(dda, np, torch, job, reps: int = 5) -> dict:
    """dda_grad_eps on the workload's solution: wall time of one gradient of
    Q_abs in the per-site permittivity (the adjoint right-hand side, one
    solve with the same product, the gradient kernel), and of the forward
    solve and gradient together (one value-and-gradient evaluation)."""
    t, o, kh, e0 = job
    kh1, e01 = kh[:1], e0[:1]
    P, res = dda.solve(t, o, kh1, e01)

    def timed(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, r

    ms_grad, (g, adj) = timed(lambda: dda.grad_eps(t, o, kh1, e01, P[0], 1.0, 0.0))

    def value_and_grad():
        Pv, _ = dda.solve(t, o, kh1, e01)
        return dda.grad_eps(t, o, kh1, e01, Pv[0], 1.0, 0.0)
    ms_both, _ = timed(value_and_grad)
    return {"grad_ms": ms_grad, "value_and_grad_ms": ms_both, "forward_iters": res[0]["iters"],
            "adjoint_iters": adj["iters"], "adjoint_rel_residual": adj["rel_residual"],
            "grad_norm": float(torch.linalg.vector_norm(g).item()),
            "note": "wall time per call; grad_ms: adjoint right-hand side, adjoint solve and gradient kernel on a "
                    "kept solution; value_and_grad_ms: the forward solve and the gradient"}


FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz


def farfield_measurement(dda, np, torch, job, reps: int = 5) -> dict:
    """dda_scattering_averages (Gauss-Legendre 48 x 64 directions, both
    polarizations) and dda_far_field on 74 directions, on the workload's
    solution.  The kernel's work is one term per (direction, site, right-hand
    side): three complex multiply-adds (24 flops), plus the site's phase
    factor w_x w_y w_z (two complex products, 12 flops).  The averages use a
    direction set about each right-hand side's own incidence direction, so
    every direction serves one right-hand side and the factor is formed for
    each term: 36 flops per term.  The rate is quoted as terms/s and as
    flops against the FP64 vector peak (the per-direction sincos of the
    factor table not counted)."""
    import workloads as w
    t, o, kh, e0 = job
    P, _ = dda.solve(t, o, kh, e0)
    n_rhs, n_sites = P.shape[0], P.shape[1]
    n_theta, n_phi = 48, 64
    theta = np.linspace(0.0, 180.0, 74)
    nh, th, ph = w.lab_directions(theta, np.zeros_like(theta))

    def timed(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps
    ms_avg = timed(lambda: dda.scattering_averages(t, o, kh, e0, P, n_theta, n_phi))
    ms_ff = timed(lambda: dda.far_field(t, o, P, nh, th, ph))
    terms = float(n_theta * n_phi) * n_sites * n_rhs
    flops_per_term = 24.0 + 12.0
    tflops = flops_per_term * terms / (ms_avg * 1e-3) / 1e12
    return {"averages_ms": ms_avg, "directions": n_theta * n_phi, "far_field_74_dirs_ms": ms_ff,
            "terms_per_s": terms / (ms_avg * 1e-3), "flops_per_term": flops_per_term, "bound": "alu",
            "achieved_tflops": tflops,
            "peak_tflops": FP64_VALU_PEAK_TFLOPS, "frac": tflops / FP64_VALU_PEAK_TFLOPS,
            "note": "wall time per call, both polarizations, host quadrature weights and result copies included; "
                    "flops exclude the sincos of the per-direction factor table"}


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


def copy_rate(torch, mib: int = 1024, reps: int = 8) -> float:
    """GB/s (read plus write) of torch's device-to-device copy of mib MiB:
    what a plain streaming kernel reaches on this device, beside the 8 TB/s
    peak, for the HBM-bound passes."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    return 2.0 * n * 4 * reps / (ms * 1e-3) / 1e9


def fp64_comparison(dda, np, torch, jobs, results, steps: int = 3) -> dict:
    """The same workload solved with the FP64 matvec at the same tolerance
    (one batched solve per step, the FP64 tensor FFT built beforehand): its
    time per step, and each efficiency's relative difference between the
    measured step and it, and between each and the FP64 oracle reference
    (tests/golden/<workload>_oracle.json, written by the oracle alone)."""
    import dataclasses
    t, o, kh, e0 = jobs[0]
    o64 = dataclasses.replace(o, precision="fp64", recompute_green=False)
    dda.solve(t, o64, kh, e0, want_P=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r64 = dda.solve(t, o64, kh, e0, want_P=False)[1]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    keys = ("qext", "qabs", "qsca")
    out = {"ms_per_step": ms, "iters": [r["iters"] for r in r64],
           "rel_diff_vs_fp64_gpu": {k: [abs(a[k] - b[k]) / abs(b[k]) for a, b in zip(results, r64)] for k in keys}}
    gold = os.path.join(ROOT, "tests", "golden", "sphere1m_oracle.json")
    if len(results) == 2 and t.n_sites == 1099136 and os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        ref = g["rhs"]
        out["rel_diff_vs_oracle"] = {k: [abs(a[k] - b[k]) / abs(b[k]) for a, b in zip(results, ref)] for k in keys}
        out["fp64_gpu_rel_diff_vs_oracle"] = {k: [abs(a[k] - b[k]) / abs(b[k]) for a, b in zip(r64, ref)]
                                              for k in keys}
        out["oracle_reference"] = (f"tests/golden/sphere1m_oracle.json: the oracle's FP64 FFT-BiCGSTAB to true "
                                   f"residual {max(r['true_residual'] for r in ref):.1e}")
    return out


def launch_groups(jobs) -> list:
    """The jobs (lists of indices) that share launches in one batched solve:
    the library merges targets whose padded grids are equal compile-time
    lengths on every axis and whose solver, precision, flags and variant
    agree (include/dda.h, dda_solve_batched)."""
    out, index = [], {}
    for i, (t, o, _, _) in enumerate(jobs):
        key = (tuple(t.grid), o.solver, o.precision, o.c().flags, o.kernel_variant)
        if all(L in CT_LENGTHS for L in t.grid) and o.share_launches and len(jobs) > 1:
            if key in index:
                out[index[key]].append(i)
                continue
            index[key] = len(out)
        out.append([i])
    return out


def measure_workload(dda, np, torch, w, wname: str, prec: str, solver: str, seed: int, steps: int, warmup: int):
    """Warm up, then time ``steps`` whole solves of a workload with the
    dominant matvec pass event-timed; returns (the bench line's fields, the
    jobs, the workload dict, the last step's results, ms per step)."""
    desc = WORKLOADS[wname][0]
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    jobs, orientations, d = build_jobs(dda, w, wname, seed, prec, solver)
    torch.cuda.synchronize()
    target_create_ms = (time.perf_counter() - t_create) * 1e3
    n_rhs = sum(len(j[2]) for j in jobs)
    log(f"workload {wname}: {len(jobs)} target(s), {n_rhs} right-hand sides, prec={prec}, "
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
    bpus = [pass_bytes(j[0], j[0].n_sites, csize, solver) for j in jobs]
    groups = launch_groups(jobs)

    def pass_traffic(name, units, launches, results):
        # per-RHS bytes times the RHS-matvecs each job executed, plus each
        # launch's shared bytes: every target of the launch's group once.
        # Several groups: the launches split between them in proportion to
        # the products each group ran (its slowest right-hand side's)
        per_rhs = sum(b[name][0] * u for b, u in zip(bpus, units))
        if len(groups) == 1:
            return per_rhs + sum(bpus[i][name][1] for i in groups[0]) * launches
        first = [sum(len(j[2]) for j in jobs[:i]) for i in range(len(jobs))]
        runs = [max(r["matvecs"] for i in g for r in results[first[i]:first[i] + len(jobs[i][2])]) + 3
                for g in groups]
        return per_rhs + sum(sum(bpus[i][name][1] for i in g) * launches * n / sum(runs)
                             for g, n in zip(groups, runs))

    # warmup; the last warmup step times every kernel category to find the
    # dominant matvec pass, which alone is timed during the measured steps
    for i in range(max(warmup, 1)):
        if i == max(warmup, 1) - 1:
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
    for i in range(steps):
        results = step()
        units = [a + b for a, b in zip(units, job_units(results))]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = dda.get_timing()
    dda.set_timing(False)
    dda.set_timing_sample(1)
    ms_per_step = (t1 - t0) * 1e3 / steps
    s_per_orientation = ms_per_step / 1e3 / orientations
    for r in results:
        if r["status"] != 0:
            raise SystemExit(f"solve did not converge: {r}")
    log(f"timed {steps} steps: {ms_per_step:.3f} ms/step; results {results[0]}")

    ms_tot, launches, all_launches = timing[dominant]
    bytes_tot = pass_traffic(dominant, units, all_launches, results)
    # algorithmic bytes per launch (all launches) over the sampled average launch time
    avg_s = ms_tot * 1e-3 / launches
    gbs = bytes_tot / all_launches / avg_s / 1e9
    variants = dda.tuned_variants(jobs[0][0], len(jobs[0][2]), prec) if len(jobs) == 1 else None
    traffic = (load_traffic(dominant, wname, prec, variants, sum(units) / all_launches)
               if len(jobs) == 1 else None)
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
        g = pass_traffic(name, cal_units, nl, res) / (ms * 1e-3) / 1e9
        passes[name] = {"ms_per_launch": ms / nl, "launches": nl, "bytes_per_rhs_matvec": bpus[0][name][0],
                        "bytes_per_launch_shared": bpus[0][name][1], "GBps": g, "frac": g / HBM_PEAK_GBS}
    matvec_ms = sum(calib[k][0] for k in PASSES)
    matvec_bytes = sum(pass_traffic(k, cal_units, calib[k][1], res) for k in PASSES)
    out = {
        "metric": METRIC,
        "value": s_per_orientation,
        "unit": "s/orientation",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32 matvec / f64 Krylov",
        "data": "synthetic",
        "config": {"workload": f"{wname}: {desc}", "solver": solver, "targets": len(jobs),
                   "launch_groups": [[list(jobs[g[0]][0].grid), len(g), sum(len(jobs[i][2]) for i in g)]
                                     for g in groups] if len(jobs) > 1 else None,
                   "n_sites": [j[0].n_sites for j in jobs][:4], "fft_grid": list(jobs[0][0].grid),
                   "rhs_per_step": n_rhs, "orientations_per_step": orientations, "precision": prec,
                   "seed": seed},
        "roofline": roofline,
        "autotuned_variants": variants,
        "target_create_ms": target_create_ms,
        "matvec": {"GBps_all_passes": matvec_bytes / (matvec_ms * 1e-3) / 1e9,
                   "units_per_step": sum(units) / steps, "passes_calibration_step": passes},
        "kernel_ms_calibration_step": {k: v[0] for k, v in calib.items()},
        "solver": {"iters": [r["iters"] for r in results][:8], "matvecs": [r["matvecs"] for r in results][:8],
                   "qext": [r["qext"] for r in results][:8], "qabs": [r["qabs"] for r in results][:8],
                   "qsca": [r["qsca"] for r in results][:8], "rel_residual": [r["rel_residual"] for r in results][:8],
                   "normal_eq_residual": [r["normal_eq_residual"] for r in results][:8],
                   "refinements": [r["refinements"] for r in results][:8]},
    }
    return out, jobs, d, results, ms_per_step


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32_matvec"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the FP64 comparisons (each right-hand side alone; the FP64-matvec solve)")
    ap.add_argument("--no-extra", action="store_true", help="skip the context measurement of the default line")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--solver", default="bicgstab", choices=["bicgstab", "qmr", "bicgstab2"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--print-profile-commands", action="store_true",
                    help="print the rocprofv3 runs behind the profiles/ summaries of --workload")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write the profiles/ summaries of --workload from those runs' outputs under DIR")
    ap.add_argument("--profile-dir", metavar="DIR", default="/root/repo/gpurun_out/tr",
                    help="with --print-profile-commands: where the runs write their outputs")
    ap.add_argument("--unprofiled", metavar="JSON", help="with --summarize: the unprofiled bench line")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.print_profile_commands or args.summarize:
        prec = args.precision or WORKLOADS[args.workload][1]
        if args.summarize:
            summarize_profiles(args.summarize, args.workload, prec, args.unprofiled)
        else:
            for k, c in profile_commands(args.workload, prec, args.profile_dir).items():
                print(f"# {k}\n{c}")
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
    prec = args.precision or WORKLOADS[args.workload][1]
    out, jobs, d, results, ms_per_step = measure_workload(dda, np, torch, w, args.workload, prec, args.solver,
                                                          args.seed, args.steps, args.warmup)
    cr = copy_rate(torch)
    out["roofline"]["plain_copy_GBps"] = cr
    out["roofline"]["frac_of_plain_copy"] = out["roofline"]["achieved"] / cr
    for p in out["matvec"]["passes_calibration_step"].values():
        p["frac_of_plain_copy"] = p["GBps"] / cr
    if prec == "fp32_matvec" and len(jobs) == 1 and not args.no_plain:
        log("solving the same workload with the FP64 matvec ...")
        out["fp64_matvec"] = fp64_comparison(dda, np, torch, jobs, results)
    if args.workload == DEFAULT_WORKLOAD and not args.no_extra:
        log(f"measuring {EXTRA_WORKLOAD} for context ...")
        xo, xjobs, _, xres, xms = measure_workload(dda, np, torch, w, EXTRA_WORKLOAD, WORKLOADS[EXTRA_WORKLOAD][1],
                                                   args.solver, args.seed, args.steps, args.warmup)
        out["also"] = {EXTRA_WORKLOAD: {k: xo[k] for k in ("value", "unit", "ms_per_step", "roofline", "dtype")}}
        out["also"][EXTRA_WORKLOAD]["note"] = ("the 51,488-site ellipsoid (FFT grid 128x96x64, FP64): its ~130 MB "
                                               "working set fits the 256 MB Infinity Cache")
    if not args.no_plain:
        log("timing the plain FP64 single-right-hand-side solves of the same workload ...")
        out["vs_plain_fp64_single_rhs"] = plain_reference(dda, np, torch, jobs, results, ms_per_step)
    if args.workload in GUIDE_CONTEXT:
        out["guide_context"] = dict(GUIDE_CONTEXT[args.workload],
                                    hardware="one 2.53 GHz CPU core, whole DDSCAT run (target generation, solve, "
                                             "scattering directions), precision not stated")
    if len(jobs) == 1 and jobs[0][0].n_sites <= 100_000:
        log("timing the far field and the averages over scattering directions ...")
        out["farfield"] = farfield_measurement(dda, np, torch, jobs[0])
    if args.workload == "twomat40":
        log("timing the adjoint gradient on the solution ...")
        out["adjoint"] = adjoint_measurement(dda, np, torch, jobs[0])
    if "nf_ext" in d:
        log("timing the near field on the solution ...")
        out["nearfield"] = nearfield_measurement(dda, np, torch, jobs[0], d, cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on one polarization ...")
        out["cpu_baseline"] = cpu_baseline(d, args.workload, results[0]["iters"])
        if args.workload == "config3":
            out["cpu_baseline"]["sample"] += " (the brick's orientations; the spheres are smaller)"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
