"""Write tests/golden/sphere1m_oracle.json: the CPU oracle's FP64 solution of
the 1,099,136-site sphere (radius 64 in a 128^3 box, m = 1.33+0.01i, x = 20,
LATTDR, incidence +x, polarizations y and z) by FFT-BiCGSTAB to a true
residual tighter than the GPU solve's 1e-5, so that its efficiencies serve as
the reference the GPU's FP64 and FP32-matvec solves are checked against
(1e-4 relative).

Calls only ``oracle`` and the seeded input generators of ``workloads``; it
runs once on the CPU (tens of minutes) and its output is committed.

    python tests/golden/make_sphere1m_oracle.py [--tol 1e-7]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from oracle import dense, fftsolve  # noqa: E402

# sites whose P is stored (seeded), for a coarse check of the solution itself
N_SAMPLE = 64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--out", default=os.path.join(HERE, "sphere1m_oracle.json"))
    args = ap.parse_args()
    d = w.workload("sphere1m")
    n = len(d["ijk"])
    k = dense.kd_from_size_parameter(d["x"], n)
    sample = np.sort(np.random.default_rng([0, 1001]).choice(n, N_SAMPLE, replace=False))
    out = {"source": "oracle.fftsolve FFT-BiCGSTAB in FP64 (this script; no GPU result is used)",
           "workload": "sphere1m", "n_sites": n, "x": d["x"], "m": [float(d["m"][0].real), float(d["m"][0].imag)],
           "kd": k, "tol": args.tol, "polarizability": "LATTDR", "rhs": [], "sample_sites": sample.tolist()}
    for q in range(len(d["khat"])):
        t0 = time.perf_counter()
        r = fftsolve.solve_case(d["ijk"], d["m"], d["x"], d["khat"][q], d["e0"][q], tol=args.tol, max_iter=2000)
        dt = time.perf_counter() - t0
        rec = {"khat": d["khat"][q].tolist(), "e0_re": np.real(d["e0"][q]).tolist(),
               "e0_im": np.imag(d["e0"][q]).tolist(), "qext": r["qext"], "qabs": r["qabs"], "qsca": r["qsca"],
               "qpha": r["qpha"], "iters": r["iters"], "matvecs": r["matvecs"], "converged": r["converged"],
               "recursive_residual": r["rel_residual"], "true_residual": r["true_residual"], "cpu_s": dt,
               "P_sample_re": np.real(r["P"][sample]).tolist(), "P_sample_im": np.imag(r["P"][sample]).tolist()}
        out["rhs"].append(rec)
        print(f"rhs {q}: {r['iters']} iterations, true residual {r['true_residual']:.3e}, "
              f"Q_ext {r['qext']:.10f} Q_abs {r['qabs']:.10f} in {dt:.0f} s", flush=True)
        del r
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
