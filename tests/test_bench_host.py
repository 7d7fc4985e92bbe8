"""Host logic of bench.py (no GPU): the measured-traffic lookup, the
profile-command contract and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _record(tmp_path, digest, variant_bytes):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "fft_z_green", "source_sha256": digest,
           "by_variant": {str(v): {"bytes_per_rhs_matvec": b} for v, b in variant_bytes.items()}}
    (prof / "fft_z_green_ellipsoid51k_fp64_traffic.json").write_text(json.dumps(rec))


def test_traffic_is_taken_for_the_run_variant_and_scaled_per_launch(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "abc")
    _record(tmp_path, "abc", {3: 50e6, 10: 40e6})
    # variants are (y forward, z, y inverse); the z slot decides
    assert bench.load_traffic("fft_z_green", "ellipsoid51k", "fp64", [4, 3, 4], 1.5) == 75e6
    assert bench.load_traffic("fft_z_green", "ellipsoid51k", "fp64", [4, 10, 4], 2.0) == 80e6
    assert bench.load_traffic("fft_z_green", "ellipsoid51k", "fp64", [4, 7, 4], 2.0) is None
    assert bench.load_traffic("fft_z_green", "ellipsoid51k", "fp64", None, 2.0) is None
    assert bench.load_traffic("fft_z_green", "brick48", "fp64", [4, 3, 4], 2.0) is None


def test_traffic_is_null_once_the_pass_sources_change(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "new")
    _record(tmp_path, "old", {3: 50e6})
    assert bench.load_traffic("fft_z_green", "ellipsoid51k", "fp64", [4, 3, 4], 1.5) is None


def test_source_digest_covers_the_pass_kernels():
    d = bench.kernel_source_digest()
    assert len(d) == 64 and d == bench.kernel_source_digest()


def test_profile_commands_run_committed_files_under_the_profiler():
    c = bench.profile_commands("sphere1m", "fp32_matvec", "/root/repo/gpurun_out/tr_x")
    assert set(c) == {"trace", "fetch", "write", "copy_fetch", "copy_write", "unprofiled"}
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write"):
        assert c[k].startswith("cd /tmp && export TMPDIR=/tmp && timeout ")
        assert "-- python -u /root/repo/bench.py" in c[k] and "/root/repo/gpurun_out/tr_x/" in c[k]
    assert "--pmc FETCH_SIZE" in c["fetch"] and "--pmc WRITE_SIZE" in c["write"]
    assert "--kernel-trace --stats" in c["trace"] and "--pmc" not in c["trace"]
    # the default workload (sphere1m, FP32 matvec) adds no flags; others do
    assert "--workload" not in c["unprofiled"] and "--precision" not in c["unprofiled"]
    assert "--precision fp64" in bench.profile_commands("sphere1m", "fp64")["unprofiled"]
    assert "--workload ellipsoid51k" in bench.profile_commands("ellipsoid51k", "fp64")["unprofiled"]
    # profiled runs hold the measured workload's kernels only
    for k in ("trace", "fetch", "write", "unprofiled"):
        assert "--no-plain --no-extra" in c[k]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def test_pass_bytes_count_each_solvers_site_vectors():
    class Tgt:
        box = (64, 48, 32)
        grid = (128, 96, 64)
    n = 51488
    site = 3 * n * 16
    b = {s: bench.pass_bytes(Tgt, n, 16, s) for s in ("bicgstab", "qmr", "bicgstab2", "plain")}
    lines = 128 * 48 * 32 * 3 * 16            # the x-transformed occupied lines of one RHS
    for s, (sc, ga) in bench.SITE_VECTORS.items():
        assert b[s]["scatter_fft_x"][0] == lines + sc * site
        assert b[s]["fft_x_gather"][0] == lines + ga * site
        # the strided passes and the shared bytes do not depend on the solver
        for k in ("fft_y_fwd", "fft_z_green", "fft_y_inv"):
            assert b[s][k] == b["bicgstab"][k]
        assert b[s]["scatter_fft_x"][1] == 4 * 64 * 48 * 32
    # pass 3: forward and inverse grids of every RHS; the tensor octant once per launch
    assert b["plain"]["fft_z_green"] == (2 * 128 * 96 * 32 * 48, 65 * 49 * 33 * 6 * 16)


def test_launch_groups_follow_the_library_merge_rule():
    """Targets share launches when their padded grids are equal compile-time
    lengths on every axis and their options agree (include/dda.h); others,
    and a single target, are groups of their own."""
    from types import SimpleNamespace as NS

    def opt(solver="bicgstab", precision="fp64", flags=0, variant=0, share=True):
        return NS(solver=solver, precision=precision, kernel_variant=variant, share_launches=share,
                  c=lambda: NS(flags=flags))

    def job(grid, o):
        return (NS(grid=grid), o, None, None)

    jobs = [job((96, 48, 32), opt()), job((64, 64, 64), opt()), job((80, 80, 80), opt()),
            job((64, 64, 64), opt()), job((64, 64, 64), opt(precision="fp32_matvec")),
            job((64, 64, 64), opt(share=False)), job((50, 50, 50), opt()), job((50, 50, 50), opt()),
            job((80, 80, 80), opt(flags=2)), job((80, 80, 80), opt())]
    assert bench.launch_groups(jobs) == [[0], [1, 3], [2, 9], [4], [5], [6], [7], [8]]
    assert bench.launch_groups(jobs[1:2]) == [[0]]
