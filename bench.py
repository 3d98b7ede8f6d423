"""Benchmark of the pseudo-hermitian ChASE hot path on one MI355X.

Workload (default): the mixed-vs-FP64 problem, m = 4000 (n = 8000),
A = Q diag(d) Q^H with d ~ U[0.5, 10], ||B||_2 = 0.3 min d, nev = 200,
nex = 60, deg = 20, tol = 1e-9, seed 0; synthetic inputs generated on the
host and uploaded before the timed region.

One step = one pass of the whole hot path: a full solve (Lanczos, Chebyshev
filter, CholeskyQR2, oblique Rayleigh-Ritz, residuals, locking) with the
FP32-filter / FP64-refine policy, followed by the same solve on the FP64
path.  ``value`` is the filter throughput of the mixed solves: filter flops
divided by the stream-timed filter time, with 8 n^2 real flops per active
column per degree (two products with H, each one real GEMM of 4 n^2 per
column on the real structure of H; ``filter_tflops.complex_model`` gives the
same time on the 16 n^2 of a complex-GEMM formulation).  The JSON line also carries both time-to-solution figures, their
ratio, the eigenvalue agreement, the roofline of the dominant kernel (the
c64 block-structured GEMM that applies H, timed launch by launch with HIP
events inside the timed steps) and the CPU oracle timed on bounded samples:
its filter on 8 columns, and its dense time to solution (the plain
definition the solver reaches) timed on an m = 3000 draw of the same
generator and scaled by n^3 (``--cpu-full`` times it on the workload).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--cpu-full]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def apply_h_source_sha256():
    import hashlib
    path = os.path.join(ROOT, "paper_2601_10557_amd", "csrc", "apply_h.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the c64 H X kernel from the committed
    rocprofv3 --pmc summary (FETCH_SIZE and WRITE_SIZE runs of this bench
    command, scaled by the same counters on a copy of known size); None if
    absent or if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "apply_h_c64_traffic_mixed_vs_fp64_m4000.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256") != apply_h_source_sha256():
        return None
    return d


def cpu_model():
    """CPU model name of the host that drives the GPU (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def blas_threads():
    from threadpoolctl import threadpool_info
    return int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))


def cpu_filter_sample(p, seconds_target=12.0):
    """The oracle's Chebyshev filter on a bounded sample of the workload:
    degree-1 filter on 8 sample columns of the same H, repeated to about
    seconds_target seconds.  Returns (TFLOP/s, seconds per call, reps)."""
    from oracle import chebyshev  # oracle: baseline leg only
    from oracle.solver import init_block
    k, deg = 8, 1
    W = init_block(p.w0_raw[:, :k], 1e-3)
    mu1, mu_nevex, mu_n = 0.5, 2.0, 12.0
    t = time.perf_counter()
    chebyshev.chebyshev_filter(p.A, p.B, W, deg, mu1, mu_nevex, mu_n)
    dt = time.perf_counter() - t
    reps = min(max(1, int(seconds_target / max(dt, 1e-3)) - 1), 40)
    t = time.perf_counter()
    for _ in range(reps):
        chebyshev.chebyshev_filter(p.A, p.B, W, deg, mu1, mu_nevex, mu_n)
    dt = (time.perf_counter() - t) / reps
    return 16.0 * p.n * p.n * k * deg / dt / 1e12, dt, reps, k


def cpu_dense_time(config, m, seed=0):
    """Seconds of the dense oracle (all positive eigenpairs of H, the plain
    definition the solver converges to) on an m-row draw of the workload's
    generator (same spectrum and coupling)."""
    from synth import config_problem
    from oracle import dense  # oracle: baseline leg only
    q = config_problem(config, seed=seed, m=m, nev=min(200, m // 4), nex=min(60, m // 8))
    t = time.perf_counter()
    dense.dense_ph_eig(q.A, q.B)
    return time.perf_counter() - t


def cpu_baseline(p, config, full=False, dense_m=3000):
    """The oracle on the host cores, beside the GPU figures of the same run.

    * value: the oracle's Chebyshev filter (TFLOP/s) on 8 of the nevex
      columns of the workload (degree 1, repeated to ~12 s).
    * time_to_solution_s: the dense oracle's time on the workload.  By
      default it is timed on a dense_m-row draw of the same generator
      (about 16 s on 16 cores) and scaled by (m / dense_m)^3, the cost
      order of the Cholesky, congruence and Hermitian eigensolve; with
      full=True the dense oracle runs on the workload itself."""
    tf, dt, reps, k = cpu_filter_sample(p)
    out = {"value": tf, "unit": "TFLOP/s", "cores": blas_threads(), "kind": "oracle",
           "sample": f"oracle chebyshev_filter, degree 1 in H^2 on {k} of {p.nevex} columns of the "
                     f"m={p.m} workload ({reps} timed repetitions, {dt:.2f} s each)",
           "cpu_model": cpu_model(), "os_cpus": os.cpu_count()}
    if full:
        t = cpu_dense_time(config, p.m)
        out["time_to_solution_s"] = {"dense_oracle": round(t, 2), "measured_at_m": p.m, "extrapolated": False,
                                     "what": "oracle.dense.dense_ph_eig on the workload itself"}
    else:
        t = cpu_dense_time(config, dense_m)
        scale = (p.m / dense_m) ** 3
        out["time_to_solution_s"] = {"dense_oracle": round(t * scale, 2), "measured_at_m": dense_m,
                                     "measured_s": round(t, 2), "extrapolated": True,
                                     "what": f"oracle.dense.dense_ph_eig on an m={dense_m} draw of the same "
                                             f"generator, scaled by (m/{dense_m})^3"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the dense oracle on the workload itself instead of a scaled draw")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a device copy of this many MiB before the timed region (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth import config_problem
    from paper_2601_10557_amd import FP32, FP64, MIXED, PHSolver, colmajor
    from paper_2601_10557_amd.solver import mfma_probe

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    t0 = time.perf_counter()
    p = config_problem(args.config, seed=0)
    log(f"generated {p.name} in {time.perf_counter() - t0:.1f}s")
    if args.calib_copy_mib > 0:
        src = torch.empty((args.calib_copy_mib << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    A = torch.from_numpy(p.A).cuda()
    B = torch.from_numpy(p.B).cuda()
    W0 = colmajor(torch.from_numpy(p.w0_raw)).cuda()
    Lz = colmajor(torch.from_numpy(p.lanczos_raw)).cuda()
    torch.cuda.synchronize()

    common = dict(deg=p.deg, tol=p.tol, max_iter=25)
    mixed = PHSolver(A, B, p.nev, p.nex, precision=MIXED, **common)
    fp64 = PHSolver(A, B, p.nev, p.nex, precision=FP64, **common)

    for i in range(args.warmup):
        mixed.solve(W0, Lz)
        fp64.solve(W0, Lz)
        log(f"warmup {i} done")
    # measured matrix-core ceilings (outside the timed region)
    probe32, probe64 = mfma_probe(0), mfma_probe(1)
    log(f"mfma probe: f32 {probe32:.1f} TFLOP/s, f64 {probe64:.1f} TFLOP/s")

    torch.cuda.synchronize()
    mixed.profile(True)
    fp64.profile(True)
    runs_m, runs_d = [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev_m, V_m, r_m, info_m = mixed.solve(W0, Lz)
        ev_d, V_d, r_d, info_d = fp64.solve(W0, Lz)
        runs_m.append(info_m)
        runs_d.append(info_d)
        log(f"step {i}: mixed {info_m.t_total:.3f}s ({info_m.iterations} it), "
            f"fp64 {info_d.t_total:.3f}s ({info_d.iterations} it)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    ms32, fl32, by32, n32 = mixed.profile_read(FP32)
    ms64, fl64, by64, n64 = fp64.profile_read(FP64)
    mixed.profile(False)
    fp64.profile(False)

    filt_flops_m = sum(r.filter_flops for r in runs_m)
    filt_time_m = sum(r.t_filter for r in runs_m)
    filt_flops_d = sum(r.filter_flops for r in runs_d)
    filt_time_d = sum(r.t_filter for r in runs_d)
    tts_m = float(np.median([r.t_total for r in runs_m]))
    tts_d = float(np.median([r.t_total for r in runs_d]))
    agree = float(np.max(np.abs(ev_m - ev_d) / np.abs(ev_d)))

    golden = os.path.join(ROOT, "tests", "golden", f"dense_evals_config{args.config}_seed0.txt")
    err_vs_dense = None
    if os.path.exists(golden):
        ref = np.loadtxt(golden)[: p.nev]
        err_vs_dense = {"mixed": float(np.max(np.abs(ev_m - ref) / ref)),
                        "fp64": float(np.max(np.abs(ev_d - ref) / ref))}

    achieved = fl32 / (ms32 * 1e-3) / 1e12 if ms32 > 0 else 0.0
    tr = measured_traffic()
    traffic, traffic_detail = None, None
    if tr is not None:
        traffic = tr["hbm_bytes_per_launch"]
        traffic_detail = {"algorithmic_bytes_per_launch": by32 / max(n32, 1),
                          "fetch_bytes_per_launch": tr["fetch_bytes_per_launch"],
                          "write_bytes_per_launch": tr["write_bytes_per_launch"],
                          "source": "profiles/apply_h_c64_traffic_mixed_vs_fp64_m4000.json"}
    roofline = {
        "kernel": "hx_kernel (c64 real GEMM on D = [A+B, i(A-B)]) with its operand pack and the fused "
                  "Chebyshev epilogue: one H X call (pack, one GEMM launch, whose remainder tiles take the "
                  "last k mod 64 columns of a split call, and the split-K reductions); 4 n^2 k real flops "
                  "per call",
        "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic, "traffic_detail": traffic_detail,
        "measured_mfma_peak": round(probe32, 1), "frac_of_measured": round(achieved / probe32, 4) if probe32 > 0 else None,
        "launches": n32, "avg_launch_us": round(ms32 * 1e3 / max(n32, 1), 2),
        "avg_flops_per_launch": fl32 / max(n32, 1),
        "algorithmic_gbs": round(by32 / (ms32 * 1e-3) / 1e9, 1) if ms32 > 0 else 0.0,
        "fp64_kernel": {"achieved": round(fl64 / (ms64 * 1e-3) / 1e12, 3) if ms64 > 0 else 0.0,
                        "peak": PEAK_FP64_TFLOPS, "measured_mfma_peak": round(probe64, 1), "launches": n64,
                        "avg_launch_us": round(ms64 * 1e3 / max(n64, 1), 2)},
    }
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline(p, args.config, full=args.cpu_full)
        ratio = cpu["time_to_solution_s"]["dense_oracle"] / tts_m
        cpu["time_to_solution_s"]["over_gpu_mixed"] = round(ratio, 1)

    value = filt_flops_m / filt_time_m / 1e12
    out = {
        "metric": "filter TFLOP/s + time-to-nev-eigenpairs at tol, FP32-mixed vs FP64, 1 MI355X",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 filter + c128 QR/RR (mixed); c128 (fp64 path)",
        "data": "synthetic",
        "config": {"workload": p.name, "m": p.m, "n": p.n, "nev": p.nev, "nex": p.nex, "deg": p.deg,
                   "tol": p.tol, "seed": 0},
        "time_to_solution_s": {"mixed": round(tts_m, 4), "fp64": round(tts_d, 4),
                               "fp64_over_mixed": round(tts_d / tts_m, 3),
                               "mixed_min_max": [round(min(r.t_total for r in runs_m), 4),
                                                 round(max(r.t_total for r in runs_m), 4)],
                               "fp64_min_max": [round(min(r.t_total for r in runs_d), 4),
                                                round(max(r.t_total for r in runs_d), 4)],
                               "statistic": f"median of {args.steps} timed solves each"},
        "filter_tflops": {"mixed": round(value, 3), "fp64_path": round(filt_flops_d / filt_time_d / 1e12, 3),
                          "flops_per_column_per_degree": "8 n^2 (real GEMM on the real structure of H)",
                          "complex_model": {"mixed": round(2 * value, 3),
                                            "fp64_path": round(2 * filt_flops_d / filt_time_d / 1e12, 3),
                                            "flops_per_column_per_degree": "16 n^2 (complex GEMM)"}},
        "iterations": {"mixed": runs_m[-1].iterations, "fp64": runs_d[-1].iterations,
                       "mixed_switch_iter": runs_m[-1].switch_iter},
        "phase_s_mixed": {k: round(getattr(runs_m[-1], k), 4) for k in
                          ("t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid", "t_total")},
        "phase_s_fp64": {k: round(getattr(runs_d[-1], k), 4) for k in
                         ("t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid", "t_total")},
        "eig_agreement_mixed_vs_fp64": agree,
        "eig_err_vs_dense_oracle": err_vs_dense,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host": {"cpu": cpu_model(), "os_cpus": os.cpu_count()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
