"""Microbenchmark of the block-structured H X kernel through the C ABI.

    python -m paper_2601_10557_amd.kernel_bench --m 4000 --k 260 [--prec c64|c128|both]
        [--reps 5] [--calib-copy-mib 1024] [--plans "cfg,splits;cfg,splits;..."]
        [--filter-deg D] [--mfma-probe]

Prints one line per (precision, k) with the best per-launch time (HIP events
on the library's stream), TFLOP/s at 8 n^2 k flops per launch and the
algorithmic GB/s.  Each stage call waits for its launches, so a call starts
on an idle device.  ``--filter-deg D`` instead times the 2 D back-to-back
launches of one degree-D filter call (fused recurrence epilogue, as inside
the solver) through the library's per-launch profile and prints their mean.
``--mfma-probe`` first prints the matrix-core throughput measured by
``chase_ph_mfma_probe`` (f32 and f64), the ceiling the H X kernels are set
against beside the published peaks.  ``--plans`` repeats each measurement with the tile plan
forced through ``CHASE_PH_APPLY_PLAN`` (a tuning aid; "auto" is the
library's own choice, "whole" its choice without the column split).  ``--calib-copy-mib`` first runs a plain device-to-device
copy of that many MiB, a reference dispatch of known traffic for hardware
counter calibration.  Random Hermitian A and symmetric B are drawn on the
device; no parity is checked here (see tests/).
"""
from __future__ import annotations

import argparse
import os

import torch

from . import FP32, FP64, PHSolver, colmajor, empty_cm
from .solver import mfma_probe


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--m", type=int, default=4000)
    ap.add_argument("--k", type=str, default="260")
    ap.add_argument("--prec", choices=["c64", "c128", "both"], default="both")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--calib-copy-mib", type=int, default=0)
    ap.add_argument("--plans", type=str, default="auto")
    ap.add_argument("--filter-deg", type=int, default=0)
    ap.add_argument("--mfma-probe", action="store_true",
                    help="also print the measured matrix-core throughput (f32 and f64)")
    args = ap.parse_args(argv)
    if args.mfma_probe:
        for kind, name, peak in ((0, "v_mfma_f32_32x32x2f32", 157.3), (1, "v_mfma_f64_16x16x4f64", 78.6)):
            print(f"mfma probe {name}: {mfma_probe(kind):.1f} TFLOP/s (published peak {peak})", flush=True)
    ks = [int(x) for x in args.k.split(",")]
    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"calibration copy: {args.calib_copy_mib} MiB read, {args.calib_copy_mib} MiB written", flush=True)
        del src, dst
    m, n = args.m, 2 * args.m
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    A = torch.randn(m, m, dtype=torch.complex128, device="cuda", generator=g)
    A = 0.5 * (A + A.conj().T.contiguous())
    B = torch.randn(m, m, dtype=torch.complex128, device="cuda", generator=g)
    B = 0.5 * (B + B.T.contiguous())
    kmax = max(ks)
    s = PHSolver(A, B, min(kmax // 2 + 8, m // 2), kmax // 2 + 8)
    precs = {"c64": [(FP32, torch.complex64)], "c128": [(FP64, torch.complex128)],
             "both": [(FP32, torch.complex64), (FP64, torch.complex128)]}[args.prec]
    for prec, dt in precs:
        name = "c64" if prec == FP32 else "c128"
        peak = 157.3 if prec == FP32 else 78.6
        elem = 8 if prec == FP32 else 16
        for k in ks:
            X = colmajor(torch.randn(n, k, dtype=dt, device="cuda", generator=g))
            Y = empty_cm(n, k, dt)
            for plan in args.plans.split(";"):
                os.environ.pop("CHASE_PH_NO_SPLIT", None)
                if plan == "auto":
                    os.environ.pop("CHASE_PH_APPLY_PLAN", None)
                elif plan == "whole":
                    os.environ.pop("CHASE_PH_APPLY_PLAN", None)
                    os.environ["CHASE_PH_NO_SPLIT"] = "1"
                else:
                    os.environ["CHASE_PH_APPLY_PLAN"] = plan
                if args.filter_deg > 0:
                    W = X.clone()
                    degs = [args.filter_deg] * k
                    s.filter(W, 10.0, 50.0, 400.0, degs=degs, prec=prec)
                    s.profile(True)
                    s.filter(W, 10.0, 50.0, 400.0, degs=degs, prec=prec)
                    ms, _, _, cnt = s.profile_read(prec)
                    s.profile(False)
                    best = ms / max(cnt, 1)
                else:
                    best = 1e30
                    for _ in range(args.reps + 1):
                        s.apply_h(X, Y, prec=prec)
                        best = min(best, s.last_timing()[0])
                fl = 8.0 * n * n * k
                by = (2.0 * m * m + 2.0 * n * k) * elem
                print(f"{name} m={m} k={k} plan={plan}: {best * 1e3:.1f} us  {fl / best / 1e9:.2f} TFLOP/s "
                      f"({fl / best / 1e9 / peak * 100:.1f}% of {peak})  {by / best / 1e6:.1f} GB/s algorithmic",
                      flush=True)
            os.environ.pop("CHASE_PH_APPLY_PLAN", None)
            os.environ.pop("CHASE_PH_NO_SPLIT", None)
    s.close()


if __name__ == "__main__":
    main()
