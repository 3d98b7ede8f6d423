"""One solve of a named synthetic workload, drawn on the device.

    python -m paper_2601_10557_amd.run_workload --config 4 [--precision mixed|fp64]
        [--max-iter 30] [--backward] [--samples 6] [--rr-backup] [--nex N]

Builds the workload with ``synth.gpu`` (seeded, seed 0 by default), runs
``chase_ph_solve`` and prints one JSON line: wall time, phase times, filter
TFLOP/s, iterations, the first and last eigenvalue, the largest residual
the solver reports, and ``host_residuals``: ``||H v - lambda v||`` for a few
returned pairs recomputed on the host from copies of A and B (numpy).  With
``--backward`` it also times ``chase_ph_eigval_backward`` for random loss
weights on the returned pairs; ``--rr-backup`` runs the non-hermitian
back-up Rayleigh quotient (Section 5.3) in every iteration.  ``--tda`` runs
Hermitian ChASE (Alg. 1) on the workload's A alone instead (FP64; the start
block and the Lanczos starts are the top m rows of the pseudo-hermitian ones;
``--nex-auto`` lets the library choose nex), checks its eigenvalues against
``numpy.linalg.eigvalsh(A)`` on the host (m <= 8000) and recomputes a few
residuals ``||A x - lambda x||``.  Per-iteration progress goes to stderr with
``CHASE_PH_VERBOSE=1``.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import FP64, MIXED, PHSolver, TDASolver, colmajor


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--max-iter", type=int, default=30)
    ap.add_argument("--backward", action="store_true")
    ap.add_argument("--samples", type=int, default=6)
    ap.add_argument("--rr-backup", action="store_true")
    ap.add_argument("--nex", type=int, default=None, help="override the workload's nex")
    ap.add_argument("--tda", action="store_true", help="Hermitian ChASE on A alone (Alg. 1)")
    ap.add_argument("--nex-auto", action="store_true", help="with --tda: the library chooses nex")
    args = ap.parse_args(argv)
    from synth.gpu import config_problem_device

    t0 = time.perf_counter()
    p = config_problem_device(args.config, seed=args.seed, nex=args.nex)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    if args.tda:
        run_tda(p, args, gen_s)
        return
    prec = MIXED if args.precision == "mixed" else FP64
    s = PHSolver(p.A, p.B, p.nev, p.nex, deg=p.deg, tol=p.tol, precision=prec, max_iter=args.max_iter,
                 opt_deg=p.deg_min != p.deg_max, deg_min=p.deg_min, deg_max=p.deg_max,
                 rr_backup=args.rr_backup)
    t0 = time.perf_counter()
    ev, V, res, info = s.solve(colmajor(p.w0_raw), colmajor(p.lanczos_raw), raise_on_noconv=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(workload=p.name, m=p.m, n=p.n, nev=p.nev, nex=p.nex, precision=args.precision,
               generate_s=round(gen_s, 2), solve_s=round(wall, 3), iterations=info.iterations,
               locked=info.locked,
               phases_s=dict(lanczos=round(info.t_lanczos, 3), filter=round(info.t_filter, 3),
                             qr=round(info.t_qr, 3), rr=round(info.t_rr, 3), resid=round(info.t_resid, 3)),
               filter_tflops=round(info.filter_flops / info.t_filter / 1e12, 2) if info.t_filter > 0 else 0.0,
               shifted_qr=info.shifted_qr_used, householder_qr=info.householder_qr_used,
               backup_rr=info.backup_rr_used)
    if len(ev):
        out.update(lambda_first=float(ev[0]), lambda_last=float(ev[-1]), max_resid=float(np.max(res)))
    if args.backward and len(ev):
        g = np.random.default_rng(3).standard_normal(len(ev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        GA, GB = s.eigval_backward(V, g)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        out["backward_s"] = round(tb, 3)
        # the kernel forms the lower triangles of the Hermitian G_A and the
        # symmetric G_B (m^2 / 2 entries each, 2 nev complex MACs per entry)
        out["backward_tflops"] = round(16.0 * p.m * p.m * len(ev) / tb / 1e12, 1)
        del GA, GB
    if args.samples > 0 and len(ev):
        idx = np.unique(np.linspace(0, len(ev) - 1, args.samples).astype(int))
        m = p.m
        Ah, Bh = p.A.cpu().numpy(), p.B.cpu().numpy()
        Vs = V[:, idx].cpu().numpy()
        x, y = Vs[:m], Vs[m:]
        hv = np.concatenate([Ah @ x + Bh @ y, -np.conj(Bh @ x.conj() + Ah @ y.conj())])
        r = np.linalg.norm(hv - Vs * ev[idx][None, :], axis=0) / np.linalg.norm(Vs, axis=0)
        out["host_residuals"] = [float(v) for v in r]
        out["solver_residuals"] = [float(v) for v in res[idx]]
    s.close()
    print(json.dumps(out), flush=True)


def run_tda(p, args, gen_s):
    m = p.m
    s = TDASolver(p.A, p.nev, p.nex, deg=p.deg, tol=p.tol, max_iter=args.max_iter, nex_auto=args.nex_auto)
    W0 = colmajor(p.w0_raw[:m].contiguous())
    Lz = colmajor(p.lanczos_raw[:m].contiguous())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, X, res, info = s.solve(W0, Lz, raise_on_noconv=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(workload=p.name + "-tda", m=m, nev=p.nev, nex=p.nex, nex_used=info.nex_used, precision="fp64",
               generate_s=round(gen_s, 2), solve_s=round(wall, 3), iterations=info.iterations, locked=info.locked,
               phases_s=dict(lanczos=round(info.t_lanczos, 3), filter=round(info.t_filter, 3),
                             qr=round(info.t_qr, 3), rr=round(info.t_rr, 3), resid=round(info.t_resid, 3)),
               filter_tflops=round(info.filter_flops / info.t_filter / 1e12, 2) if info.t_filter > 0 else 0.0)
    if len(ev):
        Ah = p.A.cpu().numpy()
        if m <= 8000:  # the host eigvalsh of a larger A takes minutes
            t0 = time.perf_counter()
            ref = np.linalg.eigvalsh(Ah)[: len(ev)]
            out["host_eigvalsh_s"] = round(time.perf_counter() - t0, 2)
            out["eig_err_vs_eigvalsh"] = float(np.max(np.abs(ev - ref)) / np.max(np.abs(ref)))
        out.update(lambda_first=float(ev[0]), lambda_last=float(ev[-1]), max_resid=float(np.max(res)))
        if args.samples > 0:
            idx = np.unique(np.linspace(0, len(ev) - 1, args.samples).astype(int))
            Xs = X[:, idx].cpu().numpy()
            r = np.linalg.norm(Ah @ Xs - Xs * ev[idx][None, :], axis=0) / np.linalg.norm(Xs, axis=0)
            out["host_residuals"] = [float(v) for v in r]
            out["solver_residuals"] = [float(v) for v in res[idx]]
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
