"""DDELM-NN time-to-solution on one MI355X.

One step = the whole hot path on one synthetic 2-D Poisson problem with the
inputs already in HBM: interface indexing (setup), feature assembly,
batched Householder QR of K_c^i and Kbar^i, local interface operators,
coarse S_Pi Cholesky, right-hand side, CG on eq. nn-mixed to relative
residual 1e-8, recovery of c and mu, and evaluation of u on the evaluation
grid.  Default workload: 8 x 8 subdomains, M = 256, 32 x 32 interior points,
32 points per edge, FP64, one right-hand side (u = sin(pi x) sin(pi y)).

Prints one JSON line (see the contract in the design notes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the CG kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters (KiB per dispatch), scaled by the same counters' reading of a plain
# copy of known size (FETCH_SIZE 0.5, WRITE_SIZE 1.0 of the bytes moved).  Valid
# only for the kernel sources they were taken with (sha256 of the three files
# below) and for the workload named; otherwise the bench reports null.
CG_SOURCES = ("kernels_cg.hpp", "kernels_solve.hpp", "kernels_common.hpp")
CG_TRAFFIC = {
    ("medium", "fp64"): dict(fetch_kib=1413423.4, write_kib=48890.3, fetch_scale=0.5, write_scale=1.0,
                             sha256="4f27056924380908c7303b5a7351e053a1b28039660cf289e6fd9d9db253026b"),
}


def cg_bytes_per_iteration(counts, M, n_pi, nrhs, elem=8):
    """Algorithmic HBM bytes of one CG iteration: every local interface
    operator (G, L, L^T, N, N^T blocks actually used) read once, the coarse
    matrices read once, plus the interface vectors."""
    nG = counts["n_P"].astype(np.int64) + counts["n_D"]
    nD = counts["n_D"].astype(np.int64)
    nP = counts["n_P"].astype(np.int64)
    mats = elem * int(np.sum(3 * nG * nD + 3 * nD * nP + 2 * nD * nD))
    coarse = 8 * (4 * n_pi * n_pi + 2 * n_pi * n_pi)
    vecs = 8 * nrhs * int(np.sum(nD)) * 12
    return mats + coarse + vecs


def cg_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in CG_SOURCES:
        with open(os.path.join(ROOT, "paper_2503_10032_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cg_traffic_bytes(workload, precision):
    """Measured HBM bytes per CG launch, or None when not measured for these sources."""
    t = CG_TRAFFIC.get((workload, precision))
    if t is None or t["sha256"] != cg_sources_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] / t["fetch_scale"] + t["write_kib"] / t["write_scale"])


def cpu_baseline(w, W, b, xi, X):
    """The FP64 oracle on the host cores, one whole step of the same workload:
    setup (features, QR, S_Pi), right-hand side, CG to 1e-8, recovery and
    evaluation on the evaluation grid."""
    from oracle import ddelm_oracle as O
    from paper_2503_10032_amd import inputs as I
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = len(os.sched_getaffinity(0))
    f_fn, g_fn = I.rhs_functions(w)
    t0 = time.perf_counter()
    geo = O.Geometry2D(w.nx, w.ny, I.edge_params(w.p), I.extra_boundary_params(w), xi)
    s = O.DDELMNN(geo, W, b, theta=w.theta)
    t1 = time.perf_counter()
    f = O.local_rhs(geo, lambda x: f_fn(x)[0], lambda x: g_fn(x)[0])
    r = s.solve(f, tol=1e-8, maxit=20000)
    t2 = time.perf_counter()
    O.evaluate(geo, W, b, r["c"], X)
    t3 = time.perf_counter()
    return {
        "value": t3 - t0, "unit": "s", "cores": int(cores), "kind": "oracle",
        "sample": (f"one whole step of the {w.name} workload (first right-hand side): setup {t1 - t0:.2f}s, "
                   f"right-hand side + CG to 1e-8 ({r['iters']} iterations) + recovery {t2 - t1:.2f}s, "
                   f"evaluation on {len(X)} points {t3 - t2:.2f}s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--cg-mode", type=int, default=0)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 5 times (the known-size kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                          "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (multi-GPU sharding is a "
              f"design note, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_10032_amd import DDELMSolver, inputs as I

    w = I.workload(args.workload)
    W, b = I.hidden_params(w.N, w.M, 2, w.a, w.seed)
    xi = I.interior_points(w)
    s_edge, s_extra = I.edge_params(w.p), I.extra_boundary_params(w)
    dev = torch.device("cuda:0")
    Wd = torch.as_tensor(W, device=dev)
    bd = torch.as_tensor(b, device=dev)
    xid = torch.as_tensor(xi, device=dev)
    X = torch.as_tensor(I.eval_grid(w), device=dev)
    f_fn, g_fn = I.rhs_functions(w)
    fI = torch.as_tensor(f_fn(xi), device=dev)
    prec = 1 if args.precision == "mixed" else 0
    probe = DDELMSolver(w.nx, w.ny, w.M, Wd, bd, xid, s_edge, s_extra, theta=w.theta, tol=1e-8,
                        max_nrhs=w.nrhs, cg_mode=args.cg_mode, precision=prec)
    gB = torch.as_tensor(g_fn(probe.boundary_points().cpu().numpy()), device=dev)
    if not args.quiet:
        print(f"bench: workload {w.name} ({w.nx}x{w.ny}, M={w.M}, nrhs={w.nrhs}) precision {args.precision}",
              file=sys.stderr, flush=True)
    counts = probe.counts()
    n_pi = probe.n_pi
    probe.close()

    def step():
        t0 = time.perf_counter()
        s = DDELMSolver(w.nx, w.ny, w.M, Wd, bd, xid, s_edge, s_extra, theta=w.theta, tol=1e-8,
                        max_nrhs=w.nrhs, cg_mode=args.cg_mode, precision=prec)
        t1 = time.perf_counter()
        s.factor()
        t2 = time.perf_counter()
        out = s.solve(fI, gB, want_mu=False)
        t3 = time.perf_counter()
        u = s.evaluate(out["coef"], X)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        ph = s.phase_times()
        ph.update({"host_setup": (t1 - t0) * 1e3, "host_factor": (t2 - t1) * 1e3, "host_solve": (t3 - t2) * 1e3,
                   "host_evaluate": (t4 - t3) * 1e3})
        s.close()
        return out, u, ph

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    phases = []
    iters = []
    for _ in range(args.steps):
        last = step()
        phases.append(last[2])
        iters.append(last[0]["stats"]["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    out, u, _ = last
    ph = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    it = int(np.median(iters))
    # accuracy against the manufactured solution (when there is one)
    err = None
    if w.rhs == "sinsin":
        Xh = X.cpu().numpy()
        uh = u[0].cpu().numpy()
        err = float(np.linalg.norm(uh - I.sinsin_u(Xh)) / np.linalg.norm(I.sinsin_u(Xh)))
    # dominant kernel and its roofline
    # local operators are float32 in mixed precision, everything else float64
    bpi = cg_bytes_per_iteration(counts, w.M, n_pi, w.nrhs, elem=4 if prec else 8)
    cg_ms = ph["cg"]
    solves = 4 * w.N * w.nrhs * it
    dominant = max((k for k in ph if not k.startswith("host_")), key=lambda k: ph[k])
    roof = {
        "kernel": "k_cg_fused (CG on eq. nn-mixed, one cooperative launch per solve)",
        "bound": "hbm", "achieved": bpi * it / (cg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "traffic": cg_traffic_bytes(w.name, args.precision),
    }
    roof["frac"] = roof["achieved"] / roof["peak"]
    res = {
        "metric": "DDELM-NN time-to-solution (rel res 1e-8) & local LS solves/s, mixed vs FP64",
        "value": ms_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: 2-D Poisson {w.nx}x{w.ny} subdomains, M={w.M}, "
                               f"{w.n_int}x{w.n_int} interior + {w.p} per edge, nrhs={w.nrhs}, theta={w.theta}, "
                               f"tol 1e-8", "precision": args.precision, "cg_iters": it},
        "local_ls_solves_per_s": solves / (cg_ms * 1e-3),
        "phase_ms": ph,
        "dominant_phase": dominant,
        "rel_l2_error_vs_exact": err,
        "roofline": roof,
        "cg_launch": {k: out["stats"][k] for k in ("cg_blocks", "cg_slices", "cg_coarse_dist")},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, W, b, xi, I.eval_grid(w))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
