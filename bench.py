"""DDELM-NN time-to-solution on one MI355X, float64 against mixed precision.

One step = the whole hot path on one synthetic 2-D Poisson problem with the
inputs already in HBM: interface indexing (setup), feature assembly,
batched Householder QR of K_c^i and Kbar^i, local interface operators,
coarse S_Pi Cholesky, right-hand sides, CG on eq. nn-mixed, recovery of c
and mu, and evaluation of u on the evaluation grid.

Default workload (large): 32 x 32 subdomains (boundary subdomains carry
extra boundary rows, so the local sizes are uneven), M = 400, 40 x 40
interior points, 40 per edge, 16 random Fourier right-hand sides in one
batch, relative residual 1e-8.  Every step is timed in three precisions:

  fp64    float64 throughout; the float64 residual of eq. nn-mixed at the
          returned mu is checked after the CG (true_rel_res <= 1e-8);
  mixed   float32 Householder QR on the matrix cores, float64 downstream,
          float32 CG operators, float64 refinement of the coupled system;
          its distance from the float64 result is reported;
  f32cg   float64 factors, float32 CG operators, float64 refinement of the
          interface residual to 1e-8.

The JSON line's value is the float64 time to solution; the other two
precisions, their errors against the float64 result and the speed ratios
are in "precisions".  Prints one JSON line.
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
FP64_MFMA_PEAK_TFS = 78.6
FP32_MFMA_PEAK_TFS = 157.3
PRECISIONS = {"fp64": 0, "mixed": 1, "f32cg": 2}

# HBM bytes per launch of the CG kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters (KiB per dispatch), scaled by the same counters' reading of a plain
# copy of known size (FETCH_SIZE 0.5, WRITE_SIZE 1.0 of the bytes moved).  Valid
# only for the kernel sources they were taken with (sha256 of the three files
# below) and for the workload named; otherwise the bench reports null.
CG_SOURCES = ("kernels_cg.hpp", "kernels_solve.hpp", "kernels_common.hpp")
CG_TRAFFIC = {
    ("large", "fp64"): dict(fetch_kib=193915486.4, write_kib=56009999.5, fetch_scale=0.5, write_scale=1.0,
                            sha256="5ec49a76e5efeaaec9be3560ce59b2087caf083144dfcbd0d7cbe7fd572511bf"),
    ("medium", "fp64"): dict(fetch_kib=1448269.2, write_kib=53905.8, fetch_scale=0.5, write_scale=1.0,
                             sha256="5ec49a76e5efeaaec9be3560ce59b2087caf083144dfcbd0d7cbe7fd572511bf"),
}


def cg_bytes_per_iteration(counts, n_pi, nrhs, elem=8):
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


def qr_flops(counts, M):
    """Algorithmic flops of the Householder QR of every K_c^i and Kbar^i
    (2 m M^2 - 2/3 M^3 each)."""
    m = counts["m"].astype(np.float64)
    return float(2 * np.sum(2.0 * m * M * M - 2.0 / 3.0 * M ** 3))


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


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def cpu_baseline(w, iters):
    """The FP64 oracle on the host cores, on a bounded sample of the workload.

    A whole oracle step of the large workload takes hours (2048 Householder
    QRs of ~1800 x 400 matrices, then S_Pi assembled column by column: one
    sweep over all 1024 subdomains for each of 961 coarse unknowns), so the
    oracle runs on a 3 x 3 partition with the same local shapes (M, interior
    grid, points per edge, extra boundary rows) and the same right-hand-side
    family; its per-subdomain costs are scaled to the full workload:
        T = N (t_setup - t_coarse) / 9 + n_Pi N t_col / 9 + nrhs I N t_op / 9
    with t_col the oracle's S_Pi column sweep, t_op one application of
    S_theta, I the GPU's CG iteration count."""
    from oracle import ddelm_oracle as O
    from paper_2503_10032_amd import inputs as I
    s3 = I.Workload("slice", 3, 3, w.M, w.a, w.seed, w.n_int, w.p, extra_boundary=w.extra_boundary,
                    rhs=w.rhs, nrhs=1, rhs_seed=w.rhs_seed)
    W, b = I.hidden_params(s3.N, s3.M, 2, s3.a, s3.seed)
    xi = I.interior_points(s3)

    def per_call(fn, min_s, min_n=3):
        """Median time of one call, repeated for at least min_s seconds."""
        ts, t_all = [], time.perf_counter()
        while len(ts) < min_n or time.perf_counter() - t_all < min_s:
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    def measure():
        t0 = time.perf_counter()
        geo = O.Geometry2D(3, 3, I.edge_params(s3.p), I.extra_boundary_params(s3), xi)
        s = O.DDELMNN(geo, W, b, theta=s3.theta, rho=I.coefficient(w))
        t1 = time.perf_counter()
        e = np.zeros(s.nP)
        e[0] = 1.0
        t_col = per_call(lambda: s.S_Pi_apply(e), 1.0)
        v = np.random.default_rng(0).standard_normal(s.nD)
        t_op = per_call(lambda: s.S_theta(v), 3.0)
        return t1 - t0 - s.nP * t_col, t_col, t_op, s.nP

    t_set, t_col, t_op, np3 = measure()
    N, nP = w.N, (w.nx - 1) * (w.ny - 1)
    est = N * t_set / 9 + nP * N * t_col / 9 + w.nrhs * iters * N * t_op / 9
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            t_set1, t_col1, t_op1, _ = measure()
        one = N * t_set1 / 9 + nP * N * t_col1 / 9 + w.nrhs * iters * N * t_op1 / 9
    except Exception:
        pass
    return {
        "value": est, "unit": "s", "cores": int(blas_threads()), "kind": "oracle",
        "value_1thread": one,
        "sample": (f"oracle on a 3x3 partition with the {w.name} workload's local shapes: setup without the "
                   f"coarse columns {t_set:.2f}s, one S_Pi column sweep {t_col:.4f}s and one S_theta application "
                   f"{t_op:.4f}s (medians of calls repeated for 1 s and 3 s); scaled as N*t_setup/9 + "
                   f"n_Pi*N*t_col/9 + nrhs*I*N*t_op/9 with N={N}, n_Pi={nP}, nrhs={w.nrhs}, I={iters}; "
                   f"measured with all BLAS threads, then again with one"),
    }


def coefficient_arrays(rho_fn, solver, xi, dev):
    """Device arrays of ddelm_set_coefficient for a coefficient callable (None
    for rho = 1), evaluated once at the interior and interface points so that
    they are resident before any timed step."""
    if rho_fn is None:
        return None
    import torch
    r, g = rho_fn(xi.reshape(-1, 2))
    rho_I = np.concatenate([r.reshape(-1, 1), g.reshape(-1, 2)], axis=1).reshape(xi.shape[0], xi.shape[1], 3)
    xp, xd = (t.cpu().numpy() for t in solver.interface_points())
    rp = rho_fn(xp)[0] if len(xp) else np.zeros(0)
    rd = rho_fn(xd)[0]
    return tuple(torch.as_tensor(np.ascontiguousarray(a), device=dev) for a in (rho_I, rp, rd))


ABLATION = [   # (label, coarse, theta): the paper's comparison columns and the cells of table chov
    ("DDELM (no coarse space)", 0, 0.0),
    ("K + A, corners", 1, 0.0), ("K + A, corners, NN", 1, 0.999),
    ("K_c + A", 3, 0.0), ("K_c + A, NN", 3, 0.999),
    ("K + A_m", 4, 0.0), ("K + A_m, NN", 4, 0.999),
    ("DDELM-CS (K_c + A_m)", 2, 0.0), ("DDELM-NN (K_c + A_m, NN)", 2, 0.999),
]


def ablation(args):
    """Iterations, time and accuracy of DDELM, DDELM-CS and DDELM-NN and of the
    K/K_c x A/A_m cells (sec. 4.2, tables chov and nn-mixed) on one workload,
    same inputs, float64; one JSON line."""
    import torch
    from paper_2503_10032_amd import DDELMSolver, inputs as I
    w = I.workload(args.workload)
    W, b = I.hidden_params(w.N, w.M, 2, w.a, w.seed)
    xi = I.interior_points(w)
    s_edge, s_extra = I.edge_params(w.p), I.extra_boundary_params(w)
    dev = torch.device("cuda:0")
    X = I.eval_grid(w)
    Xd = torch.as_tensor(X, device=dev)
    f_fn, g_fn = I.rhs_functions(w)
    if w.rhs == "sinsin":
        u_exact = torch.as_tensor(I.sinsin_u(X), device=dev)
    rows = []
    rho_fn = I.coefficient(w)
    # inputs resident on the device before any timed step (the boundary
    # points do not depend on the variant)
    Wd, bd, xid = (torch.as_tensor(a, device=dev) for a in (W, b, xi))
    fI = torch.as_tensor(f_fn(xi), device=dev)
    probe = DDELMSolver(w.nx, w.ny, w.M, Wd, bd, xid, s_edge, s_extra)
    gB = torch.as_tensor(g_fn(probe.boundary_points().cpu().numpy()), device=dev)
    probe.close()
    for label, coarse, theta in ABLATION:
        rho_dev = None
        if rho_fn is not None:
            probe = DDELMSolver(w.nx, w.ny, w.M, Wd, bd, xid, s_edge, s_extra, theta=theta, coarse=coarse)
            rho_dev = coefficient_arrays(rho_fn, probe, xi, dev)
            probe.close()

        def step():
            s = DDELMSolver(w.nx, w.ny, w.M, Wd, bd, xid, s_edge, s_extra, theta=theta, coarse=coarse, tol=1e-8,
                            max_nrhs=w.nrhs, maxit=50000)
            if rho_dev is not None:
                s.set_coefficient(*rho_dev)
            s.factor()
            out = s.solve(fI, gB, want_mu=False)
            u = s.evaluate(out["coef"], Xd)
            torch.cuda.synchronize()
            s.close()
            return out, u
        for _ in range(args.warmup):
            step()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out, u = step()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        row = {"variant": label, "coarse": coarse, "theta": theta, "cg_iters": out["stats"]["iters"],
               "ms_per_step": ms, "converged": out["stats"]["converged"],
               "true_rel_res": out["stats"]["true_rel_res"]}
        if w.rhs == "sinsin":
            row["rel_l2_error_vs_exact"] = float(torch.linalg.norm(u[0] - u_exact) / torch.linalg.norm(u_exact))
        rows.append(row)
        if not args.quiet:
            print(f"ablation: {label}: {row['cg_iters']} iterations, {ms:.1f} ms", file=sys.stderr, flush=True)
    base = {r["variant"]: r for r in rows}
    nn = base["DDELM-NN (K_c + A_m, NN)"]
    print(json.dumps({"ablation": rows, "workload": w.name,
                      "iteration_ratio_DDELM_over_NN": base["DDELM (no coarse space)"]["cg_iters"] / nn["cg_iters"],
                      "iteration_ratio_CS_over_NN": base["DDELM-CS (K_c + A_m)"]["cg_iters"] / nn["cg_iters"],
                      "time_ratio_DDELM_over_NN": base["DDELM (no coarse space)"]["ms_per_step"] / nn["ms_per_step"],
                      "time_ratio_CS_over_NN": base["DDELM-CS (K_c + A_m)"]["ms_per_step"] / nn["ms_per_step"]}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=None, help="large (default), medium, small, adjoint; medium for --ablation")
    ap.add_argument("--cg-mode", type=int, default=0)
    ap.add_argument("--precision", default="all", help="fp64, mixed, f32cg or all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--ablation", action="store_true",
                    help="DDELM / DDELM-CS / DDELM-NN and the K/K_c x A/A_m cells on the workload (default medium)")
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
    if args.ablation:
        args.workload = args.workload or "medium"
        ablation(args)
        return

    import torch
    from paper_2503_10032_amd import DDELMSolver, inputs as I
    from paper_2503_10032_amd import _lib

    w = I.workload(args.workload or "large")
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
    modes = list(PRECISIONS) if args.precision == "all" else args.precision.split(",")
    tol = 1e-8

    rho_dev = None

    def make(prec):
        s = DDELMSolver(w.nx, w.ny, w.M, Wd, bd, xid, s_edge, s_extra, theta=w.theta, tol=tol,
                        max_nrhs=w.nrhs, cg_mode=args.cg_mode, precision=PRECISIONS[prec])
        if rho_dev is not None:
            s.set_coefficient(*rho_dev)
        return s

    probe = make("fp64")
    gB = torch.as_tensor(g_fn(probe.boundary_points().cpu().numpy()), device=dev)
    counts = probe.counts()
    n_pi = probe.n_pi
    rho_dev = coefficient_arrays(I.coefficient(w), probe, xi, dev)
    probe.close()
    if not args.quiet:
        print(f"bench: workload {w.name} ({w.nx}x{w.ny}, M={w.M}, nrhs={w.nrhs}) precisions {modes}",
              file=sys.stderr, flush=True)

    def step(prec):
        t0 = time.perf_counter()
        s = make(prec)
        t1 = time.perf_counter()
        s.factor()
        t2 = time.perf_counter()
        out = s.solve(fI, gB)
        t3 = time.perf_counter()
        u = s.evaluate(out["coef"], X)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        ph = s.phase_times()
        ph.update({"host_setup": (t1 - t0) * 1e3, "host_factor": (t2 - t1) * 1e3, "host_solve": (t3 - t2) * 1e3,
                   "host_evaluate": (t4 - t3) * 1e3})
        s.close()
        return out, u, ph

    results = {}
    for prec in modes:
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phases, iters = [], []
        last = None
        for _ in range(args.steps):
            last = step(prec)
            phases.append(last[2])
            iters.append(last[0]["stats"]["iters"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out, u, _ = last
        results[prec] = dict(ms=(t1 - t0) * 1e3 / args.steps, out=out, u=u,
                             ph={k: float(np.mean([p[k] for p in phases])) for k in phases[0]},
                             iters=int(np.median(iters)))
        if not args.quiet:
            print(f"bench: {prec} {results[prec]['ms']:.1f} ms/step, {results[prec]['iters']} CG iterations",
                  file=sys.stderr, flush=True)

    main_prec = "fp64" if "fp64" in results else modes[0]
    R = results[main_prec]
    ph, it = R["ph"], R["iters"]
    st = R["out"]["stats"]

    def rel(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    prec_report = {}
    for prec, r in results.items():
        s_ = r["out"]["stats"]
        e = {"ms_per_step": r["ms"], "cg_iters": r["iters"], "converged": s_["converged"],
             "true_rel_res": None if s_["true_rel_res"] != s_["true_rel_res"] else s_["true_rel_res"],
             "refine_steps": s_["refine_steps"], "refine_corr": s_["refine_corr"],
             "cg_restarts": s_["cg_restarts"], "phase_ms": r["ph"]}
        if "fp64" in results and prec != "fp64":
            ref = results["fp64"]
            e["rel_err_u_vs_fp64"] = rel(r["u"], ref["u"])
            e["rel_err_mu_dl_vs_fp64"] = rel(r["out"]["mu_dl"], ref["out"]["mu_dl"])
            e["speedup_vs_fp64"] = ref["ms"] / r["ms"]
        prec_report[prec] = e

    # dominant kernel: the persistent CG (HBM), and the QR on the matrix cores
    elem = 8 if main_prec == "fp64" else 4
    bpi = cg_bytes_per_iteration(counts, n_pi, w.nrhs, elem=elem)
    cg_ms = ph["cg"]
    solves = 4 * w.N * w.nrhs * it
    dominant = max((k for k in ph if not k.startswith("host_")), key=lambda k: ph[k])
    roof = {
        "kernel": "k_cg_fused (CG on eq. nn-mixed, one cooperative launch per solve)",
        "bound": "hbm", "achieved": bpi * it / (cg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "traffic": cg_traffic_bytes(w.name, main_prec),
        "bytes_per_iteration": bpi, "iterations": it,
    }
    roof["frac"] = roof["achieved"] / roof["peak"]
    qf = qr_flops(counts, w.M)
    roof_qr = {"kernel": "batched Householder QR (panels + block-reflector updates)", "bound": "mfma",
               "achieved": qf / (ph["qr"] * 1e-3) / 1e12, "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
               "flops": qf}
    roof_qr["frac"] = roof_qr["achieved"] / roof_qr["peak"]
    if "mixed" in results:
        roof_qr["mixed_float32"] = {"achieved": qf / (results["mixed"]["ph"]["qr"] * 1e-3) / 1e12,
                                    "peak": FP32_MFMA_PEAK_TFS}
    err = None
    if w.rhs == "sinsin":
        Xh = X.cpu().numpy()
        uh = R["u"][0].cpu().numpy()
        err = float(np.linalg.norm(uh - I.sinsin_u(Xh)) / np.linalg.norm(I.sinsin_u(Xh)))
    res = {
        "metric": "DDELM-NN time-to-solution (rel res 1e-8) & local LS solves/s, mixed vs FP64",
        "value": R["ms"] / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: 2-D {'Poisson' if w.rho == 'one' else 'variable-coefficient Poisson (rho = tanh(GRF) + 1.1, alpha ' + format(w.rho_alpha, 'g') + ')'} {w.nx}x{w.ny} subdomains, M={w.M}, "
                               f"{w.n_int}x{w.n_int} interior + {w.p} per edge"
                               f"{' + extra boundary rows' if w.extra_boundary else ''}, nrhs={w.nrhs} "
                               f"({w.rhs} sources), theta={w.theta}, rel res {tol:g}",
                   "precision": main_prec, "cg_iters": it,
                   "timed_steps_per_precision": args.steps, "precisions_timed": list(results)},
        "true_rel_res": st["true_rel_res"],
        "converged": st["converged"],
        "local_ls_solves_per_s": solves / (cg_ms * 1e-3),
        "phase_ms": ph,
        "dominant_phase": dominant,
        "rel_l2_error_vs_exact": err,
        "precisions": prec_report,
        "roofline": roof,
        "roofline_qr": roof_qr,
        "cg_launch": {k: st[k] for k in ("cg_blocks", "cg_slices", "cg_coarse_dist")},
        "kappa_est_max": st["kappa_est_max"],
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, it)
    print(json.dumps(res), flush=True)
    _lib.load().ddelm_release_cached_memory()


if __name__ == "__main__":
    main()
