"""Write the oracle's results on two full-size workloads as JSON fixtures.

The FP64 oracle needs minutes on these problems (its coarse Schur complement
is assembled column by column, one sweep over every subdomain per coarse
unknown), too long to run inside a GPU test.  This script runs it once on
the CPU and stores sampled entries of mu_Delta, mu_Pi and of u on the
evaluation grid, with the norms of the full vectors, so that the GPU tests
can compare against them.  It calls only the oracle and the seeded input
generators.

  adjoint_fp64.json            16x16 subdomains, M = 300, U(-2,2) seed 4,
                               32x32 interior points, 32 per edge; data of the
                               adjoint workload (64 sine coefficients of f,
                               8 per side for g, seed 5); CG to 1e-12; the
                               whole mu_Delta is stored as well (the tests
                               form the GPU system's residual at it)
  large_reduced_fp64.json      32x32 subdomains with the extra boundary rows
                               of the large workload (uneven local sizes),
                               M = 24, 5x5 interior, 6 per edge, U(-2,2)
                               seed 2, 16 random Fourier right-hand sides
                               (seed 100), of which 0, 7 and 15 are solved
                               here; CG to 1e-12
  varcoef_fp64.json            the variable-coefficient workload: 16x16
                               subdomains, M = 256, U(-2,2) seed 3, 20x20
                               interior, 20 per edge, -div(rho grad u) = 1,
                               u = 0, rho = tanh(GRF) + 1.1 (alpha 32, seed
                               7); CG to 1e-10; whole mu_Delta stored,
                               and the largest 2-norm condition number of
                               the local matrices K_c^i and Kbar^i

Usage: python tests/golden/make_fullsize_refs.py [adjoint|large_reduced|varcoef ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")   # many small LAPACK calls: one thread is fastest
import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ddelm_oracle as O            # noqa: E402
from paper_2503_10032_amd import inputs as I   # noqa: E402

SAMPLE_U = 600


def workloads():
    return {
        "adjoint": dict(w=I.Workload("adjoint", 16, 16, 300, 2.0, 4, 32, 32, tol=1e-12), rhs="adjoint",
                        solve=[0], mu_stride=16, full_mu=True),
        "large_reduced": dict(w=I.Workload("large_reduced", 32, 32, 24, 2.0, 2, 5, 6, tol=1e-12, nrhs=16,
                                           extra_boundary=True, rhs="fourier", rhs_seed=100),
                              rhs="fourier", solve=[0, 7, 15], mu_stride=16),
        "varcoef": dict(w=I.Workload("varcoef", 16, 16, 256, 2.0, 3, 20, 20, tol=1e-10, rhs="one", rho="grf"),
                        rhs="one", solve=[0], mu_stride=16, full_mu=True, cond_K=True),
    }


def sample_indices(n, k):
    return np.unique(np.linspace(0, n - 1, min(k, n)).round().astype(np.int64))


def run(name):
    spec = workloads()[name]
    w = spec["w"]
    W, b = I.hidden_params(w.N, w.M, 2, w.a, w.seed)
    xi = I.interior_points(w)
    t0 = time.time()
    geo = O.Geometry2D(w.nx, w.ny, I.edge_params(w.p), I.extra_boundary_params(w), xi)
    s = O.DDELMNN(geo, W, b, theta=w.theta, rho=I.coefficient(w))
    print(f"{name}: oracle set up in {time.time() - t0:.0f} s", flush=True)
    # 2-norm condition number of the local matrices (singular values): with a
    # rough coefficient the diagonal of R underestimates it
    cond_K = max(np.linalg.cond(K) for K in s.K + s.Kb) if spec.get("cond_K") else None
    if spec["rhs"] == "adjoint":
        ap = I.adjoint_params(5)
        f_fn = lambda x: ap.f(x)[None]
        g_fn = lambda x: ap.g(x)[None]
    else:
        f_fn, g_fn = I.rhs_functions(w)     # "fourier" or "one" (f = 1, g = 0)
    X = I.eval_grid(w)
    iu = sample_indices(len(X), SAMPLE_U)
    out = dict(workload=name, nx=w.nx, ny=w.ny, M=w.M, a=w.a, seed=w.seed, n_int=w.n_int, p=w.p,
               extra_boundary=w.extra_boundary, rhs=spec["rhs"], nrhs=w.nrhs, theta=w.theta, tol=w.tol,
               rho=w.rho, rho_alpha=w.rho_alpha, rho_seed=w.rho_seed, cond_K_max=cond_K,
               u_points=iu.tolist(), results=[])
    for r in spec["solve"]:
        t1 = time.time()
        f = O.local_rhs(geo, lambda x: f_fn(x)[r], lambda x: g_fn(x)[r])
        ref = s.solve(f, tol=w.tol, maxit=20000)
        u = O.evaluate(geo, W, b, ref["c"], X)
        idl = sample_indices(s.nD, max(1, s.nD // spec["mu_stride"]))
        ipi = sample_indices(s.nP, max(1, s.nP // spec["mu_stride"]))
        out["results"].append(dict(
            rhs=r, iters=int(ref["iters"]), kappa=float(ref["kappa"]),
            mu_dl_norm=float(np.linalg.norm(ref["mu_dl"])), mu_dl_index=idl.tolist(),
            mu_dl=ref["mu_dl"][idl].tolist(),
            mu_pi_norm=float(np.linalg.norm(ref["mu_pi"])), mu_pi_index=ipi.tolist(),
            mu_pi=ref["mu_pi"][ipi].tolist(),
            u_norm=float(np.linalg.norm(u)), u=u[iu].tolist()))
        if spec.get("full_mu"):
            out["results"][-1]["mu_dl_full"] = ref["mu_dl"].tolist()
        print(f"{name}: rhs {r} solved in {time.time() - t1:.0f} s, {ref['iters']} iterations", flush=True)
    path = os.path.join(HERE, f"{name}_fp64.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(workloads())):
        run(n)
