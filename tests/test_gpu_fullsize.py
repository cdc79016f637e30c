"""Parity at the benchmark sizes, in the launch configuration bench.py times
(persistent CG, default slicing, all right-hand sides in one launch).

medium (8x8 subdomains, M = 256, FP64): the oracle runs the whole solve;
u on the evaluation grid and mu are compared.

large (32x32, M = 400, 16 right-hand sides, FP64 and mixed precision): too
large for the oracle's CG, so it is checked on samples the oracle can
compute one by one: for sampled subdomains and right-hand sides, the
oracle's local least-squares solve with the interface values mu returned by
the GPU, c_i = K_c^{i+} (f^i - B^i mu), must give the same fitted values
K_c^i c_i on the local collocation rows as the GPU's coefficients (this
checks features, QR, recovery and the consistency of c with mu), and CG must
report convergence.  The fitted values are compared rather than u at other
points: at these sizes K_c^i has a condition number near 1e13, so c carries
noise along near-null directions of K_c^i that is invisible on the
collocation rows but not elsewhere (measured 1e-5 between two float64
least-squares solvers at off-grid points).
"""
import numpy as np
import pytest

from oracle import ddelm_oracle as O
from paper_2503_10032_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _solver(w, **kw):
    from paper_2503_10032_amd import DDELMSolver
    W, b = I.hidden_params(w.N, w.M, 2, w.a, w.seed)
    xi = I.interior_points(w)
    s = DDELMSolver(w.nx, w.ny, w.M, W, b, xi, I.edge_params(w.p), I.extra_boundary_params(w), theta=w.theta,
                    max_nrhs=w.nrhs, **kw)
    return s, W, b, xi


def test_medium_workload_matches_oracle():
    _torch()
    w = I.workload("medium")
    g, W, b, xi = _solver(w, tol=1e-12)
    g.factor()
    xB = g.boundary_points().cpu().numpy()
    out = g.solve(I.sinsin_f(xi)[None], I.sinsin_u(xB)[None])
    assert out["stats"]["converged"]
    geo = O.Geometry2D(w.nx, w.ny, I.edge_params(w.p), I.extra_boundary_params(w), xi)
    ref = O.DDELMNN(geo, W, b, theta=w.theta).solve(O.local_rhs(geo, I.sinsin_f, I.sinsin_u), tol=1e-12,
                                                    maxit=20000)
    X = I.eval_grid(w)
    u = g.evaluate(out["coef"], X)[0].cpu().numpy()
    u_ref = O.evaluate(geo, W, b, ref["c"], X)
    eu = _rel(u, u_ref)
    emd = _rel(out["mu_dl"][0].cpu().numpy(), ref["mu_dl"])
    emp = _rel(out["mu_pi"][0].cpu().numpy(), ref["mu_pi"])
    print(f"medium: u {eu:.2e} mu_dl {emd:.2e} mu_pi {emp:.2e} iters {out['stats']['iters']} / {ref['iters']}")
    assert eu < 1e-9 and emd < 1e-8 and emp < 1e-8, (eu, emd, emp)


def _sampled_local_check(w, g, W, b, xi, out, subs, rhs_ids, tol):
    geo = O.Geometry2D(w.nx, w.ny, I.edge_params(w.p), I.extra_boundary_params(w), xi)
    f_fn, g_fn = I.rhs_functions(w)
    coef = out["coef"].cpu().numpy()
    mu_pi = out["mu_pi"].cpu().numpy()
    mu_dl = out["mu_dl"].cpu().numpy()
    worst = 0.0
    for i in subs:
        sb = geo.subs[i]
        K, _, _, _ = O.local_matrices(geo, i, W[i], b[i])
        for r in rhs_ids:
            f = np.concatenate([f_fn(sb.x_I)[r], g_fn(sb.x_B)[r], np.zeros(sb.n_G)])
            g0 = sb.n_I + sb.n_B
            f[g0:g0 + sb.n_P] += mu_pi[r][sb.pi_glob]            # f - B mu, B = -R on the Gamma rows
            f[g0 + sb.n_P:] += mu_dl[r][sb.dl_glob]
            c = O.LocalLS(K).solve(f)          # the oracle's Householder least-squares solve
            e = _rel(K @ coef[r, i], K @ c)
            worst = max(worst, e)
            assert e < tol, (i, r, e)
    return worst


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-4)])
def test_large_workload_sampled_local_solves(precision, tol):
    _torch()
    w = I.workload("large")
    g, W, b, xi = _solver(w, tol=1e-8, precision=precision)
    g.factor()
    f_fn, g_fn = I.rhs_functions(w)
    xB = g.boundary_points().cpu().numpy()
    out = g.solve(f_fn(xi), g_fn(xB))
    assert out["stats"]["converged"]
    if precision == 0:
        assert out["stats"]["rel_res"] <= 1e-8
    subs = [0, w.nx - 1, 5 * w.nx + 7, 17 * w.nx + 16, w.N - 1]      # corner, corner, interior, interior, corner
    worst = _sampled_local_check(w, g, W, b, xi, out, subs, [0, 7, 15], tol)
    print(f"large precision {precision}: worst sampled relative difference of fitted values {worst:.2e}")
