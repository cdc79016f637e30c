"""The allocation-free solve (ddelm_solve_noalloc) against ddelm_solve.

Both entry points run the same kernels; the allocation-free one takes its
workspace from the library's fixed scratch array instead of the context's
buffers.  Two calls in a row (the second on a smaller problem, so the
scratch holds the first call's values beyond the second's workspace), in
float64 and in mixed precision, each compared with ddelm_solve on the same
inputs; and a workspace above the scratch size is refused before any work.
"""
import numpy as np
import pytest

from paper_2503_10032_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(nx, ny, M, n_int, p, seed, nrhs, precision=0, extra=False):
    from paper_2503_10032_amd import DDELMSolver
    w = I.Workload("na", nx, ny, M, 2.0, seed, n_int, p, tol=1e-12, nrhs=nrhs, extra_boundary=extra,
                   rhs="fourier" if nrhs > 1 else "sinsin")
    W, b = I.hidden_params(w.N, M, 2, w.a, seed)
    xi = I.interior_points(w)
    g = DDELMSolver(nx, ny, M, W, b, xi, I.edge_params(p), I.extra_boundary_params(w), tol=1e-12, max_nrhs=nrhs,
                    precision=precision).factor()
    f_fn, g_fn = I.rhs_functions(w)
    xB = g.boundary_points().cpu().numpy()
    return w, g, f_fn(xi), g_fn(xB)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_solve_matches_solve_on_two_calls(precision):
    _torch()
    for k, spec in enumerate([dict(nx=4, ny=3, M=48, n_int=7, p=9, seed=2, nrhs=3, extra=True),
                              dict(nx=2, ny=2, M=40, n_int=6, p=8, seed=0, nrhs=1)]):
        w, g, fI, gB = _case(precision=precision, **spec)
        X = I.eval_grid(w)
        ref = g.solve(fI, gB)
        got = g.solve_noalloc(fI, gB)
        assert got["stats"]["converged"] == ref["stats"]["converged"]
        u_ref = g.evaluate(ref["coef"], X).cpu().numpy()
        u = g.evaluate(got["coef"], X).cpu().numpy()
        eu = _rel(u, u_ref)
        emd = _rel(got["mu_dl"].cpu().numpy(), ref["mu_dl"].cpu().numpy())
        emp = _rel(got["mu_pi"].cpu().numpy(), ref["mu_pi"].cpu().numpy())
        same = bool((got["coef"] == ref["coef"]).all())
        print(f"call {k} precision {precision}: u {eu:.2e} mu_dl {emd:.2e} mu_pi {emp:.2e} bitwise {same}")
        assert eu <= 1e-10 and emd <= 1e-10 and emp <= 1e-10, (eu, emd, emp)
        g.close()


def test_noalloc_solve_refuses_a_workspace_above_the_scratch_size():
    _torch()
    from paper_2503_10032_amd.solver import DDELMError
    w, g, fI, gB = _case(nx=16, ny=16, M=32, n_int=30, p=30, seed=1, nrhs=32)
    with pytest.raises(DDELMError, match="SHAPE.*scratch"):
        g.solve_noalloc(fI, gB)
    g.close()
