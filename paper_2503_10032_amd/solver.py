"""Python front end of the DDELM-NN library: torch tensors in, torch tensors out.

Only argument marshalling happens here; every step of the method runs in
the HIP kernels of libddelm.so.  The library must be built and a GPU must
be present, otherwise construction raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


class DDELMError(RuntimeError):
    pass


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class DDELMSolver:
    """setup -> factor -> solve(f, g) -> evaluate on one GPU.

    Parameters follow include/ddelm.h.  W (N, M, 2), b (N, M) and x_int
    (N, n_int, 2) may be numpy arrays or tensors; they are copied to the
    device as float64.
    """

    def __init__(self, nx: int, ny: int, M: int, W, b, x_int, edge_s: Sequence[float],
                 extra_s: Sequence[float] = (), lo=(0.0, 0.0), hi=(1.0, 1.0), theta: float = 0.999,
                 coarse: int = 2, tol: float = 1e-8, maxit: int = 20000, max_nrhs: int = 1,
                 cg_mode: int = 0, precision: int = 0, refine_maxit: int = 10, refine_tol: float = 1e-9,
                 inner_tol: float = 1e-3, device: str = "cuda:0"):
        if not torch.cuda.is_available():
            raise DDELMError("DDELM-NN needs a GPU (torch.cuda.is_available() is False)")
        self.lib = L.load()
        self.device = torch.device(device)
        dev = self.device
        self.W = torch.as_tensor(W, dtype=torch.float64, device=dev).contiguous()
        self.b = torch.as_tensor(b, dtype=torch.float64, device=dev).contiguous()
        self.x_int = torch.as_tensor(x_int, dtype=torch.float64, device=dev).contiguous()
        N = nx * ny
        assert self.W.shape == (N, M, 2) and self.b.shape == (N, M), "W must be (N, M, 2), b (N, M)"
        assert self.x_int.ndim == 3 and self.x_int.shape[0] == N and self.x_int.shape[2] == 2
        self._edge = np.ascontiguousarray(edge_s, dtype=np.float64)
        self._extra = np.ascontiguousarray(extra_s, dtype=np.float64)
        prob = L.Problem()
        prob.nx, prob.ny = nx, ny
        prob.lo[0], prob.lo[1] = lo
        prob.hi[0], prob.hi[1] = hi
        prob.p = len(self._edge)
        prob.edge_s = self._edge.ctypes.data_as(L.c_double_p)
        prob.n_extra = len(self._extra)
        prob.extra_s = self._extra.ctypes.data_as(L.c_double_p) if len(self._extra) else None
        prob.n_int = self.x_int.shape[1]
        prob.x_int = self.x_int.data_ptr()
        prob.M = M
        prob.W = self.W.data_ptr()
        prob.b = self.b.data_ptr()
        opt = L.Options()
        self.lib.ddelm_default_options(ctypes.byref(opt))
        opt.theta, opt.coarse, opt.precision = theta, coarse, precision
        opt.tol, opt.maxit, opt.max_nrhs, opt.cg_mode = tol, maxit, max_nrhs, cg_mode
        opt.refine_maxit, opt.refine_tol, opt.inner_tol = refine_maxit, refine_tol, inner_tol
        self.opt = opt
        self.stream = torch.cuda.current_stream(dev)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = self.lib.ddelm_setup(ctypes.byref(ctx), ctypes.byref(prob), ctypes.byref(opt),
                                      ctypes.c_void_p(self.stream.cuda_stream))
        self.ctx = ctx
        L.register(self)
        if st != L.DDELM_OK:
            msg = self.lib.ddelm_last_error(ctx).decode() if ctx else ""
            self.close()
            raise DDELMError(f"ddelm_setup: {L.STATUS_NAMES.get(st, st)}: {msg}")
        sz = L.Sizes()
        self._check(self.lib.ddelm_get_sizes(self.ctx, ctypes.byref(sz)), "get_sizes")
        self.sizes = sz
        self.N, self.M, self.n_pi, self.n_dl = sz.N, sz.M, sz.n_pi, sz.n_dl
        self.nx, self.ny = nx, ny
        self.max_nrhs = max_nrhs
        self.factored = False

    # ------------------------------------------------------------ helpers
    def _check(self, st, what):
        if st < 0:
            raise DDELMError(f"ddelm_{what}: {L.STATUS_NAMES.get(st, st)}: "
                             f"{self.lib.ddelm_last_error(self.ctx).decode()}")
        return st

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ddelm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ API
    def set_coefficient(self, rho_I, rho_pi, rho_dl):
        """Coefficient rho of -div(rho grad u) (ddelm_set_coefficient):
        rho_I (N, n_int, 3) = rho, d rho/dx, d rho/dy at the interior points,
        rho_pi (n_pi,) and rho_dl (n_dl,) = rho at the interface_points().
        All None: back to rho = 1.  The solver must be factored again."""
        dev = self.device
        if rho_I is None and rho_pi is None and rho_dl is None:
            keep = ()
            args = (None, None, None)
        else:
            keep = tuple(torch.as_tensor(t, dtype=torch.float64, device=dev).contiguous()
                         for t in (rho_I, rho_pi, rho_dl))
            assert keep[0].shape == (self.N, self.x_int.shape[1], 3), "rho_I must be (N, n_int, 3)"
            assert keep[1].shape == (self.n_pi,) and keep[2].shape == (self.n_dl,), "rho_pi (n_pi,), rho_dl (n_dl,)"
            args = tuple(t.data_ptr() if t.numel() else None for t in keep)
        with torch.cuda.device(dev):
            self._check(self.lib.ddelm_set_coefficient(self.ctx, *args), "set_coefficient")
        self.factored = False
        return self

    def coefficient_from(self, rho_fn):
        """set_coefficient from a callable x (n, 2) numpy -> (rho (n,), grad rho (n, 2)),
        evaluated at the interior points and at the interface points."""
        xi = self.x_int.cpu().numpy().reshape(-1, 2)
        r, g = rho_fn(xi)
        rho_I = np.concatenate([np.asarray(r).reshape(-1, 1), np.asarray(g).reshape(-1, 2)], axis=1)
        xp, xd = (t.cpu().numpy() for t in self.interface_points())
        rp = np.asarray(rho_fn(xp)[0]).reshape(-1) if len(xp) else np.zeros(0)
        rd = np.asarray(rho_fn(xd)[0]).reshape(-1)
        return self.set_coefficient(rho_I.reshape(self.N, -1, 3), rp, rd)

    def factor(self):
        with torch.cuda.device(self.device):
            self._check(self.lib.ddelm_factor(self.ctx), "factor")
        self.factored = True
        return self

    def counts(self):
        N = self.N
        nB, nP, nD, m = (np.zeros(N, np.int32) for _ in range(4))
        self._check(self.lib.ddelm_get_counts(self.ctx, *(a.ctypes.data_as(L.c_int_p) for a in (nB, nP, nD, m))),
                    "get_counts")
        return dict(n_B=nB, n_P=nP, n_D=nD, m=m)

    def indexing(self):
        c = self.counts()
        pi = np.zeros(max(int(c["n_P"].sum()), 1), np.int32)
        dl = np.zeros(max(int(c["n_D"].sum()), 1), np.int32)
        self._check(self.lib.ddelm_get_indexing(self.ctx, pi.ctypes.data_as(L.c_int_p),
                                                dl.ctypes.data_as(L.c_int_p)), "get_indexing")
        return pi[:int(c["n_P"].sum())], dl[:int(c["n_D"].sum())]

    def boundary_points(self) -> torch.Tensor:
        out = torch.zeros((max(self.sizes.sum_nB, 1), 2), dtype=torch.float64, device=self.device)
        self._check(self.lib.ddelm_get_boundary_points(self.ctx, out.data_ptr()), "get_boundary_points")
        return out[: self.sizes.sum_nB]

    def interface_points(self):
        xp = torch.zeros((max(self.n_pi, 1), 2), dtype=torch.float64, device=self.device)
        xd = torch.zeros((max(self.n_dl, 1), 2), dtype=torch.float64, device=self.device)
        self._check(self.lib.ddelm_get_interface_points(self.ctx, xp.data_ptr(), xd.data_ptr()), "get_interface_points")
        return xp[: self.n_pi], xd[: self.n_dl]

    def phase_times(self):
        """Device-timeline ms of the last factor/solve phases (see ddelm_get_phase_times)."""
        ms = np.zeros(8)
        self._check(self.lib.ddelm_get_phase_times(self.ctx, ms.ctypes.data_as(L.c_double_p)), "get_phase_times")
        keys = ("assemble", "qr", "local_ops", "coarse", "rhs", "cg", "recover")
        return {k: float(ms[i]) for i, k in enumerate(keys)}

    def local_matrix(self, which: int, sub: int = 0) -> torch.Tensor:
        r, c = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.ddelm_get_local_matrix(self.ctx, which, sub, None, ctypes.byref(r), ctypes.byref(c)),
                    "get_local_matrix")
        out = torch.zeros((max(r.value, 1), max(c.value, 1)), dtype=torch.float64, device=self.device)
        if r.value and c.value:
            self._check(self.lib.ddelm_get_local_matrix(self.ctx, which, sub, out.data_ptr(), ctypes.byref(r),
                                                        ctypes.byref(c)), "get_local_matrix")
        return out[: r.value, : c.value]

    def solve(self, f_I, g_B, want_mu: bool = True, mu0=None):
        """f_I (nrhs, N, n_int), g_B (nrhs, sum_nB) -> dict(coef (nrhs, N, M), mu_pi, mu_dl, stats).
        mu0 (nrhs, n_dl), optional: starting value of mu_Delta for the CG."""
        dev = self.device
        f_I = torch.as_tensor(f_I, dtype=torch.float64, device=dev).contiguous()
        g_B = torch.as_tensor(g_B, dtype=torch.float64, device=dev).contiguous()
        if f_I.ndim == 2:
            f_I = f_I[None]
        if g_B.ndim == 1:
            g_B = g_B[None]
        nrhs = f_I.shape[0]
        assert f_I.shape == (nrhs, self.N, self.sizes.n_int), f_I.shape
        assert g_B.shape == (nrhs, self.sizes.sum_nB), g_B.shape
        coef = torch.empty((nrhs, self.N, self.M), dtype=torch.float64, device=dev)
        mu_pi = torch.zeros((nrhs, self.n_pi), dtype=torch.float64, device=dev) if want_mu else None
        mu_dl = torch.zeros((nrhs, self.n_dl), dtype=torch.float64, device=dev) if want_mu else None
        m0 = None
        if mu0 is not None and self.n_dl:
            m0 = torch.as_tensor(mu0, dtype=torch.float64, device=dev).contiguous().reshape(nrhs, self.n_dl)
        st = L.Stats()
        with torch.cuda.device(dev):
            code = self._check(self.lib.ddelm_solve(self.ctx, nrhs, f_I.data_ptr(), g_B.data_ptr(), _ptr(m0),
                                                    coef.data_ptr(),
                                                    _ptr(mu_pi) if self.n_pi else None,
                                                    _ptr(mu_dl) if self.n_dl else None, ctypes.byref(st)), "solve")
        return dict(coef=coef, mu_pi=mu_pi, mu_dl=mu_dl, stats=self._stats(st, code))

    def solve_noalloc(self, f_I, g_B):
        """As solve, through ddelm_solve_noalloc: the call allocates no device
        memory (its workspace lives in the library's fixed scratch array; the
        output tensors are allocated here, before the call)."""
        dev = self.device
        f_I = torch.as_tensor(f_I, dtype=torch.float64, device=dev).contiguous()
        g_B = torch.as_tensor(g_B, dtype=torch.float64, device=dev).contiguous()
        if f_I.ndim == 2:
            f_I = f_I[None]
        if g_B.ndim == 1:
            g_B = g_B[None]
        nrhs = f_I.shape[0]
        assert f_I.shape == (nrhs, self.N, self.sizes.n_int), f_I.shape
        assert g_B.shape == (nrhs, self.sizes.sum_nB), g_B.shape
        coef = torch.empty((nrhs, self.N, self.M), dtype=torch.float64, device=dev)
        mu_pi = torch.zeros((nrhs, self.n_pi), dtype=torch.float64, device=dev)
        mu_dl = torch.zeros((nrhs, self.n_dl), dtype=torch.float64, device=dev)
        st = L.Stats()
        with torch.cuda.device(dev):
            code = self._check(self.lib.ddelm_solve_noalloc(self.ctx, nrhs, f_I.data_ptr(), g_B.data_ptr(),
                                                            coef.data_ptr(), _ptr(mu_pi) if self.n_pi else None,
                                                            _ptr(mu_dl) if self.n_dl else None, ctypes.byref(st)),
                               "solve_noalloc")
        return dict(coef=coef, mu_pi=mu_pi, mu_dl=mu_dl, stats=self._stats(st, code))

    def solve_general(self, f_loc, h=None, want_mu: bool = True):
        """General right-hand side: f_loc (nrhs, sum m) on every local row, h
        (nrhs, n_pi + n_dl) on the flux rows (None = 0)."""
        dev = self.device
        f_loc = torch.as_tensor(f_loc, dtype=torch.float64, device=dev).contiguous()
        if f_loc.ndim == 1:
            f_loc = f_loc[None]
        nrhs = f_loc.shape[0]
        summ = int(self.counts()["m"].sum())
        assert f_loc.shape == (nrhs, summ), f_loc.shape
        hh = None
        if h is not None:
            hh = torch.as_tensor(h, dtype=torch.float64, device=dev).contiguous().reshape(nrhs, self.n_pi + self.n_dl)
        coef = torch.empty((nrhs, self.N, self.M), dtype=torch.float64, device=dev)
        mu_pi = torch.zeros((nrhs, self.n_pi), dtype=torch.float64, device=dev) if want_mu else None
        mu_dl = torch.zeros((nrhs, self.n_dl), dtype=torch.float64, device=dev) if want_mu else None
        st = L.Stats()
        with torch.cuda.device(dev):
            code = self._check(self.lib.ddelm_solve_general(
                self.ctx, nrhs, f_loc.data_ptr(), _ptr(hh), coef.data_ptr(),
                _ptr(mu_pi) if self.n_pi else None, _ptr(mu_dl) if self.n_dl else None, ctypes.byref(st)),
                "solve_general")
        return dict(coef=coef, mu_pi=mu_pi, mu_dl=mu_dl, stats=self._stats(st, code))

    def evaluate(self, coef: torch.Tensor, x, grad: bool = False):
        dev = self.device
        x = torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous()
        coef = coef.contiguous()
        nrhs = coef.shape[0] if coef.ndim == 3 else 1
        npts = x.shape[0]
        u = torch.empty((nrhs, npts), dtype=torch.float64, device=dev)
        g = torch.empty((nrhs, npts, 2), dtype=torch.float64, device=dev) if grad else None
        with torch.cuda.device(dev):
            self._check(self.lib.ddelm_evaluate(self.ctx, nrhs, coef.data_ptr(), npts, x.data_ptr(), u.data_ptr(),
                                                _ptr(g)), "evaluate")
        return (u, g) if grad else u

    # ------------------------------------------------------------ adjoints
    def _stats(self, st, code):
        return dict(iters=st.iters, refine_steps=st.refine_steps, rel_res=st.rel_res, ms_rhs=st.ms_rhs,
                    ms_cg=st.ms_cg, ms_recover=st.ms_recover, converged=code == L.DDELM_OK,
                    cg_blocks=st.cg_blocks, cg_slices=st.cg_slices, cg_coarse_dist=st.cg_coarse_dist,
                    cg_restarts=st.cg_restarts, true_rel_res=st.true_rel_res, refine_corr=st.refine_corr,
                    kappa_est_max=st.kappa_est_max, start_rel_res=st.start_rel_res)

    def solve_adjoint(self, coef_bar):
        """Transpose of solve: coef_bar (nrhs, N, M) -> dict(f_I_bar (nrhs, N, n_int),
        g_B_bar (nrhs, sum_nB), stats)."""
        dev = self.device
        cb = torch.as_tensor(coef_bar, dtype=torch.float64, device=dev).contiguous()
        if cb.ndim == 2:
            cb = cb[None]
        nrhs = cb.shape[0]
        assert cb.shape == (nrhs, self.N, self.M), cb.shape
        fI = torch.empty((nrhs, self.N, self.sizes.n_int), dtype=torch.float64, device=dev)
        gB = torch.empty((nrhs, max(self.sizes.sum_nB, 1)), dtype=torch.float64, device=dev)
        st = L.Stats()
        with torch.cuda.device(dev):
            code = self._check(self.lib.ddelm_solve_adjoint(self.ctx, nrhs, cb.data_ptr(), fI.data_ptr(),
                                                            gB.data_ptr() if self.sizes.sum_nB else None,
                                                            ctypes.byref(st)), "solve_adjoint")
        return dict(f_I_bar=fI, g_B_bar=gB[:, : self.sizes.sum_nB], stats=self._stats(st, code))

    def solve_adjoint_general(self, coef_bar, mu_pi_bar=None, mu_dl_bar=None):
        """Transpose of solve_general: cotangents of (coef, mu_pi, mu_dl) ->
        dict(f_loc_bar (nrhs, sum m), h_bar (nrhs, n_pi + n_dl), stats)."""
        dev = self.device
        cb = torch.as_tensor(coef_bar, dtype=torch.float64, device=dev).contiguous()
        if cb.ndim == 2:
            cb = cb[None]
        nrhs = cb.shape[0]
        assert cb.shape == (nrhs, self.N, self.M), cb.shape

        def opt(t, n):
            if t is None or n == 0:
                return None
            t = torch.as_tensor(t, dtype=torch.float64, device=dev).contiguous().reshape(nrhs, n)
            return t

        mp, md = opt(mu_pi_bar, self.n_pi), opt(mu_dl_bar, self.n_dl)
        summ = int(self.counts()["m"].sum())
        fb = torch.empty((nrhs, summ), dtype=torch.float64, device=dev)
        hb = torch.zeros((nrhs, max(self.n_pi + self.n_dl, 1)), dtype=torch.float64, device=dev)
        st = L.Stats()
        with torch.cuda.device(dev):
            code = self._check(self.lib.ddelm_solve_adjoint_general(
                self.ctx, nrhs, cb.data_ptr(), _ptr(mp), _ptr(md), fb.data_ptr(),
                hb.data_ptr() if self.n_pi + self.n_dl else None, ctypes.byref(st)), "solve_adjoint_general")
        return dict(f_loc_bar=fb, h_bar=hb[:, : self.n_pi + self.n_dl], stats=self._stats(st, code))

    def evaluate_adjoint(self, x, u_bar, grad_bar=None):
        """Transpose of evaluate in the coefficients: u_bar (nrhs, npts) and
        optionally grad_bar (nrhs, npts, 2) -> coef_bar (nrhs, N, M)."""
        dev = self.device
        x = torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous()
        ub = torch.as_tensor(u_bar, dtype=torch.float64, device=dev).contiguous()
        if ub.ndim == 1:
            ub = ub[None]
        nrhs, npts = ub.shape
        assert x.shape == (npts, 2), x.shape
        gb = None
        if grad_bar is not None:
            gb = torch.as_tensor(grad_bar, dtype=torch.float64, device=dev).contiguous().reshape(nrhs, npts, 2)
        cb = torch.empty((nrhs, self.N, self.M), dtype=torch.float64, device=dev)
        with torch.cuda.device(dev):
            self._check(self.lib.ddelm_evaluate_adjoint(self.ctx, nrhs, npts, x.data_ptr(), ub.data_ptr(), _ptr(gb),
                                                        cb.data_ptr()), "evaluate_adjoint")
        return cb
