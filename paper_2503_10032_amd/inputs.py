"""Seeded synthetic inputs for the DDELM-NN workloads.

This module only draws and describes inputs: hidden-layer parameters,
collocation point sets, edge parameterisations and the right-hand-side
functions f and g of the Poisson problems.  It holds none of the method's
arithmetic, so both the GPU library's tests and the CPU oracle can be fed
from it without sharing any solver code.

Workload shapes follow the paper's experiments (section 4: tanh hidden
layer, uniform training grid per subdomain, 2-D Poisson with a manufactured
solution or a random Fourier source as in the GRF equation).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    """One synthetic 2-D Poisson problem on a uniform grid of subdomains."""

    name: str
    nx: int
    ny: int
    M: int                  # neurons per subdomain
    a: float                # hidden weights and biases ~ U(-a, a)
    seed: int
    n_int: int              # interior collocation grid is n_int x n_int per subdomain
    p: int                  # points per interface/boundary edge, both ends included
    theta: float = 0.999
    tol: float = 1e-10
    nrhs: int = 1
    extra_boundary: bool = False   # boundary subdomains get edge midpoints as extra rows
    lo: tuple = (0.0, 0.0)
    hi: tuple = (1.0, 1.0)
    rhs: str = "sinsin"     # "sinsin" (manufactured), "fourier" or "one" (f = 1, g = 0)
    rhs_seed: int = 100
    rho: str = "one"        # coefficient of -div(rho grad u): "one" or "grf" (tanh(GRF) + 1.1)
    rho_alpha: float = 32.0
    rho_seed: int = 7

    @property
    def N(self) -> int:
        return self.nx * self.ny


def workload(name: str) -> Workload:
    """The named synthetic workloads.

    small    2x2 subdomains, M=64, U(-2,2), 16x16 interior, 16 per edge, tol 1e-10
    medium   8x8, M=256, U(-3,3), 32x32 interior, 32 per edge (FP64, one RHS)
    large    32x32, M=400, U(-2,2), 40x40 interior, 40 per edge, uneven
             boundary subdomains, 16 random Fourier right-hand sides
    adjoint  16x16, M=300, U(-2,2), 32x32 interior, 32 per edge
    varcoef  16x16, M=256, U(-2,2), 20x20 interior, 20 per edge: the
             variable-coefficient problem -div(rho grad u) = 1, u = 0 on the
             boundary, rho = tanh(GRF) + 1.1 with alpha = 32 (65,536 neurons
             in total and a 320 x 320 training grid, as in the paper's table)
    """
    if name == "small":
        return Workload("small", 2, 2, 64, 2.0, 0, 16, 16, tol=1e-10)
    if name == "medium":
        return Workload("medium", 8, 8, 256, 3.0, 1, 32, 32, tol=1e-8)
    if name == "large":
        return Workload("large", 32, 32, 400, 2.0, 2, 40, 40, tol=1e-8, nrhs=16,
                        extra_boundary=True, rhs="fourier", rhs_seed=100)
    if name == "adjoint":
        return Workload("adjoint", 16, 16, 300, 2.0, 4, 32, 32, tol=1e-10)
    if name == "varcoef":
        return Workload("varcoef", 16, 16, 256, 2.0, 3, 20, 20, tol=1e-8, rhs="one", rho="grf")
    raise KeyError(name)


def hidden_params(N: int, M: int, d: int, a: float, seed: int):
    """W ~ U(-a,a) of shape (N, M, d), then b ~ U(-a,a) of shape (N, M).

    The weights act on per-subdomain local coordinates in [-1, 1]^d.
    """
    rng = np.random.default_rng(seed)
    W = rng.uniform(-a, a, size=(N, M, d))
    b = rng.uniform(-a, a, size=(N, M))
    return np.ascontiguousarray(W), np.ascontiguousarray(b)


def paper_hidden_params(nx: int, ny: int, M: int, c: float, seed: int, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    """Hidden parameters drawn with the paper's initialisation (sec. 4.1, eq.
    init_be), returned in the local coordinates the library uses.

    Per subdomain Omega_i (a box of half widths (hx, hy) about its centre):
    r = diam(Omega_i)/2, B_r = the closed r-neighbourhood of Omega_i (so
    diam(B_r) = 2 diam(Omega_i)), l = c M^{1/d} / diam(B_r) with d = 2;
    w ~ U([-l, l]^2) acting on global coordinates, b = -w . xi with xi drawn
    uniformly from B_r (by rejection from its bounding box).  With
    x = centre + (hx, hy) * xi_loc the same neuron reads
    w . x + b = (w * (hx, hy)) . xi_loc + w . (centre - xi).
    Returns W (N, M, 2) and b (N, M) like hidden_params."""
    rng = np.random.default_rng(seed)
    N = nx * ny
    hx = (hi[0] - lo[0]) / nx
    hy = (hi[1] - lo[1]) / ny
    diam = math.hypot(hx, hy)
    r = 0.5 * diam
    ell = c * math.sqrt(M) / (2.0 * diam)
    W = np.empty((N, M, 2))
    b = np.empty((N, M))
    for iy in range(ny):
        for ix in range(nx):
            i = iy * nx + ix
            x0, y0 = lo[0] + ix * hx, lo[1] + iy * hy
            x1, y1 = x0 + hx, y0 + hy
            w = rng.uniform(-ell, ell, size=(M, 2))
            xi = np.empty((0, 2))
            while len(xi) < M:
                cand = rng.uniform((x0 - r, y0 - r), (x1 + r, y1 + r), size=(2 * M, 2))
                dx = np.maximum(np.maximum(x0 - cand[:, 0], cand[:, 0] - x1), 0.0)
                dy = np.maximum(np.maximum(y0 - cand[:, 1], cand[:, 1] - y1), 0.0)
                xi = np.concatenate([xi, cand[dx * dx + dy * dy <= r * r]])
            xi = xi[:M]
            centre = np.array([x0 + 0.5 * hx, y0 + 0.5 * hy])
            W[i] = w * np.array([0.5 * hx, 0.5 * hy])
            b[i] = np.einsum("mk,mk->m", w, centre - xi)
    return np.ascontiguousarray(W), np.ascontiguousarray(b)


def interior_points(w: Workload) -> np.ndarray:
    """Uniform strictly-interior grid, shape (N, n*n, 2), x fastest.

    Subdomain i = iy*nx + ix covers [ix*hx, (ix+1)*hx] x [iy*hy, (iy+1)*hy];
    its interior points sit at (k+1)/(n+1) of the cell width per axis.
    """
    n = w.n_int
    hx = (w.hi[0] - w.lo[0]) / w.nx
    hy = (w.hi[1] - w.lo[1]) / w.ny
    t = (np.arange(n) + 1.0) / (n + 1.0)
    out = np.empty((w.N, n * n, 2))
    for iy in range(w.ny):
        for ix in range(w.nx):
            X = w.lo[0] + (ix + t) * hx
            Y = w.lo[1] + (iy + t) * hy
            gx, gy = np.meshgrid(X, Y, indexing="xy")
            out[iy * w.nx + ix, :, 0] = gx.ravel()
            out[iy * w.nx + ix, :, 1] = gy.ravel()
    return out


def edge_params(p: int) -> np.ndarray:
    """Equispaced edge parameters s_k = k/(p-1), exactly 0 and 1 at the ends."""
    s = np.arange(p, dtype=np.float64) / (p - 1)
    s[0], s[-1] = 0.0, 1.0
    return s


def extra_boundary_params(w: Workload) -> np.ndarray:
    """Edge midpoints, used as extra boundary rows on sides lying on the boundary."""
    if not w.extra_boundary:
        return np.zeros(0)
    s = edge_params(w.p)
    return 0.5 * (s[:-1] + s[1:])


# ---------------------------------------------------------------- RHS functions

def sinsin_u(x: np.ndarray) -> np.ndarray:
    return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1])


def sinsin_f(x: np.ndarray) -> np.ndarray:
    """-Laplace of sin(pi x) sin(pi y)."""
    return 2.0 * np.pi ** 2 * sinsin_u(x)


def sinsin_grad(x: np.ndarray) -> np.ndarray:
    gx = np.pi * np.cos(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1])
    gy = np.pi * np.sin(np.pi * x[..., 0]) * np.cos(np.pi * x[..., 1])
    return np.stack([gx, gy], axis=-1)


def zero_g(x: np.ndarray) -> np.ndarray:
    return np.zeros(x.shape[:-1])


@dataclasses.dataclass
class FourierRHS:
    """f_r(x) = sum_k A[r,k] psi_k(x) with psi_k = sin or cos(2 pi k_j . x).

    32 modes: 16 integer wavevectors k_j in {-4..4}^2 \\ {0}, each as sin and
    cos; coefficients A ~ N(0, 1).  Shape of the random Fourier source of the
    GRF equation in the paper's Poisson experiment.
    """

    A: np.ndarray           # (nrhs, 32)
    kvec: np.ndarray        # (16, 2) integer wavevectors

    def basis(self, x: np.ndarray) -> np.ndarray:
        ph = 2.0 * np.pi * (x[..., None, 0] * self.kvec[:, 0] + x[..., None, 1] * self.kvec[:, 1])
        return np.concatenate([np.sin(ph), np.cos(ph)], axis=-1)   # (..., 32)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        return np.einsum("...k,rk->r...", self.basis(x), self.A)   # (nrhs, ...)


def fourier_rhs(nrhs: int, seed: int) -> FourierRHS:
    rng_k = np.random.default_rng(seed + 1)
    cand = np.array([(i, j) for i in range(-4, 5) for j in range(-4, 5) if (i, j) != (0, 0)])
    kvec = cand[rng_k.choice(len(cand), size=16, replace=False)].astype(np.float64)
    A = np.random.default_rng(seed).standard_normal((nrhs, 32))
    return FourierRHS(A=A, kvec=kvec)


@dataclasses.dataclass
class AdjointParams:
    """Source and boundary data parameterised by 64 + 32 coefficients.

    f = sum_{k1,k2=1..8} th[k1,k2] sin(k1 pi x) sin(k2 pi y);
    on side s (0 bottom, 1 right, 2 top, 3 left) g = sum_{j=1..8} eta[s,j] sin(j pi t)
    with t the coordinate running along that side.
    """

    theta: np.ndarray       # (64,)
    eta: np.ndarray         # (32,)

    @staticmethod
    def f_basis(x: np.ndarray) -> np.ndarray:
        k = np.arange(1, 9, dtype=np.float64)
        sx = np.sin(np.pi * x[..., 0, None] * k)
        sy = np.sin(np.pi * x[..., 1, None] * k)
        return (sx[..., :, None] * sy[..., None, :]).reshape(x.shape[:-1] + (64,))

    @staticmethod
    def g_basis(x: np.ndarray, tol: float = 1e-12) -> np.ndarray:
        """(..., 32) basis values; a point on two sides (a domain corner) gets
        both contributions, which vanish there anyway (sin(j pi t) at t=0,1)."""
        j = np.arange(1, 9, dtype=np.float64)
        out = np.zeros(x.shape[:-1] + (32,))
        on = [np.abs(x[..., 1]) < tol, np.abs(x[..., 0] - 1.0) < tol,
              np.abs(x[..., 1] - 1.0) < tol, np.abs(x[..., 0]) < tol]
        tcoord = [x[..., 0], x[..., 1], x[..., 0], x[..., 1]]
        for s in range(4):
            out[..., 8 * s:8 * s + 8] = np.where(on[s][..., None], np.sin(np.pi * tcoord[s][..., None] * j), 0.0)
        return out

    def f(self, x):
        return self.f_basis(x) @ self.theta

    def g(self, x):
        return self.g_basis(x) @ self.eta


def adjoint_params(seed: int = 5) -> AdjointParams:
    rng = np.random.default_rng(seed)
    return AdjointParams(theta=rng.standard_normal(64), eta=rng.standard_normal(32))


def observation_points(n: int = 10000, seed: int = 6) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, 2))


def eval_grid(w: Workload) -> np.ndarray:
    """Uniform global evaluation grid with 2*n_int*nx + 1 points per axis."""
    kx = 2 * w.n_int * w.nx + 1
    ky = 2 * w.n_int * w.ny + 1
    X = np.linspace(w.lo[0], w.hi[0], kx)
    Y = np.linspace(w.lo[1], w.hi[1], ky)
    gx, gy = np.meshgrid(X, Y, indexing="xy")
    return np.stack([gx.ravel(), gy.ravel()], axis=-1)


def rhs_functions(w: Workload):
    """(f, g) callables returning arrays of shape (nrhs, npts)."""
    if w.rhs == "one":
        return (lambda x: np.ones((w.nrhs,) + x.shape[:-1])), (lambda x: np.zeros((w.nrhs,) + x.shape[:-1]))
    if w.rhs == "sinsin":
        f1 = lambda x: sinsin_f(x)[None]
        g1 = lambda x: sinsin_u(x)[None]
        return f1, g1
    if w.rhs == "fourier":
        fr = fourier_rhs(w.nrhs, w.rhs_seed)
        return (lambda x: fr(x)), (lambda x: np.zeros((w.nrhs,) + x.shape[:-1]))
    raise KeyError(w.rhs)


# ---------------------------------------------------------------- coefficients

@dataclasses.dataclass
class GRF:
    """Approximate Gaussian random field grf(x) = sum_i a_i sin(w_i . x + b_i)
    with n terms, a_i ~ N(0, alpha^4/n), w_i ~ N(0, alpha^2 I), b_i ~ U(0, 2 pi)
    (eq. grf, n = 256); a larger alpha gives a more oscillatory field."""

    a: np.ndarray           # (n,)
    w: np.ndarray           # (n, 2)
    b: np.ndarray           # (n,)

    # Elementwise products and a sum along the last axis (no BLAS product),
    # so a point's value does not depend on which batch it is evaluated in.
    def _phase(self, x: np.ndarray) -> np.ndarray:
        return x[..., 0, None] * self.w[:, 0] + x[..., 1, None] * self.w[:, 1] + self.b

    def __call__(self, x: np.ndarray) -> np.ndarray:
        return (np.sin(self._phase(x)) * self.a).sum(axis=-1)

    def grad(self, x: np.ndarray) -> np.ndarray:
        c = np.cos(self._phase(x)) * self.a
        return np.stack([(c * self.w[:, 0]).sum(axis=-1), (c * self.w[:, 1]).sum(axis=-1)], axis=-1)


def grf(alpha: float, seed: int, n: int = 256) -> GRF:
    """Draws a, then w, then b from one generator seeded with `seed`."""
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, alpha * alpha / math.sqrt(n), size=n)
    w = rng.normal(0.0, alpha, size=(n, 2))
    b = rng.uniform(0.0, 2.0 * math.pi, size=n)
    return GRF(a=a, w=w, b=b)


@dataclasses.dataclass
class TanhGRFCoefficient:
    """rho(x) = tanh(grf(x)) + shift of the variable-coefficient Poisson
    problem (sec. 4.3, shift 1.1), so 0.1 < rho < 2.1 for shift 1.1.

    Called on points x (..., 2) it returns (rho(x), grad rho(x)) with shapes
    (...) and (..., 2)."""

    field: GRF
    shift: float = 1.1

    def __call__(self, x: np.ndarray):
        x = np.asarray(x, dtype=np.float64)
        flat = x.reshape(-1, 2)
        t = np.tanh(self.field(flat))
        g = (1.0 - t * t)[:, None] * self.field.grad(flat)
        return (t + self.shift).reshape(x.shape[:-1]), g.reshape(x.shape)


def coefficient(w: Workload):
    """The workload's coefficient as a callable x -> (rho, grad rho), or None
    for rho = 1."""
    if w.rho == "one":
        return None
    if w.rho == "grf":
        return TanhGRFCoefficient(grf(w.rho_alpha, w.rho_seed))
    raise KeyError(w.rho)
