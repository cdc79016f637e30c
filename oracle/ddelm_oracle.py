"""Plain FP64 CPU oracle for DDELM-NN (coarse space + Neumann-Neumann acceleration).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It shares no code with the HIP library.

Everything follows the paper (Lee & Ryoo, "A Neumann-Neumann Acceleration
with Coarse Space for Domain Decomposition of Extreme Learning Machines"):

  * local networks NN^i(x) = sum_j c_j tanh(w_j . x + b_j)      (sec. 2.2)
  * the DDELM block system [K B; A 0][c; mu] = [f; 0]            (eq. ddelm)
  * partition of the interface into corners Pi and the rest Delta,
    elimination of A_Pi, K~, B~, A~, f~, D~, d~                    (sec. 3, eq. coarse)
  * K~^+ applied through the coarse Schur complement S_Pi, assembled in
    full and Cholesky-factored; (K~^+)^T [phi; 0] by the paper's recipe
  * Neumann-Neumann map P = Abar Kbar^+ Bbar and the theta-mixed normal
    equation (eq. nn-mixed), solved by CG on mu_Delta           (sec. 3.1)
  * change of variables T^i (fig. change) and mean-flux rows A_m  (sec. 3.2)
  * optionally the variable-coefficient operator -div(rho grad u)
    (sec. 4.3): interior rows rho (-Laplace phi) - grad rho . grad phi,
    flux rows the conormal derivative rho dphi/dn

Readings where the paper is silent (all listed in the design notes):
  - hidden weights act on local coordinates xi = (x - centre)/(h/2);
  - interior collocation points are given; edges carry p points including
    both ends; edge ends on the domain boundary are boundary points;
  - Pi = subdomain corners not on the domain boundary; Delta = the other
    interface points; global orders as in `Geometry2D`;
  - T on an edge with one end on the boundary is the hat from the Pi end;
  - an A_m corner row is the sum, over this subdomain's interface edges
    meeting the corner, of the edge-mean flux excluding the opposite end;
  - Kbar and Abar use point values (no T, no A_m), Abar is summed;
  - CG stops on the recurrence residual ||r_k|| <= tol ||b||, from mu=0;
  - with a coefficient rho, the flux continuity and Neumann rows use the
    conormal derivative rho dphi/dn (rho is continuous, so this is the same
    interface condition as dphi/dn, with rows scaled by rho).

Precision: float64 throughout.  Library primitives used as steps: numpy QR
(LAPACK Householder), scipy Cholesky and triangular solves, pinv/lstsq in
the dense reference.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg as sla

SIDES = ("bottom", "right", "top", "left")
NORMAL = {"bottom": (0.0, -1.0), "right": (1.0, 0.0), "top": (0.0, 1.0), "left": (-1.0, 0.0)}


# ============================================================== geometry

@dataclasses.dataclass
class Sub:
    """Point sets and row layout of one subdomain."""
    ix: int
    iy: int
    center: np.ndarray
    half: np.ndarray                 # half widths (h/2 per axis)
    x_I: np.ndarray                  # (n_I, 2)
    x_B: np.ndarray                  # (n_B, 2)
    pi_glob: List[int]               # global Pi indices of the local Pi points (sorted)
    dl_glob: List[int]               # global Delta indices of the local Delta points (sorted)
    x_G: np.ndarray                  # (n_G, 2), local Gamma order = Pi block then Delta block
    T: np.ndarray                    # (n_G, n_G) transition W' -> W (identity without change of vars)
    # flux description per local Gamma row: list of (weight, point, normal) terms
    flux_terms: list
    # Delta rows of Kbar: point flux; normal per Delta point
    dl_normal: np.ndarray            # (n_D, 2)

    @property
    def n_I(self):
        return len(self.x_I)

    @property
    def n_B(self):
        return len(self.x_B)

    @property
    def n_P(self):
        return len(self.pi_glob)

    @property
    def n_D(self):
        return len(self.dl_glob)

    @property
    def n_G(self):
        return self.n_P + self.n_D

    @property
    def m(self):
        return self.n_I + self.n_B + self.n_G


class Geometry2D:
    """Uniform nx x ny partition of a box, with the paper's interface split.

    Subdomain i = iy*nx + ix.  Lattice vertices (jx, jy), 0<=jx<=nx, 0<=jy<=ny.
    Interior edges: vertical edge on line x_jx between rows iy, iy+1 has index
    iy*(nx-1) + (jx-1) (1<=jx<=nx-1); horizontal edge on line y_jy between
    columns ix, ix+1 has index (nx-1)*ny + (jy-1)*nx + ix (1<=jy<=ny-1).
    Pi: interior vertices, index (jy-1)*(nx-1) + (jx-1).
    Delta: edge-interior points, index edge*(p-2) + (k-1), k = 1..p-2 along
    increasing coordinate; with coarse == 0 the interior vertices are Delta
    points too, numbered after all edge points in the Pi order.

    coarse: 0 = no coarse space (vanilla DDELM), K and plain A;
            1 = corners as Pi, K and plain A;
            2 = corners as Pi, K_c and A_m (the paper's default);
            3 = corners as Pi, K_c and plain A;
            4 = corners as Pi, K and A_m
    (3 and 4 are the remaining cells of the ablation of sec. 4.2, table chov).
    """

    def __init__(self, nx, ny, s_edge, s_extra, x_int, lo=(0.0, 0.0), hi=(1.0, 1.0), coarse=2):
        self.nx, self.ny = nx, ny
        self.lo = np.asarray(lo, float)
        self.hi = np.asarray(hi, float)
        self.h = (self.hi - self.lo) / np.array([nx, ny], float)
        self.s = np.asarray(s_edge, float)
        self.s_extra = np.asarray(s_extra, float)
        self.p = len(self.s)
        self.coarse = coarse
        p = self.p
        n_vert_edges = (nx - 1) * ny
        n_horiz_edges = (ny - 1) * nx
        self.n_edges = n_vert_edges + n_horiz_edges
        self.n_pi = (nx - 1) * (ny - 1) if coarse > 0 else 0
        n_cross = (nx - 1) * (ny - 1)
        self.n_dl = self.n_edges * (p - 2) + (n_cross if coarse == 0 else 0)
        self.subs: List[Sub] = []
        for iy in range(ny):
            for ix in range(nx):
                self.subs.append(self._build_sub(ix, iy, np.asarray(x_int[iy * nx + ix], float)))

    # -- lattice helpers
    def vertex_xy(self, jx, jy):
        return np.array([self.lo[0] + jx * self.h[0], self.lo[1] + jy * self.h[1]])

    def vertex_on_boundary(self, jx, jy):
        return jx == 0 or jx == self.nx or jy == 0 or jy == self.ny

    def cross_index(self, jx, jy):
        return (jy - 1) * (self.nx - 1) + (jx - 1)

    def side_info(self, ix, iy, side):
        """(on_boundary, v0, v1, edge_index_or_None, coord(s)) of one side.

        v0 is the end at s=0 (smaller coordinate), v1 the end at s=1."""
        nx, ny = self.nx, self.ny
        if side == "bottom":
            on, v0, v1 = iy == 0, (ix, iy), (ix + 1, iy)
            e = None if on else (nx - 1) * ny + (iy - 1) * nx + ix
            f = lambda s: np.array([self.lo[0] + (ix + s) * self.h[0], self.lo[1] + iy * self.h[1]])
        elif side == "top":
            on, v0, v1 = iy + 1 == ny, (ix, iy + 1), (ix + 1, iy + 1)
            e = None if on else (nx - 1) * ny + iy * nx + ix
            f = lambda s: np.array([self.lo[0] + (ix + s) * self.h[0], self.lo[1] + (iy + 1) * self.h[1]])
        elif side == "left":
            on, v0, v1 = ix == 0, (ix, iy), (ix, iy + 1)
            e = None if on else iy * (nx - 1) + (ix - 1)
            f = lambda s: np.array([self.lo[0] + ix * self.h[0], self.lo[1] + (iy + s) * self.h[1]])
        else:  # right
            on, v0, v1 = ix + 1 == nx, (ix + 1, iy), (ix + 1, iy + 1)
            e = None if on else iy * (nx - 1) + ix
            f = lambda s: np.array([self.lo[0] + (ix + 1) * self.h[0], self.lo[1] + (iy + s) * self.h[1]])
        return on, v0, v1, e, f

    def _build_sub(self, ix, iy, x_I):
        p, s = self.p, self.s
        center = np.array([self.lo[0] + (ix + 0.5) * self.h[0], self.lo[1] + (iy + 0.5) * self.h[1]])
        half = 0.5 * self.h
        # ---- boundary points (canonical order: sides bottom,right,top,left on the
        # domain boundary, each by increasing s, skipping repeats; then extras)
        xb, keys = [], set()
        for side in SIDES:
            on, v0, v1, e, f = self.side_info(ix, iy, side)
            if not on:
                continue
            for k in range(p):
                if k == 0:
                    key = ("v",) + v0
                elif k == p - 1:
                    key = ("v",) + v1
                else:
                    key = ("b", side, k)
                if key in keys:
                    continue
                keys.add(key)
                xb.append(f(s[k]))
        for side in SIDES:
            on, v0, v1, e, f = self.side_info(ix, iy, side)
            if on:
                for se in self.s_extra:
                    xb.append(f(se))
        x_B = np.array(xb).reshape(-1, 2)
        # ---- interface points
        corners = [(ix, iy), (ix + 1, iy), (ix, iy + 1), (ix + 1, iy + 1)]
        inner_corners = [c for c in corners if not self.vertex_on_boundary(*c)]
        pis, dls = [], []   # (global index, xy, info)
        if self.coarse > 0:
            for c in inner_corners:
                pis.append((self.cross_index(*c), self.vertex_xy(*c), c))
        else:
            base = self.n_edges * (p - 2)
            for c in inner_corners:
                dls.append((base + self.cross_index(*c), self.vertex_xy(*c), ("v", c)))
        iface_sides = []
        for side in SIDES:
            on, v0, v1, e, f = self.side_info(ix, iy, side)
            if on:
                continue
            iface_sides.append((side, v0, v1, e, f))
            for k in range(1, p - 1):
                dls.append((e * (p - 2) + (k - 1), f(s[k]), ("e", side, k)))
        pis.sort(key=lambda t: t[0])
        dls.sort(key=lambda t: t[0])
        x_G = np.array([t[1] for t in pis] + [t[1] for t in dls]).reshape(-1, 2)
        nP, nD = len(pis), len(dls)
        nG = nP + nD
        pos_pi = {t[2]: a for a, t in enumerate(pis)}             # vertex -> local row
        # ---- transition matrix T^i (fig. change): columns are the W' basis,
        # rows point values.  A corner's W' function is the hat that is 1 at the
        # corner and falls linearly (in s) to 0 at the other end of each of this
        # subdomain's interface edges through that corner.
        T = np.eye(nG)
        if self.coarse in (2, 3):
            for a, t in enumerate(dls):
                info = t[2]
                if info[0] != "e":
                    continue
                side, k = info[1], info[2]
                _, v0, v1, _, _ = self.side_info(ix, iy, side)
                row = nP + a
                if v0 in pos_pi:
                    T[row, pos_pi[v0]] = 1.0 - s[k]
                if v1 in pos_pi:
                    T[row, pos_pi[v1]] = s[k]
        # ---- flux rows: list of (weight, xy, normal) terms per local Gamma row
        flux_terms = []
        for a, t in enumerate(pis):
            c = t[2]
            terms = []
            incident = [sd for sd in iface_sides if sd[1] == c or sd[2] == c]
            if self.coarse in (2, 4):
                # mean flux over each incident edge, excluding the opposite end
                for side, v0, v1, e, f in incident:
                    n = np.array(NORMAL[side])
                    ks = range(0, p - 1) if v0 == c else range(1, p)
                    for k in ks:
                        terms.append((1.0 / (p - 1), f(s[k]), n))
            else:
                n = sum(np.array(NORMAL[sd[0]]) for sd in incident)
                terms.append((1.0, t[1], n))
            flux_terms.append(terms)
        dl_normal = np.zeros((nD, 2))
        for a, t in enumerate(dls):
            info = t[2]
            if info[0] == "e":
                n = np.array(NORMAL[info[1]])
            else:
                c = info[1]
                incident = [sd for sd in iface_sides if sd[1] == c or sd[2] == c]
                n = sum(np.array(NORMAL[sd[0]]) for sd in incident)
            dl_normal[a] = n
            flux_terms.append([(1.0, t[1], n)])
        return Sub(ix, iy, center, half, x_I, x_B, [t[0] for t in pis], [t[0] for t in dls],
                   x_G, T, flux_terms, dl_normal)

    # -- global point lists (for tests of the indexing)
    def pi_points(self):
        out = np.zeros((self.n_pi, 2))
        for sb in self.subs:
            for a, g in enumerate(sb.pi_glob):
                out[g] = sb.x_G[a]
        return out

    def delta_points(self):
        out = np.zeros((self.n_dl, 2))
        for sb in self.subs:
            for a, g in enumerate(sb.dl_glob):
                out[g] = sb.x_G[sb.n_P + a]
        return out


# ============================================================== features (sec. 2.2)

def tanh_features(W, b, half, center, x):
    """phi_j(x), grad phi_j(x) and -Laplace phi_j(x) at points x (n, 2).

    phi_j = tanh(w_j . xi + b_j), xi = (x - center)/half.  With t = tanh(z):
      d phi/dx_k = w_jk (1 - t^2) / half_k
      d2 phi/dx_k^2 = -2 t (1 - t^2) w_jk^2 / half_k^2
    """
    xi = (x - center) / half                       # (n, 2)
    z = xi @ W.T + b                               # (n, M)
    t = np.tanh(z)
    dt = 1.0 - t * t
    grad = dt[:, :, None] * (W / half)[None, :, :]  # (n, M, 2)
    lap = -2.0 * t * dt * ((W / half) ** 2).sum(axis=1)[None, :]
    return t, grad, -lap


def local_matrices(geo: Geometry2D, i: int, W: np.ndarray, b: np.ndarray, rho=None):
    """K^i (or K_c^i), A^i (or A_m^i) rows at local Gamma, Kbar^i and Abar^i.

    rho: None for the Poisson operator -Laplace u, else a callable
    x (n, 2) -> (rho(x) (n,), grad rho(x) (n, 2)) for -div(rho grad u)
    (sec. 4.3, variable-coefficient Poisson).  Then an interior row is
    -div(rho grad phi) = rho (-Laplace phi) - grad rho . grad phi, and every
    flux row (the A / A_m rows and the Delta rows of Kbar) takes the conormal
    derivative rho dphi/dn at each of its points; value rows do not change.
    """
    sb = geo.subs[i]
    phi_I, grad_I, Lphi_I = tanh_features(W, b, sb.half, sb.center, sb.x_I)
    phi_B, _, _ = tanh_features(W, b, sb.half, sb.center, sb.x_B)
    phi_G, grad_G, _ = tanh_features(W, b, sb.half, sb.center, sb.x_G)
    if rho is not None:
        r_I, dr_I = rho(sb.x_I)
        Lphi_I = r_I[:, None] * Lphi_I - np.einsum("nmk,nk->nm", grad_I, dr_I)
    # K_c: Gamma rows are (T^i)^{-1} C phi(x_Gamma)  (sec. 3.2)
    CG = np.linalg.inv(sb.T) @ phi_G
    K = np.vstack([Lphi_I, phi_B, CG])
    # flux rows
    A = np.zeros((sb.n_G, W.shape[0]))
    for r, terms in enumerate(sb.flux_terms):
        for wgt, xy, n in terms:
            _, g, _ = tanh_features(W, b, sb.half, sb.center, xy[None, :])
            scale = 1.0 if rho is None else rho(xy[None, :])[0][0]
            A[r] += wgt * scale * (g[0] @ n)
    # Kbar: Dirichlet at Pi, point flux at Delta (sec. 3.1); Abar: trace at Delta
    nP = sb.n_P
    flux_D = np.einsum("nmk,nk->nm", grad_G[nP:], sb.dl_normal)
    if rho is not None:
        flux_D = rho(sb.x_G[nP:])[0][:, None] * flux_D
    Kbar = np.vstack([Lphi_I, phi_B, phi_G[:nP], flux_D])
    Abar = phi_G[nP:]
    return K, A, Kbar, Abar


# ============================================================== the solver

class LocalLS:
    """Thin Householder QR of a local matrix; K^+ y and (K^+)^T z."""

    def __init__(self, K):
        self.Q, self.R = np.linalg.qr(K, mode="reduced")

    def solve(self, y):          # K^+ y
        return sla.solve_triangular(self.R, self.Q.T @ y, lower=False)

    def solve_T(self, z):        # (K^+)^T z
        return self.Q @ sla.solve_triangular(self.R, z, lower=False, trans="T")


class DDELMNN:
    """DDELM with coarse space and theta-mixed Neumann-Neumann acceleration.

    Vectors over the local row spaces are lists (one array per subdomain);
    interface vectors are global arrays over Pi or Delta.
    """

    def __init__(self, geo: Geometry2D, W, b, theta=0.999, rho=None):
        self.geo = geo
        self.theta = float(theta)
        self.N = len(geo.subs)
        self.K, self.A, self.Kb, self.Ab = [], [], [], []
        for i in range(self.N):
            K, A, Kb, Ab = local_matrices(geo, i, W[i], b[i], rho=rho)
            self.K.append(K); self.A.append(A); self.Kb.append(Kb); self.Ab.append(Ab)
        self.ls = [LocalLS(K) for K in self.K]
        self.lsb = [LocalLS(Kb) for Kb in self.Kb] if self.theta != 0.0 else None
        self.nP, self.nD = geo.n_pi, geo.n_dl
        self._build_coarse()

    # ---------------- block operators of the DDELM system (eq. ddelm)
    def _gamma_rows(self, i):
        sb = self.geo.subs[i]
        g0 = sb.n_I + sb.n_B
        return g0, g0 + sb.n_P, g0 + sb.n_G        # start of Pi rows, Delta rows, end

    def B_Pi(self, mu_pi):           # B^i = [0; 0; -R^i]: Pi part
        out = []
        for i, sb in enumerate(self.geo.subs):
            y = np.zeros(sb.m)
            p0, d0, e = self._gamma_rows(i)
            y[p0:d0] = -mu_pi[sb.pi_glob]
            out.append(y)
        return out

    def B_Dl(self, mu_dl):
        out = []
        for i, sb in enumerate(self.geo.subs):
            y = np.zeros(sb.m)
            p0, d0, e = self._gamma_rows(i)
            y[d0:e] = -mu_dl[sb.dl_glob]
            out.append(y)
        return out

    def B_Pi_T(self, ys):
        out = np.zeros(self.nP)
        for i, sb in enumerate(self.geo.subs):
            p0, d0, e = self._gamma_rows(i)
            np.add.at(out, sb.pi_glob, -ys[i][p0:d0])
        return out

    def B_Dl_T(self, ys):
        out = np.zeros(self.nD)
        for i, sb in enumerate(self.geo.subs):
            p0, d0, e = self._gamma_rows(i)
            np.add.at(out, sb.dl_glob, -ys[i][d0:e])
        return out

    def A_Pi(self, cs):              # A = [A^1 ... A^N], rows at Pi
        out = np.zeros(self.nP)
        for i, sb in enumerate(self.geo.subs):
            np.add.at(out, sb.pi_glob, self.A[i][:sb.n_P] @ cs[i])
        return out

    def A_Dl(self, cs):
        out = np.zeros(self.nD)
        for i, sb in enumerate(self.geo.subs):
            np.add.at(out, sb.dl_glob, self.A[i][sb.n_P:] @ cs[i])
        return out

    def A_Pi_T(self, y):
        return [self.A[i][:sb.n_P].T @ y[sb.pi_glob] for i, sb in enumerate(self.geo.subs)]

    def A_Dl_T(self, y):
        return [self.A[i][sb.n_P:].T @ y[sb.dl_glob] for i, sb in enumerate(self.geo.subs)]

    def Kmul(self, cs):
        return [self.K[i] @ cs[i] for i in range(self.N)]

    def Kplus(self, ys):
        return [self.ls[i].solve(ys[i]) for i in range(self.N)]

    def KplusT(self, zs):
        return [self.ls[i].solve_T(zs[i]) for i in range(self.N)]

    @staticmethod
    def _add(xs, ys, a=1.0):
        return [x + a * y for x, y in zip(xs, ys)]

    # ---------------- D_{alpha beta} = -A_alpha K^+ B_beta  (sec. 3)
    def D_PiPi(self, mu_pi):
        return -self.A_Pi(self.Kplus(self.B_Pi(mu_pi)))

    def D_PiPi_T(self, y):
        return -self.B_Pi_T(self.KplusT(self.A_Pi_T(y)))

    def D_PiDl(self, mu_dl):
        return -self.A_Pi(self.Kplus(self.B_Dl(mu_dl)))

    def D_PiDl_T(self, y):
        return -self.B_Dl_T(self.KplusT(self.A_Pi_T(y)))

    # ---------------- coarse Schur complement S_Pi, assembled in full + Cholesky
    def S_Pi_apply(self, mu_pi):
        Bm = self.B_Pi(mu_pi)
        KKB = self.Kmul(self.Kplus(Bm))
        return (self.B_Pi_T(Bm) + self.D_PiPi_T(self.D_PiPi(mu_pi)) - self.B_Pi_T(KKB))

    def _build_coarse(self):
        n = self.nP
        S = np.zeros((n, n))
        for k in range(n):
            e = np.zeros(n); e[k] = 1.0
            S[:, k] = self.S_Pi_apply(e)
        self.S_Pi = S
        self.S_Pi_chol = sla.cho_factor(S, lower=True) if n > 0 else None

    def S_Pi_solve(self, r):
        if self.nP == 0:
            return np.zeros(0)
        return sla.cho_solve(self.S_Pi_chol, r)

    # ---------------- K~ and its pseudo-inverse
    def Kt_mul(self, cs, mu_pi):
        top = self._add(self.Kmul(cs), self.B_Pi(mu_pi))
        return top, self.D_PiPi(mu_pi)

    def Kt_plus(self, phi, psi):
        """[c; mu_Pi] = K~^+ [phi; psi] through S_Pi."""
        KKphi = self.Kmul(self.Kplus(phi))
        rhs = self.B_Pi_T(phi) - self.B_Pi_T(KKphi) + self.D_PiPi_T(psi)
        mu_pi = self.S_Pi_solve(rhs)
        cs = self.Kplus(self._add(phi, self.B_Pi(mu_pi), -1.0))
        return cs, mu_pi

    def Kt_plus_T(self, phi, psi=None):
        """(K~^+)^T [phi; psi] (phi over the c blocks, psi over Pi).

        With psi = 0 this is the paper's recipe; a nonzero psi only adds to
        the right-hand side of the coarse solve, since K~^+ reaches mu_Pi
        through S_Pi^{-1} alone (transpose of `Kt_plus`)."""
        KpTphi = self.KplusT(phi)
        r = -self.B_Pi_T(KpTphi)
        if psi is not None:
            r = r + psi
        nu = self.S_Pi_solve(r)
        Bnu = self.B_Pi(nu)
        KKBnu = self.Kmul(self.Kplus(Bnu))
        top = [KpTphi[i] - KKBnu[i] + Bnu[i] for i in range(self.N)]
        return top, self.D_PiPi(nu)

    # ---------------- B~, A~, D~
    def Bt(self, mu_dl):
        return self.B_Dl(mu_dl), self.D_PiDl(mu_dl)

    def Bt_T(self, top, bot):
        return self.B_Dl_T(top) + self.D_PiDl_T(bot)

    def Dt(self, mu_dl):             # D~ = -A~ K~^+ B~
        cs, _ = self.Kt_plus(*self.Bt(mu_dl))
        return -self.A_Dl(cs)

    def Dt_T(self, y):               # D~^T = -B~^T (K~^+)^T A~^T
        top, bot = self.Kt_plus_T(self.A_Dl_T(y))
        return -self.Bt_T(top, bot)

    # ---------------- Neumann-Neumann map P = Abar Kbar^+ Bbar
    def _Bbar(self, lam):
        out = []
        for i, sb in enumerate(self.geo.subs):
            y = np.zeros(sb.m)
            y[sb.m - sb.n_D:] = -lam[sb.dl_glob]
            out.append(y)
        return out

    def _Bbar_T(self, ys):
        out = np.zeros(self.nD)
        for i, sb in enumerate(self.geo.subs):
            np.add.at(out, sb.dl_glob, -ys[i][sb.m - sb.n_D:])
        return out

    def P(self, lam):
        cb = [self.lsb[i].solve(y) for i, y in enumerate(self._Bbar(lam))]
        out = np.zeros(self.nD)
        for i, sb in enumerate(self.geo.subs):
            np.add.at(out, sb.dl_glob, self.Ab[i] @ cb[i])
        return out

    def P_T(self, y):
        zs = [self.Ab[i].T @ y[sb.dl_glob] for i, sb in enumerate(self.geo.subs)]
        return self._Bbar_T([self.lsb[i].solve_T(z) for i, z in enumerate(zs)])

    def Mtheta(self, lam):
        if self.theta == 0.0:
            return lam.copy()
        return self.theta * self.P_T(self.P(lam)) + (1.0 - self.theta) * lam

    # ---------------- eq. nn-mixed
    def S_theta(self, v):
        top, bot = self.Bt(v)
        BtBt = self.Bt_T(top, bot)
        cs, mu_pi = self.Kt_plus(top, bot)
        ktop, kbot = self.Kt_mul(cs, mu_pi)
        BtKK = self.Bt_T(ktop, kbot)
        return BtBt + self.Dt_T(self.Mtheta(self.Dt(v))) - BtKK

    def rhs(self, f, h=None):
        """Right-hand side of eq. nn-mixed for local RHS f (list) and an optional
        flux right-hand side h = (h_Pi, h_Delta) of the second block row."""
        hP = np.zeros(self.nP) if h is None else h[0]
        hD = np.zeros(self.nD) if h is None else h[1]
        Kpf = self.Kplus(f)
        d_pi = hP - self.A_Pi(Kpf)                       # d_Pi = h_Pi - A_Pi K^+ f
        cs, mu_pi = self.Kt_plus(f, d_pi)                # K~^+ f~
        d_t = hD - self.A_Dl(cs)                         # d~ = h_Delta - A~ K~^+ f~
        ktop, kbot = self.Kt_mul(cs, mu_pi)
        b = (self.Bt_T(f, d_pi) - self.Bt_T(ktop, kbot)
             + self.Dt_T(self.Mtheta(d_t)))
        return b, d_pi

    def recover(self, f, d_pi, mu_dl):
        """[c; mu_Pi] = K~^+ (f~ - B~ mu_Delta)  (eq. coarse_sol_2)."""
        top, bot = self.Bt(mu_dl)
        return self.Kt_plus(self._add(f, top, -1.0), d_pi - bot)

    def solve_direct(self, f, h=None):
        """Same result with S_theta assembled column by column and a dense
        Cholesky solve in place of CG (small problems only)."""
        b, d_pi = self.rhs(f, h)
        if self.nD:
            S = assemble_S_theta(self)
            mu_dl = sla.cho_solve(sla.cho_factor(0.5 * (S + S.T), lower=True), b)
        else:
            mu_dl = np.zeros(0)
        cs, mu_pi = self.recover(f, d_pi, mu_dl)
        return dict(c=cs, mu_pi=mu_pi, mu_dl=mu_dl, iters=0, relres=0.0, b=b)

    def solve(self, f, h=None, tol=1e-10, maxit=10000, x0=None):
        b, d_pi = self.rhs(f, h)
        info = {}
        mu_dl, it, relres = cg(self.S_theta, b, tol, maxit, x0, info=info)
        cs, mu_pi = self.recover(f, d_pi, mu_dl)
        return dict(c=cs, mu_pi=mu_pi, mu_dl=mu_dl, iters=it, relres=relres, b=b, kappa=info.get("kappa", 1.0))

    # ---------------- adjoint (transpose) of solve, derived from its equations
    def adjoint(self, cbar, mubar_pi=None, mubar_dl=None, tol=1e-12, maxit=10000, direct=False):
        """Transpose of the linear map (f, h) -> (c, mu_Pi, mu_Delta) of `solve`.

        The forward map, in the notation of sec. 3:
          f~ = [f; d_Pi],  d_Pi = h_Pi - A_Pi K^+ f,
          b  = B~^T (I - K~ K~^+) f~ + D~^T M (h_Delta - A~ K~^+ f~),
               M = theta P^T P + (1 - theta) I             (eq. nn-mixed)
          mu_Delta = S_theta^{-1} b,
          [c; mu_Pi] = K~^+ (f~ - B~ mu_Delta)             (eq. coarse_sol_2).
        K~ K~^+, S_theta and M are symmetric, so the transpose is
          g = (K~^+)^T [cbar; mubar_Pi],
          bbar = S_theta^{-1} (mubar_Delta - B~^T g),
          fbar~ = g + (I - K~ K~^+) B~ bbar - (K~^+)^T A~^T M D~ bbar,
          hbar_Delta = M D~ bbar,  hbar_Pi = fbar~ (Pi part),
          fbar = fbar~ (c part) - (K^+)^T A_Pi^T hbar_Pi.
        Returns (fbar as a list over subdomains, (hbar_Pi, hbar_Delta), CG iterations).
        direct=True solves with the assembled S_theta (small problems)."""
        nP, nD = self.nP, self.nD
        mP = np.zeros(nP) if mubar_pi is None else np.asarray(mubar_pi, float)
        mD = np.zeros(nD) if mubar_dl is None else np.asarray(mubar_dl, float)
        gtop, gbot = self.Kt_plus_T(cbar, mP)
        rhs = mD - self.Bt_T(gtop, gbot)
        it = 0
        if nD == 0:
            bbar = np.zeros(0)
        elif direct:
            S = assemble_S_theta(self)
            bbar = sla.cho_solve(sla.cho_factor(0.5 * (S + S.T), lower=True), rhs)
        else:
            bbar, it, _ = cg(self.S_theta, rhs, tol, maxit)
        top, bot = self.Bt(bbar)
        cs, mp = self.Kt_plus(top, bot)
        ktop, kbot = self.Kt_mul(cs, mp)
        q = self.Mtheta(self.Dt(bbar))
        ttop, tbot = self.Kt_plus_T(self.A_Dl_T(q))
        ft_top = [gtop[i] + top[i] - ktop[i] - ttop[i] for i in range(self.N)]
        ft_bot = gbot + bot - kbot - tbot
        corr = self.KplusT(self.A_Pi_T(ft_bot))
        fbar = [ft_top[i] - corr[i] for i in range(self.N)]
        return fbar, (ft_bot, q), it


def cg(apply, b, tol, maxit, x0=None, info=None):
    """Plain conjugate gradients; stops when ||r_k|| <= tol ||b||.

    If `info` is a dict, info["kappa"] receives the condition-number estimate
    of the operator from the CG coefficients: CG is the Lanczos process, whose
    tridiagonal matrix T (T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_{j,j+1} = sqrt(beta_j)/alpha_j) has Ritz values inside the spectrum that
    approach its ends; kappa = largest / smallest Ritz value."""
    n = len(b)
    x = np.zeros(n) if x0 is None else x0.copy()
    if n == 0:
        return x, 0, 0.0
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0
    r = b - apply(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = r @ r
    it = 0
    alphas, betas = [], []
    while np.sqrt(rr) > tol * bn and it < maxit:
        w = apply(p)
        alpha = rr / (p @ w)
        x += alpha * p
        r -= alpha * w
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        alphas.append(alpha)
        betas.append(rr_new / rr)
        rr = rr_new
        it += 1
    if info is not None and alphas:
        k = len(alphas)
        d = np.array([1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0) for j in range(k)])
        e = np.array([np.sqrt(betas[j]) / alphas[j] for j in range(k - 1)])
        ritz = sla.eigvalsh_tridiagonal(d, e)
        info["kappa"] = float(ritz[-1] / ritz[0])
    return x, it, np.sqrt(rr) / bn


# ============================================================== problem-level helpers

def local_rhs(geo: Geometry2D, f_fn, g_fn):
    """f^i = [f(x_I); g(x_B); 0] for each subdomain."""
    out = []
    for sb in geo.subs:
        out.append(np.concatenate([f_fn(sb.x_I), g_fn(sb.x_B), np.zeros(sb.n_G)]))
    return out


def local_rhs_from_values(geo: Geometry2D, f_I: Sequence[np.ndarray], g_B: Sequence[np.ndarray]):
    return [np.concatenate([f_I[i], g_B[i], np.zeros(sb.n_G)]) for i, sb in enumerate(geo.subs)]


def owner_of(geo: Geometry2D, x):
    """Lowest-index subdomain whose closed box contains each point."""
    rel = (np.asarray(x) - geo.lo) / geo.h
    ix = np.clip(np.ceil(rel[:, 0]) - 1, 0, geo.nx - 1).astype(int)
    iy = np.clip(np.ceil(rel[:, 1]) - 1, 0, geo.ny - 1).astype(int)
    return iy * geo.nx + ix


def evaluate(geo: Geometry2D, W, b, cs, x, grad=False):
    """u(x) = NN^i(x) on the owning subdomain (and optionally grad u)."""
    x = np.asarray(x, float)
    own = owner_of(geo, x)
    u = np.zeros(len(x))
    g = np.zeros((len(x), 2))
    for i in np.unique(own):
        sel = own == i
        sb = geo.subs[i]
        t, gr, _ = tanh_features(W[i], b[i], sb.half, sb.center, x[sel])
        u[sel] = t @ cs[i]
        g[sel] = np.einsum("nmk,m->nk", gr, cs[i])
    return (u, g) if grad else u


def evaluate_adjoint(geo: Geometry2D, W, b, x, ubar, gbar=None):
    """Transpose of `evaluate` in the coefficients: for each subdomain i,
    cbar_i = Phi_i(x_own)^T ubar_own (+ the gradient features against gbar)."""
    x = np.asarray(x, float)
    own = owner_of(geo, x)
    out = []
    for i, sb in enumerate(geo.subs):
        sel = own == i
        t, gr, _ = tanh_features(W[i], b[i], sb.half, sb.center, x[sel])
        cb = t.T @ ubar[sel]
        if gbar is not None:
            cb = cb + np.einsum("nmk,nk->m", gr, gbar[sel])
        out.append(cb)
    return out


def rel_errors(u_ref, u, g_ref=None, g=None):
    l2 = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    if g_ref is None:
        return l2
    num = np.sqrt(np.sum((u - u_ref) ** 2) + np.sum((g - g_ref) ** 2))
    den = np.sqrt(np.sum(u_ref ** 2) + np.sum(g_ref ** 2))
    return l2, num / den


# ============================================================== dense reference (tiny inputs)

def dense_system(solver: DDELMNN):
    """Global matrices of eq. ddelm and of the Neumann-Neumann construction."""
    geo = solver.geo
    ms = [sb.m for sb in geo.subs]
    Ms = [solver.K[i].shape[1] for i in range(solver.N)]
    ro = np.concatenate([[0], np.cumsum(ms)])
    co = np.concatenate([[0], np.cumsum(Ms)])
    nP, nD = solver.nP, solver.nD
    K = sla.block_diag(*solver.K)
    Kb = sla.block_diag(*solver.Kb) if solver.lsb is not None else None
    BP = np.zeros((ro[-1], nP)); BD = np.zeros((ro[-1], nD))
    AP = np.zeros((nP, co[-1])); AD = np.zeros((nD, co[-1]))
    Bb = np.zeros((ro[-1], nD)); Ab = np.zeros((nD, co[-1]))
    for i, sb in enumerate(geo.subs):
        g0 = ro[i] + sb.n_I + sb.n_B
        for a, gidx in enumerate(sb.pi_glob):
            BP[g0 + a, gidx] = -1.0
            AP[gidx, co[i]:co[i + 1]] += solver.A[i][a]
        for a, gidx in enumerate(sb.dl_glob):
            BD[g0 + sb.n_P + a, gidx] = -1.0
            AD[gidx, co[i]:co[i + 1]] += solver.A[i][sb.n_P + a]
            Bb[ro[i] + sb.m - sb.n_D + a, gidx] = -1.0
            Ab[gidx, co[i]:co[i + 1]] += solver.Ab[i][a]
    return dict(K=K, BP=BP, BD=BD, AP=AP, AD=AD, Kb=Kb, Bb=Bb, Ab=Ab, ro=ro, co=co)


def dense_reference_solve(solver: DDELMNN, f: List[np.ndarray], h=None):
    """The DDELM-NN result by its definition, with pinv and one stacked lstsq.

    Eq. nn-mixed together with eq. coarse_sol_2 are the normal equations, and
    their Schur complement, of the weighted least-squares problem
        min || K~ [c; mu_Pi] + B~ mu_Delta - f~ ||^2
            + || M^{1/2} (D~ mu_Delta - d~) ||^2,   M = theta P^T P + (1-theta) I,
    so solving that problem directly gives the same (c, mu_Pi, mu_Delta).
    """
    S = dense_system(solver)
    K, BP, BD, AP, AD = S["K"], S["BP"], S["BD"], S["AP"], S["AD"]
    nP, nD = solver.nP, solver.nD
    fv = np.concatenate(f)
    hP = np.zeros(nP) if h is None else h[0]
    hD = np.zeros(nD) if h is None else h[1]
    Kp = np.linalg.pinv(K)
    DPP = -AP @ Kp @ BP
    DPD = -AP @ Kp @ BD
    dP = hP - AP @ Kp @ fv
    Kt = np.block([[K, BP], [np.zeros((nP, K.shape[1])), DPP]])
    Bt = np.vstack([BD, DPD])
    At = np.hstack([AD, np.zeros((nD, nP))])
    ft = np.concatenate([fv, dP])
    Ktp = np.linalg.pinv(Kt)
    Dt = -At @ Ktp @ Bt
    dt = hD - At @ Ktp @ ft
    th = solver.theta
    if th != 0.0:
        P = S["Ab"] @ np.linalg.pinv(S["Kb"]) @ S["Bb"]
        Mth = th * P.T @ P + (1.0 - th) * np.eye(nD)
    else:
        Mth = np.eye(nD)
    ev, V = np.linalg.eigh(0.5 * (Mth + Mth.T))
    Mh = (V * np.sqrt(np.clip(ev, 0.0, None))) @ V.T
    nx_ = Kt.shape[1]
    big = np.block([[Kt, Bt], [np.zeros((nD, nx_)), Mh @ Dt]])
    rhs = np.concatenate([ft, Mh @ dt])
    sol = np.linalg.lstsq(big, rhs, rcond=None)[0]
    xs, mu_dl = sol[:nx_], sol[nx_:]
    co = S["co"]
    cs = [xs[co[i]:co[i + 1]] for i in range(solver.N)]
    mu_pi = xs[co[-1]:]
    return dict(c=cs, mu_pi=mu_pi, mu_dl=mu_dl, S_theta_dense=Bt.T @ Bt + Dt.T @ Mth @ Dt
                - Bt.T @ Kt @ Ktp @ Bt)


def monolithic_solve(solver: DDELMNN, f: List[np.ndarray]):
    """Direct solve of the square coupled system [K B; A 0][c; mu] = [f; 0]."""
    S = dense_system(solver)
    K = S["K"]
    B = np.hstack([S["BP"], S["BD"]])
    A = np.vstack([S["AP"], S["AD"]])
    nG = B.shape[1]
    big = np.block([[K, B], [A, np.zeros((nG, nG))]])
    assert big.shape[0] == big.shape[1], "monolithic pin needs square local systems"
    rhs = np.concatenate([np.concatenate(f), np.zeros(nG)])
    sol = np.linalg.solve(big, rhs)
    co = S["co"]
    cs = [sol[co[i]:co[i + 1]] for i in range(solver.N)]
    return dict(c=cs, mu_pi=sol[co[-1]:co[-1] + solver.nP], mu_dl=sol[co[-1] + solver.nP:])


def assemble_S_theta(solver: DDELMNN):
    """S_theta column by column from the matrix-free operator."""
    n = solver.nD
    S = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n); e[k] = 1.0
        S[:, k] = solver.S_theta(e)
    return S
