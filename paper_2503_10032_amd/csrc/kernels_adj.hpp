// Adjoint (transposed) DDELM-NN solve and adjoint of the evaluation.
//
// The solve maps (f, h) -> (c, mu_Pi, mu_Delta) linearly.  In the local form
// used by the forward kernels it is the chain
//   al = (Q^T f)[:M],  cf0 = R^{-1} al,
//   rho = Q_G,P al - f_P,  s = Q_G,D al - f_D,  psi = -A_P cf0,  l = -A_D cf0 (+ h_D),
//   [mu1; e1] = X1 [sum rho; sum psi + h_P],  lam = l - L_DP mu1,
//   eta = M sum lam (M = theta P^T P + (1 - theta) I),
//   [nu; e'] = X1[:, :nP] sum L_DP^T eta,
//   b = sum (s + L_DD^T eta - G_DP (mu1 + nu) + L_PD^T (e1 + e')),
//   mu_Delta = S_theta^{-1} b,
//   mu_Pi = mu1 - (X1 [sum G_PD mu_Delta; sum L_PD mu_Delta])[:nP],
//   c = cf0 + E [mu_Pi; mu_Delta],   E = R^{-1} Q_G^T.
// The kernels below apply the transpose of each stage in reverse order.
// S_theta and M are symmetric, so the transposed solve is one more CG with
// the forward operator, and the M stage reuses the forward P kernels.
#pragma once
#include "tanh_fast.hpp"
#include "kernels_rhs.hpp"

namespace ddelm {

// yP / yD (Pi / Delta slots) = E_i^T cbar_i
template <typename T>
__global__ void k_adj_Et(int M, int N, const int* __restrict__ pi_off, const int* __restrict__ dl_off,
                         const QRDesc* __restrict__ desc, const T* __restrict__ qrA, const double* __restrict__ cbar,
                         int sumP, int sumD, double* __restrict__ yP, double* __restrict__ yD) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i], nd = dl_off[i + 1] - d0;
  extern __shared__ double cs[];
  for (int k = threadIdx.x; k < M; k += kBlock) cs[k] = cbar[((size_t)r * N + i) * M + k];
  __syncthreads();
  const QRDesc d = desc[i];
  const T* E = qrA + d.off + (long long)M * d.ld;
  for (int a = threadIdx.x; a < np + nd; a += kBlock) {
    double acc = 0.0;
    for (int k = 0; k < M; ++k) acc += (double)E[(long long)a * d.ld + k] * cs[k];
    if (a < np) yP[(size_t)r * sumP + p0 + a] = acc;
    else yD[(size_t)r * sumD + d0 + a - np] = acc;
  }
}

// out[r][off + g] = sum over the owner slots of g of loc[r][slot] (+ add[r][g]),
// one thread per (g, r).  out may alias add when stride == n and off == 0.
__global__ void k_owner_sum(int n, const int* __restrict__ own_ptr, const int* __restrict__ own_slot,
                            const double* __restrict__ loc, int sumS, const double* add, double* out,
                            int out_stride, int out_off) {
  const int g = blockIdx.x * kBlock + threadIdx.x, r = blockIdx.y;
  if (g >= n) return;
  double s = 0.0;
  for (int o = own_ptr[g]; o < own_ptr[g + 1]; ++o) s += loc[(size_t)r * sumS + own_slot[o]];
  if (add) s += add[(size_t)r * n + g];
  out[(size_t)r * out_stride + out_off + g] = s;
}

// out[r][q] = scale * sum_{k < nrow} X1[r0 + k][q] in[r][k] for q < nq
// (X1 column-major, leading dimension ld)
__global__ void k_x1t(const double* __restrict__ X1, int ld, int r0, int nrow, const double* __restrict__ in,
                      int in_stride, int nq, double scale, double* __restrict__ out, int out_stride) {
  const int q = blockIdx.x * kBlock + threadIdx.x, r = blockIdx.y;
  if (q >= nq) return;
  double s = 0.0;
  for (int k = 0; k < nrow; ++k) s += X1[(long long)q * ld + r0 + k] * in[(size_t)r * in_stride + k];
  out[(size_t)r * out_stride + q] = scale * s;
}

// transposed recovery: zD (Delta slots) = yD + G_PD^T u_rho(Pi^i) + L_PD^T u_psi(Pi^i),
// u = [u_rho; u_psi] global (2 nP per rhs)
template <typename T>
__global__ void k_adj_rec(const OpArgs<T> a, const double* __restrict__ yD, const double* __restrict__ u,
                          double* __restrict__ zD) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0, d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  const T* G = a.Gm + a.offG[i];
  const T* L = a.Lm + a.offG[i];
  const double* ur = u + (size_t)r * 2 * a.nP;
  for (int t = threadIdx.x; t < nd; t += kBlock) {
    double acc = yD[(size_t)r * a.sumD + d0 + t];
    for (int b = 0; b < np; ++b) {
      const int q = a.pi_l2g[p0 + b];
      const long long e = (long long)(np + t) * ng + b;
      acc += (double)G[e] * ur[q] + (double)L[e] * ur[a.nP + q];
    }
    zD[(size_t)r * a.sumD + d0 + t] = acc;
  }
}

// transpose of the last right-hand-side stage for bbar (global Delta):
//   mloc (Pi slots) = -G_DP^T bbar_i,  eloc (Pi slots) = L_PD bbar_i,
//   etaD (Delta slots) = L_DD bbar_i
template <typename T>
__global__ void k_adj_A1(const OpArgs<T> a, const double* __restrict__ bbar, double* __restrict__ mloc,
                         double* __restrict__ eloc, double* __restrict__ etaD) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0, d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  extern __shared__ double bs[];
  for (int k = threadIdx.x; k < nd; k += kBlock) bs[k] = bbar[(size_t)r * a.nD + a.dl_l2g[d0 + k]];
  __syncthreads();
  const T* G = a.Gm + a.offG[i];
  const T* L = a.Lm + a.offG[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    if (t < np) {
      double sm = 0.0, se = 0.0;
      for (int k = 0; k < nd; ++k) {
        sm -= (double)G[(long long)t * ng + np + k] * bs[k];
        se += (double)L[(long long)(np + k) * ng + t] * bs[k];
      }
      mloc[(size_t)r * a.sumP + p0 + t] = sm;
      eloc[(size_t)r * a.sumP + p0 + t] = se;
    } else {
      const int row = t - np;
      double s = 0.0;
      for (int k = 0; k < nd; ++k) s += (double)L[(long long)(np + k) * ng + np + row] * bs[k];
      etaD[(size_t)r * a.sumD + d0 + row] = s;
    }
  }
}

// lam_loc (Delta slots; their owner sum is the cotangent of eta) = etaD + L_DP nubar(Pi^i)
template <typename T>
__global__ void k_adj_A2(const OpArgs<T> a, const double* __restrict__ etaD, const double* __restrict__ nubar) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0, d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  const T* L = a.Lm + a.offG[i];
  for (int t = threadIdx.x; t < nd; t += kBlock) {
    double acc = etaD[(size_t)r * a.sumD + d0 + t];
    for (int b = 0; b < np; ++b)
      acc += (double)L[(long long)b * ng + np + t] * nubar[(size_t)r * a.nP + a.pi_l2g[p0 + b]];
    a.lam_loc[(size_t)r * a.sumD + d0 + t] = acc;
  }
}

// lbar_i = theta sum z + (1 - theta) sum lam at the Delta points of i (the
// cotangent of lambda, M applied to that of eta), into Delta slots;
// mloc (Pi slots) -= L_DP^T lbar_i
template <typename T>
__global__ void k_adj_A3(const OpArgs<T> a, double* __restrict__ lbar, double* __restrict__ mloc) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0, d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  extern __shared__ double ls[];
  for (int k = threadIdx.x; k < nd; k += kBlock) {
    const int g = a.dl_l2g[d0 + k];
    const double l = dl_sum(a.dl_own_ptr, a.dl_own_slot, a.lam_loc + (size_t)r * a.sumD, g);
    double v = l;
    if (a.theta != 0.0)
      v = a.theta * dl_sum(a.dl_own_ptr, a.dl_own_slot, a.z_loc + (size_t)r * a.sumD, g) + (1.0 - a.theta) * l;
    ls[k] = v;
    lbar[(size_t)r * a.sumD + d0 + k] = v;
  }
  __syncthreads();
  const T* L = a.Lm + a.offG[i];
  for (int b = threadIdx.x; b < np; b += kBlock) {
    double s = 0.0;
    for (int k = 0; k < nd; ++k) s += (double)L[(long long)b * ng + np + k] * ls[k];
    mloc[(size_t)r * a.sumP + p0 + b] -= s;
  }
}

// cotangent of h_Delta: theta sum z + (1 - theta) sum lam at every global Delta point
template <typename T>
__global__ void k_adj_hD(const OpArgs<T> a, double* __restrict__ hbD) {
  const int g = blockIdx.x * kBlock + threadIdx.x, r = blockIdx.y;
  if (g >= a.nD) return;
  const double l = dl_sum(a.dl_own_ptr, a.dl_own_slot, a.lam_loc + (size_t)r * a.sumD, g);
  double v = l;
  if (a.theta != 0.0)
    v = a.theta * dl_sum(a.dl_own_ptr, a.dl_own_slot, a.z_loc + (size_t)r * a.sumD, g) + (1.0 - a.theta) * l;
  hbD[(size_t)r * a.nD + g] = v;
}

// Per subdomain, with u = [u_rho; u_psi] the cotangent of the coarse input:
//   Fb[:M]  = cbar_i - A_m^T [u_psi(Pi^i); lbar_i]       (cotangent of cf0)
//   Fb[M:m] = 0
//   pbarG   = [u_rho(Pi^i); bbar(Delta^i)]               (cotangent of the projections)
template <typename T, typename TA>
__global__ void k_adj_F(int M, int N, int nP, int nD, const int* __restrict__ sizes, const int* __restrict__ pi_off,
                        const int* __restrict__ dl_off, const int* __restrict__ pi_l2g,
                        const int* __restrict__ dl_l2g, const long long* __restrict__ offAm,
                        const TA* __restrict__ Am, const double* __restrict__ cbar, const double* __restrict__ u,
                        const double* __restrict__ lbar, const double* __restrict__ bbar, int sumD,
                        const long long* __restrict__ offm, long long summ, T* __restrict__ Fb,
                        double* __restrict__ pbarG, int sumG) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int m = sizes[5 * i + 3], ng = sizes[5 * i + 4];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  const int g0 = p0 + d0;
  extern __shared__ double ys[];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double v, pb;
    if (t < np) {
      const int q = pi_l2g[p0 + t];
      v = u[(size_t)r * 2 * nP + nP + q];
      pb = u[(size_t)r * 2 * nP + q];
    } else {
      v = lbar[(size_t)r * sumD + d0 + t - np];
      pb = bbar[(size_t)r * nD + dl_l2g[d0 + t - np]];
    }
    ys[t] = v;
    pbarG[(size_t)r * sumG + g0 + t] = pb;
  }
  __syncthreads();
  const TA* A = Am + offAm[i];
  T* Fi = Fb + (size_t)r * summ + offm[i];
  for (int k = threadIdx.x; k < M; k += kBlock) {
    double acc = cbar[((size_t)r * N + i) * M + k];
    for (int t = 0; t < ng; ++t) acc -= (double)A[(long long)k * ng + t] * ys[t];
    Fi[k] = (T)acc;
  }
  for (int row = M + threadIdx.x; row < m; row += kBlock) Fi[row] = T(0);
}

// Fb[:M] += Q_G^T pbar_i   (after R^{-T} has been applied to Fb[:M])
template <typename T>
__global__ void k_adj_alpha(int M, const int* __restrict__ sizes, const int* __restrict__ pi_off,
                            const int* __restrict__ dl_off, const long long* __restrict__ offQG,
                            const T* __restrict__ QG, const double* __restrict__ pbarG, int sumG,
                            const long long* __restrict__ offm, long long summ, T* __restrict__ Fb) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int ng = sizes[5 * i + 4];
  extern __shared__ double pb[];
  const double* src = pbarG + (size_t)r * sumG + pi_off[i] + dl_off[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) pb[t] = src[t];
  __syncthreads();
  const T* Q = QG + offQG[i];
  T* Fi = Fb + (size_t)r * summ + offm[i];
  for (int k = threadIdx.x; k < M; k += kBlock) {
    double acc = (double)Fi[k];
    for (int t = 0; t < ng; ++t) acc += (double)Q[(long long)t * M + k] * pb[t];
    Fi[k] = (T)acc;
  }
}

// fbar = Fb (after Q) - pbar on the interface rows, in float64, for all m
// rows; the interface rows also go to fbGP / fbGD in slot order (if given)
template <typename T>
__global__ void k_adj_fout(const int* __restrict__ sizes, const int* __restrict__ pi_off,
                           const int* __restrict__ dl_off, const long long* __restrict__ offm, long long summ,
                           const T* __restrict__ Fb, const double* __restrict__ pbarG, int sumG, int sumP, int sumD,
                           double* __restrict__ fbar, double* __restrict__ fbGP, double* __restrict__ fbGD) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int nI = sizes[5 * i + 1], nB = sizes[5 * i + 2], m = sizes[5 * i + 3];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  const size_t base = (size_t)r * summ + offm[i];
  for (int row = threadIdx.x; row < m; row += kBlock) {
    double v = (double)Fb[base + row];
    const int g = row - nI - nB;
    if (g >= 0) {
      v -= pbarG[(size_t)r * sumG + p0 + d0 + g];
      if (fbGP) {
        if (g < np) fbGP[(size_t)r * sumP + p0 + g] = v;
        else fbGD[(size_t)r * sumD + d0 + g - np] = v;
      }
    }
    fbar[base + row] = v;
  }
}

// f_I_bar [nrhs][N][n_int] and g_B_bar [nrhs][sum n_B] (may be null) from the
// rows of fbar
__global__ void k_adj_out(int N, int n_int, const int* __restrict__ sizes, const long long* __restrict__ offm,
                          const long long* __restrict__ offB, long long summ, long long sumB,
                          const double* __restrict__ fbar, double* __restrict__ fIbar, double* __restrict__ gBbar) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int nB = sizes[5 * i + 2];
  const size_t base = (size_t)r * summ + offm[i];
  for (int row = threadIdx.x; row < n_int + nB; row += kBlock) {
    const double v = fbar[base + row];
    if (row < n_int) fIbar[((size_t)r * N + i) * n_int + row] = v;
    else if (gBbar) gBbar[(size_t)r * sumB + offB[i] + row - n_int] = v;
  }
}

// Refinement of a float32 adjoint: z <- z - Op^T w, with Op the coupled
// system [K B; A 0] and w = (fw, hw) the last adjoint increment.
// c part here: zc_i -= K_i^T fw_i + A_m^i^T hw(Gamma^i) (float64 features);
// the mu parts (z_mu += sum of the interface rows of fw) are owner sums.
__global__ void k_adj_resid(int M, int nP, int nD, const int* __restrict__ sizes, const int* __restrict__ pi_off,
                            const int* __restrict__ dl_off, const int* __restrict__ pi_l2g,
                            const int* __restrict__ dl_l2g, const long long* __restrict__ offK,
                            const double* __restrict__ K64, const long long* __restrict__ offAm,
                            const double* __restrict__ A64, const long long* __restrict__ offm, long long summ,
                            const double* __restrict__ fw, const double* __restrict__ hwP,
                            const double* __restrict__ hwD, int N, double* __restrict__ zc) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int m = sizes[5 * i + 3], ng = sizes[5 * i + 4];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  extern __shared__ double sh[];
  double* fs = sh;          // [m]
  double* hs = sh + m;      // [ng]
  for (int row = threadIdx.x; row < m; row += kBlock) fs[row] = fw[(size_t)r * summ + offm[i] + row];
  for (int t = threadIdx.x; t < ng; t += kBlock)
    hs[t] = t < np ? (hwP ? hwP[(size_t)r * nP + pi_l2g[p0 + t]] : 0.0)
                   : (hwD ? hwD[(size_t)r * nD + dl_l2g[d0 + t - np]] : 0.0);
  __syncthreads();
  const double* K = K64 + offK[i];
  const double* A = A64 + offAm[i];
  for (int k = threadIdx.x; k < M; k += kBlock) {
    double acc = 0.0;
    for (int row = 0; row < m; ++row) acc += K[(long long)k * m + row] * fs[row];
    for (int t = 0; t < ng; ++t) acc += A[(long long)k * ng + t] * hs[t];
    zc[((size_t)r * N + i) * M + k] -= acc;
  }
}

// ---------------------------------------------------------------- evaluation adjoint
// cbar[r][i][j] = sum over the points p owned by subdomain i (the owner rule
// of k_evaluate) of ubar[r][p] phi_j(x_p) + gbar[r][p] . grad phi_j(x_p).
// Grid (N, ceil(M / kBlock), nrhs); the points are scanned in chunks of
// kBlock, the owned ones compacted into LDS in ascending order, so the
// summation order is fixed.
__global__ void __launch_bounds__(kBlock) k_eval_adj(int nx, int ny, int M, int N, double lo0, double lo1, double h0,
                                                     double h1, const double* __restrict__ W,
                                                     const double* __restrict__ bias, long long npts,
                                                     const double* __restrict__ x, const double* __restrict__ ubar,
                                                     const double* __restrict__ gbar, double* __restrict__ cbar) {
  const int i = blockIdx.x, r = blockIdx.z;
  const int j = blockIdx.y * kBlock + threadIdx.x;
  const int ix = i % nx, iy = i / nx;
  const double hx = 0.5 * h0, hy = 0.5 * h1;
  const double cx = lo0 + (ix + 0.5) * h0, cy = lo1 + (iy + 0.5) * h1;
  const bool active = j < M;
  const double w0 = active ? W[((size_t)i * M + j) * 2] : 0.0;
  const double w1 = active ? W[((size_t)i * M + j) * 2 + 1] : 0.0;
  const double bj = active ? bias[(size_t)i * M + j] : 0.0;
  __shared__ long long idx[kBlock];
  __shared__ int wcnt[kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc = 0.0;
  for (long long base = 0; base < npts; base += kBlock) {
    const long long p = base + threadIdx.x;
    bool own = false;
    if (p < npts) {
      const double px = x[2 * p], py = x[2 * p + 1];
      int jx = (int)ceil((px - lo0) / h0) - 1, jy = (int)ceil((py - lo1) / h1) - 1;
      jx = jx < 0 ? 0 : (jx > nx - 1 ? nx - 1 : jx);
      jy = jy < 0 ? 0 : (jy > ny - 1 ? ny - 1 : jy);
      own = jx == ix && jy == iy;
    }
    const unsigned long long mask = __ballot(own);
    const int pre = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wv] = __popcll(mask);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (w < wv) off += wcnt[w];
      tot += wcnt[w];
    }
    if (own) idx[off + pre] = p;
    __syncthreads();
    if (active) {
      for (int q = 0; q < tot; ++q) {
        const long long pq = idx[q];
        const double xi0 = (x[2 * pq] - cx) / hx, xi1 = (x[2 * pq + 1] - cy) / hy;
        const double t = tanh_fast(w0 * xi0 + w1 * xi1 + bj);
        acc += ubar[(size_t)r * npts + pq] * t;
        if (gbar) {
          const double dt = 1.0 - t * t;
          acc += dt * (gbar[((size_t)r * npts + pq) * 2] * (w0 / hx) +
                       gbar[((size_t)r * npts + pq) * 2 + 1] * (w1 / hy));
        }
      }
    }
    __syncthreads();
  }
  if (active) cbar[((size_t)r * N + i) * M + j] = acc;
}

}  // namespace ddelm
