// Right-hand side, refinement residual, recovery, CG bookkeeping and
// evaluation kernels.  T is the storage type of the local factors (double,
// or float in mixed precision); interface vectors are always double.
#pragma once
#include "tanh_fast.hpp"
#include "kernels_qr.hpp"
#include "kernels_solve.hpp"

namespace ddelm {

// sizes[5*i + ...]: 0 M, 1 n_I, 2 n_B, 3 m, 4 n_G

// f^i = [f_I; g_B; 0] into F[r][offm[i] + row] (type T) and optionally into
// F64 (the double copy kept for refinement residuals)
template <typename T>
__global__ void k_rhs_assemble(int N, int n_int, const int* __restrict__ sizes, const long long* __restrict__ offm,
                               const long long* __restrict__ offB, long long summ, long long sumB,
                               const double* __restrict__ fI, const double* __restrict__ gB, T* __restrict__ F,
                               double* __restrict__ F64) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int nB = sizes[5 * i + 2], m = sizes[5 * i + 3];
  const size_t base = (size_t)r * summ + offm[i];
  for (int row = threadIdx.x; row < m; row += kBlock) {
    double v = 0.0;
    if (row < n_int) v = fI[((size_t)r * N + i) * n_int + row];
    else if (row < n_int + nB) v = gB[(size_t)r * sumB + offB[i] + row - n_int];
    F[base + row] = (T)v;
    if (F64) F64[base + row] = v;
  }
}

// A general local right-hand side, given row by row for every subdomain
// (f64 [nrhs][sum m]), into F (type T) and its interface rows in slot order.
template <typename T>
__global__ void k_rhs_split(const int* __restrict__ sizes, const int* __restrict__ pi_off,
                            const int* __restrict__ dl_off, const long long* __restrict__ offm, long long summ,
                            int sumP, int sumD, const double* __restrict__ ff, T* __restrict__ F,
                            double* __restrict__ F64, double* __restrict__ fGP, double* __restrict__ fGD) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int nI = sizes[5 * i + 1], nB = sizes[5 * i + 2], m = sizes[5 * i + 3];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  const size_t base = (size_t)r * summ + offm[i];
  for (int row = threadIdx.x; row < m; row += kBlock) {
    const double v = ff[base + row];
    F[base + row] = (T)v;
    if (F64) F64[base + row] = v;
    const int g = row - nI - nB;
    if (g >= 0) {
      if (g < np) fGP[(size_t)r * sumP + p0 + g] = v;
      else fGD[(size_t)r * sumD + d0 + g - np] = v;
    }
  }
}

// p_G = Q_G (Q^T f)[:M];  rho_loc = p_P - f_P (Pi slots), s_loc = p_D - f_D
// (Delta slots), where f_P, f_D are the interface rows of f before Q^T was
// applied (fGP, fGD; null when they are zero).  One workgroup per
// (subdomain, group of P right-hand sides), Q_G read once per group.
template <typename T, int P>
__global__ void __launch_bounds__(kBlock) k_rhs_proj(int M, int nrhs, const int* __restrict__ sizes,
                                                     const int* __restrict__ pi_off, const int* __restrict__ dl_off,
                                                     const long long* __restrict__ offQG, const T* __restrict__ QG,
                                                     const long long* __restrict__ offm, long long summ,
                                                     const T* __restrict__ F, int sumP, int sumD,
                                                     const double* __restrict__ fGP, const double* __restrict__ fGD,
                                                     double* __restrict__ rho_loc, double* __restrict__ s_loc) {
  const int i = blockIdx.x, r0 = blockIdx.y * P, nr = min(P, nrhs - r0);
  const int ng = sizes[5 * i + 4];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  extern __shared__ double al[];   // [M][P]
  for (int e = threadIdx.x; e < M * P; e += kBlock) {
    const int k = e / P, j = e % P;
    al[e] = j < nr ? (double)F[(size_t)(r0 + j) * summ + offm[i] + k] : 0.0;
  }
  __syncthreads();
  constexpr int kU = 8;   // elements of Q loaded together per thread
  const T* Q = QG + offQG[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = 0.0;
    for (int k0 = 0; k0 < M; k0 += kU) {
      double q[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) q[u] = k0 + u < M ? (double)Q[(long long)t * M + k0 + u] : 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (k0 + u < M) {
#pragma unroll
          for (int j = 0; j < P; ++j) acc[j] += q[u] * al[(k0 + u) * P + j];
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      const int r = r0 + j;
      if (t < np) {
        const size_t e = (size_t)r * sumP + p0 + t;
        rho_loc[e] = acc[j] - (fGP ? fGP[e] : 0.0);
      } else {
        const size_t e = (size_t)r * sumD + d0 + t - np;
        s_loc[e] = acc[j] - (fGD ? fGD[e] : 0.0);
      }
    }
  }
}

// ad = A_m c_f0;  psi_loc = -ad_P, l_loc = -ad_D (+ h_D at the first owner of
// each Delta point, so that the owner sum gives h_D - A_D K^+ f).  One
// workgroup per (subdomain, group of P right-hand sides), A_m read once per
// group.
template <typename T, typename TA, int P>
__global__ void __launch_bounds__(kBlock) k_rhs_flux(int M, int nD, int nrhs, const int* __restrict__ sizes,
                                                     const int* __restrict__ pi_off, const int* __restrict__ dl_off,
                                                     const int* __restrict__ dl_l2g, const int* __restrict__ dl_own_ptr,
                                                     const int* __restrict__ dl_own_slot,
                                                     const long long* __restrict__ offAm, const TA* __restrict__ Am,
                                                     const long long* __restrict__ offm, long long summ,
                                                     const T* __restrict__ F, int sumP, int sumD,
                                                     const double* __restrict__ hD, double* __restrict__ psi_loc,
                                                     double* __restrict__ l_loc) {
  const int i = blockIdx.x, r0 = blockIdx.y * P, nr = min(P, nrhs - r0);
  const int ng = sizes[5 * i + 4];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  extern __shared__ double cf[];   // [M][P]
  for (int e = threadIdx.x; e < M * P; e += kBlock) {
    const int k = e / P, j = e % P;
    cf[e] = j < nr ? (double)F[(size_t)(r0 + j) * summ + offm[i] + k] : 0.0;
  }
  __syncthreads();
  const TA* A = Am + offAm[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = 0.0;
    for (int k = 0; k < M; ++k) {
      const double av = (double)A[(long long)k * ng + t];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] += av * cf[k * P + j];
    }
    int own = 1, g = 0;
    if (t >= np && hD) {
      const int slot = d0 + t - np;
      g = dl_l2g[slot];
      own = dl_own_slot[dl_own_ptr[g]] == slot;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      const int r = r0 + j;
      if (t < np) {
        psi_loc[(size_t)r * sumP + p0 + t] = -acc[j];
      } else {
        double v = -acc[j];
        if (hD && own) v += hD[(size_t)r * nD + g];
        l_loc[(size_t)r * sumD + d0 + t - np] = v;
      }
    }
  }
}

// c^i = c_f0 + E [mu_P(Pi^i); mu_D(Delta^i)], E = R^{-1} Q_G^T kept in the K_c
// matrix (rows 0..M-1 of columns M.., leading dimension m).  accumulate = 1
// adds the result to coef instead of overwriting it.  One workgroup per
// (subdomain, group of P right-hand sides), E read once per group.
template <typename T, int P>
__global__ void __launch_bounds__(kBlock) k_recover(int M, int nP, int nD, int nrhs, const int* __restrict__ pi_off,
                                                    const int* __restrict__ dl_off, const int* __restrict__ pi_l2g,
                                                    const int* __restrict__ dl_l2g, const QRDesc* __restrict__ desc,
                                                    const T* __restrict__ qrA, const long long* __restrict__ offm,
                                                    long long summ, const T* __restrict__ F,
                                                    const double* __restrict__ mu_pi, const double* __restrict__ mu_dl,
                                                    int N, double* __restrict__ coef, int accumulate) {
  const int i = blockIdx.x, r0 = blockIdx.y * P, nr = min(P, nrhs - r0);
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i], nd = dl_off[i + 1] - d0;
  extern __shared__ double mus[];   // [np + nd][P]
  for (int e = threadIdx.x; e < (np + nd) * P; e += kBlock) {
    const int a = e / P, j = e % P, r = r0 + j;
    mus[e] = j >= nr ? 0.0
                     : (a < np ? mu_pi[(size_t)r * nP + pi_l2g[p0 + a]] : mu_dl[(size_t)r * nD + dl_l2g[d0 + a - np]]);
  }
  __syncthreads();
  const QRDesc d = desc[i];
  const T* E = qrA + d.off + (long long)M * d.ld;
  for (int k = threadIdx.x; k < M; k += kBlock) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = j < nr ? (double)F[(size_t)(r0 + j) * summ + offm[i] + k] : 0.0;
    for (int a = 0; a < np + nd; ++a) {
      const double ev = (double)E[(long long)a * d.ld + k];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] += ev * mus[a * P + j];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      const size_t e = ((size_t)(r0 + j) * N + i) * M + k;
      coef[e] = accumulate ? coef[e] + acc[j] : acc[j];
    }
  }
}

// Residual of the coupled system [K B; A 0][c; mu] = [f; 0] in float64:
//   R = f - K c - B mu   (B mu is -mu on the interface rows),
//   flux slots  aP/aD = (A_m c) at the local Pi / Delta rows.
// K64 (m x M) and A64 (n_G x M) are the float64 feature matrices.  One
// workgroup per (subdomain, group of P right-hand sides): rows along the
// threads, the group's P coefficient vectors in LDS (cs[k][j]), so every
// element of K and A read from memory serves P products.  Dynamic LDS:
// M * P doubles.
template <int P>
__global__ void __launch_bounds__(kBlock) k_residual(
    int M, int nP, int nD, int nrhs, const int* __restrict__ sizes, const int* __restrict__ pi_off,
    const int* __restrict__ dl_off, const int* __restrict__ pi_l2g, const int* __restrict__ dl_l2g,
    const long long* __restrict__ offK, const double* __restrict__ K64, const long long* __restrict__ offAm,
    const double* __restrict__ A64, const long long* __restrict__ offm, long long summ,
    const double* __restrict__ F64, const double* __restrict__ coef, const double* __restrict__ mu_pi,
    const double* __restrict__ mu_dl, int N, int sumP, int sumD, double* __restrict__ R64,
    double* __restrict__ fGP, double* __restrict__ fGD, double* __restrict__ aP, double* __restrict__ aD) {
  const int i = blockIdx.x, r0 = blockIdx.y * P;
  const int nr = min(P, nrhs - r0);
  const int nI = sizes[5 * i + 1], nB = sizes[5 * i + 2], m = sizes[5 * i + 3], ng = sizes[5 * i + 4];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  extern __shared__ double cs[];
  for (int e = threadIdx.x; e < M * P; e += kBlock) {
    const int k = e / P, j = e % P;
    cs[e] = j < nr ? coef[((size_t)(r0 + j) * N + i) * M + k] : 0.0;
  }
  __syncthreads();
  constexpr int kU = 8;   // matrix elements loaded together per thread
  const double* K = K64 + offK[i];
  const long long base = offm[i];
  for (int row = threadIdx.x; row < m; row += kBlock) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = j < nr ? F64[(size_t)(r0 + j) * summ + base + row] : 0.0;
    for (int k0 = 0; k0 < M; k0 += kU) {
      double kv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) kv[u] = k0 + u < M ? K[(long long)(k0 + u) * m + row] : 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (k0 + u < M) {
#pragma unroll
          for (int j = 0; j < P; ++j) acc[j] -= kv[u] * cs[(k0 + u) * P + j];
        }
      }
    }
    const int g = row - nI - nB;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      const int r = r0 + j;
      double v = acc[j];
      if (g >= 0) {
        if (g < np) {
          v += mu_pi[(size_t)r * nP + pi_l2g[p0 + g]];
          fGP[(size_t)r * sumP + p0 + g] = v;
        } else {
          v += mu_dl[(size_t)r * nD + dl_l2g[d0 + g - np]];
          fGD[(size_t)r * sumD + d0 + g - np] = v;
        }
      }
      R64[(size_t)r * summ + base + row] = v;
    }
  }
  const double* A = A64 + offAm[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = 0.0;
    for (int k = 0; k < M; ++k) {
      const double av = A[(long long)k * ng + t];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] += av * cs[k * P + j];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      const int r = r0 + j;
      if (t < np) aP[(size_t)r * sumP + p0 + t] = acc[j];
      else aD[(size_t)r * sumD + d0 + t - np] = acc[j];
    }
  }
}

// h = h0 - (A c) at the global interface points: hP[r][p], hD[r][g]
// (h0P, h0D: the flux right-hand side of the original system, may be null)
__global__ void k_flux_residual(int nP, int nD, int sumP, int sumD, const int* __restrict__ pi_own_ptr,
                                const int* __restrict__ pi_own_slot, const int* __restrict__ dl_own_ptr,
                                const int* __restrict__ dl_own_slot, const double* __restrict__ aP,
                                const double* __restrict__ aD, const double* __restrict__ h0P,
                                const double* __restrict__ h0D, double* __restrict__ hP, double* __restrict__ hD) {
  const int e = blockIdx.x * kBlock + threadIdx.x, r = blockIdx.y;
  if (e < nP) {
    double s = 0.0;
    for (int o = pi_own_ptr[e]; o < pi_own_ptr[e + 1]; ++o) s += aP[(size_t)r * sumP + pi_own_slot[o]];
    hP[(size_t)r * nP + e] = (h0P ? h0P[(size_t)r * nP + e] : 0.0) - s;
  } else if (e < nP + nD) {
    const int g = e - nP;
    double s = 0.0;
    for (int o = dl_own_ptr[g]; o < dl_own_ptr[g + 1]; ++o) s += aD[(size_t)r * sumD + dl_own_slot[o]];
    hD[(size_t)r * nD + g] = (h0D ? h0D[(size_t)r * nD + g] : 0.0) - s;
  }
}

template <typename TS, typename TD>
__global__ void k_convert(const TS* __restrict__ s, TD* __restrict__ d, long long n) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock)
    d[e] = (TD)s[e];
}

// y += x; partial sums of x.x and y.y per rhs (rows of length n), one block per (chunk, rhs)
__global__ void k_axpy_norms(const double* __restrict__ x, double* __restrict__ y, int n, int nblk,
                             double* __restrict__ part) {
  __shared__ double red[kWaves];
  const int r = blockIdx.y, blk = blockIdx.x;
  double sx = 0.0, sy = 0.0;
  for (int g = blk * kBlock + threadIdx.x; g < n; g += nblk * kBlock) {
    const size_t e = (size_t)r * n + g;
    const double xv = x[e];
    const double yv = y[e] + xv;
    y[e] = yv;
    sx += xv * xv;
    sy += yv * yv;
  }
  sx = block_sum(sx, red);
  sy = block_sum(sy, red);
  if (threadIdx.x == 0) {
    part[((size_t)r * nblk + blk) * 2] = sx;
    part[((size_t)r * nblk + blk) * 2 + 1] = sy;
  }
}

// mu_Pi = pi_f - mu_Pi(v)
__global__ void k_mu_pi(int nP, int nrhs, const double* __restrict__ pif, const double* __restrict__ c1,
                        double* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nP * nrhs) return;
  const int r = e / nP, p = e % nP;
  out[e] = pif[e] - c1[(size_t)r * 2 * nP + p];
}

__global__ void k_save_pif(int nP, int nrhs, const double* __restrict__ c1, double* __restrict__ pif) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nP * nrhs) return;
  const int r = e / nP, p = e % nP;
  pif[e] = c1[(size_t)r * 2 * nP + p];
}

// set the unit entries of the appended identity columns
template <typename T>
__global__ void k_set_units(const long long* __restrict__ pos, long long n, T* __restrict__ A) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) A[pos[e]] = T(1);
}

// X1 = [[Sinv, Z^T], [-Z, I - W]] (column-major, 2n x 2n) with Z = D Sinv, W = D Z^T
__global__ void k_assemble_X1(int n, const double* __restrict__ Sinv, const double* __restrict__ Z,
                              const double* __restrict__ W, double* __restrict__ X1) {
  const long long tot = 4ll * n * n;
  const int ld = 2 * n;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < tot; e += (long long)gridDim.x * kBlock) {
    const int r = (int)(e % ld), c = (int)(e / ld);
    double v;
    if (r < n && c < n) v = Sinv[(long long)c * n + r];
    else if (r < n) v = Z[(long long)r * n + (c - n)];               // Z^T[r][c-n] = Z[c-n][r]
    else if (c < n) v = -Z[(long long)c * n + (r - n)];
    else v = (r == c ? 1.0 : 0.0) - W[(long long)(c - n) * n + (r - n)];
    X1[e] = v;
  }
}

// ---------------------------------------------------------------- CG kernels (one launch per phase)

// w = sum of owners, partial p.w
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_wdot(OpArgs<T> a, CGState s) {
  __shared__ double red[kWaves];
  const int r = blockIdx.y, blk = blockIdx.x;
  double acc = 0.0;
  for (int g = blk * kBlock + threadIdx.x; g < s.n; g += s.nblk * kBlock) {
    const double wv = dl_sum(a.dl_own_ptr, a.dl_own_slot, a.w_loc + (size_t)r * a.sumD, g);
    s.w[(size_t)r * s.n + g] = wv;
    acc += wv * s.p[(size_t)r * s.n + g];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) s.part[(size_t)r * s.nblk + blk] = acc;
}

// alpha = rr / p.w (one block per rhs)
__global__ void __launch_bounds__(kBlock) k_cg_alpha(CGState s) {
  __shared__ double red[kWaves];
  const int r = blockIdx.x;
  const double pw = cg_reduce_parts(s.part, s.nblk, r, red);
  if (threadIdx.x == 0) {
    double* sc = s.scal + (size_t)r * 8;
    sc[2] = pw;
    sc[3] = (sc[5] != 0.0 || pw == 0.0) ? 0.0 : sc[0] / pw;
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_axpy(CGState s) {
  __shared__ double red[kWaves];
  const int r = blockIdx.y, blk = blockIdx.x;
  const double al = s.scal[(size_t)r * 8 + 3];
  double acc = 0.0;
  for (int g = blk * kBlock + threadIdx.x; g < s.n; g += s.nblk * kBlock) {
    const size_t e = (size_t)r * s.n + g;
    s.x[e] += al * s.p[e];
    const double rv = s.r[e] - al * s.w[e];
    s.r[e] = rv;
    acc += rv * rv;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) s.part[(size_t)r * s.nblk + blk] = acc;
}

__global__ void __launch_bounds__(kBlock) k_cg_beta(CGState s) {
  __shared__ double red[kWaves];
  const int r = blockIdx.x;
  const double rr = cg_reduce_parts(s.part, s.nblk, r, red);
  if (threadIdx.x == 0) {
    double* sc = s.scal + (size_t)r * 8;
    if (sc[5] != 0.0) {
      sc[4] = 0.0;
    } else {
      sc[4] = sc[0] > 0.0 ? rr / sc[0] : 0.0;
      sc[0] = rr;
      sc[6] += 1.0;
      if (!(rr == rr) || isinf(rr)) sc[7] = 1.0;
      if (sqrt(rr) <= s.tol * sqrt(sc[1]) || !(rr == rr)) sc[5] = 1.0;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_pupd(CGState s) {
  const int r = blockIdx.y, blk = blockIdx.x;
  const double be = s.scal[(size_t)r * 8 + 4];
  for (int g = blk * kBlock + threadIdx.x; g < s.n; g += s.nblk * kBlock) {
    const size_t e = (size_t)r * s.n + g;
    s.p[e] = s.r[e] + be * s.p[e];
  }
}

// r = p = b, x = 0; partial b.b
__global__ void __launch_bounds__(kBlock) k_cg_init(CGState s, const double* __restrict__ b) {
  __shared__ double red[kWaves];
  const int r = blockIdx.y, blk = blockIdx.x;
  double acc = 0.0;
  for (int g = blk * kBlock + threadIdx.x; g < s.n; g += s.nblk * kBlock) {
    const size_t e = (size_t)r * s.n + g;
    const double bv = b[e];
    s.x[e] = 0.0;
    s.r[e] = bv;
    s.p[e] = bv;
    acc += bv * bv;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) s.part[(size_t)r * s.nblk + blk] = acc;
}

__global__ void __launch_bounds__(kBlock) k_cg_init2(CGState s) {
  __shared__ double red[kWaves];
  const int r = blockIdx.x;
  const double bb = cg_reduce_parts(s.part, s.nblk, r, red);
  if (threadIdx.x == 0) {
    double* sc = s.scal + (size_t)r * 8;
    sc[0] = bb; sc[1] = s.bref ? s.bref[r] : bb; sc[2] = 0; sc[3] = 0; sc[4] = 0;
    sc[5] = (bb == 0.0) ? 1.0 : 0.0;
    sc[6] = 0; sc[7] = 0;
  }
}

// r = b - w (when r is not null) and, per right-hand side rh, ||b - w||^2
// (out[rh]) and ||b||^2 (out[nrhs + rh], nrhs = gridDim.x); w may be null
// (then the residual is b).  One workgroup per right-hand side, fixed
// summation order.
__global__ void __launch_bounds__(kBlock) k_resid_norms(int n, const double* __restrict__ b,
                                                        const double* __restrict__ w, double* __restrict__ r,
                                                        double* __restrict__ out) {
  __shared__ double red[kWaves];
  const int rh = blockIdx.x;
  double ss = 0.0, bb = 0.0;
  for (int g = threadIdx.x; g < n; g += kBlock) {
    const size_t e = (size_t)rh * n + g;
    const double bv = b[e], d = w ? bv - w[e] : bv;
    if (r) r[e] = d;
    ss += d * d;
    bb += bv * bv;
  }
  ss = block_sum(ss, red);
  bb = block_sum(bb, red);
  if (threadIdx.x == 0) {
    out[rh] = ss;
    out[gridDim.x + rh] = bb;
  }
}

// x += d (element-wise, n * nrhs values)
__global__ void __launch_bounds__(kBlock) k_add_to(long long n, const double* __restrict__ d, double* __restrict__ x) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock)
    x[e] += d[e];
}

// ---------------------------------------------------------------- evaluation
// u[r][p] (and grad[r][p][:]) for the right-hand sides r0 .. r0+NRB-1 (< nrhs)
// at point p = blockIdx.x * kBlock + threadIdx.x, r0 = blockIdx.y * NRB: one
// tanh per (point, neuron) serves every right-hand side of the group.  GRAD:
// the gradient is wanted (otherwise it is not accumulated).
template <int NRB, bool GRAD>
__global__ void __launch_bounds__(kBlock) k_evaluate(int nx, int ny, int M, int N, double lo0, double lo1, double h0,
                                                     double h1, const double* __restrict__ W,
                                                     const double* __restrict__ bias, const double* __restrict__ coef,
                                                     long long npts, const double* __restrict__ x,
                                                     double* __restrict__ u, double* __restrict__ grad, int nrhs) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= npts) return;
  const int r0 = blockIdx.y * NRB;
  const double px = x[2 * e], py = x[2 * e + 1];
  int ix = (int)ceil((px - lo0) / h0) - 1, iy = (int)ceil((py - lo1) / h1) - 1;
  ix = ix < 0 ? 0 : (ix > nx - 1 ? nx - 1 : ix);
  iy = iy < 0 ? 0 : (iy > ny - 1 ? ny - 1 : iy);
  const int i = iy * nx + ix;
  const double hx = 0.5 * h0, hy = 0.5 * h1;
  const double cx = lo0 + (ix + 0.5) * h0, cy = lo1 + (iy + 0.5) * h1;
  const double xi0 = (px - cx) / hx, xi1 = (py - cy) / hy;
  double acc[NRB], g0[NRB], g1[NRB];
#pragma unroll
  for (int k = 0; k < NRB; ++k) acc[k] = g0[k] = g1[k] = 0.0;
  for (int j = 0; j < M; ++j) {
    const double w0 = W[((size_t)i * M + j) * 2], w1 = W[((size_t)i * M + j) * 2 + 1];
    const double t = tanh_fast(w0 * xi0 + w1 * xi1 + bias[(size_t)i * M + j]);
    const double dt = 1.0 - t * t;
#pragma unroll
    for (int k = 0; k < NRB; ++k) {
      if (r0 + k < nrhs) {
        const double c = coef[((size_t)(r0 + k) * N + i) * M + j];
        acc[k] += c * t;
        if (GRAD) {
          const double d = c * dt;
          g0[k] += d * w0;
          g1[k] += d * w1;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NRB; ++k) {
    if (r0 + k >= nrhs) continue;
    const int r = r0 + k;
    u[(size_t)r * npts + e] = acc[k];
    if (GRAD) {
      grad[((size_t)r * npts + e) * 2] = g0[k] / hx;
      grad[((size_t)r * npts + e) * 2 + 1] = g1[k] / hy;
    }
  }
}

// Two-stage QR: the interface rows of the local vectors F (n_G rows) move
// between their place in the full row order (from row t_i = m - n_G) and the
// reduced order of the second stage (from row M).  down = 0: up, after Q1^T;
// down = 1: down, before Q1, with rows M..t_i-1 (the part of the first
// stage's vector below its M leading rows) cleared.  Whole blocks are read
// before any is written, so the ranges may overlap.
template <typename T>
__global__ void k_move_rows(int M, const int* __restrict__ sizes, const long long* __restrict__ offm, long long summ,
                            T* __restrict__ F, int down) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int m = sizes[5 * i + 3], ng = sizes[5 * i + 4], t = m - ng;
  extern __shared__ double buf[];
  T* Fi = F + (size_t)r * summ + offm[i];
  const int src = down ? M : t, dst = down ? t : M;
  for (int k = threadIdx.x; k < ng; k += kBlock) buf[k] = (double)Fi[src + k];
  __syncthreads();
  if (down)
    for (int row = M + threadIdx.x; row < t; row += kBlock) Fi[row] = T(0);
  for (int k = threadIdx.x; k < ng; k += kBlock) Fi[dst + k] = (T)buf[k];
}

// ---------------------------------------------------------------- evaluation on the matrix cores
//
// For many points the evaluation runs in tiles of 16 points of one subdomain:
// the points are binned by owning subdomain first (counting sort), then every
// wave takes one tile and forms U (16 x 16) = T (16 x M) C^T (M x 16) on f64
// MFMA, T = tanh(w . xi + b) computed lane by lane as the A operand (lane l:
// point l & 15, neuron 4 s + (l >> 4) of step s, so each tanh is evaluated
// exactly once) and C^T (coefficients of 16 right-hand sides, transposed so
// that a neuron's 16 values are contiguous) as the B operand.  Each point's
// value is computed on its own, so the order of the points inside a bin (set
// by the atomics of the binning) does not change any result.

// Owning subdomain of a point: the box is split uniformly, points outside it
// are clamped to the nearest subdomain (as k_evaluate does).
__device__ __forceinline__ int owner_of_point(double px, double py, int nx, int ny, double lo0, double lo1,
                                              double h0, double h1) {
  int ix = (int)ceil((px - lo0) / h0) - 1, iy = (int)ceil((py - lo1) / h1) - 1;
  ix = ix < 0 ? 0 : (ix > nx - 1 ? nx - 1 : ix);
  iy = iy < 0 ? 0 : (iy > ny - 1 ? ny - 1 : iy);
  return iy * nx + ix;
}

// Points of one wave mostly share their subdomain, so the wave adds its
// points to a bin with one atomic per distinct subdomain: the lanes of the
// first pending subdomain find each other by a ballot, their leader takes the
// slots, and each lane's slot is the leader's plus its rank among them.
// Returns the lane's slot in its bin (-1 for lanes without a point).
__device__ __forceinline__ int bin_slot(bool has, int key, int* __restrict__ ctr) {
  const int lane = threadIdx.x & 63;
  int slot = -1;
  bool done = !has;
  for (;;) {
    const unsigned long long pending = __ballot(!done);
    if (pending == 0) break;
    const int lead = __ffsll((long long)pending) - 1;
    const int k = __shfl(key, lead);
    const bool mine = !done && key == k;
    const unsigned long long m = __ballot(mine);
    int base = 0;
    if (lane == lead) base = atomicAdd(&ctr[k], __popcll(m));
    base = __shfl(base, lead);
    if (mine) {
      slot = base + __popcll(m & ((1ull << lane) - 1ull));
      done = true;
    }
  }
  return slot;
}

__global__ void k_bin_count(int nx, int ny, double lo0, double lo1, double h0, double h1, long long npts,
                            const double* __restrict__ x, int* __restrict__ cnt) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  const bool has = e < npts;
  const int i = has ? owner_of_point(x[2 * e], x[2 * e + 1], nx, ny, lo0, lo1, h0, h1) : 0;
  bin_slot(has, i, cnt);
}

__global__ void k_bin_scatter(int nx, int ny, double lo0, double lo1, double h0, double h1, long long npts,
                              const double* __restrict__ x, const long long* __restrict__ off,
                              int* __restrict__ cursor, int* __restrict__ perm) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  const bool has = e < npts;
  const int i = has ? owner_of_point(x[2 * e], x[2 * e + 1], nx, ny, lo0, lo1, h0, h1) : 0;
  const int slot = bin_slot(has, i, cursor);
  if (has) perm[off[i] + slot] = (int)e;
}

// coefT[g][i][j][c] = coef[16 g + c][i][j] (zero for 16 g + c >= nrhs)
__global__ void k_coef_transpose(int N, int M, int nrhs, int ngroups, const double* __restrict__ coef,
                                 double* __restrict__ coefT) {
  const long long n = (long long)ngroups * N * M * 16;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock) {
    const int c = (int)(e % 16);
    const long long q = e / 16;                  // (g, i, j)
    const int j = (int)(q % M);
    const long long gi = q / M;                  // g * N + i
    const int i = (int)(gi % N), g = (int)(gi / N);
    const int r = 16 * g + c;
    coefT[e] = r < nrhs ? coef[((size_t)r * N + i) * M + j] : 0.0;
  }
}

template <bool GRAD>
__global__ void __launch_bounds__(kBlock) k_evaluate_mfma(int nx, int M, int N, double lo0, double lo1, double h0,
                                                          double h1, const double* __restrict__ W,
                                                          const double* __restrict__ bias,
                                                          const double* __restrict__ coefT,
                                                          const long long* __restrict__ off,
                                                          const long long* __restrict__ toff, long long ntiles,
                                                          const int* __restrict__ perm, long long npts,
                                                          const double* __restrict__ x, double* __restrict__ u,
                                                          double* __restrict__ grad, int nrhs) {
  typedef Mfma<double>::v4 v4;
  const long long tile = (long long)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (tile >= ntiles) return;                    // uniform over the wave
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int g = blockIdx.y;                      // right-hand-side group of 16
  // subdomain of the tile: toff[i] <= tile < toff[i + 1] (bins without points have no tiles)
  int lo = 0, hi = N;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (toff[mid] <= tile) lo = mid;
    else hi = mid;
  }
  const int i = lo;
  const long long p0 = off[i] + (tile - toff[i]) * 16, pend = off[i + 1];
  const int ix = i % nx, iy = i / nx;
  const double hx = 0.5 * h0, hy = 0.5 * h1;
  const double cx = lo0 + (ix + 0.5) * h0, cy = lo1 + (iy + 0.5) * h1;
  // this lane's point for the A operand (rows past the bin repeat its last point; never stored)
  const long long ea = perm[min(p0 + lr, pend - 1)];
  const double xi0 = (x[2 * ea] - cx) / hx, xi1 = (x[2 * ea + 1] - cy) / hy;
  const double* Wi = W + (size_t)i * M * 2;
  const double* bi = bias + (size_t)i * M;
  const double* Ci = coefT + ((size_t)g * N + i) * M * 16;
  v4 acc = {0.0, 0.0, 0.0, 0.0}, a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < M; j0 += 4) {
    const int j = j0 + lk;
    const int jc = j < M ? j : M - 1;
    const double w0 = Wi[2 * jc], w1 = Wi[2 * jc + 1];
    const double cb = j < M ? Ci[(size_t)jc * 16 + lr] : 0.0;      // B[neuron j][rhs lr]
    const double t = tanh_fast(w0 * xi0 + w1 * xi1 + bi[jc]);
    acc = Mfma<double>::mma(t, cb, acc);
    if (GRAD) {
      const double dt = 1.0 - t * t;
      a0 = Mfma<double>::mma(dt * w0, cb, a0);
      a1 = Mfma<double>::mma(dt * w1, cb, a1);
    }
  }
  const int r = 16 * g + lr;
  if (r >= nrhs) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const long long p = p0 + Mfma<double>::drow(lane, v);
    if (p >= pend) continue;
    const long long e = perm[p];
    u[(size_t)r * npts + e] = acc[v];
    if (GRAD) {
      grad[((size_t)r * npts + e) * 2] = a0[v] / hx;
      grad[((size_t)r * npts + e) * 2 + 1] = a1[v] / hy;
    }
  }
}

}  // namespace ddelm
