// Solve-time kernels: the interface operator of eq. nn-mixed in local
// (per-subdomain) form, the right-hand side, CG updates and recovery.
//
// Per subdomain i, with the local interface ordered [Pi^i; Delta^i] and
// Q_G the rows of Q_i (K_c^i = Q_i R_i) at the interface rows:
//   G_i = I - Q_G Q_G^T                      (interface block of I - K K^+)
//   L_i = A_m^i R_i^{-1} Q_G^T = A_m^i K^{i+} E_G   (local Dirichlet-to-Neumann)
//   N_i = Abar^i Kbar^{i+} E_flux            (local Neumann-to-Dirichlet)
// With v_i the Delta values of subdomain i, the operator of eq. nn-mixed is
//   S v = sum_i R_D^T [ G_DD v_i - G_DP (mu + nu)_i + L_PD^T (e + e')_i + L_DD^T eta_i ]
// where   [mu; e]  = X1 [sum R_P^T G_PD v_i ; sum R_P^T L_PD v_i]
//          lambda  = sum R_D^T (L_DD v_i - L_DP mu_i)          (= D~ v)
//          eta     = theta P^T P lambda + (1-theta) lambda,  P = -sum R_D^T N_i R_D
//         [nu; e'] = X1[:, :nP] sum R_P^T L_DP^T eta_i
// and X1 = [[S^-1, S^-1 D^T], [-D S^-1, I - D S^-1 D^T]], D = D_PiPi,
// S = S_Pi.  The right-hand side of eq. nn-mixed has the same structure
// with the first-stage local vectors replaced by those of f (see rhs_*).
#pragma once
#include "kernels_common.hpp"

namespace ddelm {

template <typename T>
struct OpArgs {
  int N, nP, nD, nrhs;
  int sumP, sumD;
  double theta;
  const int* pi_off;       // [N+1]
  const int* dl_off;       // [N+1]
  const int* pi_l2g;       // [sumP]
  const int* dl_l2g;       // [sumD]
  const int* pi_own_ptr;   // [nP+1]
  const int* pi_own_slot;
  const int* dl_own_ptr;   // [nD+1]
  const int* dl_own_slot;
  const long long* offG;   // [N] offsets of G, L, LT (n_G^2 each)
  const long long* offN;   // [N] offsets of N, NT (n_D^2 each)
  const T* Gm;
  const T* Lm;
  const T* LTm;
  const T* Nm;
  const T* NTm;
  const double* X1;        // (2 nP)^2, column-major
  // local work vectors, [nrhs][sumD] or [nrhs][sumP]
  double* s_loc;
  double* l_loc;
  double* rho_loc;
  double* psi_loc;
  double* lam_loc;
  double* y_loc;
  double* z_loc;
  double* t_loc;
  double* nu_loc;
  double* w_loc;
  double* c1;              // [nrhs][2 nP]: mu_Pi, e
  double* c2;              // [nrhs][2 nP]: nu, -D nu
  const double* hP;        // optional [nrhs][nP] flux right-hand side at Pi (may be null)
  const double* hD;        // optional [nrhs][nD] at Delta (may be null)
};

// LDS needed by the local phases: 2 * max n_G doubles + reductions.
// The local stages below take the right-hand sides r0 .. r0 + nr - 1 (nr <=
// P) of one subdomain i together: the gathered vectors sit in LDS as
// [point][P], so every element of a local operator read from memory serves
// all of them.

// ---------------------------------------------------------------- stage 1
// s = G_DD v_i, l = L_DD v_i (Delta slots), rho = G_PD v_i, psi = L_PD v_i (Pi slots).
template <typename T, int P>
__device__ void ph_local_v(const OpArgs<T>& a, const double* __restrict__ v, int i, int r0, int nr, double* sm) {
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
  const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  double* vs = sm;
  for (int e = threadIdx.x; e < nd * P; e += kBlock) {
    const int k = e / P, j = e % P;
    vs[e] = j < nr ? v[(size_t)(r0 + j) * a.nD + a.dl_l2g[d0 + k]] : 0.0;
  }
  __syncthreads();
  const T* G = a.Gm + a.offG[i];
  const T* L = a.Lm + a.offG[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double sg[P], sl[P];
#pragma unroll
    for (int j = 0; j < P; ++j) sg[j] = sl[j] = 0.0;
    for (int b = 0; b < nd; ++b) {
      const long long e = (long long)(np + b) * ng + t;
      const double g = (double)G[e], l = (double)L[e];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        sg[j] += g * vs[b * P + j];
        sl[j] += l * vs[b * P + j];
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      const int r = r0 + j;
      if (t < np) {
        a.rho_loc[(size_t)r * a.sumP + p0 + t] = sg[j];
        a.psi_loc[(size_t)r * a.sumP + p0 + t] = sl[j];
      } else {
        a.s_loc[(size_t)r * a.sumD + d0 + t - np] = sg[j];
        a.l_loc[(size_t)r * a.sumD + d0 + t - np] = sl[j];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- coarse stages
// out[r][row] = sum_q X1[row][q] u[q] for rows [row0, row0+nrows_here), with
// u = [sum_owners A; sum_owners B (+ h)] (ncol_in = 2 nP) or u = sum_owners A
// (ncol_in = nP, first block column of X1).
__device__ void ph_coarse(int nP, const int* __restrict__ own_ptr, const int* __restrict__ own_slot,
                          const double* __restrict__ X1, const double* __restrict__ Aloc,
                          const double* __restrict__ Bloc, const double* __restrict__ h, int sumP, int r,
                          int row_block, double* __restrict__ out, double sign_bottom, double* sm) {
  const int nin = Bloc ? 2 * nP : nP;
  double* u = sm;
  for (int p = threadIdx.x; p < nP; p += kBlock) {
    double sa = 0.0, sb = 0.0;
    for (int e = own_ptr[p]; e < own_ptr[p + 1]; ++e) {
      sa += Aloc[(size_t)r * sumP + own_slot[e]];
      if (Bloc) sb += Bloc[(size_t)r * sumP + own_slot[e]];
    }
    u[p] = sa;
    if (Bloc) u[nP + p] = sb + (h ? h[(size_t)r * nP + p] : 0.0);
  }
  __syncthreads();
  const int ld = 2 * nP;
  const int row = row_block * kBlock + threadIdx.x;
  if (row < 2 * nP) {
    double acc = 0.0;
    for (int q = 0; q < nin; ++q) acc += X1[(long long)q * ld + row] * u[q];
    out[(size_t)r * ld + row] = row < nP ? acc : sign_bottom * acc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- stage 3
// lam_loc = l - L_DP mu_i
template <typename T>
__device__ void ph_local_lam(const OpArgs<T>& a, int i, int r) {
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
  const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  const T* L = a.Lm + a.offG[i];
  const double* mu = a.c1 + (size_t)r * 2 * a.nP;
  for (int t = threadIdx.x; t < nd; t += kBlock) {
    double acc = a.l_loc[(size_t)r * a.sumD + d0 + t];
    for (int b = 0; b < np; ++b) acc -= (double)L[(long long)b * ng + np + t] * mu[a.pi_l2g[p0 + b]];
    a.lam_loc[(size_t)r * a.sumD + d0 + t] = acc;
  }
}

// gather-sum of a local Delta vector at the Delta points of subdomain i
__device__ __forceinline__ double dl_sum(const int* __restrict__ own_ptr, const int* __restrict__ own_slot,
                                         const double* __restrict__ loc, int g) {
  double s = 0.0;
  for (int e = own_ptr[g]; e < own_ptr[g + 1]; ++e) s += loc[own_slot[e]];
  return s;
}

// ---------------------------------------------------------------- stages 4 and 5
// out = -B_i (sum over owners of src at the Delta points of i):
//   y = -N_i lambda_i (B = N, src = lam_loc) and z = -N_i^T (P lambda)_i (B = N^T, src = y_loc)
template <typename T, int P>
__device__ void ph_local_N(const OpArgs<T>& a, const T* __restrict__ B, const double* __restrict__ src,
                           double* __restrict__ out, int i, int r0, int nr, double* sm) {
  const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  double* ls = sm;
  for (int e = threadIdx.x; e < nd * P; e += kBlock) {
    const int k = e / P, j = e % P;
    ls[e] = j < nr ? dl_sum(a.dl_own_ptr, a.dl_own_slot, src + (size_t)(r0 + j) * a.sumD, a.dl_l2g[d0 + k]) : 0.0;
  }
  __syncthreads();
  const T* Bi = B + a.offN[i];
  for (int t = threadIdx.x; t < nd; t += kBlock) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = 0.0;
    for (int b = 0; b < nd; ++b) {
      const double m = (double)Bi[(long long)b * nd + t];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] += m * ls[b * P + j];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      out[(size_t)(r0 + j) * a.sumD + d0 + t] = -acc[j];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- stage 6
// eta = theta P^T P lambda + (1-theta) lambda at the Delta points of i;
// nu_loc = L_DP^T eta (Pi slots), t = L_DD^T eta (Delta slots).
// With theta == 0 the Neumann-Neumann stages are skipped and eta = lambda.
template <typename T, int P>
__device__ void ph_local_eta(const OpArgs<T>& a, int i, int r0, int nr, double* sm) {
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
  const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  double* es = sm;
  for (int e = threadIdx.x; e < nd * P; e += kBlock) {
    const int k = e / P, j = e % P;
    double val = 0.0;
    if (j < nr) {
      const int g = a.dl_l2g[d0 + k];
      const double l = dl_sum(a.dl_own_ptr, a.dl_own_slot, a.lam_loc + (size_t)(r0 + j) * a.sumD, g);
      if (a.theta != 0.0) {
        const double pp = dl_sum(a.dl_own_ptr, a.dl_own_slot, a.z_loc + (size_t)(r0 + j) * a.sumD, g);
        val = a.theta * pp + (1.0 - a.theta) * l;
      } else {
        val = l;
      }
    }
    es[e] = val;
  }
  __syncthreads();
  const T* LT = a.LTm + a.offG[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = 0.0;
    for (int b = 0; b < nd; ++b) {
      const double m = (double)LT[(long long)(np + b) * ng + t];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] += m * es[b * P + j];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j >= nr) break;
      const int r = r0 + j;
      if (t < np) a.nu_loc[(size_t)r * a.sumP + p0 + t] = acc[j];
      else a.t_loc[(size_t)r * a.sumD + d0 + t - np] = acc[j];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- stage 8
// w_loc = s + t - G_DP (mu + nu) + L_PD^T (e + e')
template <typename T>
__device__ void ph_local_w(const OpArgs<T>& a, int i, int r) {
  const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
  const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
  const int ng = np + nd;
  const T* G = a.Gm + a.offG[i];
  const T* LT = a.LTm + a.offG[i];
  const double* c1 = a.c1 + (size_t)r * 2 * a.nP;
  const double* c2 = a.c2 + (size_t)r * 2 * a.nP;
  for (int t = threadIdx.x; t < nd; t += kBlock) {
    double acc = a.s_loc[(size_t)r * a.sumD + d0 + t] + a.t_loc[(size_t)r * a.sumD + d0 + t];
    for (int b = 0; b < np; ++b) {
      const int q = a.pi_l2g[p0 + b];
      acc -= (double)G[(long long)b * ng + np + t] * (c1[q] + c2[q]);
      acc += (double)LT[(long long)b * ng + np + t] * (c1[a.nP + q] + c2[a.nP + q]);
    }
    a.w_loc[(size_t)r * a.sumD + d0 + t] = acc;
  }
}

// ---------------------------------------------------------------- phase kernels (one launch each)
// Launched on (N, ceil(nrhs / P)) workgroups with P * (max n_G or 2 nP) doubles of LDS.
template <typename T, int P>
__global__ void __launch_bounds__(kBlock) k_ph_local_v(OpArgs<T> a, const double* __restrict__ v, int nrhs) {
  extern __shared__ double sm[];
  const int r0 = blockIdx.y * P;
  ph_local_v<T, P>(a, v, blockIdx.x, r0, min(P, nrhs - r0), sm);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_ph_coarse1(OpArgs<T> a) {
  extern __shared__ double sm[];
  ph_coarse(a.nP, a.pi_own_ptr, a.pi_own_slot, a.X1, a.rho_loc, a.psi_loc, a.hP, a.sumP, blockIdx.y, blockIdx.x,
            a.c1, 1.0, sm);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_ph_lam(OpArgs<T> a) { ph_local_lam(a, blockIdx.x, blockIdx.y); }

template <typename T, int P>
__global__ void __launch_bounds__(kBlock) k_ph_P1(OpArgs<T> a, int nrhs) {
  extern __shared__ double sm[];
  const int r0 = blockIdx.y * P;
  ph_local_N<T, P>(a, a.Nm, a.lam_loc, a.y_loc, blockIdx.x, r0, min(P, nrhs - r0), sm);
}

template <typename T, int P>
__global__ void __launch_bounds__(kBlock) k_ph_P2(OpArgs<T> a, int nrhs) {
  extern __shared__ double sm[];
  const int r0 = blockIdx.y * P;
  ph_local_N<T, P>(a, a.NTm, a.y_loc, a.z_loc, blockIdx.x, r0, min(P, nrhs - r0), sm);
}

template <typename T, int P>
__global__ void __launch_bounds__(kBlock) k_ph_eta(OpArgs<T> a, int nrhs) {
  extern __shared__ double sm[];
  const int r0 = blockIdx.y * P;
  ph_local_eta<T, P>(a, blockIdx.x, r0, min(P, nrhs - r0), sm);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_ph_coarse2(OpArgs<T> a) {
  extern __shared__ double sm[];
  ph_coarse(a.nP, a.pi_own_ptr, a.pi_own_slot, a.X1, a.nu_loc, nullptr, nullptr, a.sumP, blockIdx.y, blockIdx.x,
            a.c2, 1.0, sm);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_ph_w(OpArgs<T> a) { ph_local_w(a, blockIdx.x, blockIdx.y); }

// w[r][g] = sum over owners of w_loc (+ optional hD), one thread per (g, r)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ph_sum_w(OpArgs<T> a, double* __restrict__ w) {
  const int g = blockIdx.x * kBlock + threadIdx.x, r = blockIdx.y;
  if (g >= a.nD) return;
  w[(size_t)r * a.nD + g] = dl_sum(a.dl_own_ptr, a.dl_own_slot, a.w_loc + (size_t)r * a.sumD, g);
}

// ---------------------------------------------------------------- CG
struct CGState {
  double* x;        // [nrhs][n]
  double* r;
  double* p;
  double* w;
  double* part;     // [nrhs][nblk] block partial sums
  double* scal;     // [nrhs][8]: 0 rr, 1 bb, 2 pw, 3 alpha, 4 beta, 5 done flag, 6 iters
  int n, nrhs, nblk;
  double tol;
  int maxit;
  const double* bref;   // [nrhs] squared norm the stopping test is relative to (null: ||r_0||^2)
};

// partial dot products of two vectors, one block per (chunk, rhs)
__device__ void cg_partial_dot(const double* __restrict__ x, const double* __restrict__ y, int n, int nblk, int blk,
                               int r, double* __restrict__ part, double* red) {
  double s = 0.0;
  for (int g = blk * kBlock + threadIdx.x; g < n; g += nblk * kBlock) s += x[(size_t)r * n + g] * y[(size_t)r * n + g];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(size_t)r * nblk + blk] = s;
}

__device__ double cg_reduce_parts(const double* __restrict__ part, int nblk, int r, double* red) {
  double s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kBlock) s += part[(size_t)r * nblk + k];
  return block_sum(s, red);
}

}  // namespace ddelm
