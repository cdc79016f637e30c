// Setup-time kernels: feature assembly, batched Householder QR, triangular
// solves, small batched GEMMs, coarse assembly, Cholesky and inverse.
#pragma once
#include "tanh_fast.hpp"
#include "geometry.hpp"
#include "kernels_common.hpp"

namespace ddelm {

// ---------------------------------------------------------------- features
//
// Row r of a local matrix of subdomain i is  sum_terms wgt * op(phi_j)(x),
// phi_j(x) = tanh(w_j . xi + b_j), xi = ((x - cx)/hx, (y - cy)/hy):
//   value      t
//   -Laplace   2 t (1 - t^2) (w0^2/hx^2 + w1^2/hy^2)
//   flux       (1 - t^2) (w0 nx/hx + w1 ny/hy)
// With a coefficient rho (operator -div(rho grad u), sec. 4.3) an interior
// row is rho (-Laplace phi) - grad rho . grad phi, grad phi = (1 - t^2)
// (w0/hx, w1/hy), and a flux term is multiplied by rho at its point, looked up
// by the term's global interface index.
// Output: column-major, element (r, j) at out[off[i] + j*ld[i] + r].
struct FeatArgs {
  int lead;              // implicit interior rows per subdomain (-Laplace at xint)
  const double* xint;    // [N][lead][2]
  const int* row0;       // [N+1] first stored row
  const int* ptr;        // [stored rows+1]
  const Term* terms;
  const double* W;       // [N][M][2]
  const double* bias;    // [N][M]
  const double* geom;    // [N][4]: cx, cy, hx, hy
  const long long* off;  // [N]
  const int* ld;         // [N]
  int M;
  int sub0;              // first subdomain of this launch
  const double* rho_int;   // [N][lead][3] rho, d rho/dx, d rho/dy at xint, or nullptr (rho = 1)
  const double* rho_iface; // [#Pi + #Delta] rho at the interface points, or nullptr
  const int* first_row;    // [N] rows below it are not assembled, or nullptr (all rows)
};

// One feature value of a stored-row term, t = tanh(w . xi + b) at the term's point.
__device__ __forceinline__ double term_value(const FeatArgs& a, const Term& tm, double t, double gx, double gy,
                                             double lap) {
  const double dt = 1.0 - t * t;
  if (tm.op == OP_VALUE) return t;
  if (tm.op == OP_NEG_LAPLACE) return 2.0 * t * dt * lap;
  const double v = dt * (gx * tm.nx + gy * tm.ny);
  return a.rho_iface ? a.rho_iface[tm.iface] * v : v;
}

// Rows with more terms than this (the mean-flux rows at the corners, 2(p-1)
// terms) are left to k_features_long, which spreads a row's terms over the
// lanes of a wave instead of looping over them in one thread.
constexpr int kLongTerms = 8;

constexpr int kFeatCols = 8;   // neurons per wave in k_features

template <typename T>
__global__ void __launch_bounds__(kBlock) k_features(FeatArgs a, T* __restrict__ out) {
  // A wave takes 64 consecutive rows and kFeatCols consecutive neurons: the
  // row's data (point, coefficient, term range) is read once for all of its
  // neurons and each neuron's weights are wave-uniform; every element is
  // computed with the same operations as one element per thread would be.
  const int i = a.sub0 + blockIdx.z;
  const int r = blockIdx.x * 64 + (threadIdx.x & 63);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j0 = (blockIdx.y * kWaves + wv) * kFeatCols;
  const int nrows = a.lead + a.row0[i + 1] - a.row0[i];
  if (r >= nrows || j0 >= a.M || (a.first_row && r < a.first_row[i])) return;
  const int j1 = min(j0 + kFeatCols, a.M);
  const double cx = a.geom[4 * i], cy = a.geom[4 * i + 1], hx = a.geom[4 * i + 2], hy = a.geom[4 * i + 3];
  T* o = out + a.off[i] + (long long)j0 * a.ld[i] + r;
  const long long ldo = a.ld[i];
  const double* Wi = a.W + (size_t)i * a.M * 2;
  const double* bi = a.bias + (size_t)i * a.M;
  if (r < a.lead) {            // interior row: -Laplace(phi) at the interior point
    const double px = a.xint[((size_t)i * a.lead + r) * 2], py = a.xint[((size_t)i * a.lead + r) * 2 + 1];
    const double xs = (px - cx) / hx, ys = (py - cy) / hy;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    if (a.rho_int) {
      const double* q = a.rho_int + ((size_t)i * a.lead + r) * 3;
      q0 = q[0]; q1 = q[1]; q2 = q[2];
    }
    for (int j = j0; j < j1; ++j, o += ldo) {
      const double w0 = Wi[2 * j], w1 = Wi[2 * j + 1], bj = bi[j];
      const double gx = w0 / hx, gy = w1 / hy;
      const double lap = gx * gx + gy * gy;
      const double t = tanh_fast(w0 * xs + w1 * ys + bj);
      const double dt = 1.0 - t * t;
      double v = 2.0 * t * dt * lap;
      if (a.rho_int) v = q0 * v - dt * (q1 * gx + q2 * gy);
      *o = (T)v;
    }
    return;
  }
  const int row = a.row0[i] + r - a.lead;
  const int q0 = a.ptr[row], q1 = a.ptr[row + 1];
  if (q1 - q0 > kLongTerms) return;
  for (int j = j0; j < j1; ++j, o += ldo) {
    const double w0 = Wi[2 * j], w1 = Wi[2 * j + 1], bj = bi[j];
    const double gx = w0 / hx, gy = w1 / hy;
    const double lap = gx * gx + gy * gy;
    double acc = 0.0;
    for (int q = q0; q < q1; ++q) {
      const Term tm = a.terms[q];
      const double t = tanh_fast(w0 * ((tm.x - cx) / hx) + w1 * ((tm.y - cy) / hy) + bj);
      acc += tm.wgt * term_value(a, tm, t, gx, gy, lap);
    }
    *o = (T)acc;
  }
}

// Rows with many terms: list[k] = (subdomain, local row) for k < nlong (all
// in this launch's subdomains).  Block (k, column group): wave w takes column
// j = 4 * blockIdx.y + w, its lanes the row's terms, then a wave sum.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_features_long(FeatArgs a, const int* __restrict__ list, T* __restrict__ out) {
  const int i = list[2 * blockIdx.x], r = list[2 * blockIdx.x + 1];
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= a.M) return;
  const double cx = a.geom[4 * i], cy = a.geom[4 * i + 1], hx = a.geom[4 * i + 2], hy = a.geom[4 * i + 3];
  const double w0 = a.W[((size_t)i * a.M + j) * 2], w1 = a.W[((size_t)i * a.M + j) * 2 + 1];
  const double bj = a.bias[(size_t)i * a.M + j];
  const double gx = w0 / hx, gy = w1 / hy;
  const double lap = gx * gx + gy * gy;
  const int row = a.row0[i] + r - a.lead;
  double acc = 0.0;
  for (int q = a.ptr[row] + lane; q < a.ptr[row + 1]; q += 64) {
    const Term tm = a.terms[q];
    const double t = tanh_fast(w0 * ((tm.x - cx) / hx) + w1 * ((tm.y - cy) / hy) + bj);
    acc += tm.wgt * term_value(a, tm, t, gx, gy, lap);
  }
  acc = wave_sum(acc);
  if (lane == 0) out[a.off[i] + (long long)j * a.ld[i] + r] = (T)acc;
}

// ---------------------------------------------------------------- Householder QR
//
// A batch of column-major matrices.  Reflector j of matrix b lives below the
// diagonal of column j (v_j[j] = 1 implicit), tau[b][j] its scale, so that
// H_j = I - tau_j v_j v_j^T and K = H_0 H_1 ... H_{M-1} [R; 0].
struct QRDesc {
  long long off;   // element offset of the matrix
  int m;           // rows
  int ld;          // leading dimension
  int ncols;       // columns stored (factored columns first)
  int nrefl;       // reflectors (= factored columns)
  long long tau;   // offset into tau
  int zhi;         // rows (j, zhi) of column j are zero and stay zero (an upper
                   // triangle on top of dense rows); 0 when there is no such band
};

// Reduced matrices of the two-stage QR.  Matrix b (K_c^i for b < N, Kbar^i
// for b >= N, i = b mod N) is the (M + n_G) x ncols matrix [R1 0; G E]: R1
// the upper triangle of the first-stage factor (rows 0..M-1 of the K_c^i
// features after their QR over the first t_i rows), G the interface rows of
// the full features (rows t_i.. of K_c^i, or of Kbar^i in kbfull, same
// layout), E the unit columns of the interface rows (K_c^i) or of the flux
// rows (Kbar^i, from its row n_P of G on: uoff).
template <typename T>
__global__ void k_stage2_assemble(const QRDesc* __restrict__ d2, const QRDesc* __restrict__ d1, int N, int M,
                                  const int* __restrict__ uoff, const T* __restrict__ top,
                                  const T* __restrict__ kbfull, T* __restrict__ A) {
  const int b = blockIdx.y, i = b % N;
  const QRDesc d = d2[b], t = d1[i];
  const T* full = b < N ? top : kbfull;
  // columns over the workgroups, rows over the threads (no index division)
  for (int col = blockIdx.x; col < d.ncols; col += gridDim.x) {
    T* dst = A + d.off + (long long)col * d.ld;
    for (int row = threadIdx.x; row < d.ld; row += kBlock) {
      T v;
      if (col < M) {
        if (row < M) v = row <= col ? top[t.off + (long long)col * t.ld + row] : T(0);
        else v = full[t.off + (long long)col * t.ld + t.m + (row - M)];
      } else {
        v = row == M + uoff[b] + (col - M) ? T(1) : T(0);
      }
      dst[row] = v;
    }
  }
}

// Condition estimate of a triangular factor from its diagonal: for matrix b,
// out[b] = max_j |R_jj| / min_j |R_jj| over the nrefl diagonal entries of the
// factored matrix (infinity when a diagonal entry is zero).  One workgroup
// per matrix.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_diag_ratio(const QRDesc* __restrict__ desc, const T* __restrict__ A,
                                                       double* __restrict__ out) {
  __shared__ double red[kWaves];
  const QRDesc d = desc[blockIdx.x];
  double mx = 0.0, mn = INFINITY;
  for (int j = threadIdx.x; j < d.nrefl; j += kBlock) {
    const double v = fabs((double)A[d.off + (long long)j * d.ld + j]);
    mx = fmax(mx, v);
    mn = fmin(mn, v);
  }
  // max and min through the sum helper's storage: one value per wave
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    mn = fmin(mn, __shfl_xor(mn, o, 64));
  }
  __shared__ double rmn[kWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { red[wid] = mx; rmn[wid] = mn; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kWaves; ++k) { mx = fmax(mx, red[k]); mn = fmin(mn, rmn[k]); }
    mx = fmax(mx, red[0]);
    mn = fmin(mn, rmn[0]);
    out[blockIdx.x] = mn > 0.0 ? mx / mn : INFINITY;
  }
}

// Zero the columns after the factored ones (the appended unit columns) of
// every matrix; the factored columns are written in full by the feature
// assembly.  blockIdx.y = matrix.
template <typename T>
__global__ void k_zero_appended(const QRDesc* __restrict__ desc, T* __restrict__ A) {
  const QRDesc d = desc[blockIdx.y];
  const long long beg = d.off + (long long)d.ld * d.nrefl, n = (long long)d.ld * (d.ncols - d.nrefl);
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock)
    A[beg + e] = T(0);
}

// ---------------------------------------------------------------- triangular solves
//
// X <- R^{-1} X (trans = 0) or R^{-T} X (trans = 1) for the n x n upper
// triangle R of matrix b (R at A + desc.off, leading dimension desc.ld,
// n = desc.nrefl), X = n x nc columns at X + xoff[b], leading dimension
// ldx[b].  Up to kTRSMC columns per workgroup, staged in LDS.
constexpr int kTRSMC = 8;    // right-hand-side columns per workgroup
constexpr int kTRB = 16;     // rows per block of the substitution

template <typename T, int kTRSMC>
__global__ void __launch_bounds__(kBlock, 4) k_trsm(const QRDesc* __restrict__ desc, const T* __restrict__ A,
                                                 T* __restrict__ X, const long long* __restrict__ xoff,
                                                 const int* __restrict__ ldx, const int* __restrict__ xn,
                                                 int trans, int nmat, int ntile) {
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);          // [kTRSMC][n]: a column per RHS, rows along the lanes
  // 1-D grid over (matrix, column tile), arranged so that all tiles of one
  // matrix land on the same XCD (workgroup id mod 8) close together in
  // time: R is read from memory once and then from that XCD's L2
  const int id = blockIdx.x;
  const int b = (id % 8) + 8 * ((id / 8) / ntile);
  const int tile = (id / 8) % ntile;
  if (b >= nmat) return;
  const QRDesc d = desc[b];
  const int n = d.nrefl;
  const int cbeg = tile * kTRSMC;
  const int ctot = xn[b];
  if (cbeg >= ctot) return;
  const int nc = min(kTRSMC, ctot - cbeg);
  const T* R = A + d.off;
  T* Xm = X + xoff[b];
  const int L = ldx[b];
  {
    constexpr int kU = 8;      // loads issued together per thread
    for (int e0 = threadIdx.x; e0 < n * kTRSMC; e0 += kU * kBlock) {
      T v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * kBlock, c = e / n, r = e % n;
        v[u] = (e < n * kTRSMC && c < nc) ? Xm[(long long)(cbeg + c) * L + r] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (e0 + u * kBlock < n * kTRSMC) xs[e0 + u * kBlock] = v[u];
    }
  }
  __syncthreads();
  // Substitution by blocks of kTRB rows.  The diagonal block is staged in
  // LDS with the reciprocals of its diagonal, and solved by kTRSMC lanes of
  // the first wave, one column each, with the block's unknowns in registers
  // and column by column (each solved unknown is removed from all remaining
  // rows at once), so the dependent chain is one multiply and one
  // multiply-add per row rather than a row-long sum and a division.  Then
  // every thread takes one row not yet solved: its kTRB entries of R are
  // loaded in one batch and applied to all columns (the solved values are
  // broadcast from LDS).
  __shared__ T Rd[kTRB][kTRB + 1];
  __shared__ T rinv[kTRB];
  const int nblk = (n + kTRB - 1) / kTRB;
  for (int s = 0; s < nblk; ++s) {
    const int bk = trans ? s : nblk - 1 - s;
    const int r0 = bk * kTRB, r1 = min(n, r0 + kTRB), nb = r1 - r0;
    for (int e = threadIdx.x; e < kTRB * kTRB; e += kBlock) {
      const int i = e % kTRB, j = e / kTRB;             // Rd[i][j] = R(r0 + i, r0 + j)
      const T v = (i < nb && j < nb) ? R[(long long)(r0 + j) * d.ld + r0 + i] : (i == j ? T(1) : T(0));
      Rd[i][j] = v;
      if (i == j) rinv[i] = T(1) / v;
    }
    __syncthreads();
    if (threadIdx.x < kTRSMC) {
      const int c = threadIdx.x;
      T x[kTRB];
#pragma unroll
      for (int k = 0; k < kTRB; ++k) x[k] = k < nb ? xs[c * n + r0 + k] : T(0);
      // rows past the end of R have a unit diagonal and zero coupling, so they stay 0
      if (!trans) {
#pragma unroll
        for (int k = kTRB - 1; k >= 0; --k) {
          x[k] *= rinv[k];
#pragma unroll
          for (int j = 0; j < k; ++j) x[j] -= Rd[j][k] * x[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < kTRB; ++k) {
          x[k] *= rinv[k];
#pragma unroll
          for (int j = k + 1; j < kTRB; ++j) x[j] -= Rd[k][j] * x[k];
        }
      }
#pragma unroll
      for (int k = 0; k < kTRB; ++k)
        if (k < nb) xs[c * n + r0 + k] = x[k];
    }
    __syncthreads();
    // rows still to solve: above the block (back substitution) or below it (forward)
    const int u0 = trans ? r1 : 0, u1 = trans ? n : r0;
    for (int r = u0 + threadIdx.x; r < u1; r += kBlock) {
      // one address per element, chosen before the load: two alternative
      // loads into one register would make each wait for the previous one
      const T* rp = trans ? R + (long long)r * d.ld + r0 : R + (long long)r0 * d.ld + r;
      const long long rs = trans ? 1 : d.ld;
      T rv[kTRB];
#pragma unroll
      for (int j = 0; j < kTRB; ++j) rv[j] = j < nb ? rp[j * rs] : T(0);
#pragma unroll
      for (int c = 0; c < kTRSMC; ++c) {
        T acc = xs[c * n + r];
#pragma unroll
        for (int j = 0; j < kTRB; ++j)
          if (j < nb) acc -= rv[j] * xs[c * n + r0 + j];   // rows past n are not in xs
        xs[c * n + r] = acc;
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * kTRSMC; e += kBlock) {
    const int c = e / n, r = e % n;
    if (c < nc) Xm[(long long)(cbeg + c) * L + r] = xs[e];
  }
}

// ---------------------------------------------------------------- batched GEMM
//
// C = alpha * op(A) * B + beta * C, all column-major; op(A) = A (m x k) or
// A^T (A stored k x m).  The kernel (k_gemm_mfma) is with the other MFMA
// kernels.
struct GemmDesc {
  long long a, b, c;     // element offsets
  int lda, ldb, ldc;
  int m, n, k;
};

// ---------------------------------------------------------------- small helpers

// dst[b] (rows x cols, ld_dst) <- src[b] rows [r0, r0+rows), cols [c0, c0+cols)
// (ld_src); optional transpose.  One launch per batch via blockIdx.z.
struct CopyDesc {
  long long src, dst;
  int lds, ldd;
  int rows, cols;
  int trans;
  int pad;
};

template <typename TS, typename TD>
__global__ void __launch_bounds__(kBlock) k_copy2d(const CopyDesc* __restrict__ desc, const TS* __restrict__ S,
                                                   TD* __restrict__ D) {
  const CopyDesc c = desc[blockIdx.y];
  // columns over the workgroups, rows over the threads (no index division)
  for (int col = blockIdx.x; col < c.cols; col += gridDim.x)
    for (int r = threadIdx.x; r < c.rows; r += kBlock) {
      const TS v = S[c.src + (long long)col * c.lds + r];
      if (c.trans) D[c.dst + (long long)r * c.ldd + col] = (TD)v;
      else D[c.dst + (long long)col * c.ldd + r] = (TD)v;
    }
}

#ifndef DDELM_KERNEL_SUBSET   // plain kernels: defined once, in the unit that launches them
// Interior points must lie in the closed box of their subdomain
// (box[4 i .. 4 i + 3] = x0, x1, y0, y1); *first_bad becomes the lowest
// subdomain index with a point outside (or a NaN coordinate).  It starts at
// 0xffffffff.
__global__ void k_check_interior(const double* __restrict__ x, const double* __restrict__ box, int N, int n_int,
                                 unsigned* __restrict__ first_bad) {
  const long long n = (long long)N * n_int;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock) {
    const int i = (int)(e / n_int);
    const double px = x[2 * e], py = x[2 * e + 1];
    const double* b = box + 4 * (size_t)i;
    if (!(px >= b[0] && px <= b[1] && py >= b[2] && py <= b[3])) atomicMin(first_bad, (unsigned)i);
  }
}

#endif

// Zero several buffers in one launch: blockIdx.y = buffer, n in 32-bit words.
constexpr int kZeroMax = 24;
struct ZeroList {
  unsigned* p[kZeroMax];
  long long n[kZeroMax];
};
#ifndef DDELM_KERNEL_SUBSET   // plain kernels: defined once, in the unit that launches them
__global__ void k_zero_many(ZeroList z) {
  unsigned* __restrict__ p = z.p[blockIdx.y];
  const long long n = z.n[blockIdx.y];
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock) p[e] = 0u;
}

__global__ void k_fill(double* __restrict__ p, long long n, double v) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock) p[e] = v;
}
#endif

// identity blocks: for each batch entry, add `v` on the diagonal of an n x n
// block at off (column-major, ld = n)
template <typename T>
__global__ void k_add_diag_t(const long long* __restrict__ off, const int* __restrict__ n, T* __restrict__ P, T v) {
  const int b = blockIdx.x;
  for (int k = threadIdx.x; k < n[b]; k += kBlock) P[off[b] + (long long)k * n[b] + k] += v;
}

// ---------------------------------------------------------------- coarse problem
//
// Sum the local corner blocks into global nP x nP matrices (column-major):
//   Dpp[p][q] = sum_i L_i[a_p][a_q],  Gs[p][q] = sum_i G_i[a_p][a_q]
// over subdomains i holding both corners.  One thread per row p; owners in
// subdomain order, so the sums are deterministic.
template <typename T>
__global__ void k_coarse_assemble(int nP, const int* __restrict__ own_ptr, const int* __restrict__ own_slot,
                                  const int* __restrict__ slot_sub, const int* __restrict__ pi_off,
                                  const int* __restrict__ pi_l2g, const long long* __restrict__ offG,
                                  const int* __restrict__ nG, const T* __restrict__ Gm, const T* __restrict__ Lm,
                                  double* __restrict__ Dpp, double* __restrict__ Gs) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= nP) return;
  for (int e = own_ptr[p]; e < own_ptr[p + 1]; ++e) {
    const int slot = own_slot[e];
    const int i = slot_sub[slot];
    const int ap = slot - pi_off[i];
    const int np = pi_off[i + 1] - pi_off[i];
    const int ng = nG[i];
    for (int bq = 0; bq < np; ++bq) {
      const int q = pi_l2g[pi_off[i] + bq];
      Dpp[(long long)q * nP + p] += (double)Lm[offG[i] + (long long)bq * ng + ap];
      Gs[(long long)q * nP + p] += (double)Gm[offG[i] + (long long)bq * ng + ap];
    }
  }
}

// Blocked right-looking Cholesky (lower, column-major, in place) of the
// coarse Schur complement: for each block column k0 of width at most kCB,
// k_chol_diag factors the diagonal block in LDS, k_chol_panel solves the
// rows below against it (one thread per row), and the trailing matrix is
// updated by one GEMM (A22 -= L21 L21^T) on the host side.  Only the lower
// triangle is meaningful afterwards.  err[0] |= 2 if a pivot is not positive.
constexpr int kCB = 32;

#ifndef DDELM_KERNEL_SUBSET   // plain kernels: defined once, in the unit that launches them
__global__ void __launch_bounds__(kBlock) k_chol_diag(double* __restrict__ S, int n, int k0, int nb,
                                                      unsigned* __restrict__ err) {
  __shared__ double A[kCB][kCB + 1];   // A[col][row]
  for (int e = threadIdx.x; e < nb * nb; e += kBlock) {
    const int r = e % nb, c = e / nb;
    A[c][r] = S[(long long)(k0 + c) * n + k0 + r];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (threadIdx.x == 0) {
      double d = A[j][j];
      if (!(d > 0.0)) {
        atomicOr(err, 2u);
        d = 1.0;
      }
      A[j][j] = sqrt(d);
    }
    __syncthreads();
    const double inv = 1.0 / A[j][j];
    for (int r = j + 1 + threadIdx.x; r < nb; r += kBlock) A[j][r] *= inv;
    __syncthreads();
    const int m = nb - j - 1;
    for (int e = threadIdx.x; e < m * m; e += kBlock) {
      const int r = j + 1 + e % m, c = j + 1 + e / m;
      if (r >= c) A[c][r] -= A[j][r] * A[j][c];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nb * nb; e += kBlock) {
    const int r = e % nb, c = e / nb;
    if (r >= c) S[(long long)(k0 + c) * n + k0 + r] = A[c][r];
  }
}

// L21 = A21 L11^{-T} for the rows k0 + nb .. n-1 of block column k0
__global__ void __launch_bounds__(kBlock) k_chol_panel(double* __restrict__ S, int n, int k0, int nb) {
  __shared__ double L[kCB][kCB + 1];   // L[col][row] of the factored diagonal block
  for (int e = threadIdx.x; e < nb * nb; e += kBlock) {
    const int r = e % nb, c = e / nb;
    L[c][r] = S[(long long)(k0 + c) * n + k0 + r];
  }
  __syncthreads();
  const int r = k0 + nb + blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  double x[kCB];
#pragma unroll
  for (int j = 0; j < kCB; ++j) x[j] = j < nb ? S[(long long)(k0 + j) * n + r] : 0.0;
#pragma unroll
  for (int j = 0; j < kCB; ++j) {
    if (j < nb) {
      double v = x[j];
#pragma unroll
      for (int l = 0; l < kCB; ++l)
        if (l < j) v -= x[l] * L[l][j];
      x[j] = v / L[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < kCB; ++j)
    if (j < nb) S[(long long)(k0 + j) * n + r] = x[j];
}

// Columns of S^{-1} from the Cholesky factor (lower, column-major):
// solve L y = e_k then L^T x = y; 4 columns per workgroup, in LDS.  Both
// substitutions go by blocks of kIB rows: the block's triangle is staged in
// LDS and solved by four threads (one column each, the block's unknowns in
// registers), then every thread updates one (row, column) of the rest with
// the block's kIB solved values: three barriers per block instead of two
// per row.
constexpr int kIB = 32;
__global__ void __launch_bounds__(kBlock) k_chol_inverse(const double* __restrict__ Lf, int n,
                                                         double* __restrict__ Sinv) {
  extern __shared__ unsigned char smem_raw[];
  double* x = reinterpret_cast<double*>(smem_raw);   // [n][4]
  __shared__ double Lb[kIB][kIB + 1];                // Lb[i][j] = L(kb + i, kb + j)
  const int c0 = blockIdx.x * 4;
  for (int e = threadIdx.x; e < n * 4; e += kBlock) {
    const int r = e / 4, c = e % 4;
    x[e] = (r == c0 + c) ? 1.0 : 0.0;
  }
  const int nblk = (n + kIB - 1) / kIB;
  for (int pass = 0; pass < 2; ++pass) {          // 0: L y = e, 1: L^T x = y
    for (int q = 0; q < nblk; ++q) {
      const int bk = pass == 0 ? q : nblk - 1 - q;
      const int kb = bk * kIB, nb = min(kIB, n - kb);
      for (int e = threadIdx.x; e < kIB * kIB; e += kBlock) {
        const int i = e % kIB, j = e / kIB;
        Lb[i][j] = (i < nb && j < nb) ? Lf[(long long)(kb + j) * n + kb + i] : 0.0;
      }
      __syncthreads();
      if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        double xr[kIB];
#pragma unroll
        for (int k = 0; k < kIB; ++k) xr[k] = k < nb ? x[(kb + k) * 4 + c] : 0.0;
        if (pass == 0) {
#pragma unroll
          for (int k = 0; k < kIB; ++k) {
            if (k < nb) {
              xr[k] /= Lb[k][k];
#pragma unroll
              for (int r = k + 1; r < kIB; ++r) xr[r] -= Lb[r][k] * xr[k];
            }
          }
        } else {
#pragma unroll
          for (int k = kIB - 1; k >= 0; --k) {
            if (k < nb) {
              xr[k] /= Lb[k][k];
#pragma unroll
              for (int r = 0; r < k; ++r) xr[r] -= Lb[k][r] * xr[k];
            }
          }
        }
#pragma unroll
        for (int k = 0; k < kIB; ++k)
          if (k < nb) x[(kb + k) * 4 + c] = xr[k];
      }
      __syncthreads();
      // rows below the block (forward) or above it (backward)
      const int u0 = pass == 0 ? kb + nb : 0, u1 = pass == 0 ? n : kb;
      for (int e = u0 * 4 + threadIdx.x; e < u1 * 4; e += kBlock) {
        const int r = e / 4, c = e % 4;
        double acc = x[e];
        for (int k = 0; k < nb; ++k) {
          const double l = pass == 0 ? Lf[(long long)(kb + k) * n + r] : Lf[(long long)r * n + kb + k];
          acc -= l * x[(kb + k) * 4 + c];
        }
        x[e] = acc;
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < n * 4; e += kBlock) {
    const int r = e / 4, c = e % 4;
    if (c0 + c < n) Sinv[(long long)(c0 + c) * n + r] = x[e];
  }
}
#endif

}  // namespace ddelm
