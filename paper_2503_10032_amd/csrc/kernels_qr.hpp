// Blocked Householder QR with compact-WY updates on the matrix cores.
//
// Panels are 16 columns wide.  The panel kernel factors 16 columns held in
// registers and builds the upper-triangular T of the block reflector
//   H_k H_{k+1} ... H_{k+15} = I - V T V^T            (forward, columnwise)
// The update kernel then applies the block reflector to any set of columns,
//   C <- (I - V T^T V^T) C  (Q^T C)   or   C <- (I - V T V^T) C  (Q C),
// as W = V^T C, W <- T^T W (or T W), C <- C - V W, with both products on
// 16x16x4 MFMA (f64 or f32).  V^T C contracts over rows, which are
// contiguous in the column-major storage, so the operands of that product
// are staged through LDS; C - V W is computed transposed (rows along the
// lanes) straight from global memory.
#pragma once
#include "kernels_common.hpp"
#include "kernels_setup.hpp"

namespace ddelm {

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element v of lane l holds D[drow(l, v)][l & 15]
  __device__ static __forceinline__ int drow(int l, int v) { return (l >> 4) + 4 * v; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int drow(int l, int v) { return 4 * (l >> 4) + v; }
};
// Operands: lane l supplies A[l & 15][l >> 4] and B[l >> 4][l & 15].

constexpr int kNB = 16;   // panel width

// element (row, j) of the block reflector V of panel k of matrix Am (rows
// relative to the matrix): 0 above the diagonal, 1 on it, stored below it
template <typename T>
__device__ __forceinline__ T v_elem(const T* Am, int ld, int m, int k, int row, int j) {
  const int rr = row - k;
  if (row >= m || rr < j) return T(0);
  if (rr == j) return T(1);
  return Am[(long long)(k + j) * ld + row];
}

// Row skipping for matrices with a zero band (QRDesc::zhi): the reflectors
// of columns [k, k + w) are zero in rows [k + w, zhi), and applying them
// leaves those rows unchanged, so row loops that start at k jump from the
// band's first row to zhi.  Rows at or past zhi are left alone.
__device__ __forceinline__ int skip_band(int r, int kw, int zhi) { return (r >= kw && r < zhi) ? zhi : r; }

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (a full __syncthreads waits for them as well).
// For loops whose threads exchange data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// Row of panel-local index l (l = 0, 1, ...) for the panel of columns
// [k, k + kNB): the panel's own rows first, then the rows from zhi on.
template <int NB>
__device__ __forceinline__ int band_row(int k, int l, int zhi) { return (zhi > k + NB && l >= NB) ? zhi + (l - NB) : k + l; }

// ---------------------------------------------------------------- panel
// One workgroup of NT threads per matrix (kPanelThreads, or 256 when the
// panel has at most 256 rows); rows k + tid + q*NT.
constexpr int kPanelThreads = 512;

// Column JJ of a panel (compile-time, so each column only touches the
// columns it needs and picks its own column without selects).  One reduction
// per column: with x the current column below the diagonal (rows r > j),
// alpha = x_j and s = 1/(alpha - beta), v_j = [1; s x] and
//   v_j . a_c = a_c[j] + s sum_{r>j} x_r a_c[r]        (c > JJ, applies H_j)
//   v_c . v_j = v_c[j] + s sum_{r>j} x_r v_c[r]        (c < JJ, builds T)
// so the squared norm of x (slot JJ) and the 15 sums share one reduction.
// Sum over the panel's workgroup of kNB values per thread with a single
// barrier.  Within a wave, a reduce-scatter over each row of 16 lanes: four
// butterfly steps through DPP moves (row mirror, half-row mirror, two quad
// permutations; partners differ in lane bit 3, 2, 1, 0), in each of which
// the lane whose bit is clear keeps the lower half of its values and adds
// its partner's copy of them, so lane i of a row ends with the row's sum of
// value i (15 moves and adds per lane instead of 16 full wave reductions);
// then the four rows are added by two lane shuffles.  Lanes 0..kNB-1 write
// the wave's sums to one LDS slot per wave; every wave then adds the NW
// partial sums itself (lanes 0..kNB-1) and broadcasts them by readlane.
// `red` holds NW * kNB values (NW waves); callers alternate two buffers, so
// a wave that runs ahead cannot overwrite sums still being read.
template <typename T, int NW>
__device__ __forceinline__ void panel_sum(const T* v, T* out, T* red) {
  static_assert(kNB == 16, "one value per lane of a 16-lane row");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T a8[8], a4[4], a2[2];
  {
    const bool h = lane & 8;     // partner 15 - i
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const T snd = h ? v[j] : v[j + 8];
      a8[j] = (h ? v[j + 8] : v[j]) + dpp_move<0x140, 0xf>(snd);   // row_mirror
    }
  }
  {
    const bool h = lane & 4;     // partner 7 - i within the half row
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T snd = h ? a8[j] : a8[j + 4];
      a4[j] = (h ? a8[j + 4] : a8[j]) + dpp_move<0x141, 0xf>(snd);   // row_half_mirror
    }
  }
  {
    const bool h = lane & 2;     // partner i ^ 2
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const T snd = h ? a4[j] : a4[j + 2];
      a2[j] = (h ? a4[j + 2] : a4[j]) + dpp_move<0x4E, 0xf>(snd);   // quad_perm [2,3,0,1]
    }
  }
  T w;
  {
    const bool h = lane & 1;     // partner i ^ 1
    const T snd = h ? a2[0] : a2[1];
    w = (h ? a2[1] : a2[0]) + dpp_move<0xB1, 0xf>(snd);             // quad_perm [1,0,3,2]
  }
  w += __shfl_xor(w, 16, 64);
  w += __shfl_xor(w, 32, 64);
  if (lane < kNB) red[wid * kNB + lane] = w;
  __syncthreads();
  T s = 0;
  if (lane < kNB) {
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[k * kNB + lane];
  }
#pragma unroll
  for (int c = 0; c < kNB; ++c) {
    if constexpr (sizeof(T) == 8) {
      const int lo = __builtin_amdgcn_readlane(__double2loint(s), c);
      const int hi = __builtin_amdgcn_readlane(__double2hiint(s), c);
      out[c] = __hiloint2double(hi, lo);
    } else {
      out[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s), c));
    }
  }
}

template <typename T, int RPT, int JJ, int NT>
__device__ __forceinline__ void panel_column(const QRDesc& d, int k, T (&a)[RPT][kNB], T* red2, T* rowj2,
                                             T (&Ts)[kNB][kNB]) {
  const int j = k + JJ;
  T* red = red2 + (JJ & 1) * (NT / 64) * kNB;     // alternating buffers, see panel_sum
  T* rowj = rowj2 + (JJ & 1) * kNB;
  T part[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) part[c] = 0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = band_row<kNB>(k, threadIdx.x + q * NT, d.zhi);
    const T x = a[q][JJ];
    if (r > j && r < d.m) {
#pragma unroll
      for (int c = 0; c < kNB; ++c) part[c] += x * a[q][c];   // slot JJ: x . x
    }
    if (r == j) {
#pragma unroll
      for (int c = 0; c < kNB; ++c) rowj[c] = a[q][c];
    }
  }
  T w[kNB];
  panel_sum<T, NT / 64>(part, w, red);
  const T ss = w[JJ];
  const T alpha = rowj[JJ];
  T beta = alpha, tj = 0, scale = 0;
  if (ss > T(0)) {
    beta = -copysign(sqrt(alpha * alpha + ss), alpha);
    tj = (beta - alpha) / beta;
    scale = T(1) / (alpha - beta);
  }
#pragma unroll
  for (int c = 0; c < kNB; ++c) w[c] = rowj[c] + scale * w[c];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = band_row<kNB>(k, threadIdx.x + q * NT, d.zhi);
    if (r >= j && r < d.m) {
      const T vj = (r == j) ? T(1) : a[q][JJ] * scale;
      a[q][JJ] = (r == j) ? beta : vj;
#pragma unroll
      for (int c = JJ + 1; c < kNB; ++c) a[q][c] -= tj * w[c] * vj;
    }
  }
  // T(0:JJ, JJ) = -tau_j T(0:JJ, 0:JJ) z, z_c = v_c . v_j = w_c (c < JJ); T(JJ, JJ) = tau_j
  if (threadIdx.x < JJ) {      // thread i forms T(i, JJ)
    const int i = threadIdx.x;
    T s = 0;
#pragma unroll
    for (int c = 0; c < JJ; ++c)
      if (c >= i) s += Ts[i][c] * w[c];
    Ts[i][JJ] = -tj * s;
  }
  // (read by the next columns after their reduction's barrier)
  if (threadIdx.x == 0) Ts[JJ][JJ] = tj;
}

template <typename T, int RPT, int JJ, int NT>
__device__ __forceinline__ void panel_columns(const QRDesc& d, int k, int ncol, T (&a)[RPT][kNB], T* red, T* rowj,
                                              T (&Ts)[kNB][kNB]) {
  if constexpr (JJ < kNB) {
    if (JJ < ncol) {
      panel_column<T, RPT, JJ, NT>(d, k, a, red, rowj, Ts);
      panel_columns<T, RPT, JJ + 1, NT>(d, k, ncol, a, red, rowj, Ts);
    }
  }
}

template <typename T, int RPT, int NT>
__global__ void __launch_bounds__(NT) k_qr_panel16(const QRDesc* __restrict__ desc, T* __restrict__ A,
                                                              T* __restrict__ tau, T* __restrict__ Tbuf, int k,
                                                              int panel, int npanel) {
  const QRDesc d = desc[blockIdx.x];
  if (k >= d.nrefl) return;
  __shared__ T red[2 * (NT / 64) * kNB];
  __shared__ T rowj[2 * kNB];
  __shared__ T Ts[kNB][kNB];
  T* Am = A + d.off;
  const int ncol = min(kNB, d.nrefl - k);
  for (int e = threadIdx.x; e < kNB * kNB; e += NT) Ts[e / kNB][e % kNB] = T(0);
  T a[RPT][kNB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = band_row<kNB>(k, threadIdx.x + q * NT, d.zhi);
#pragma unroll
    for (int c = 0; c < kNB; ++c) a[q][c] = (r < d.m && c < ncol) ? Am[(long long)(k + c) * d.ld + r] : T(0);
  }
  panel_columns<T, RPT, 0, NT>(d, k, ncol, a, red, rowj, Ts);
  __syncthreads();
  if (threadIdx.x < ncol) tau[d.tau + k + threadIdx.x] = Ts[threadIdx.x][threadIdx.x];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = band_row<kNB>(k, threadIdx.x + q * NT, d.zhi);
#pragma unroll
    for (int c = 0; c < kNB; ++c)
      if (r < d.m && c < ncol) Am[(long long)(k + c) * d.ld + r] = a[q][c];
  }
  T* Tout = Tbuf + ((long long)blockIdx.x * npanel + panel) * kNB * kNB;
  for (int e = threadIdx.x; e < kNB * kNB; e += NT) Tout[e] = Ts[e / kNB][e % kNB];
}

// ---------------------------------------------------------------- block reflector application
//
// Target of matrix b: columns c0 + blockIdx.y*32 + (0..32) of C + coff[b]
// (leading dimension ldc[b], cn[b] columns in total); rows k..m-1 change.
// transT = 1 applies Q^T (I - V T^T V^T); transT = 0 applies Q (I - V T V^T).
constexpr int kUC = 32;   // columns per workgroup

// Off32: as for k_qr_wy64 below (32-bit byte offsets from the matrix start).
template <typename T, bool Off32 = false>
__global__ void __launch_bounds__(kBlock) k_qr_wy(const QRDesc* __restrict__ desc, const T* __restrict__ A,
                                                  const T* __restrict__ Tbuf, int k, int panel, int npanel,
                                                  T* __restrict__ C, const long long* __restrict__ coff,
                                                  const int* __restrict__ ldc, const int* __restrict__ cn, int c0,
                                                  int transT) {
  typedef typename Mfma<T>::v4 v4;
  const QRDesc d = desc[blockIdx.x];
  if (k >= d.nrefl) return;
  const int cbeg = c0 + blockIdx.y * kUC;
  const int ctot = cn[blockIdx.x];
  if (cbeg >= ctot) return;
  const int ncol = min(kUC, ctot - cbeg);
  const int L = ldc[blockIdx.x];
  const T* Am = A + d.off;
  T* Cm = C + coff[blockIdx.x];
  // element (row, col) of the matrix (leading dimension ld) and of C (L)
  auto aref = [&](int col, int row) -> const T& {
    if constexpr (Off32)
      return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(Am) +
                                         (unsigned)((col * d.ld + row) * (int)sizeof(T)));
    else
      return Am[(long long)col * d.ld + row];
  };
  auto cref = [&](int col, int row) -> T& {
    if constexpr (Off32)
      return *reinterpret_cast<T*>(reinterpret_cast<char*>(Cm) + (unsigned)((col * L + row) * (int)sizeof(T)));
    else
      return Cm[(long long)col * L + row];
  };
  __shared__ T Vs[64][kNB + 1];
  __shared__ T Cs[64][kUC + 1];
  __shared__ T Wp[kWaves][kNB][kUC + 1];
  __shared__ T Ts[kNB][kNB];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const T* Tin = Tbuf + ((long long)blockIdx.x * npanel + panel) * kNB * kNB;
  for (int e = threadIdx.x; e < kNB * kNB; e += kBlock) Ts[e / kNB][e % kNB] = Tin[e];
  // ---- W = V^T C over rows k..m-1, 64-row chunks staged in LDS; the loads
  //      of the next two chunks (4 V and 8 C elements per thread each, in
  //      two register sets used in turn) are in flight during this chunk's
  //      products, and the barriers order the LDS accesses only
  v4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  // every load reads an element inside the matrix (indices clamped) and the
  // value (0 or 1 above and on the diagonal, 0 past the last row or column)
  // is selected when the chunk is stored to LDS: straight-line loads whose
  // waits count only the chunk being stored
  auto load_chunk = [&](int r0, T (&vv)[4], T (&cc)[8]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + u * kBlock;
      vv[u] = aref(k + e / 64, min(r0 + e % 64, d.m - 1));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + u * kBlock;
      cc[u] = cref(cbeg + min(e / 64, ncol - 1), min(r0 + e % 64, d.m - 1));
    }
  };
  // chunk at r0 held in (vv, cc): to LDS, its products; then (vv, cc) takes
  // the chunk at rl
  auto chunk = [&](int r0, T (&vv)[4], T (&cc)[8], int rl) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const int row = r0 + e % 64, j = e / 64, rr = row - k;
      Vs[e % 64][j] = (row >= d.m || rr < j) ? T(0) : (rr == j ? T(1) : vv[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const int c = e / 64, row = r0 + e % 64;
      Cs[e % 64][c] = (row < d.m && c < ncol) ? cc[u] : T(0);
    }
    lds_barrier();
    load_chunk(min(rl, d.m), vv, cc);   // past the end: unused, no branch
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int rr = wv * 16 + ks * 4 + (lane >> 4);
      const T av = Vs[rr][lane & 15];
      acc0 = Mfma<T>::mma(av, Cs[rr][lane & 15], acc0);
      acc1 = Mfma<T>::mma(av, Cs[rr][16 + (lane & 15)], acc1);
    }
    lds_barrier();
  };
  auto next_chunk = [&](int r) { return r < d.m ? skip_band(r + 64, k + kNB, d.zhi) : d.m; };
  {
    T va[4], ca[8], vb[4], cb[8];
    int r0 = k, r1 = next_chunk(k);
    load_chunk(r0, va, ca);
    load_chunk(r1, vb, cb);
    while (r0 < d.m) {
      const int r2 = next_chunk(r1);
      chunk(r0, va, ca, r2);
      if (r1 >= d.m) break;
      const int r3 = next_chunk(r2);
      chunk(r1, vb, cb, r3);
      r0 = r2;
      r1 = r3;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = Mfma<T>::drow(lane, v);
    Wp[wv][i][lane & 15] = acc0[v];
    Wp[wv][i][16 + (lane & 15)] = acc1[v];
  }
  __syncthreads();
  // W summed over waves into Wp[0]; then Wn = -T^T W (Q^T) or -T W (Q) into Wp[1]
  for (int e = threadIdx.x; e < kNB * kUC; e += kBlock) {
    const int i = e / kUC, c = e % kUC;
    Wp[0][i][c] = Wp[0][i][c] + Wp[1][i][c] + Wp[2][i][c] + Wp[3][i][c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kNB * kUC; e += kBlock) {
    const int i = e / kUC, c = e % kUC;
    T s = 0;
    if (transT) {
      for (int ip = 0; ip <= i; ++ip) s += Ts[ip][i] * Wp[0][ip][c];
    } else {
      for (int ip = i; ip < kNB; ++ip) s += Ts[i][ip] * Wp[0][ip][c];
    }
    Wp[1][i][c] = -s;
  }
  __syncthreads();
  // ---- C^T <- C^T + Wn^T V^T for 16-row blocks (rows along the lanes); two
  //      register sets used in turn keep the loads of the next two blocks in
  //      flight during this block's products (clamped indices, values
  //      selected at use, as above)
  auto load_rows = [&](int rb, T (&cn)[8], T (&bn)[4]) {
    const int row = min(rb + (lane & 15), d.m - 1);
#pragma unroll
    for (int cg = 0; cg < 2; ++cg)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = min(cg * 16 + Mfma<T>::drow(lane, v), ncol - 1);
        cn[4 * cg + v] = cref(cbeg + c, row);
      }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) bn[ks] = aref(k + ks * 4 + (lane >> 4), row);
  };
  // block at rb held in (cn, bn): its products and stores; then (cn, bn)
  // takes the block at rl
  auto block = [&](int rb, T (&cn)[8], T (&bn)[4], int rl) {
    const int row = rb + (lane & 15), rr = row - k;
    v4 acc[2];
    T bv[4];
#pragma unroll
    for (int cg = 0; cg < 2; ++cg)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cg][v] = cn[4 * cg + v];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int j = ks * 4 + (lane >> 4);
      bv[ks] = (row >= d.m || rr < j) ? T(0) : (rr == j ? T(1) : bn[ks]);
    }
    load_rows(min(rl, d.m), cn, bn);
#pragma unroll
    for (int cg = 0; cg < 2; ++cg)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const T av = Wp[1][ks * 4 + (lane >> 4)][cg * 16 + (lane & 15)];
        acc[cg] = Mfma<T>::mma(av, bv[ks], acc[cg]);
      }
#pragma unroll
    for (int cg = 0; cg < 2; ++cg)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = cg * 16 + Mfma<T>::drow(lane, v);
        if (row < d.m && c < ncol) cref(cbeg + c, row) = acc[cg][v];
      }
  };
  // 64-row groups of the four waves, the band skipped between groups
  auto next_rb = [&](int r) {
    return r < d.m ? skip_band(r - wv * 16 + kWaves * 16, k + kNB, d.zhi) + wv * 16 : d.m;
  };
  {
    T ca[8], va[4], cb[8], vb[4];
    int r0 = k + wv * 16, r1 = next_rb(r0);
    load_rows(min(r0, d.m), ca, va);
    load_rows(min(r1, d.m), cb, vb);
    while (r0 < d.m) {
      const int r2 = next_rb(r1);
      block(r0, ca, va, r2);
      if (r1 >= d.m) break;
      const int r3 = next_rb(r2);
      block(r1, cb, vb, r3);
      r0 = r2;
      r1 = r3;
    }
  }
}

}  // namespace ddelm

namespace ddelm {

// ---------------------------------------------------------------- 64-column blocks
//
// Four 16-column panels make one block.  Inside a block each panel's
// reflector is applied only to the block's remaining columns; the four
// panel T factors are then merged into the T of the whole block,
//   Q1 Q2 = I - [V1 V2] [[T1, -T1 V1^T V2 T2], [0, T2]] [V1 V2]^T,
// and the block reflector updates the trailing matrix once per 64 columns,
// which streams it a quarter as often as panel-by-panel updates.
constexpr int kBB = 64;    // block width
constexpr int kBC = 64;    // columns of C per workgroup in the block update

// T of block blk (columns kb .. kb+bw-1) from the panel T factors and V^T V.
// One workgroup per matrix.  Tbig[b][blk] is 64 x 64 row-major, zero beyond bw.
// The Gram matrix and the merge are formed in float64 whatever T is (a
// float32 Gram summed over ~10^3 rows would add rounding that the
// panel-by-panel application does not have).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_qr_tmerge(const QRDesc* __restrict__ desc, const T* __restrict__ A,
                                                      const T* __restrict__ Tbuf, T* __restrict__ Tbig, int kb,
                                                      int blk, int npanel, int nblock) {
  const QRDesc d = desc[blockIdx.x];
  if (kb >= d.nrefl) return;
  const int bw = min(kBB, d.nrefl - kb);
  const int npb = (bw + kNB - 1) / kNB;
  __shared__ double Ts[kBB][kBB + 1];
  __shared__ double Gs[kBB][kBB + 1];
  __shared__ double Vc[64][kBB + 1];
  const T* Am = A + d.off;
  for (int e = threadIdx.x; e < kBB * kBB; e += kBlock) Ts[e / kBB][e % kBB] = 0.0;
  __syncthreads();
  for (int e = threadIdx.x; e < npb * kNB * kNB; e += kBlock) {
    const int pp = e / (kNB * kNB), i = (e / kNB) % kNB, j = e % kNB;
    const int p = kb / kNB + pp;
    Ts[pp * kNB + i][pp * kNB + j] = (double)Tbuf[((long long)blockIdx.x * npanel + p) * kNB * kNB + i * kNB + j];
  }
  // G = V^T V over the rows of the block's reflectors on f64 MFMA.  The
  // merge reads only the blocks G(p, q), p < q, of 16 x 16 (panels p and q):
  // six tiles, two for waves 0 and 1 and one for waves 2 and 3.  Loads read
  // clamped in-matrix addresses with no branches and the reflector values
  // are selected when a chunk is stored to LDS; the loop's barriers order
  // LDS accesses only, so the next chunk's loads stay in flight.
  typedef Mfma<double>::v4 v4d;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tp0 = wv < 2 ? 0 : wv - 1, tq0 = wv == 0 ? 1 : 3;   // (0,1) (0,3) (1,3) (2,3)
  const int tp1 = wv, tq1 = 2;                                  // (0,2) (1,2) for waves 0, 1
  const bool two_tiles = wv < 2;
  v4d acc0 = v4d{0, 0, 0, 0}, acc1 = v4d{0, 0, 0, 0};
  if (npb > 1) {
    T vv[16];
    auto load_chunk = [&](int r0) {
      const int row = min(r0 + (int)threadIdx.x % 64, d.m - 1);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int c = (threadIdx.x + u * kBlock) / 64;
        vv[u] = Am[(long long)(kb + min(c, bw - 1)) * d.ld + row];
      }
    };
    load_chunk(kb);
    for (int r0 = kb; r0 < d.m;) {
      const int rn = skip_band(r0 + 64, kb + kBB, d.zhi);
      {
        const int row = r0 + threadIdx.x % 64, rr = row - kb;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = threadIdx.x + u * kBlock, c = e / 64;
          Vc[e % 64][c] = (c >= bw || row >= d.m || rr < c) ? 0.0 : (rr == c ? 1.0 : (double)vv[u]);
        }
      }
      lds_barrier();
      load_chunk(min(rn, d.m));   // next chunk in flight during the products (past the end: unused)
#pragma unroll 4
      for (int ks = 0; ks < 16; ++ks) {
        const int rr = ks * 4 + (lane >> 4);
        acc0 = Mfma<double>::mma(Vc[rr][16 * tp0 + (lane & 15)], Vc[rr][16 * tq0 + (lane & 15)], acc0);
        if (two_tiles)
          acc1 = Mfma<double>::mma(Vc[rr][16 * tp1 + (lane & 15)], Vc[rr][16 * tq1 + (lane & 15)], acc1);
      }
      lds_barrier();
      r0 = rn;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Gs[16 * tp0 + Mfma<double>::drow(lane, v)][16 * tq0 + (lane & 15)] = acc0[v];
      if (two_tiles) Gs[16 * tp1 + Mfma<double>::drow(lane, v)][16 * tq1 + (lane & 15)] = acc1[v];
    }
  }
  __syncthreads();
  // merge: T(0:n0, n0:n0+16) = -T(0:n0, 0:n0) G(0:n0, n0:n0+16) T(n0:n0+16, n0:n0+16)
  for (int q = 1; q < npb; ++q) {
    const int n0 = q * kNB;
    for (int e = threadIdx.x; e < n0 * kNB; e += kBlock) {
      const int i = e / kNB, c = e % kNB;
      double y = 0.0;
      for (int l = i; l < n0; ++l) y += Ts[i][l] * Gs[l][n0 + c];
      Vc[i][c] = y;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n0 * kNB; e += kBlock) {
      const int i = e / kNB, c = e % kNB;
      double z = 0.0;
      for (int l = 0; l <= c; ++l) z += Vc[i][l] * Ts[n0 + l][n0 + c];
      Ts[i][n0 + c] = -z;
    }
    __syncthreads();
  }
  T* Tout = Tbig + ((long long)blockIdx.x * nblock + blk) * kBB * kBB;
  for (int e = threadIdx.x; e < kBB * kBB; e += kBlock) Tout[e] = (T)Ts[e / kBB][e % kBB];
}

// Apply the block reflector of block blk (columns kb .. kb+bw-1) of every
// matrix to columns [c0, cn[b]) of C + coff[b] (leading dimension ldc[b]):
// transT = 1 applies Q^T = I - V T^T V^T, transT = 0 applies Q = I - V T V^T.
// 1-D grid over (matrix, BC-column tile), arranged so that all tiles of one
// matrix land on the same XCD (workgroup id mod 8) and share its L2 for V.
// BC = 64 for the factorisation's trailing updates; BC = 16 applies Q or Q^T
// to up to 16 right-hand sides without the products of 48 empty columns.
// Off32: every element of a matrix and of its C block lies within 2^31 bytes
// of the block's start (checked by the caller), so addresses are a uniform
// base plus a 32-bit byte offset (fewer registers than 64-bit addresses per
// column).
template <typename T, int BC = kBC, bool Off32 = false>
__global__ void __launch_bounds__(kBlock, Off32 ? 2 : 1) k_qr_wy64(const QRDesc* __restrict__ desc, const T* __restrict__ A,
                                                    const T* __restrict__ Tbig, int kb, int blk, int nblock,
                                                    int nmat, int ntile, T* __restrict__ C,
                                                    const long long* __restrict__ coff, const int* __restrict__ ldc,
                                                    const int* __restrict__ cn, int c0, int transT) {
  typedef typename Mfma<T>::v4 v4;
  static_assert(BC == 16 || BC == 64, "column tiles of 16 or 64");
  constexpr int NT = BC / 16;           // 16-column MFMA tiles
  constexpr int CPT = 64 * BC / kBlock;   // elements of a 64-row C chunk per thread
  const int id = blockIdx.x;
  const int b = (id % 8) + 8 * ((id / 8) / ntile);
  const int tile = (id / 8) % ntile;
  if (b >= nmat) return;
  const QRDesc d = desc[b];
  if (kb >= d.nrefl) return;
  const int bw = min(kBB, d.nrefl - kb);
  const int cbeg = c0 + tile * BC;
  const int ctot = cn[b];
  if (cbeg >= ctot) return;
  const int ncol = min(BC, ctot - cbeg);
  const int L = ldc[b];
  const T* Am = A + d.off;
  T* Cm = C + coff[b];
  // element (row, col) of the matrix (column-major, leading dimension ld)
  // and of the C block (leading dimension L)
  auto aref = [&](int col, int row) -> const T& {
    if constexpr (Off32)
      return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(Am) +
                                         (unsigned)((col * d.ld + row) * (int)sizeof(T)));
    else
      return Am[(long long)col * d.ld + row];
  };
  auto cref = [&](int col, int row) -> T& {
    if constexpr (Off32)
      return *reinterpret_cast<T*>(reinterpret_cast<char*>(Cm) + (unsigned)((col * L + row) * (int)sizeof(T)));
    else
      return Cm[(long long)col * L + row];
  };
  __shared__ T Vs[64][kBB + 1];      // V chunk, later T
  __shared__ T Cs[64][BC + 1];       // C chunk, later W
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // ---- W = V^T C: wave wv forms rows 16 wv .. 16 wv + 15 of W (NT tiles of 16 columns)
  v4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4{0, 0, 0, 0};
  // Loads read elements inside the matrix (indices clamped) with no
  // branches; the values (0 or 1 above and on the diagonal of V, 0 past the
  // last row or column) are selected when a chunk is stored to LDS.  The
  // barriers of this loop order LDS accesses only, so the next chunk's loads
  // stay in flight across them.
  T vv[16], cc[CPT];
  auto load_chunk = [&](int r0) {
    const int row = min(r0 + (int)threadIdx.x % 64, d.m - 1);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int c = (threadIdx.x + u * kBlock) / 64;
      vv[u] = aref(kb + min(c, bw - 1), row);
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int c = (threadIdx.x + u * kBlock) / 64;
      cc[u] = cref(cbeg + min(c, ncol - 1), row);
    }
  };
  load_chunk(kb);
  for (int r0 = kb; r0 < d.m;) {
    const int rn = skip_band(r0 + 64, kb + kBB, d.zhi);
    {
      const int row = r0 + threadIdx.x % 64, rr = row - kb;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = threadIdx.x + u * kBlock, c = e / 64;
        Vs[e % 64][c] = (c >= bw || row >= d.m || rr < c) ? T(0) : (rr == c ? T(1) : vv[u]);
      }
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int e = threadIdx.x + u * kBlock, c = e / 64;
        Cs[e % 64][c] = (row < d.m && c < ncol) ? cc[u] : T(0);
      }
    }
    lds_barrier();
    load_chunk(min(rn, d.m));   // next chunk in flight during the products (past the end: unused)
#pragma unroll 4
    for (int ks = 0; ks < 16; ++ks) {
      const int rr = ks * 4 + (lane >> 4);
      const T av = Vs[rr][16 * wv + (lane & 15)];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = Mfma<T>::mma(av, Cs[rr][16 * t + (lane & 15)], acc[t]);
    }
    lds_barrier();
    r0 = rn;
  }
  // W into Cs, T into Vs
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * wv + Mfma<T>::drow(lane, v);
#pragma unroll
    for (int t = 0; t < NT; ++t) Cs[i][16 * t + (lane & 15)] = acc[t][v];
  }
  const T* Tin = Tbig + ((long long)b * nblock + blk) * kBB * kBB;
  for (int e = threadIdx.x; e < kBB * kBB; e += kBlock) Vs[e / kBB][e % kBB] = Tin[e];
  __syncthreads();
  // ---- W <- -T^T W (Q^T) or -T W (Q) on the matrix cores: wave wv forms
  //      rows 16 wv .. 16 wv + 15 (NT tiles of 16 columns); the zero
  //      triangle of T is multiplied too (as one row chunk of V^T C)
  {
    v4 tacc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) tacc[t] = v4{0, 0, 0, 0};
#pragma unroll 4
    for (int ks = 0; ks < 16; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      const T av = transT ? Vs[kk][16 * wv + (lane & 15)] : Vs[16 * wv + (lane & 15)][kk];
#pragma unroll
      for (int t = 0; t < NT; ++t) tacc[t] = Mfma<T>::mma(av, Cs[kk][16 * t + (lane & 15)], tacc[t]);
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * wv + Mfma<T>::drow(lane, v);
#pragma unroll
      for (int t = 0; t < NT; ++t) Cs[i][16 * t + (lane & 15)] = -tacc[t][v];
    }
  }
  __syncthreads();
  // ---- C <- C + V W for 16-row blocks (rows along the lanes)
  // loads of the next 16-row block are issued before the products of this one
  T cn_[4 * NT], bn_[16];
  // (clamped indices, values selected at use, as above)
  auto load_rows = [&](int rb) {
    const int row = min(rb + (lane & 15), d.m - 1);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * t + Mfma<T>::drow(lane, v);
        cn_[4 * t + v] = cref(cbeg + min(c, ncol - 1), row);
      }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int jj = ks * 4 + (lane >> 4);
      bn_[ks] = aref(kb + min(jj, bw - 1), row);
    }
  };
  auto next_rb = [&](int r) { return skip_band(r - wv * 16 + kWaves * 16, kb + kBB, d.zhi) + wv * 16; };
  int rb = kb + wv * 16;
  if (rb < d.m) load_rows(rb);
  for (; rb < d.m; rb = next_rb(rb)) {
    // W is read from LDS in every row block rather than held in registers
    // across the loop (64 doubles per lane), which keeps two waves per SIMD
    asm volatile("" ::: "memory");
    const int row = rb + (lane & 15);
    v4 cacc[NT];
    T bv[16];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) cacc[t][v] = cn_[4 * t + v];
    {
      const int rr = row - kb;
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const int jj = ks * 4 + (lane >> 4);
        bv[ks] = (jj >= bw || row >= d.m || rr < jj) ? T(0) : (rr == jj ? T(1) : bn_[ks]);
      }
    }
    load_rows(min(next_rb(rb), d.m));
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int jj = ks * 4 + (lane >> 4);
#pragma unroll
      for (int t = 0; t < NT; ++t) cacc[t] = Mfma<T>::mma(Cs[jj][16 * t + (lane & 15)], bv[ks], cacc[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * t + Mfma<T>::drow(lane, v);
        if (row < d.m && c < ncol) cref(cbeg + c, row) = cacc[t][v];
      }
  }
}

}  // namespace ddelm

namespace ddelm {

// Batched C = alpha op(A) B + beta C on f64 MFMA (operands of any storage
// type are widened to double).  One workgroup per 32 x 32 tile of C (each
// wave a 16 x 16 quarter), k in chunks of 32 staged through LDS, the next
// chunk's loads issued before the current chunk's products.
constexpr int kGT = 32;
template <typename TA, typename TB, typename TC>
__global__ void __launch_bounds__(kBlock) k_gemm_mfma(const GemmDesc* __restrict__ desc, const TA* __restrict__ A,
                                                      const TB* __restrict__ B, TC* __restrict__ C, int transA,
                                                      double alpha, double beta, int nx, int ny, int nmat) {
  typedef Mfma<double>::v4 v4;
  // 1-D grid over (matrix, tile).  With 8 or more products, all tiles of
  // one product land on the same XCD (workgroup id mod 8) close together in
  // time and share its L2 for their row and column strips; fewer products
  // spread their tiles over all XCDs.
  const int ntl = nx * ny;
  const int id = blockIdx.x;
  const bool grouped = nmat >= 8;
  const int b = grouped ? (id % 8) + 8 * ((id / 8) / ntl) : id / ntl;
  const int t = grouped ? (id / 8) % ntl : id % ntl;
  if (b >= nmat) return;
  const GemmDesc g = desc[b];
  const int row0 = (t % nx) * kGT, col0 = (t / nx) * kGT;
  if (row0 >= g.m || col0 >= g.n) return;
  __shared__ double As[kGT][kGT + 1];   // As[k][row]
  __shared__ double Bs[kGT][kGT + 1];   // Bs[col][k]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = wv & 1, wc = wv >> 1;
  constexpr int kPer = kGT * kGT / kBlock;   // elements of each operand per thread and chunk
  double av[kPer], bv[kPer];
  // element u of this thread: A along rows (transA = 0) or along k (transA = 1), B along k
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const int lo = e % kGT, hi = e / kGT;
      const int r = transA ? hi : lo, kk = transA ? lo : hi;
      const int rg = row0 + r, kg = k0 + kk;
      const long long ia = transA ? g.a + (long long)rg * g.lda + kg : g.a + (long long)kg * g.lda + rg;
      av[u] = (rg < g.m && kg < g.k) ? (double)A[ia] : 0.0;
      const int cg = col0 + hi, kb = k0 + lo;
      bv[u] = (cg < g.n && kb < g.k) ? (double)B[g.b + (long long)cg * g.ldb + kb] : 0.0;
    }
  };
  v4 acc = v4{0, 0, 0, 0};
  load(0);
  for (int k0 = 0; k0 < g.k; k0 += kGT) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const int lo = e % kGT, hi = e / kGT;
      if (transA) As[lo][hi] = av[u];
      else As[hi][lo] = av[u];
      Bs[hi][lo] = bv[u];
    }
    __syncthreads();
    if (k0 + kGT < g.k) load(k0 + kGT);
#pragma unroll
    for (int ks = 0; ks < kGT / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      acc = Mfma<double>::mma(As[kk][16 * wr + (lane & 15)], Bs[16 * wc + (lane & 15)][kk], acc);
    }
    __syncthreads();
  }
  const int col = col0 + 16 * wc + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = row0 + 16 * wr + Mfma<double>::drow(lane, v);
    if (row < g.m && col < g.n) {
      TC* cp = C + g.c + (long long)col * g.ldc + row;
      const double prev = beta != 0.0 ? (double)*cp : 0.0;
      *cp = (TC)(alpha * acc[v] + beta * prev);
    }
  }
}

// Q^T C (transT = 1, blocks in order) or Q C (transT = 0, blocks reversed)
// for a few columns (ncols <= NR <= 4), one workgroup of an_threads(NR)
// threads per matrix applying every 64-reflector block in one launch.  The
// columns stay in LDS for the whole launch; per block: W = V^T C (wave w
// takes reflectors 16 (w % 4) .. + 15 and the 128-row chunks w / 4 modulo
// the number of row groups, lanes the rows; the groups' sums are added in
// LDS), W <- -T^T W or -T W, then C += V W (threads take rows).  Two row
// groups (512 threads) where the registers allow it.
__host__ __device__ constexpr int an_threads(int nr) { return nr <= 2 ? 512 : 256; }
template <typename T, int NR>
__global__ void __launch_bounds__(an_threads(NR)) k_qr_apply_narrow(const QRDesc* __restrict__ desc, const T* __restrict__ A,
                                                            const T* __restrict__ Tbig, int nblock, T* __restrict__ C,
                                                            const long long* __restrict__ coff,
                                                            const int* __restrict__ ldc, int ncols, int transT) {
  extern __shared__ unsigned char smem_raw[];
  T* cs = reinterpret_cast<T*>(smem_raw);          // [m][NR]
  __shared__ T Ts[kBB][kBB + 1];
  constexpr int kAN = an_threads(NR), kRG = kAN / 256;   // threads, row groups
  __shared__ T Ws[kRG][kBB][NR];
  __shared__ T Wn[kBB][NR];
  const QRDesc d = desc[blockIdx.x];
  const int m = d.m, L = ldc[blockIdx.x];
  T* Cm = C + coff[blockIdx.x];
  const T* Am = A + d.off;
  for (int e = threadIdx.x; e < m * NR; e += kAN) {
    const int c = e / m, r = e % m;
    cs[r * NR + c] = c < ncols ? Cm[(long long)c * L + r] : T(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wg = wv & 3, wh = wv >> 2;      // reflector group, row half
  for (int q = 0; q < nblock; ++q) {
    const int blk = transT ? q : nblock - 1 - q;
    const int kb = blk * kBB;
    if (kb >= d.nrefl) continue;
    const int bw = min(kBB, d.nrefl - kb);
    const T* Tin = Tbig + ((long long)blockIdx.x * nblock + blk) * kBB * kBB;
    for (int e = threadIdx.x; e < kBB * kBB; e += kAN) Ts[e / kBB][e % kBB] = Tin[e];
    // rows by their index l along [kb, m) with the zero band skipped
    const int nl = d.zhi > kb + kBB ? kBB + m - d.zhi : m - kb;
    // ---- W = V^T C
    T acc[16][NR];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
#pragma unroll
      for (int c = 0; c < NR; ++c) acc[jj][c] = T(0);
    for (int l0 = 128 * wh; l0 < nl; l0 += 128 * kRG) {
      T vv[2][16], cv[2][NR];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int l = l0 + u * 64 + lane;
        const int r = l < nl ? band_row<kBB>(kb, l, d.zhi) : m;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          const int j = 16 * wg + jj;
          vv[u][jj] = j < bw ? v_elem(Am, d.ld, m, kb, r, j) : T(0);
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) cv[u][c] = r < m ? cs[r * NR + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
#pragma unroll
          for (int c = 0; c < NR; ++c) acc[jj][c] += vv[u][jj] * cv[u][c];
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const T v = wave_sum(acc[jj][c]);
        if (lane == 0) Ws[wh][16 * wg + jj][c] = v;
      }
    __syncthreads();
    // ---- W <- -T^T W (Q^T) or -T W (Q)
    for (int e = threadIdx.x; e < kBB * NR; e += kAN) {
      const int i = e / NR, c = e % NR;
      T s = T(0);
      if (transT) {
        for (int ip = 0; ip <= i; ++ip) {
          T w = Ws[0][ip][c];
#pragma unroll
          for (int h = 1; h < kRG; ++h) w += Ws[h][ip][c];
          s += Ts[ip][i] * w;
        }
      } else {
        for (int ip = i; ip < kBB; ++ip) {
          T w = Ws[0][ip][c];
#pragma unroll
          for (int h = 1; h < kRG; ++h) w += Ws[h][ip][c];
          s += Ts[i][ip] * w;
        }
      }
      Wn[i][c] = -s;
    }
    __syncthreads();
    // ---- C += V W, two rows per thread with their loads issued together
    for (int l = threadIdx.x; l < nl; l += 2 * kAN) {
      const int r = band_row<kBB>(kb, l, d.zhi);
      const int r2 = l + kAN < nl ? band_row<kBB>(kb, l + kAN, d.zhi) : m;
      T a[2][NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        a[0][c] = cs[r * NR + c];
        a[1][c] = r2 < m ? cs[r2 * NR + c] : T(0);
      }
      for (int j0 = 0; j0 < bw; j0 += 16) {
        T v0[16], v1[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          v0[jj] = j0 + jj < bw ? v_elem(Am, d.ld, m, kb, r, j0 + jj) : T(0);
          v1[jj] = j0 + jj < bw ? v_elem(Am, d.ld, m, kb, r2, j0 + jj) : T(0);
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
#pragma unroll
          for (int c = 0; c < NR; ++c) {
            const T w = j0 + jj < bw ? Wn[j0 + jj][c] : T(0);
            a[0][c] += v0[jj] * w;
            a[1][c] += v1[jj] * w;
          }
      }
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        cs[r * NR + c] = a[0][c];
        if (r2 < m) cs[r2 * NR + c] = a[1][c];
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * ncols; e += kAN) {
    const int c = e / m, r = e % m;
    Cm[(long long)c * L + r] = cs[r * NR + c];
  }
}

}  // namespace ddelm
