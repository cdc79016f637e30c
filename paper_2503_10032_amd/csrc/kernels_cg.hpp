// Persistent CG on eq. nn-mixed: the whole CG loop in one cooperative launch.
//
// Work units are (subdomain i, row slice q): each subdomain's local operator
// rows are split into S slices so that small problems still spread over
// many compute units.  Every unit handles all right-hand sides together, so
// a matrix element read from memory serves nrhs products.
//
// The iteration is the Chronopoulos-Gear form of CG (one operator
// application and one fused reduction per step, see below).  Per pass
// (theta != 0) the phases are separated by 6 grid-wide synchronisations:
//   A  CG update at the unit's Delta points (u = A r of the pass before as
//      the sum of its owners' rows); rows of [G; L](:, Delta) r; partial (r, r)
//   B  coarse solve at the subdomain's corners (mu_Pi, e), lam rows
//   C  y = -N lambda rows               D  z = -N^T (P lambda) rows
//   E  eta, rows of L^T(:, Delta) eta
//   F  coarse nu at the corners, rows of u = A r; partial (u, r)
// (u, r) needs no assembled u: it is the sum over subdomains of each
// subdomain's rows of u times r at the same points.
// With few coarse unknowns the coarse solves are done redundantly by every
// unit for its own corners (rows of X1 against the full coarse right-hand
// side), which removes synchronisations.  With many (nP * nrhs large) every
// unit gathering the whole coarse right-hand side costs more than two extra
// synchronisations, so B and F are split: the coarse right-hand side is
// gathered once, distributed over workgroups (B1, F1); the rows of X1 times
// it are distributed over workgroups with X1 read about once (B2, F2); the
// units then read their corner values (B3, F3).  Scalar reductions are
// repeated by every workgroup in the same order, so all take identical
// decisions.
//
// Synchronisation: every workgroup publishes an epoch in its own flag once
// its memory operations have completed, then waits for all flags to reach
// that epoch (one thread per flag).  Data exchanged between workgroups moves
// through coherent loads and stores (see ld_co/st_co).  The waits are bounded.
#pragma once
#include "kernels_common.hpp"
#include "kernels_solve.hpp"

namespace ddelm {

constexpr int kFlagStride = 16;   // one flag per 64-byte line

// Coherent loads of values written by other workgroups are issued in
// batches of kLB elements before any of them is used: each such load goes to
// memory, and a loop that consumed every value right after loading it would
// pay one full round trip per element.
constexpr int kLB = 8;
constexpr int kMaxOwn = 4;   // owners of an interface point: 2 on an edge, 4 at a vertex

// Coherent (agent-scope) loads and stores for every value that one workgroup
// writes and another reads inside the kernel.  They bypass the per-XCD L2
// copies, so no cache write-back or invalidation fences are needed; the
// read-only matrices stay cached.
__device__ __forceinline__ double ld_co(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_co(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Values that stay inside one workgroup between phases (written and read by
// the same unit, which keeps its workgroup for the whole launch) need no
// agent-scope coherence: plain accesses when `own` (one unit per
// subdomain), coherent ones otherwise (row slices of a subdomain sit in
// different workgroups).
__device__ __forceinline__ double ld_wg(const double* p, bool own) { return own ? *p : ld_co(p); }
__device__ __forceinline__ void st_wg(double* p, double v, bool own) {
  if (own) *p = v;
  else st_co(p, v);
}

// Grid-wide synchronisation: wait until this wave's memory operations have
// completed, publish the epoch in this workgroup's flag, then wait (bounded)
// until every workgroup's flag has reached it.  Together with ld_co/st_co for
// the exchanged data this orders all cross-workgroup traffic.
__device__ __forceinline__ void flag_sync(unsigned* flags, unsigned nb, unsigned epoch, unsigned* err) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(&flags[blockIdx.x * kFlagStride], epoch, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned t = threadIdx.x; t < nb; t += kBlock) {
    unsigned long long spins = 0;
    while (__hip_atomic_load(&flags[t * kFlagStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1ull << 27)) {
        __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

template <typename T>
struct FusedArgs {
  OpArgs<T> a;
  int S;                 // row slices per subdomain
  int nrhs;
  double tol;
  int maxit;
  const double* bref;    // [nrhs] squared norm the stopping test is relative to (null: ||r_0||^2)
  double* x;             // [nrhs][nD]
  double* r;             // [nrhs][nD] r buffers (alternate by pass); r holds b on entry
  double* r1;
  double* p0;            // [nrhs][nD] p buffers (alternate by pass)
  double* p1;
  double* s0;            // [nrhs][nD] s = A p buffers (alternate by pass)
  double* s1;
  double* part;          // [3][nrhs][nb] workgroup partials: (u, r); (r, r) of even and of odd passes
  double* mu_slot;       // [nrhs][sumP]  mu_Pi at the corner slots
  double* e_slot;        // [nrhs][sumP]
  double* scal;          // [nrhs][8] out: rr, bb, -, -, -, done, iters, nonfinite
  double* rsl;           // [nrhs][sumD] with one unit per subdomain (S == 1): r, s and p at
  double* ssl;           // every slot of the unit's Delta points, kept by the unit itself
  double* psl;
  unsigned* flags;       // [nb * kFlagStride]
  unsigned* err;
  int lds_ys, lds_part, lds_cu;   // LDS offsets (doubles) of the output, partial-sum and coarse areas
  int lds_total;         // doubles of dynamic LDS
  int dist;              // 1: distributed coarse phases
  const double* X1t;     // X1 transposed (row-major X1), for the distributed coarse rows
  double* ug;            // [nrhs][2 nP] gathered coarse right-hand side (distributed mode)
  double* cg1;           // [nrhs][2 nP] X1 times it (distributed mode)
  // index tables in LDS (ints after the lds_total doubles): for each of the
  // workgroup's units (at most tab_units; 0 = no tables) and each local Delta
  // point, the global index (bit 30: this slot is the first owner) and the
  // slots of its owners (-1 padded); for the coarse gathers of the redundant
  // mode, the owner slots of every Pi point.
  int tab_units, tab_nd, tab_pi;
};

constexpr int kTabUnits = 4;
constexpr int kOwnerFlag = 1 << 30;

// Owner slots of the Delta point k of the unit's table, as one 16-byte LDS read.
__device__ __forceinline__ int4 tab_slots(const int* tslot, int k) {
  return reinterpret_cast<const int4*>(tslot)[k];
}

// Distributed coarse gather: for the Pi points of this workgroup's share,
// ug[r][p] = sum over owners of A, ug[r][nP + p] = sum over owners of B (B may be null).
template <typename T>
__device__ __forceinline__ void coarse_gather(const OpArgs<T>& a, const double* A, const double* B, int nrhs,
                                              double* ug) {
  const unsigned nb = gridDim.x;
  const int chunk = (a.nP + (int)nb - 1) / (int)nb;
  const int p0 = blockIdx.x * chunk, p1 = min(a.nP, p0 + chunk);
  for (int e = threadIdx.x; e < (p1 - p0) * nrhs; e += kBlock) {
    const int pq = p0 + e / nrhs, r = e % nrhs;
    double s1 = 0.0, s2 = 0.0;
    for (int o = a.pi_own_ptr[pq]; o < a.pi_own_ptr[pq + 1]; ++o) {
      const int sl = a.pi_own_slot[o];
      s1 += ld_co(&A[(size_t)r * a.sumP + sl]);
      if (B) s2 += ld_co(&B[(size_t)r * a.sumP + sl]);
    }
    st_co(&ug[(size_t)r * 2 * a.nP + pq], s1);
    if (B) st_co(&ug[(size_t)r * 2 * a.nP + a.nP + pq], s2);
  }
}

// Distributed coarse rows: out[r][row] = sum_{c < ncol} X1[row][c] ug[r][c]
// for this workgroup's share of the 2 nP rows.
// One row per wave (the large case): the columns are taken in chunks of
// Cw = lds_cap / nrhs (a multiple of 64); all right-hand sides of a chunk are
// staged in LDS at once, the chunk of the wave's X1 row is loaded beside them,
// and the wave keeps one accumulator per right-hand side across the chunks,
// so X1 is read once and a chunk costs one or two batches of coherent loads.
// Otherwise the right-hand sides are staged in groups of G = lds_cap / ncol
// (the launch makes lds_cap >= ncol) and each wave streams a 512-column tile
// of each of its rows per pass and applies it to the whole group.
template <int NR>
__device__ __forceinline__ void coarse_rows(const double* __restrict__ X1t, int nP, int ncol, const double* ug,
                                            int nrhs, double* lds, int lds_cap, double* out) {
  constexpr int kST = NR >= 16 ? 8 : 16;   // staged elements per thread whose loads are issued together
  const unsigned nb = gridDim.x;
  const int ld = 2 * nP;
  const int chunk = (ld + (int)nb - 1) / (int)nb;
  const int row0 = blockIdx.x * chunk, row1 = min(ld, row0 + chunk);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int Cw = (lds_cap / max(nrhs, 1)) / 64 * 64;
  if (chunk <= kWaves && Cw >= 64) {
    const int row = row0 + wid;
    double acc[NR];
#pragma unroll
    for (int g = 0; g < NR; ++g) acc[g] = 0.0;
    for (int c0 = 0; c0 < ncol; c0 += Cw) {
      const int cw = min(Cw, ncol - c0);
      constexpr int kXJ = NR >= 16 ? 4 : 8;
      double xv[kXJ];                     // this lane's X1 elements of the chunk, 64 apart
      const int nj = (cw + 63) / 64;
      if (row1 > row0) {
        const int n = nrhs * cw;
        for (int e0 = threadIdx.x; e0 < n; e0 += kST * kBlock) {
          double v[kST];
#pragma unroll
          for (int u = 0; u < kST; ++u) {
            const int e = e0 + u * kBlock;
            v[u] = e < n ? ld_co(&ug[(size_t)(e / cw) * ld + c0 + e % cw]) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kST; ++u)
            if (e0 + u * kBlock < n) lds[e0 + u * kBlock] = v[u];
        }
      }
      __syncthreads();
      for (int jb = 0; jb < nj; jb += kXJ) {
#pragma unroll
        for (int j = 0; j < kXJ; ++j) {
          const int c = (jb + j) * 64 + lane;
          xv[j] = (row < row1 && jb + j < nj && c < cw) ? X1t[(long long)row * ld + c0 + c] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kXJ; ++j) {
          const int c = (jb + j) * 64 + lane;
          if (row < row1 && jb + j < nj && c < cw) {
#pragma unroll
            for (int g = 0; g < NR; ++g)
              if (g < nrhs) acc[g] += xv[j] * lds[g * cw + c];
          }
        }
      }
      __syncthreads();
    }
    if (row < row1) {
#pragma unroll
      for (int g = 0; g < NR; ++g) {
        if (g < nrhs) {
          const double sum = wave_sum(acc[g]);
          if (lane == 0) st_co(&out[(size_t)g * ld + row], sum);
        }
      }
    }
    return;
  }
  const int G = max(1, min(nrhs, lds_cap / max(ncol, 1)));
  for (int g0 = 0; g0 < nrhs; g0 += G) {
    const int gn = min(G, nrhs - g0);
    if (row1 > row0) {
      const int n = gn * ncol;
      for (int e0 = threadIdx.x; e0 < n; e0 += kST * kBlock) {
        double v[kST];
#pragma unroll
        for (int u = 0; u < kST; ++u) {
          const int e = e0 + u * kBlock;
          v[u] = e < n ? ld_co(&ug[(size_t)(g0 + e / ncol) * ld + e % ncol]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kST; ++u)
          if (e0 + u * kBlock < n) lds[e0 + u * kBlock] = v[u];
      }
    }
    __syncthreads();
    for (int row = row0 + wid; row < row1; row += kWaves) {
      double acc[NR];
#pragma unroll
      for (int g = 0; g < NR; ++g) acc[g] = 0.0;
      const double* xrow = X1t + (long long)row * ld;
      for (int c0 = 0; c0 < ncol; c0 += 64 * 8) {
        double xv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = c0 + k * 64 + lane;
          xv[k] = c < ncol ? xrow[c] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = c0 + k * 64 + lane;
          if (c < ncol) {
#pragma unroll
            for (int g = 0; g < NR; ++g)
              if (g < gn) acc[g] += xv[k] * lds[g * ncol + c];
          }
        }
      }
#pragma unroll
      for (int g = 0; g < NR; ++g) {
        if (g < gn) {
          const double sum = wave_sum(acc[g]);
          if (lane == 0) st_co(&out[(size_t)(g0 + g) * ld + row], sum);
        }
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void slice_rows(int n, int S, int q, int& r0, int& r1) {
  const int len = (n + S - 1) / S;
  r0 = min(n, q * len);
  r1 = min(n, r0 + len);
}

// y_m[t][r] = sum_{k<K} A_m[(c0 + k) * lda + r0 + t] * x[k*NR + r] for rows t < R and
// matrices m < NM; results in out[(m*R + t)*NR + r] (LDS).  The 256 threads
// are split into nsplit groups over k; partial sums meet in `part` (LDS,
// kBlock * NM * NR doubles).
// Many right-hand sides: the same products as a small GEMM on f64 MFMA,
// Y (R x NR) = A (R x K) X (K x NR) in 16-row tiles (tile w, w + 4, ... for
// wave w; NR <= 16 right-hand sides padded to the 16 MFMA columns), the
// matrix streamed from memory as the A operand (lane l: row l & 15, column
// l >> 4 of each 16 x 4 step, so 16 consecutive rows of a column per load)
// and X read from LDS as the B operand.  A wave's work is one sequence of
// batches of kMB steps (4 columns each) over its tiles; the loads of batch
// s + 1 are issued before the products of batch s, so a wave always has one
// batch in flight while it computes (the matrix stream is latency bound: a
// batch costs one memory round trip).  Float32 matrices are widened to
// float64.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T, int NM, int kMB>
__device__ __forceinline__ void mfma_load_batch(const T* A0, const T* A1, int lda, int r0, int R, int c0, int K,
                                                int tile, int kb, double (&va)[kMB], double (&vb)[kMB]) {
  // Branch-free: every lane loads from a clamped (in-range, so finite)
  // element; nothing is masked here.  Rows past R only feed output rows that
  // are never stored, and columns past K meet a zero x in the product, so the
  // loads of a batch stay one unconditional group and the wait before the
  // products can count them exactly.
  const int lane = threadIdx.x & 63;
  const int rowc = min(tile * 16 + (lane & 15), R - 1);
  const T* a0 = A0 + (long long)c0 * lda + r0 + rowc;
  const T* a1 = NM > 1 ? A1 + (long long)c0 * lda + r0 + rowc : nullptr;
#pragma unroll
  for (int u = 0; u < kMB; ++u) {
    const long long kc = min(kb * 4 * kMB + 4 * u + (lane >> 4), K - 1);
    va[u] = (double)a0[kc * lda];
    if (NM > 1) vb[u] = (double)a1[kc * lda];
  }
}

template <int NR, int NM, int kMB>
__device__ __forceinline__ void mfma_batch(int R, int K, int tile, int kb, int nkb, const double (&va)[kMB],
                                           const double (&vb)[kMB], const double* x, double* out, f64x4& acc0,
                                           f64x4& acc1) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int u = 0; u < kMB; ++u) {
    const int kk = kb * 4 * kMB + 4 * u + lk;
    const double xv = x[min(kk, K - 1) * NR + min(lr, NR - 1)];
    const double xb = (kk < K && lr < NR) ? xv : 0.0;
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], xb, acc0, 0, 0, 0);
    if (NM > 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(vb[u], xb, acc1, 0, 0, 0);
  }
  if (kb == nkb - 1) {
    // accumulator element v of lane l holds row (l >> 4) + 4 v, right-hand side l & 15
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int orow = tile * 16 + lk + 4 * v;
      if (orow < R && lr < NR) {
        out[orow * NR + lr] = acc0[v];
        if (NM > 1) out[(R + orow) * NR + lr] = acc1[v];
      }
      acc0[v] = 0.0;
      acc1[v] = 0.0;
    }
  }
}

template <typename T, int NR, int NM>
__device__ __forceinline__ void mv_rows_mfma(const T* A0, const T* A1, int lda, int r0, int R, int c0, int K,
                                             const double* x, double* out) {
  constexpr int kMB = 8;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int ntile = (R + 15) / 16;
  const int nkb = (K + 4 * kMB - 1) / (4 * kMB);                // batches per tile
  const int mytiles = wv < ntile ? (ntile - wv + kWaves - 1) / kWaves : 0;
  const int nsteps = mytiles * nkb;
  if (nsteps > 0) {
    f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    double pa[kMB], pb[kMB], qa[kMB], qb[kMB];
    // batch s: tile wv + (s / nkb) * kWaves, column batch s % nkb.  Two
    // register sets alternate (p for even s, q for odd s).  Every load and
    // product is unconditional, so the waits before the products count the
    // loads exactly: batches past the wave's last tile (an odd count's last
    // q batch, the final prefetch) load clamped elements and store nothing.
    mfma_load_batch<T, NM, kMB>(A0, A1, lda, r0, R, c0, K, wv, 0, pa, pb);
    for (int s = 0; s < nsteps; s += 2) {
      mfma_load_batch<T, NM, kMB>(A0, A1, lda, r0, R, c0, K, wv + ((s + 1) / nkb) * kWaves, (s + 1) % nkb, qa, qb);
      mfma_batch<NR, NM, kMB>(R, K, wv + (s / nkb) * kWaves, s % nkb, nkb, pa, pb, x, out, acc0, acc1);
      mfma_load_batch<T, NM, kMB>(A0, A1, lda, r0, R, c0, K, wv + ((s + 2) / nkb) * kWaves, (s + 2) % nkb, pa, pb);
      mfma_batch<NR, NM, kMB>(R, K, wv + ((s + 1) / nkb) * kWaves, (s + 1) % nkb, nkb, qa, qb, x, out, acc0, acc1);
    }
  }
  __syncthreads();
}

template <typename T, int NR, int NM>
__device__ __forceinline__ void mv_rows(const T* A0, const T* A1, int lda, int r0, int R, int c0, int K,
                                        const double* x, int nrhs, double* out, double* part) {
  if (R <= 0) {
    __syncthreads();
    return;
  }
  if constexpr (NR >= 8) {
    mv_rows_mfma<T, NR, NM>(A0, A1, lda, r0, R, c0, K, x, out);
    return;
  }
  // rows per pass: 64, 128 or 256 so that no thread of the block idles for
  // the whole pass (a 192-row pass would leave a quarter of them without work)
  int Rp = R <= 64 ? 64 : (R <= 128 ? 128 : ((R > 192 && R <= 256) ? 256 : 64));
  const int nsplit = kBlock / Rp;
  for (int rb = 0; rb < R; rb += Rp) {
    const int t = threadIdx.x % Rp, j = threadIdx.x / Rp;
    const int row = rb + t;
    double acc[NM][NR];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[m][r] = 0.0;
    if (row < R && j < nsplit) {
      const T* a0 = A0 + (long long)c0 * lda + r0 + row;
      const T* a1 = NM > 1 ? A1 + (long long)c0 * lda + r0 + row : nullptr;
      // batches of kU columns, the last one predicated: all loads of a batch
      // are issued before its products, so each thread keeps kU * NM loads in
      // flight and a row costs ceil(K / (kU * nsplit)) memory round trips.
      // The matrix stream is latency bound, so with many right-hand sides
      // (one wave per SIMD) the batch is deeper; with few, 16 columns
      // measured faster.
      constexpr int kU = NR >= 8 ? 32 : 16;
      for (int k = j; k < K; k += kU * nsplit) {
        double v0[kU], v1[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int kk = k + u * nsplit;
          v0[u] = kk < K ? (double)a0[(long long)kk * lda] : 0.0;
          if (NM > 1) v1[u] = kk < K ? (double)a1[(long long)kk * lda] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int kk = k + u * nsplit;
          if (kk < K) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
              const double xv = x[kk * NR + r];
              acc[0][r] += v0[u] * xv;
              if (NM > 1) acc[NM - 1][r] += v1[u] * xv;
            }
          }
        }
      }
    }
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
      for (int r = 0; r < NR; ++r) part[((m * nsplit + j) * Rp + t) * NR + r] = acc[m][r];
    __syncthreads();
    for (int e = threadIdx.x; e < NM * Rp * NR; e += kBlock) {
      const int m = e / (Rp * NR), rem = e % (Rp * NR), tt = rem / NR, r = rem % NR;
      if (rb + tt < R && r < nrhs) {
        double s = 0.0;
        for (int jj = 0; jj < nsplit; ++jj) s += part[((m * nsplit + jj) * Rp + tt) * NR + r];
        out[(m * R + rb + tt) * NR + r] = s;
      }
    }
    __syncthreads();
  }
}

// Element loops over (point k, right-hand side r) of a unit run RHS-major:
// thread t takes r = t / kTPR and the points k = t % kTPR + kTPR j, so that
// the lanes of a wave touch consecutive points of one right-hand side.  The
// interface vectors are stored [r][point] and the points of a unit (and their
// owner slots) run along its edges in consecutive global order, so a wave's
// coherent loads and stores fall on a few cache lines instead of one line
// per right-hand side.
template <int NR>
struct RhsMajor {
  static constexpr int kTPR = kBlock / NR;       // threads per right-hand side
  int r, k0;
  __device__ __forceinline__ RhsMajor() : r(threadIdx.x / kTPR), k0(threadIdx.x % kTPR) {}
};

// sum over owners of a local Delta vector, for all Delta points of subdomain i
// into xs[k*NR + r] (LDS); optionally mixes two vectors (theta*A + (1-theta)*B).
// Columns r >= nrhs of xs are zeroed.
template <int NR>
__device__ __forceinline__ void gather_dl(const int* own_ptr, const int* own_slot, const int* l2g, int d0, int nd,
                                          const double* A, const double* B, double ca, double cb, int sumD, int nrhs,
                                          double* xs) {
  constexpr int kTPR = RhsMajor<NR>::kTPR;
  const RhsMajor<NR> th;
  for (int kb = th.k0; kb < nd; kb += kLB * kTPR) {
    double va[kLB][kMaxOwn], vb[kLB][kMaxOwn];
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int k = kb + u * kTPR;
      int o0 = 0, cnt = 0;
      if (k < nd && th.r < nrhs) {
        const int g = l2g[d0 + k];
        o0 = own_ptr[g];
        cnt = own_ptr[g + 1] - o0;
      }
#pragma unroll
      for (int o = 0; o < kMaxOwn; ++o) {
        va[u][o] = 0.0;
        vb[u][o] = 0.0;
        if (o < cnt) {
          const size_t sl = (size_t)th.r * sumD + own_slot[o0 + o];
          va[u][o] = ld_co(&A[sl]);
          if (B) vb[u][o] = ld_co(&B[sl]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int k = kb + u * kTPR;
      if (k < nd) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int o = 0; o < kMaxOwn; ++o) {
          sa += va[u][o];
          sb += vb[u][o];
        }
        xs[k * NR + th.r] = B ? ca * sa + cb * sb : sa;
      }
    }
  }
}

// Sum over the workgroup of one value per thread, split by right-hand side
// for the RHS-major element loops: out[r] is the sum over the threads
// t / kTPR == r.  `red` must hold kBlock / min(kTPR, 64) values.  Fixed
// order: the same bits on every run.
template <int NR>
__device__ __forceinline__ void block_sum_grp(double v, double* dst, size_t stride, int nrhs, double* red) {
  constexpr int kTPR = RhsMajor<NR>::kTPR;
  constexpr int kW = kTPR < 64 ? kTPR : 64;      // lanes of one right-hand side inside a wave
  constexpr int kE = kBlock / kW;                // partial sums in `red`
#pragma unroll
  for (int o = 1; o < kW; o <<= 1) v += __shfl_xor(v, o, 64);   // sums within aligned groups of kW lanes
  const int lane = threadIdx.x & 63;
  __syncthreads();
  if (lane % kW == 0) red[threadIdx.x / kW] = v;
  __syncthreads();
  if ((int)threadIdx.x < nrhs) {
    constexpr int kPer = kE / NR;                // partial sums per right-hand side
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) t += red[threadIdx.x * kPer + j];
    st_co(dst + threadIdx.x * stride, t);
  }
}

// Two values per thread summed by right-hand side as in block_sum_grp, into
// the shared arrays sa[r], sb[r] (visible to every thread on return).
// `red` must hold 2 kBlock / min(kTPR, 64) values.  Fixed order.
template <int NR>
__device__ __forceinline__ void block_sum_grp2(double a, double b, double* sa, double* sb, int nrhs, double* red) {
  constexpr int kTPR = RhsMajor<NR>::kTPR;
  constexpr int kW = kTPR < 64 ? kTPR : 64;
  constexpr int kE = kBlock / kW;
#pragma unroll
  for (int o = 1; o < kW; o <<= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  const int lane = threadIdx.x & 63;
  __syncthreads();
  if (lane % kW == 0) {
    red[threadIdx.x / kW] = a;
    red[kE + threadIdx.x / kW] = b;
  }
  __syncthreads();
  if ((int)threadIdx.x < nrhs) {
    constexpr int kPer = kE / NR;
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      ta += red[threadIdx.x * kPer + j];
      tb += red[kE + threadIdx.x * kPer + j];
    }
    sa[threadIdx.x] = ta;
    sb[threadIdx.x] = tb;
  }
  __syncthreads();
}

// gather_dl with the owner slots read from the LDS table of the unit
template <int NR>
__device__ __forceinline__ void gather_dl_tab(const int* tslot, int nd, const double* A, const double* B, double ca,
                                              double cb, int sumD, int nrhs, double* xs) {
  constexpr int kTPR = RhsMajor<NR>::kTPR;
  const RhsMajor<NR> th;
  for (int kb = th.k0; kb < nd; kb += kLB * kTPR) {
    double va[kLB][kMaxOwn], vb[kLB][kMaxOwn];
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int k = kb + u * kTPR;
      int4 sl = make_int4(-1, -1, -1, -1);
      if (k < nd && th.r < nrhs) sl = tab_slots(tslot, k);
      const int so[kMaxOwn] = {sl.x, sl.y, sl.z, sl.w};
#pragma unroll
      for (int o = 0; o < kMaxOwn; ++o) {
        va[u][o] = 0.0;
        vb[u][o] = 0.0;
        if (so[o] >= 0) {
          const size_t q = (size_t)th.r * sumD + so[o];
          va[u][o] = ld_co(&A[q]);
          if (B) vb[u][o] = ld_co(&B[q]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int k = kb + u * kTPR;
      if (k < nd) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int o = 0; o < kMaxOwn; ++o) {
          sa += va[u][o];
          sb += vb[u][o];
        }
        xs[k * NR + th.r] = B ? ca * sa + cb * sb : sa;
      }
    }
  }
}

template <typename T, int NR>
__global__ void __launch_bounds__(kBlock, 2) k_cg_fused(FusedArgs<T> f) {
  extern __shared__ double lds[];
  __shared__ double red[kWaves];
  __shared__ double redv[kWaves * (NR > 2 ? NR : 2)];
  __shared__ double sc_rr[NR], sc_bb[NR], sc_done[NR], sc_it[NR], sc_beta[NR], sc_alpha[NR], sc_gprev[NR];
  __shared__ double sc_gt[NR], sc_dt[NR];   // the reduced (r, r) and (u, r) of the pass before
  __shared__ double cor[2][4][NR];          // per corner: (mu, e) or (nu, -D nu)
  __shared__ double cms[2][4][NR];          // per corner: (mu, e) read back in F
  const OpArgs<T>& a = f.a;
  const unsigned nb = gridDim.x;
  const int nrhs = f.nrhs;
  const int nunits = a.N * f.S;
  constexpr int kTPR = RhsMajor<NR>::kTPR;
  const RhsMajor<NR> th;
  // One unit per subdomain: every unit keeps r, s and p at its own Delta slots
  // (the same values the points' other units and owner compute, bit for bit)
  // and reads the vectors it produced itself with plain accesses.
  const bool slot_state = f.S == 1;
  // LDS layout: inputs [max n_D][NR], outputs [2][max n_G][NR], partial sums
  // [kBlock][2][NR], coarse right-hand side [2 nP] (one rhs at a time)
  double* xs = lds;
  double* ys = lds + f.lds_ys;
  double* part = lds + f.lds_part;
  double* cu = lds + f.lds_cu;
  unsigned epoch = 0;                        // flags are zeroed before every launch
  int* tab = reinterpret_cast<int*>(lds + f.lds_total);
  int* tg = tab;                                            // [tab_units][tab_nd]
  int* tsl = tab + kTabUnits * f.tab_nd;                    // [tab_units][tab_nd][4], 16-byte aligned
  int* tpi = tsl + 4 * kTabUnits * f.tab_nd;                // [nP][4] when tab_pi
  if (f.tab_units) {
    for (int t = 0; t < f.tab_units; ++t) {
      const int u = blockIdx.x + t * (int)nb;
      if (u >= nunits) break;
      const int i = u / f.S, d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
      for (int k = threadIdx.x; k < nd; k += kBlock) {
        const int g = a.dl_l2g[d0 + k];
        const int o0 = a.dl_own_ptr[g], cnt = a.dl_own_ptr[g + 1] - o0;
        int sl[kMaxOwn];
#pragma unroll
        for (int o = 0; o < kMaxOwn; ++o) sl[o] = o < cnt ? a.dl_own_slot[o0 + o] : -1;
        tg[t * f.tab_nd + k] = g | (sl[0] == d0 + k ? kOwnerFlag : 0);
        reinterpret_cast<int4*>(tsl)[t * f.tab_nd + k] = make_int4(sl[0], sl[1], sl[2], sl[3]);
      }
    }
    if (f.tab_pi) {
      for (int pq = threadIdx.x; pq < a.nP; pq += kBlock) {
        const int o0 = a.pi_own_ptr[pq], cnt = a.pi_own_ptr[pq + 1] - o0;
        int sl[kMaxOwn];
#pragma unroll
        for (int o = 0; o < kMaxOwn; ++o) sl[o] = o < cnt ? a.pi_own_slot[o0 + o] : -1;
        reinterpret_cast<int4*>(tpi)[pq] = make_int4(sl[0], sl[1], sl[2], sl[3]);
      }
    }
    __syncthreads();
  }

  // Chronopoulos-Gear CG.  With u_k = A r_k, gamma_k = (r_k, r_k) and
  // delta_k = (u_k, r_k):
  //   beta_k  = gamma_k / gamma_{k-1}                      (beta_0 = 0)
  //   alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
  //   p_k = r_k + beta_k p_{k-1},   s_k = u_k + beta_k s_{k-1}   (s_k = A p_k)
  //   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k
  // (the same iterates as CG in exact arithmetic).  Pass `it` applies the
  // operator to r_it.  Its phase A first forms p_{it-1}, s_{it-1}, x_it and
  // r_it at the unit's Delta points from the reduction of the pass before:
  // every unit computes its points' values, the first owner stores them, so
  // the update needs no synchronisation of its own.  r, p and s alternate
  // between two buffers by pass, so the other units still read a point's
  // previous value in the same phase.
  // ---- prologue: x = 0, p_{-1} = s_{-1} = 0 (r_0 = b is in rb[0])
  for (int r = 0; r < nrhs; ++r)
    for (int g = blockIdx.x * kBlock + threadIdx.x; g < a.nD; g += nb * kBlock) {
      const size_t e = (size_t)r * a.nD + g;
      st_co(&f.x[e], 0.0);      // x is updated by the owner unit's workgroup, so coherent stores throughout
      st_co(&f.p1[e], 0.0);
      st_co(&f.s1[e], 0.0);
    }
  if (threadIdx.x == 0)
    for (int r = 0; r < NR; ++r) {
      sc_rr[r] = 0.0; sc_bb[r] = 0.0; sc_done[r] = 0.0; sc_it[r] = 0.0;
      sc_beta[r] = 0.0; sc_alpha[r] = 0.0; sc_gprev[r] = 0.0;
    }
  flag_sync(f.flags, nb, ++epoch, f.err);

  int it = 0;
  for (;; ++it) {
    if (it > 0) {
      // ---- reduce gamma_{it-1}, delta_{it-1}; convergence test; alpha, beta (identical in every workgroup)
      // RHS-major: a thread sums the partials of its right-hand side th.r over
      // the workgroups k = th.k0 + kTPR j, the loads of a batch issued together
      {
        constexpr int kRB = 8;
        double gs = 0.0, ds = 0.0;
        if (th.r < nrhs) {
          const double* pg = &f.part[(size_t)((1 + ((it - 1) & 1)) * nrhs + th.r) * nb];
          const double* pd = &f.part[(size_t)th.r * nb];
          for (int kb = th.k0; kb < (int)nb; kb += kRB * kTPR) {
            double vg[kRB], vd[kRB];
#pragma unroll
            for (int u = 0; u < kRB; ++u) {
              const int k = kb + u * kTPR;
              vg[u] = k < (int)nb ? ld_co(pg + k) : 0.0;
              vd[u] = k < (int)nb ? ld_co(pd + k) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kRB; ++u) {
              gs += vg[u];
              ds += vd[u];
            }
          }
        }
        block_sum_grp2<NR>(gs, ds, sc_gt, sc_dt, nrhs, redv);
      }
      if (threadIdx.x == 0) {
        for (int r = 0; r < nrhs; ++r) {
          const double gam = sc_gt[r], del = sc_dt[r];
          if (sc_done[r] == 0.0) {
            sc_rr[r] = gam;
            if (it == 1) sc_bb[r] = f.bref ? f.bref[r] : gam;
            if (gam == 0.0 || sqrt(gam) <= f.tol * sqrt(sc_bb[r]) || !(gam == gam)) sc_done[r] = 1.0;
          }
          if (sc_done[r] == 0.0 && it - 1 < f.maxit) {
            const double beta = it == 1 ? 0.0 : gam / sc_gprev[r];
            const double den = it == 1 ? del : del - beta * gam / sc_alpha[r];
            sc_beta[r] = beta;
            sc_alpha[r] = den != 0.0 ? gam / den : 0.0;
            sc_gprev[r] = gam;
            sc_it[r] += 1.0;
          } else {
            sc_beta[r] = 0.0;
            sc_alpha[r] = 0.0;
          }
        }
      }
      __syncthreads();
      bool all_done = true;
      for (int r = 0; r < nrhs; ++r) all_done = all_done && sc_done[r] != 0.0;
      if (all_done || it - 1 >= f.maxit) break;
    }
    // (selects rather than indexed pointer arrays, which would live in scratch memory)
    const bool odd = it & 1;
    const double* r_old = odd ? f.r : f.r1;   // r_{it-1}
    double* r_cur = odd ? f.r1 : f.r;         // r_it (r_0 = b when it == 0)
    const double* p_old = odd ? f.p1 : f.p0;  // p_{it-2}
    double* p_new = odd ? f.p0 : f.p1;        // p_{it-1}
    const double* s_old = odd ? f.s1 : f.s0;
    double* s_new = odd ? f.s0 : f.s1;

    // ---- A: CG update at the unit's Delta points, rows of [G; L](:, Delta) r_it
    // (RHS-major element loops: every thread's elements belong to the
    // right-hand side th.r)
    double gacc = 0.0;
    for (int u = blockIdx.x, t = 0; u < nunits; u += nb, ++t) {
      const bool use_tab = t < f.tab_units;
      const int i = u / f.S, q = u % f.S;
      const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
      const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
      const int ng = np + nd;
      int r0, r1;
      slice_rows(ng, f.S, q, r0, r1);
      constexpr int kLA = 5;     // points per thread whose loads are issued together
      for (int kb = th.k0; kb < nd; kb += kLA * kTPR) {
        double rv[kLA], pv[kLA], sv[kLA], wv[kLA][kMaxOwn];
        int gg[kLA];
        bool own[kLA];
#pragma unroll
        for (int v = 0; v < kLA; ++v) {
          const int k = kb + v * kTPR;
          rv[v] = pv[v] = sv[v] = 0.0;
#pragma unroll
          for (int o = 0; o < kMaxOwn; ++o) wv[v][o] = 0.0;
          gg[v] = 0;
          own[v] = false;
          if (k < nd && th.r < nrhs) {
            int so[kMaxOwn];
            if (use_tab) {
              const int tv = tg[t * f.tab_nd + k];
              gg[v] = tv & ~kOwnerFlag;
              own[v] = (tv & kOwnerFlag) != 0;
              const int4 sl = tab_slots(tsl + 4 * t * f.tab_nd, k);
              so[0] = sl.x; so[1] = sl.y; so[2] = sl.z; so[3] = sl.w;
            } else {
              gg[v] = a.dl_l2g[d0 + k];
              const int o0 = a.dl_own_ptr[gg[v]], cnt = a.dl_own_ptr[gg[v] + 1] - o0;
#pragma unroll
              for (int o = 0; o < kMaxOwn; ++o) so[o] = o < cnt ? a.dl_own_slot[o0 + o] : -1;
              own[v] = so[0] == d0 + k;
            }
            const size_t ge = (size_t)th.r * a.nD + gg[v];
            const size_t es = (size_t)th.r * a.sumD + d0 + k;
            if (it == 0) {
              rv[v] = r_cur[ge];              // b, written before the launch
            } else if (slot_state) {
              // r_{it-1}, s_{it-2}, p_{it-2} as this unit computed them (zero before pass 2)
              rv[v] = f.rsl[es];
              if (it >= 2) {
                sv[v] = f.ssl[es];
                if (own[v]) pv[v] = f.psl[es];
              }
            } else {
              rv[v] = ld_co(&r_old[ge]);
              if (own[v] && q == 0) pv[v] = ld_co(&p_old[ge]);     // p is only updated by the owner
              sv[v] = ld_co(&s_old[ge]);
            }
            if (it != 0) {
              // u_{it-1} at the point: the owners' rows from phase F of the pass before
#pragma unroll
              for (int o = 0; o < kMaxOwn; ++o)
                if (so[o] >= 0) wv[v][o] = ld_co(&a.w_loc[(size_t)th.r * a.sumD + so[o]]);
            }
          }
        }
#pragma unroll
        for (int v = 0; v < kLA; ++v) {
          const int k = kb + v * kTPR;
          if (k >= nd) continue;
          double x = 0.0;
          if (th.r < nrhs) {
            if (it == 0) {
              x = rv[v];
            } else {
              double uu = 0.0;
#pragma unroll
              for (int o = 0; o < kMaxOwn; ++o) uu += wv[v][o];
              const double be = sc_beta[th.r], al = sc_alpha[th.r];
              const double pn = rv[v] + be * pv[v];
              const double sn = uu + be * sv[v];
              x = rv[v] - al * sn;
              const size_t ge = (size_t)th.r * a.nD + gg[v];
              if (slot_state) {
                const size_t es = (size_t)th.r * a.sumD + d0 + k;
                f.ssl[es] = sn;
                if (own[v]) f.psl[es] = pn;
              } else if (q == 0 && own[v]) {
                st_co(&p_new[ge], pn);
                st_co(&s_new[ge], sn);
                st_co(&r_cur[ge], x);
              }
              // the solution is read and written only by this thread (the
              // owner's unit stays with its workgroup), so plain accesses;
              // the prologue's zero stands for x_0 and is not read back
              if (q == 0 && own[v]) f.x[ge] = (it == 1 ? 0.0 : f.x[ge]) + al * pn;
            }
            if (slot_state) f.rsl[(size_t)th.r * a.sumD + d0 + k] = x;
            if (q == 0 && own[v]) gacc += x * x;
          }
          xs[k * NR + th.r] = x;
        }
      }
      __syncthreads();
      mv_rows<T, NR, 2>(a.Gm + a.offG[i], a.Lm + a.offG[i], ng, r0, r1 - r0, np, nd, xs, nrhs, ys, part);
      for (int tt = th.k0; tt < r1 - r0 && th.r < nrhs; tt += kTPR) {
        const int r = th.r;
        const int row = r0 + tt;
        const double sg = ys[(0 * (r1 - r0) + tt) * NR + r], sl = ys[(1 * (r1 - r0) + tt) * NR + r];
        if (row < np) {
          st_co(&a.rho_loc[(size_t)r * a.sumP + p0 + row], sg);
          st_co(&a.psi_loc[(size_t)r * a.sumP + p0 + row], sl);
        } else {
          st_wg(&a.s_loc[(size_t)r * a.sumD + d0 + row - np], sg, slot_state);   // read in F by this unit
          st_wg(&a.l_loc[(size_t)r * a.sumD + d0 + row - np], sl, slot_state);   // read in B by this unit
        }
      }
      __syncthreads();
    }
    block_sum_grp<NR>(gacc, &f.part[(size_t)(1 + (it & 1)) * nrhs * nb + blockIdx.x], nb, nrhs, redv);
    flag_sync(f.flags, nb, ++epoch, f.err);

    // ---- B: coarse solve at the corners, lam rows
    if (f.dist) {
      coarse_gather(a, a.rho_loc, a.psi_loc, nrhs, f.ug);
      flag_sync(f.flags, nb, ++epoch, f.err);
      coarse_rows<NR>(f.X1t, a.nP, 2 * a.nP, f.ug, nrhs, lds, f.lds_total, f.cg1);
      flag_sync(f.flags, nb, ++epoch, f.err);
    }
    for (int u = blockIdx.x, t = 0; u < nunits; u += nb, ++t) {
      const bool use_tab = t < f.tab_units;
      const int i = u / f.S, q = u % f.S;
      const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
      const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
      const int ng = np + nd;
      if (np > 0 && f.dist) {
        for (int e = threadIdx.x; e < 2 * np * nrhs; e += kBlock) {
          const int kind = e / (np * nrhs), b = (e / nrhs) % np, r = e % nrhs;
          cor[kind][b][r] = ld_co(&f.cg1[(size_t)r * 2 * a.nP + (kind ? a.nP : 0) + a.pi_l2g[p0 + b]]);
        }
        __syncthreads();
        if (q == 0) {
          for (int e = threadIdx.x; e < np * nrhs; e += kBlock) {
            const int b = e / nrhs, r = e % nrhs;
            st_wg(&f.mu_slot[(size_t)r * a.sumP + p0 + b], cor[0][b][r], slot_state);
            st_wg(&f.e_slot[(size_t)r * a.sumP + p0 + b], cor[1][b][r], slot_state);
          }
        }
      } else if (np > 0) {
        for (int r = 0; r < nrhs; ++r) {
          for (int pq = threadIdx.x; pq < a.nP; pq += kBlock) {
            double s1 = 0.0, s2 = 0.0;
            if (f.tab_pi) {
              const int4 sl4 = reinterpret_cast<const int4*>(tpi)[pq];
              const int so[kMaxOwn] = {sl4.x, sl4.y, sl4.z, sl4.w};
              double v1[kMaxOwn], v2[kMaxOwn];
#pragma unroll
              for (int o = 0; o < kMaxOwn; ++o) {
                v1[o] = so[o] >= 0 ? ld_co(&a.rho_loc[(size_t)r * a.sumP + so[o]]) : 0.0;
                v2[o] = so[o] >= 0 ? ld_co(&a.psi_loc[(size_t)r * a.sumP + so[o]]) : 0.0;
              }
#pragma unroll
              for (int o = 0; o < kMaxOwn; ++o) {
                s1 += v1[o];
                s2 += v2[o];
              }
            } else {
              for (int o = a.pi_own_ptr[pq]; o < a.pi_own_ptr[pq + 1]; ++o) {
                const int sl = a.pi_own_slot[o];
                s1 += ld_co(&a.rho_loc[(size_t)r * a.sumP + sl]);
                s2 += ld_co(&a.psi_loc[(size_t)r * a.sumP + sl]);
              }
            }
            cu[pq] = s1;
            cu[a.nP + pq] = s2;
          }
          __syncthreads();
          // 2*np dot products of length 2 nP, one wave each (round robin)
          const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
          for (int dd = wid; dd < 2 * np; dd += kWaves) {
            const int b = dd >> 1, kind = dd & 1;
            const int row = (kind ? a.nP : 0) + a.pi_l2g[p0 + b];
            double s = 0.0;
            for (int c = lane; c < 2 * a.nP; c += 64) s += a.X1[(long long)c * 2 * a.nP + row] * cu[c];
            s = wave_sum(s);
            if (lane == 0) cor[kind][b][r] = s;
          }
          __syncthreads();
        }
        if (q == 0) {
          for (int e = threadIdx.x; e < np * nrhs; e += kBlock) {
            const int b = e / nrhs, r = e % nrhs;
            st_wg(&f.mu_slot[(size_t)r * a.sumP + p0 + b], cor[0][b][r], slot_state);
            st_wg(&f.e_slot[(size_t)r * a.sumP + p0 + b], cor[1][b][r], slot_state);
          }
        }
      }
      int r0, r1;
      slice_rows(nd, f.S, q, r0, r1);
      {
        // the slice's rows of the Pi columns of L, staged in LDS (xs is free here)
        const T* L = a.Lm + a.offG[i];
        for (int e = threadIdx.x; e < np * (r1 - r0); e += kBlock) {
          const int b = e / (r1 - r0), tt = e % (r1 - r0);
          xs[e] = (double)L[(long long)b * ng + np + r0 + tt];
        }
        __syncthreads();
      }
      for (int kb = th.k0; kb < r1 - r0 && th.r < nrhs; kb += kLB * kTPR) {
        const int r = th.r;
        double lv[kLB];
#pragma unroll
        for (int u = 0; u < kLB; ++u) {
          const int tt = kb + u * kTPR;
          lv[u] = tt < r1 - r0 ? ld_wg(&a.l_loc[(size_t)r * a.sumD + d0 + r0 + tt], slot_state) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kLB; ++u) {
          const int tt = kb + u * kTPR;
          if (tt >= r1 - r0) continue;
          const int row = r0 + tt;
          double acc = lv[u];
          for (int b = 0; b < np; ++b) acc -= xs[b * (r1 - r0) + tt] * cor[0][b][r];
          st_co(&a.lam_loc[(size_t)r * a.sumD + d0 + row], acc);
        }
      }
      __syncthreads();
    }
    flag_sync(f.flags, nb, ++epoch, f.err);

    if (a.theta != 0.0) {
      // ---- C: y = -N lambda rows
      for (int u = blockIdx.x, t = 0; u < nunits; u += nb, ++t) {
        const bool use_tab = t < f.tab_units;
        const int i = u / f.S, q = u % f.S;
        const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
        int r0, r1;
        slice_rows(nd, f.S, q, r0, r1);
        if (use_tab) gather_dl_tab<NR>(tsl + 4 * t * f.tab_nd, nd, a.lam_loc, nullptr, 1.0, 0.0, a.sumD, nrhs, xs);
        else gather_dl<NR>(a.dl_own_ptr, a.dl_own_slot, a.dl_l2g, d0, nd, a.lam_loc, nullptr, 1.0, 0.0, a.sumD,
                           nrhs, xs);
        __syncthreads();
        mv_rows<T, NR, 1>(a.Nm + a.offN[i], nullptr, nd, r0, r1 - r0, 0, nd, xs, nrhs, ys, part);
        for (int tt = th.k0; tt < r1 - r0 && th.r < nrhs; tt += kTPR)
          st_co(&a.y_loc[(size_t)th.r * a.sumD + d0 + r0 + tt], -ys[tt * NR + th.r]);
        __syncthreads();
      }
      flag_sync(f.flags, nb, ++epoch, f.err);
      // ---- D: z = -N^T (P lambda) rows
      for (int u = blockIdx.x, t = 0; u < nunits; u += nb, ++t) {
        const bool use_tab = t < f.tab_units;
        const int i = u / f.S, q = u % f.S;
        const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
        int r0, r1;
        slice_rows(nd, f.S, q, r0, r1);
        if (use_tab) gather_dl_tab<NR>(tsl + 4 * t * f.tab_nd, nd, a.y_loc, nullptr, 1.0, 0.0, a.sumD, nrhs, xs);
        else gather_dl<NR>(a.dl_own_ptr, a.dl_own_slot, a.dl_l2g, d0, nd, a.y_loc, nullptr, 1.0, 0.0, a.sumD,
                           nrhs, xs);
        __syncthreads();
        mv_rows<T, NR, 1>(a.NTm + a.offN[i], nullptr, nd, r0, r1 - r0, 0, nd, xs, nrhs, ys, part);
        for (int tt = th.k0; tt < r1 - r0 && th.r < nrhs; tt += kTPR)
          st_co(&a.z_loc[(size_t)th.r * a.sumD + d0 + r0 + tt], -ys[tt * NR + th.r]);
        __syncthreads();
      }
      flag_sync(f.flags, nb, ++epoch, f.err);
    }

    // ---- E: eta, rows of L^T(:, Delta) eta
    for (int u = blockIdx.x, t = 0; u < nunits; u += nb, ++t) {
      const bool use_tab = t < f.tab_units;
      const int i = u / f.S, q = u % f.S;
      const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
      const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
      const int ng = np + nd;
      int r0, r1;
      slice_rows(ng, f.S, q, r0, r1);
      {
        const double* zA = a.theta != 0.0 ? a.z_loc : a.lam_loc;
        const double* zB = a.theta != 0.0 ? a.lam_loc : nullptr;
        const double ca = a.theta != 0.0 ? a.theta : 1.0, cb = a.theta != 0.0 ? 1.0 - a.theta : 0.0;
        if (use_tab) gather_dl_tab<NR>(tsl + 4 * t * f.tab_nd, nd, zA, zB, ca, cb, a.sumD, nrhs, xs);
        else gather_dl<NR>(a.dl_own_ptr, a.dl_own_slot, a.dl_l2g, d0, nd, zA, zB, ca, cb, a.sumD, nrhs, xs);
      }
      __syncthreads();
      mv_rows<T, NR, 1>(a.LTm + a.offG[i], nullptr, ng, r0, r1 - r0, np, nd, xs, nrhs, ys, part);
      for (int tt = th.k0; tt < r1 - r0 && th.r < nrhs; tt += kTPR) {
        const int r = th.r, row = r0 + tt;
        if (row < np) st_co(&a.nu_loc[(size_t)r * a.sumP + p0 + row], ys[tt * NR + r]);
        else st_wg(&a.t_loc[(size_t)r * a.sumD + d0 + row - np], ys[tt * NR + r], slot_state);
      }
      __syncthreads();
    }
    flag_sync(f.flags, nb, ++epoch, f.err);

    // ---- F: coarse nu at the corners, rows of u = A r_it; partial (u, r_it)
    double dacc = 0.0;    // right-hand side th.r
    if (f.dist) {
      coarse_gather(a, a.nu_loc, (const double*)nullptr, nrhs, f.ug);
      flag_sync(f.flags, nb, ++epoch, f.err);
      coarse_rows<NR>(f.X1t, a.nP, a.nP, f.ug, nrhs, lds, f.lds_total, f.cg1);
      flag_sync(f.flags, nb, ++epoch, f.err);
    }
    for (int u = blockIdx.x, t = 0; u < nunits; u += nb, ++t) {
      const bool use_tab = t < f.tab_units;
      const int i = u / f.S, q = u % f.S;
      const int p0 = a.pi_off[i], np = a.pi_off[i + 1] - p0;
      const int d0 = a.dl_off[i], nd = a.dl_off[i + 1] - d0;
      const int ng = np + nd;
      if (np > 0 && f.dist) {
        for (int e = threadIdx.x; e < 2 * np * nrhs; e += kBlock) {
          const int kind = e / (np * nrhs), b = (e / nrhs) % np, r = e % nrhs;
          cor[kind][b][r] = ld_co(&f.cg1[(size_t)r * 2 * a.nP + (kind ? a.nP : 0) + a.pi_l2g[p0 + b]]);
        }
        __syncthreads();
      } else if (np > 0) {
        for (int r = 0; r < nrhs; ++r) {
          for (int pq = threadIdx.x; pq < a.nP; pq += kBlock) {
            double s1 = 0.0;
            if (f.tab_pi) {
              const int4 sl4 = reinterpret_cast<const int4*>(tpi)[pq];
              const int so[kMaxOwn] = {sl4.x, sl4.y, sl4.z, sl4.w};
              double v1[kMaxOwn];
#pragma unroll
              for (int o = 0; o < kMaxOwn; ++o) v1[o] = so[o] >= 0 ? ld_co(&a.nu_loc[(size_t)r * a.sumP + so[o]]) : 0.0;
#pragma unroll
              for (int o = 0; o < kMaxOwn; ++o) s1 += v1[o];
            } else {
              for (int o = a.pi_own_ptr[pq]; o < a.pi_own_ptr[pq + 1]; ++o)
                s1 += ld_co(&a.nu_loc[(size_t)r * a.sumP + a.pi_own_slot[o]]);
            }
            cu[pq] = s1;
          }
          __syncthreads();
          const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
          for (int dd = wid; dd < 2 * np; dd += kWaves) {
            const int b = dd >> 1, kind = dd & 1;
            const int row = (kind ? a.nP : 0) + a.pi_l2g[p0 + b];
            double s = 0.0;
            for (int c = lane; c < a.nP; c += 64) s += a.X1[(long long)c * 2 * a.nP + row] * cu[c];
            s = wave_sum(s);
            if (lane == 0) cor[kind][b][r] = s;
          }
          __syncthreads();
        }
      }
      // mu and e at the corners (from B) next to nu and -D nu (cor)
      for (int e = threadIdx.x; e < 2 * np * nrhs; e += kBlock) {
        const int kind = e / (np * nrhs), b = (e / nrhs) % np, r = e % nrhs;
        cms[kind][b][r] = ld_wg(&(kind ? f.e_slot : f.mu_slot)[(size_t)r * a.sumP + p0 + b], slot_state);
      }
      __syncthreads();
      int r0, r1;
      slice_rows(nd, f.S, q, r0, r1);
      const int nrow = r1 - r0;
      {
        // the slice's rows of the Pi columns of G and L^T, staged in LDS
        // (xs is free in this phase): gw[b][t] = G(np + r0 + t, b), lw likewise
        const T* G = a.Gm + a.offG[i];
        const T* LT = a.LTm + a.offG[i];
        for (int e = threadIdx.x; e < np * nrow; e += kBlock) {
          const int b = e / nrow, tt = e % nrow;
          xs[e] = (double)G[(long long)b * ng + np + r0 + tt];
          xs[np * nrow + e] = (double)LT[(long long)b * ng + np + r0 + tt];
        }
        __syncthreads();
      }
      const double* gw = xs;
      const double* lw = xs + np * nrow;
      for (int kb = th.k0; kb < nrow && th.r < nrhs; kb += kLB * kTPR) {
        const int r = th.r;
        double sv[kLB], tv[kLB], rc[kLB];
#pragma unroll
        for (int u = 0; u < kLB; ++u) {
          const int tt = kb + u * kTPR;
          sv[u] = 0.0;
          tv[u] = 0.0;
          rc[u] = 0.0;
          if (tt < nrow) {
            const int k = r0 + tt;
            const size_t el = (size_t)r * a.sumD + d0 + k;
            const int g = use_tab ? tg[t * f.tab_nd + k] & ~kOwnerFlag : a.dl_l2g[d0 + k];
            sv[u] = ld_wg(&a.s_loc[el], slot_state);
            tv[u] = ld_wg(&a.t_loc[el], slot_state);
            rc[u] = slot_state ? f.rsl[el] : ld_co(&r_cur[(size_t)r * a.nD + g]);
          }
        }
#pragma unroll
        for (int u = 0; u < kLB; ++u) {
          const int tt = kb + u * kTPR;
          if (tt >= nrow) continue;
          const int row = r0 + tt;
          double acc = sv[u] + tv[u];
          for (int b = 0; b < np; ++b) {
            acc -= gw[b * nrow + tt] * (cms[0][b][r] + cor[0][b][r]);
            acc += lw[b * nrow + tt] * (cms[1][b][r] + cor[1][b][r]);
          }
          st_co(&a.w_loc[(size_t)r * a.sumD + d0 + row], acc);
          dacc += acc * rc[u];
        }
      }
      __syncthreads();
    }
    block_sum_grp<NR>(dacc, &f.part[blockIdx.x], nb, nrhs, redv);
    flag_sync(f.flags, nb, ++epoch, f.err);
  }

  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int r = 0; r < nrhs; ++r) {
      double* sc = f.scal + (size_t)r * 8;
      sc[0] = sc_rr[r]; sc[1] = sc_bb[r]; sc[5] = sc_done[r]; sc[6] = sc_it[r];
      sc[7] = (sc_rr[r] == sc_rr[r]) ? 0.0 : 1.0;
      sc[2] = (double)epoch;
    }
  }
}

}  // namespace ddelm
