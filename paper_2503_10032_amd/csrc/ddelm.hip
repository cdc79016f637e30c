// C ABI of the DDELM-NN library: context, setup, factorisation, solve and
// evaluation on one gfx950 GPU.  See include/ddelm.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ddelm.h"
#include "geometry.hpp"
#include "kernels_setup.hpp"
#include "kernels_solve.hpp"
#include "kernels_cg.hpp"
#include "kernels_qr.hpp"

using namespace ddelm;

namespace {

struct HipError {
  hipError_t e;
  const char* what;
  int line;
};

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) throw HipError{e_, #x, __LINE__}; \
  } while (0)

struct StatusError {
  ddelm_status st;
  std::string msg;
};

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    free();
    n = count;
    if (count == 0) return;
    hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      n = 0;
      throw StatusError{DDELM_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    alloc(h.size());
    if (!h.empty()) HIPCHK(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void zero(hipStream_t s) {
    if (n) HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
  void free() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DBuf() { free(); }
};

struct RowSetDev {
  DBuf<int> row0, ptr;
  DBuf<Term> terms;
  void upload(const RowSet& r, hipStream_t s) {
    row0.upload(r.row0, s);
    ptr.upload(r.ptr, s);
    terms.upload(r.terms, s);
  }
};

// Device copies of small per-call descriptor arrays: one device buffer and one
// pinned host staging buffer, filled by a bump pointer and reset at the start
// of every API call (the previous call has drained the stream).
struct Arena {
  char* dev = nullptr;
  char* host = nullptr;
  size_t cap = 0, used = 0;
  void ensure(size_t c) {
    if (c <= cap) return;
    release();
    HIPCHK(hipMalloc((void**)&dev, c));
    HIPCHK(hipHostMalloc((void**)&host, c, hipHostMallocDefault));
    cap = c;
  }
  void release() {
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    dev = host = nullptr;
    cap = used = 0;
  }
  void reset() { used = 0; }
  template <typename T>
  T* put(const T* data, size_t n, hipStream_t s) {
    const size_t bytes = n * sizeof(T);
    const size_t off = (used + 255) & ~size_t(255);
    if (off + bytes > cap) throw StatusError{DDELM_E_NOMEM, "descriptor arena exhausted"};
    if (bytes) {
      std::memcpy(host + off, data, bytes);
      HIPCHK(hipMemcpyAsync(dev + off, host + off, bytes, hipMemcpyHostToDevice, s));
    }
    used = off + bytes;
    return reinterpret_cast<T*>(dev + off);
  }
  template <typename T>
  T* put(const std::vector<T>& v, hipStream_t s) { return put(v.data(), v.size(), s); }
  ~Arena() { release(); }
};

__host__ __device__ inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace

struct ddelm_ctx_s {
  hipStream_t stream = nullptr;
  ddelm_options opt;
  Geometry geo;
  int N = 0, M = 0, n_int = 0;
  int nP = 0, nD = 0, sumP = 0, sumD = 0;
  bool factored = false;
  bool use_nn = true;     // theta != 0: Kbar factored and P applied
  std::string err;
  int device = 0;
  int num_cu = 0;

  // problem copies
  DBuf<double> W, b, geom, x_int;
  RowSetDev rsK, rsA, rsKb, rsAb;
  // sizes per subdomain
  std::vector<int> h_m, h_nG, h_nD, h_nP, h_nB;
  std::vector<long long> h_offB;     // offsets into g_B
  std::vector<long long> h_offm;     // offsets into packed row space (sum m)
  long long summ = 0;
  // QR: 2N matrices (K_c then Kbar), fp64
  DBuf<double> qrA, tau, Tbuf;
  int npanel = 0;
  DBuf<QRDesc> qrdesc;
  std::vector<QRDesc> h_qrdesc;
  int max_ncols = 0;
  DBuf<long long> qr_coff;
  DBuf<int> qr_ldc, qr_cn;
  // local matrices
  DBuf<double> Am, CD;                 // n_G x M, n_D x M per subdomain
  std::vector<long long> h_offAm, h_offCD;
  DBuf<double> QG;                     // M x n_G per subdomain (Q_G^T)
  std::vector<long long> h_offQG;
  DBuf<double> Gm, Lm, LTm, Nm, NTm;
  std::vector<long long> h_offG, h_offN;
  DBuf<long long> offG, offN;
  // coarse
  DBuf<double> Spi, Sfac, Sinv, Dpp, Gs, Zm, Ztm, Wm, X1;
  DBuf<unsigned> flags;                // [0] barrier err, [1] cholesky err, [2..3] barrier
  // indexing on device
  DBuf<int> pi_off, dl_off, pi_l2g, dl_l2g, pi_own_ptr, pi_own_slot, dl_own_ptr, dl_own_slot, pi_slot_sub;
  DBuf<int> nG_dev;
  // solve workspaces
  int cap_nrhs = 0;
  DBuf<double> F;                      // [nrhs][summ]
  DBuf<long long> f_off;               // per subdomain offset into F
  DBuf<int> f_ld, f_cn, f_cnM;
  DBuf<double> s_loc, l_loc, rho_loc, psi_loc, lam_loc, y_loc, z_loc, t_loc, nu_loc, w_loc, c1, c2, pif;
  DBuf<double> cg_x, cg_r, cg_p, cg_p1, cg_w, cg_b, cg_part, cg_scal, mu_slot, e_slot;
  int cg_blocks = 0, cg_slices = 0;
  DBuf<unsigned> bar;
  DBuf<int> sizes_dev;                 // per subdomain M, n_I, n_B, m, n_G
  Arena arena;
  DBuf<long long> offm_d, offB_d, offQG_d, offAm_d;
  // phase timing (HIP events on the stream)
  hipEvent_t ev[10] = {};
  double phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  void mark(int k) {
    if (!ev[k]) HIPCHK(hipEventCreate(&ev[k]));
    HIPCHK(hipEventRecord(ev[k], stream));
  }
  double span(int a, int b) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[a], ev[b]));
    return (double)ms;
  }
  ~ddelm_ctx_s() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }

  void fail(ddelm_status st, const std::string& m) { throw StatusError{st, m}; }
};

namespace {

template <typename F>
ddelm_status run_guarded(ddelm_ctx c, F&& fn) {
  try {
    fn();
    return DDELM_OK;
  } catch (const StatusError& e) {
    if (c) c->err = e.msg;
    return e.st;
  } catch (const HipError& e) {
    if (c) c->err = std::string("HIP error ") + hipGetErrorString(e.e) + " at " + e.what + " (line " +
                    std::to_string(e.line) + ")";
    return DDELM_E_HIP;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return DDELM_E_HIP;
  }
}

// --------------------------------------------------------------- launch helpers

template <typename T>
void launch_qr_panel(int rpt, dim3 grid, hipStream_t s, const QRDesc* d, T* A, T* tau, int k) {
  switch (rpt) {
#define CASE(R) case R: k_qr_panel<T, R><<<grid, kBlock, 0, s>>>(d, A, tau, k); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12)
#undef CASE
    default: throw StatusError{DDELM_E_SHAPE, "local row count too large (max 3072)"};
  }
  HIPCHK(hipGetLastError());
}

template <typename T>
void launch_qr_panel16(int rpt, dim3 grid, hipStream_t s, const QRDesc* d, T* A, T* tau, T* Tb, int k, int panel,
                       int npanel) {
  switch (rpt) {
#define CASE(R) case R: k_qr_panel16<T, R><<<grid, kPanelThreads, 0, s>>>(d, A, tau, Tb, k, panel, npanel); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
    default: throw StatusError{DDELM_E_SHAPE, "local row count too large (max 3072)"};
  }
  HIPCHK(hipGetLastError());
}

template <typename T>
void launch_qr_apply(int rpt, dim3 grid, hipStream_t s, const QRDesc* d, const T* A, const T* tau, int j0, int j1,
                     T* C, const long long* coff, const int* ldc, const int* cn, int c0, int reverse) {
  switch (rpt) {
#define CASE(R) case R: k_qr_apply<T, R><<<grid, kBlock, 0, s>>>(d, A, tau, j0, j1, C, coff, ldc, cn, c0, reverse); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12)
#undef CASE
    default: throw StatusError{DDELM_E_SHAPE, "local row count too large (max 3072)"};
  }
  HIPCHK(hipGetLastError());
}

template <typename T>
void gemm_batch(ddelm_ctx c, const std::vector<GemmDesc>& h, const T* A, const T* B, T* C, int transA, double alpha,
                double beta) {
  if (h.empty()) return;
  int mm = 0, nn = 0;
  for (auto& g : h) { mm = std::max(mm, g.m); nn = std::max(nn, g.n); }
  if (mm == 0 || nn == 0) return;
  const GemmDesc* d = c->arena.put(h, c->stream);
  dim3 grid(ceil_div(mm, 16), ceil_div(nn, 16), (unsigned)h.size());
  k_gemm<T, T><<<grid, kBlock, 0, c->stream>>>(d, A, B, C, transA, alpha, beta);
  HIPCHK(hipGetLastError());
}

template <typename T>
void copy_batch(ddelm_ctx c, const std::vector<CopyDesc>& h, const T* S, T* D) {
  if (h.empty()) return;
  long long mx = 0;
  for (auto& cd : h) mx = std::max(mx, (long long)cd.rows * cd.cols);
  if (mx == 0) return;
  const CopyDesc* d = c->arena.put(h, c->stream);
  dim3 grid(std::min(ceil_div(mx, kBlock), 1024), (unsigned)h.size());
  k_copy2d<T, T><<<grid, kBlock, 0, c->stream>>>(d, S, D);
  HIPCHK(hipGetLastError());
}

void fill(hipStream_t s, double* p, long long n, double v) {
  if (n <= 0) return;
  k_fill<<<std::min(ceil_div(n, kBlock), 4096), kBlock, 0, s>>>(p, n, v);
  HIPCHK(hipGetLastError());
}

int rows_per_thread(int m) { return ceil_div(m, kBlock); }

// --------------------------------------------------------------- feature assembly into column-major blocks
void assemble_features(ddelm_ctx c, const RowSetDev& rs, int max_rows, double* out, const std::vector<long long>& off,
                       const std::vector<int>& ld, int sub0, int nsub) {
  if (max_rows == 0 || nsub == 0) return;
  FeatArgs a;
  a.row0 = rs.row0.p; a.ptr = rs.ptr.p; a.terms = rs.terms.p;
  a.W = c->W.p; a.bias = c->b.p; a.geom = c->geom.p;
  a.off = c->arena.put(off, c->stream); a.ld = c->arena.put(ld, c->stream); a.M = c->M; a.sub0 = sub0;
  dim3 grid(ceil_div(max_rows, 64), ceil_div(c->M, 4), nsub);
  k_features<double><<<grid, kBlock, 0, c->stream>>>(a, out);
  HIPCHK(hipGetLastError());
}

OpArgs<double> op_args(ddelm_ctx c, int nrhs) {
  OpArgs<double> a;
  a.N = c->N; a.nP = c->nP; a.nD = c->nD; a.nrhs = nrhs;
  a.sumP = c->sumP; a.sumD = c->sumD; a.theta = c->use_nn ? c->opt.theta : 0.0;
  a.pi_off = c->pi_off.p; a.dl_off = c->dl_off.p; a.pi_l2g = c->pi_l2g.p; a.dl_l2g = c->dl_l2g.p;
  a.pi_own_ptr = c->pi_own_ptr.p; a.pi_own_slot = c->pi_own_slot.p;
  a.dl_own_ptr = c->dl_own_ptr.p; a.dl_own_slot = c->dl_own_slot.p;
  a.offG = c->offG.p; a.offN = c->offN.p;
  a.Gm = c->Gm.p; a.Lm = c->Lm.p; a.LTm = c->LTm.p; a.Nm = c->Nm.p; a.NTm = c->NTm.p;
  a.X1 = c->X1.p;
  a.s_loc = c->s_loc.p; a.l_loc = c->l_loc.p; a.rho_loc = c->rho_loc.p; a.psi_loc = c->psi_loc.p;
  a.lam_loc = c->lam_loc.p; a.y_loc = c->y_loc.p; a.z_loc = c->z_loc.p; a.t_loc = c->t_loc.p;
  a.nu_loc = c->nu_loc.p; a.w_loc = c->w_loc.p; a.c1 = c->c1.p; a.c2 = c->c2.p;
  a.hP = nullptr; a.hD = nullptr;
  return a;
}

size_t local_smem(ddelm_ctx c) {
  return sizeof(double) * (size_t)std::max({c->geo.max_nG, 2 * c->nP, 1});
}

}  // namespace

// =============================================================== kernels that need the context layout

namespace {

// f^i = [f_I; g_B; 0] into F[r][off_m[i] + row]
__global__ void k_rhs_assemble(int N, int n_int, const int* __restrict__ sizes, const long long* __restrict__ offm,
                               const long long* __restrict__ offB, long long summ, long long sumB,
                               const double* __restrict__ fI, const double* __restrict__ gB, double* __restrict__ F) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int nB = sizes[5 * i + 2], m = sizes[5 * i + 3];
  double* Fi = F + (size_t)r * summ + offm[i];
  for (int row = threadIdx.x; row < m; row += kBlock) {
    double v = 0.0;
    if (row < n_int) v = fI[((size_t)r * N + i) * n_int + row];
    else if (row < n_int + nB) v = gB[(size_t)r * sumB + offB[i] + row - n_int];
    Fi[row] = v;
  }
}

// p_G = Q_G (Q^T f)[:M]; rho_loc = p_P (Pi slots), s_loc = p_D (Delta slots)
// (interface rows of f are zero in a standard solve)
__global__ void k_rhs_proj(int M, const int* __restrict__ sizes, const int* __restrict__ pi_off,
                           const int* __restrict__ dl_off, const long long* __restrict__ offQG,
                           const double* __restrict__ QG, const long long* __restrict__ offm, long long summ,
                           const double* __restrict__ F, int sumP, int sumD, double* __restrict__ rho_loc,
                           double* __restrict__ s_loc) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int ng = sizes[5 * i + 4];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  extern __shared__ double al[];
  const double* Fi = F + (size_t)r * summ + offm[i];
  for (int k = threadIdx.x; k < M; k += kBlock) al[k] = Fi[k];
  __syncthreads();
  const double* Q = QG + offQG[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double acc = 0.0;
    for (int k = 0; k < M; ++k) acc += Q[(long long)t * M + k] * al[k];
    if (t < np) rho_loc[(size_t)r * sumP + p0 + t] = acc;
    else s_loc[(size_t)r * sumD + d0 + t - np] = acc;
  }
}

// ad = A_m c_f0; psi_loc = -ad_P, l_loc = -ad_D
__global__ void k_rhs_flux(int M, const int* __restrict__ sizes, const int* __restrict__ pi_off,
                           const int* __restrict__ dl_off, const long long* __restrict__ offAm,
                           const double* __restrict__ Am, const long long* __restrict__ offm, long long summ,
                           const double* __restrict__ F, int sumP, int sumD, double* __restrict__ psi_loc,
                           double* __restrict__ l_loc) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int ng = sizes[5 * i + 4];
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i];
  extern __shared__ double cf[];
  const double* Fi = F + (size_t)r * summ + offm[i];
  for (int k = threadIdx.x; k < M; k += kBlock) cf[k] = Fi[k];
  __syncthreads();
  const double* A = Am + offAm[i];
  for (int t = threadIdx.x; t < ng; t += kBlock) {
    double acc = 0.0;
    for (int k = 0; k < M; ++k) acc += A[(long long)k * ng + t] * cf[k];
    if (t < np) psi_loc[(size_t)r * sumP + p0 + t] = -acc;
    else l_loc[(size_t)r * sumD + d0 + t - np] = -acc;
  }
}

// c^i = c_f0 + E [mu_P(Pi^i); mu_D(Delta^i)]  with E = R^{-1} Q_G^T stored in
// the K_c matrix (rows 0..M-1 of columns M.., leading dimension m)
__global__ void k_recover(int M, int nP, int nD, const int* __restrict__ sizes, const int* __restrict__ pi_off,
                          const int* __restrict__ dl_off, const int* __restrict__ pi_l2g,
                          const int* __restrict__ dl_l2g, const QRDesc* __restrict__ desc,
                          const double* __restrict__ qrA, const long long* __restrict__ offm, long long summ,
                          const double* __restrict__ F, const double* __restrict__ mu_pi,
                          const double* __restrict__ mu_dl, int N, double* __restrict__ coef) {
  const int i = blockIdx.x, r = blockIdx.y;
  const int p0 = pi_off[i], np = pi_off[i + 1] - p0, d0 = dl_off[i], nd = dl_off[i + 1] - d0;
  extern __shared__ double mus[];
  for (int a = threadIdx.x; a < np + nd; a += kBlock)
    mus[a] = a < np ? mu_pi[(size_t)r * nP + pi_l2g[p0 + a]] : mu_dl[(size_t)r * nD + dl_l2g[d0 + a - np]];
  __syncthreads();
  const QRDesc d = desc[i];
  const double* E = qrA + d.off + (long long)M * d.ld;
  const double* Fi = F + (size_t)r * summ + offm[i];
  for (int k = threadIdx.x; k < M; k += kBlock) {
    double acc = Fi[k];
    for (int a = 0; a < np + nd; ++a) acc += E[(long long)a * d.ld + k] * mus[a];
    coef[((size_t)r * N + i) * M + k] = acc;
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
__global__ void k_set_units(const long long* __restrict__ pos, long long n, double* __restrict__ A) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) A[pos[e]] = 1.0;
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
__global__ void __launch_bounds__(kBlock) k_cg_wdot(OpArgs<double> a, CGState s) {
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
    sc[0] = bb; sc[1] = bb; sc[2] = 0; sc[3] = 0; sc[4] = 0;
    sc[5] = (bb == 0.0) ? 1.0 : 0.0;
    sc[6] = 0; sc[7] = 0;
  }
}

// ---------------------------------------------------------------- evaluation
__global__ void k_evaluate(int nx, int ny, int M, int N, double lo0, double lo1, double h0, double h1,
                           const double* __restrict__ W, const double* __restrict__ bias,
                           const double* __restrict__ coef, long long npts, const double* __restrict__ x,
                           double* __restrict__ u, double* __restrict__ grad, int r) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= npts) return;
  const double px = x[2 * e], py = x[2 * e + 1];
  int ix = (int)ceil((px - lo0) / h0) - 1, iy = (int)ceil((py - lo1) / h1) - 1;
  ix = ix < 0 ? 0 : (ix > nx - 1 ? nx - 1 : ix);
  iy = iy < 0 ? 0 : (iy > ny - 1 ? ny - 1 : iy);
  const int i = iy * nx + ix;
  const double hx = 0.5 * h0, hy = 0.5 * h1;
  const double cx = lo0 + (ix + 0.5) * h0, cy = lo1 + (iy + 0.5) * h1;
  const double xi0 = (px - cx) / hx, xi1 = (py - cy) / hy;
  const double* c = coef + ((size_t)r * N + i) * M;
  double acc = 0.0, g0 = 0.0, g1 = 0.0;
  for (int j = 0; j < M; ++j) {
    const double w0 = W[((size_t)i * M + j) * 2], w1 = W[((size_t)i * M + j) * 2 + 1];
    const double t = tanh(w0 * xi0 + w1 * xi1 + bias[(size_t)i * M + j]);
    acc += c[j] * t;
    const double dt = c[j] * (1.0 - t * t);
    g0 += dt * w0;
    g1 += dt * w1;
  }
  u[(size_t)r * npts + e] = acc;
  if (grad) {
    grad[((size_t)r * npts + e) * 2] = g0 / hx;
    grad[((size_t)r * npts + e) * 2 + 1] = g1 / hy;
  }
}

}  // namespace

// =============================================================== host implementation

namespace {

void alloc_solve_workspace(ddelm_ctx c, int nrhs) {
  if (nrhs <= c->cap_nrhs) return;
  hipStream_t s = c->stream;
  c->F.alloc((size_t)nrhs * c->summ);
  const size_t D = (size_t)nrhs * std::max(c->sumD, 1), P = (size_t)nrhs * std::max(c->sumP, 1);
  for (DBuf<double>* b : {&c->s_loc, &c->l_loc, &c->lam_loc, &c->y_loc, &c->z_loc, &c->t_loc, &c->w_loc}) b->alloc(D);
  for (DBuf<double>* b : {&c->rho_loc, &c->psi_loc, &c->nu_loc}) b->alloc(P);
  const size_t C = (size_t)nrhs * std::max(2 * c->nP, 1);
  c->c1.alloc(C);
  c->c2.alloc(C);
  c->pif.alloc((size_t)nrhs * std::max(c->nP, 1));
  const size_t V = (size_t)nrhs * std::max(c->nD, 1);
  for (DBuf<double>* b : {&c->cg_x, &c->cg_r, &c->cg_p, &c->cg_p1, &c->cg_w, &c->cg_b}) b->alloc(V);
  c->mu_slot.alloc(P);
  c->e_slot.alloc(P);
  c->mu_slot.zero(s);
  c->e_slot.zero(s);
  c->cg_part.alloc((size_t)2 * nrhs * 4096);
  c->cg_scal.alloc((size_t)nrhs * 8);
  // zero everything once so unused Pi/Delta slots never hold garbage
  for (DBuf<double>* b : {&c->s_loc, &c->l_loc, &c->lam_loc, &c->y_loc, &c->z_loc, &c->t_loc, &c->w_loc, &c->rho_loc,
                          &c->psi_loc, &c->nu_loc, &c->c1, &c->c2, &c->pif})
    b->zero(s);
  std::vector<long long> foff(c->N);
  std::vector<int> fld(c->N, (int)c->summ), fcn(c->N, nrhs);
  for (int i = 0; i < c->N; ++i) foff[i] = c->h_offm[i];
  c->f_off.upload(foff, s);
  c->f_ld.upload(fld, s);
  c->f_cn.upload(fcn, s);
  c->cap_nrhs = nrhs;
  HIPCHK(hipStreamSynchronize(s));
}

// one application of the operator phases after the first stage
void run_phases_after_stage1(ddelm_ctx c, OpArgs<double>& a, int nrhs, const double* hP) {
  hipStream_t s = c->stream;
  const size_t sm = local_smem(c);
  const dim3 gl(c->N, nrhs);
  if (c->nP > 0) {
    OpArgs<double> ah = a;
    ah.hP = hP;
    k_ph_coarse1<double><<<dim3(ceil_div(2 * c->nP, kBlock), nrhs), kBlock, sm, s>>>(ah);
    HIPCHK(hipGetLastError());
  }
  k_ph_lam<double><<<gl, kBlock, 0, s>>>(a);
  HIPCHK(hipGetLastError());
  if (a.theta != 0.0) {
    k_ph_P1<double><<<gl, kBlock, sm, s>>>(a);
    k_ph_P2<double><<<gl, kBlock, sm, s>>>(a);
    HIPCHK(hipGetLastError());
  }
  k_ph_eta<double><<<gl, kBlock, sm, s>>>(a);
  HIPCHK(hipGetLastError());
  if (c->nP > 0) {
    k_ph_coarse2<double><<<dim3(ceil_div(2 * c->nP, kBlock), nrhs), kBlock, sm, s>>>(a);
    HIPCHK(hipGetLastError());
  }
  k_ph_w<double><<<gl, kBlock, 0, s>>>(a);
  HIPCHK(hipGetLastError());
}

CGState cg_state(ddelm_ctx c, int nrhs, int nblk) {
  CGState s;
  s.x = c->cg_x.p; s.r = c->cg_r.p; s.p = c->cg_p.p; s.w = c->cg_w.p;
  s.part = c->cg_part.p; s.scal = c->cg_scal.p;
  s.n = c->nD; s.nrhs = nrhs; s.nblk = nblk;
  s.tol = c->opt.tol; s.maxit = c->opt.maxit;
  return s;
}

int cg_multilaunch(ddelm_ctx c, int nrhs) {
  hipStream_t s = c->stream;
  const int nblk = std::max(1, std::min(256, ceil_div(c->nD, kBlock)));
  CGState st = cg_state(c, nrhs, nblk);
  OpArgs<double> a = op_args(c, nrhs);
  const size_t sm = local_smem(c);
  k_cg_init<<<dim3(nblk, nrhs), kBlock, 0, s>>>(st, c->cg_b.p);
  k_cg_init2<<<nrhs, kBlock, 0, s>>>(st);
  HIPCHK(hipGetLastError());
  std::vector<double> sc((size_t)nrhs * 8);
  int it = 0;
  const int check_every = 16;
  while (it < c->opt.maxit) {
    const int nstep = std::min(check_every, c->opt.maxit - it);
    for (int k = 0; k < nstep; ++k) {
      k_ph_local_v<double><<<dim3(c->N, nrhs), kBlock, sm, s>>>(a, st.p);
      run_phases_after_stage1(c, a, nrhs, nullptr);
      k_cg_wdot<<<dim3(nblk, nrhs), kBlock, 0, s>>>(a, st);
      k_cg_alpha<<<nrhs, kBlock, 0, s>>>(st);
      k_cg_axpy<<<dim3(nblk, nrhs), kBlock, 0, s>>>(st);
      k_cg_beta<<<nrhs, kBlock, 0, s>>>(st);
      k_cg_pupd<<<dim3(nblk, nrhs), kBlock, 0, s>>>(st);
      HIPCHK(hipGetLastError());
    }
    it += nstep;
    HIPCHK(hipMemcpyAsync(sc.data(), c->cg_scal.p, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool all = true;
    for (int r = 0; r < nrhs; ++r) all = all && sc[8 * r + 5] != 0.0;
    if (all) break;
  }
  return it;
}

template <int NR>
void launch_fused(ddelm_ctx c, int nrhs) {
  hipStream_t s = c->stream;
  const Geometry& g = c->geo;
  FusedArgs<double> f;
  f.a = op_args(c, nrhs);
  int S = 1;
  if (const char* env = getenv("DDELM_CG_SLICES")) S = std::max(1, std::min(8, atoi(env)));
  else S = std::max(1, std::min(4, 128 / std::max(c->N, 1)));
  f.S = S;
  f.nrhs = nrhs;
  f.tol = c->opt.tol;
  f.maxit = c->opt.maxit;
  f.x = c->cg_x.p; f.r = c->cg_r.p; f.p0 = c->cg_p.p; f.p1 = c->cg_p1.p; f.w = c->cg_w.p;
  f.part = c->cg_part.p; f.mu_slot = c->mu_slot.p; f.e_slot = c->e_slot.p; f.scal = c->cg_scal.p;
  f.err = c->flags.p;
  const int xs = std::max(g.max_nD, 1) * NR;
  const int ys = 2 * std::max(g.max_nG, 1) * NR;
  const int part = kBlock * 2 * NR;
  const int cu = std::max(2 * c->nP, 1);
  f.lds_ys = xs;
  f.lds_part = xs + ys;
  f.lds_cu = xs + ys + part;
  const size_t smem = sizeof(double) * (size_t)(xs + ys + part + cu);
  if (smem > 160 * 1024) c->fail(DDELM_E_SHAPE, "CG workspace exceeds the LDS of one compute unit");
  const void* fn = (const void*)k_cg_fused<double, NR>;
  if (smem > 65536) HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  int per_cu = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, smem));
  if (per_cu < 1) c->fail(DDELM_E_SHAPE, "CG kernel cannot be resident");
  int nb = std::min(c->num_cu * std::min(per_cu, 2), c->N * S);
  if (const char* env = getenv("DDELM_CG_BLOCKS")) nb = std::max(1, std::min(nb, atoi(env)));
  nb = std::max(1, std::min(nb, 4096));
  f.flags = c->bar.p;
  HIPCHK(hipMemcpyAsync(f.r, c->cg_b.p, (size_t)nrhs * c->nD * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(c->bar.p, 0, (size_t)nb * kFlagStride * sizeof(unsigned), s));
  void* args[] = {(void*)&f};
  HIPCHK(hipLaunchCooperativeKernel(fn, dim3(nb), dim3(kBlock), args, smem, s));
  c->cg_blocks = nb;
  c->cg_slices = S;
}

void cg_persistent(ddelm_ctx c, int nrhs) {
  if (nrhs <= 1) launch_fused<1>(c, nrhs);
  else if (nrhs <= 2) launch_fused<2>(c, nrhs);
  else if (nrhs <= 4) launch_fused<4>(c, nrhs);
  else if (nrhs <= 8) launch_fused<8>(c, nrhs);
  else if (nrhs <= 16) launch_fused<16>(c, nrhs);
  else c->fail(DDELM_E_ARG, "the persistent CG handles at most 16 right-hand sides");
}

}  // namespace

// =============================================================== C ABI

extern "C" {

void ddelm_default_options(ddelm_options* o) {
  if (!o) return;
  o->theta = 0.999;
  o->coarse = 2;
  o->precision = 0;
  o->tol = 1e-8;
  o->maxit = 20000;
  o->max_nrhs = 1;
  o->cg_mode = 0;
  o->refine_maxit = 10;
  o->refine_tol = 1e-9;
  o->inner_tol = 1e-6;
}

ddelm_status ddelm_setup(ddelm_ctx* out, const ddelm_problem* prob, const ddelm_options* opt, void* stream) {
  if (!out || !prob) return DDELM_E_ARG;
  *out = nullptr;
  ddelm_ctx c = new ddelm_ctx_s();
  ddelm_status st = run_guarded(c, [&]() {
    c->stream = (hipStream_t)stream;
    if (opt) c->opt = *opt;
    else ddelm_default_options(&c->opt);
    const ddelm_options& o = c->opt;
    if (!(o.theta >= 0.0 && o.theta <= 1.0)) c->fail(DDELM_E_ARG, "theta must lie in [0, 1]");
    if (o.coarse < 0 || o.coarse > 2) c->fail(DDELM_E_ARG, "coarse must be 0, 1 or 2");
    if (o.coarse == 0 && o.theta != 0.0)
      c->fail(DDELM_E_ARG, "theta must be 0 without a coarse space (Kbar needs Dirichlet corner rows)");
    if (o.precision != 0) c->fail(DDELM_E_ARG, "precision 1 (mixed) is not available in this build");
    if (!(o.tol > 0.0 && o.tol < 1.0)) c->fail(DDELM_E_ARG, "tol must lie in (0, 1)");
    if (o.maxit < 1) c->fail(DDELM_E_ARG, "maxit must be >= 1");
    if (o.max_nrhs < 1 || o.max_nrhs > 64) c->fail(DDELM_E_ARG, "max_nrhs must lie in [1, 64]");
    if (o.cg_mode < 0 || o.cg_mode > 2) c->fail(DDELM_E_ARG, "cg_mode must be 0, 1 or 2");
    if (prob->M < 1 || prob->M > 1024) c->fail(DDELM_E_SHAPE, "M must lie in [1, 1024]");
    if (!prob->edge_s || !prob->x_int || !prob->W || !prob->b) c->fail(DDELM_E_ARG, "null array in problem");
    if (prob->n_extra < 0 || (prob->n_extra > 0 && !prob->extra_s)) c->fail(DDELM_E_ARG, "bad extra_s");
    HIPCHK(hipGetDevice(&c->device));
    HIPCHK(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    const int N = prob->nx * prob->ny;
    if (prob->nx < 1 || prob->ny < 1 || (long long)prob->nx * prob->ny > (1 << 20))
      c->fail(DDELM_E_SHAPE, "nx, ny out of range");
    if (prob->n_int < 1) c->fail(DDELM_E_SHAPE, "n_int must be >= 1");
    c->N = N; c->M = prob->M; c->n_int = prob->n_int;
    std::vector<double> xint((size_t)N * prob->n_int * 2);
    HIPCHK(hipMemcpyAsync(xint.data(), prob->x_int, xint.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::string e = c->geo.build(prob->nx, prob->ny, prob->lo, prob->hi, prob->p, prob->edge_s, prob->n_extra,
                                 prob->extra_s, prob->n_int, xint, o.coarse);
    if (!e.empty()) c->fail(DDELM_E_SHAPE, e);
    Geometry& g = c->geo;
    c->nP = g.n_pi; c->nD = g.n_dl;
    c->sumP = g.pi_off[N]; c->sumD = g.dl_off[N];
    c->use_nn = o.theta != 0.0 && o.coarse > 0;
    if (g.max_m > kBlock * 12) c->fail(DDELM_E_SHAPE, "local row count above 3072");
    if (g.max_nG > 4096) c->fail(DDELM_E_SHAPE, "too many interface points per subdomain");
    c->h_m.resize(N); c->h_nG.resize(N); c->h_nD.resize(N); c->h_nP.resize(N); c->h_nB.resize(N);
    c->h_offB.assign(N + 1, 0); c->h_offm.assign(N + 1, 0);
    std::vector<int> sizes(5 * (size_t)N);
    for (int i = 0; i < N; ++i) {
      const SubInfo& sb = g.subs[i];
      c->h_m[i] = sb.m(); c->h_nG[i] = sb.n_G(); c->h_nD[i] = sb.n_D; c->h_nP[i] = sb.n_P; c->h_nB[i] = sb.n_B;
      if (sb.m() < c->M) c->fail(DDELM_E_SHAPE, "M exceeds the row count of subdomain " + std::to_string(i));
      c->h_offB[i + 1] = c->h_offB[i] + sb.n_B;
      c->h_offm[i + 1] = c->h_offm[i] + sb.m();
      sizes[5 * i] = c->M; sizes[5 * i + 1] = sb.n_I; sizes[5 * i + 2] = sb.n_B; sizes[5 * i + 3] = sb.m();
      sizes[5 * i + 4] = sb.n_G();
    }
    c->summ = c->h_offm[N];
    hipStream_t s = c->stream;
    // problem copies
    c->W.alloc((size_t)N * c->M * 2);
    HIPCHK(hipMemcpyAsync(c->W.p, prob->W, c->W.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    c->b.alloc((size_t)N * c->M);
    HIPCHK(hipMemcpyAsync(c->b.p, prob->b, c->b.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    c->x_int.upload(xint, s);
    std::vector<double> geom(4 * (size_t)N);
    for (int i = 0; i < N; ++i) {
      geom[4 * i] = g.subs[i].cx; geom[4 * i + 1] = g.subs[i].cy;
      geom[4 * i + 2] = g.subs[i].hx; geom[4 * i + 3] = g.subs[i].hy;
    }
    c->geom.upload(geom, s);
    c->rsK.upload(g.rowsK, s); c->rsA.upload(g.rowsA, s); c->rsKb.upload(g.rowsKb, s); c->rsAb.upload(g.rowsAb, s);
    c->sizes_dev.upload(sizes, s);
    c->pi_off.upload(g.pi_off, s); c->dl_off.upload(g.dl_off, s);
    c->pi_l2g.upload(g.pi_loc2glob, s); c->dl_l2g.upload(g.dl_loc2glob, s);
    c->pi_own_ptr.upload(g.pi_own_ptr, s); c->pi_own_slot.upload(g.pi_own_slot, s);
    c->dl_own_ptr.upload(g.dl_own_ptr, s); c->dl_own_slot.upload(g.dl_own_slot, s);
    std::vector<int> slot_sub(std::max(c->sumP, 1), 0);
    for (int i = 0; i < N; ++i)
      for (int a = g.pi_off[i]; a < g.pi_off[i + 1]; ++a) slot_sub[a] = i;
    c->pi_slot_sub.upload(slot_sub, s);
    std::vector<int> nGv(c->h_nG);
    c->nG_dev.upload(nGv, s);
    {
      long long units = 0;
      for (int i = 0; i < N; ++i) units += c->h_nG[i] + c->h_nD[i];
      c->arena.ensure((size_t)(1 << 20) + (size_t)N * 1024 + (size_t)units * 16);
    }
    c->flags.alloc(8);
    c->flags.zero(s);
    c->bar.alloc((size_t)4096 * kFlagStride);
    c->bar.zero(s);
    HIPCHK(hipStreamSynchronize(s));
  });
  if (st != DDELM_OK) {
    // keep the context only to report the error through ddelm_last_error
    *out = c;
    return st;
  }
  *out = c;
  return DDELM_OK;
}

ddelm_status ddelm_factor(ddelm_ctx c) {
  if (!c) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    hipStream_t s = c->stream;
    const int N = c->N, M = c->M;
    const Geometry& g = c->geo;
    const bool nn = c->use_nn;
    HIPCHK(hipStreamSynchronize(s));
    c->arena.reset();
    const int nmat = nn ? 2 * N : N;
    // ---- layout of the QR matrices: K_c^i: m x (M + n_G), Kbar^i: m x (M + n_D)
    c->h_qrdesc.assign(nmat, QRDesc());
    long long off = 0, toff = 0;
    c->max_ncols = 0;
    for (int b = 0; b < nmat; ++b) {
      const int i = b % N;
      QRDesc d;
      d.off = off; d.m = c->h_m[i]; d.ld = c->h_m[i];
      d.ncols = M + (b < N ? c->h_nG[i] : c->h_nD[i]);
      d.nrefl = M; d.tau = toff; d.pad = 0;
      c->h_qrdesc[b] = d;
      off += (long long)d.ld * d.ncols;
      toff += M;
      c->max_ncols = std::max(c->max_ncols, d.ncols);
    }
    c->qrA.alloc(off);
    c->tau.alloc(toff);
    c->qrA.zero(s);
    c->qrdesc.upload(c->h_qrdesc, s);
    {
      std::vector<long long> coff(nmat);
      std::vector<int> ldc(nmat), cn(nmat);
      for (int b = 0; b < nmat; ++b) { coff[b] = c->h_qrdesc[b].off; ldc[b] = c->h_qrdesc[b].ld; cn[b] = c->h_qrdesc[b].ncols; }
      c->qr_coff.upload(coff, s); c->qr_ldc.upload(ldc, s); c->qr_cn.upload(cn, s);
    }
    c->mark(0);
    // ---- features: K_c (and Kbar) into the first M columns; A_m, Abar separately
    {
      std::vector<long long> o1(N), o2(N);
      std::vector<int> l1(N);
      for (int i = 0; i < N; ++i) { o1[i] = c->h_qrdesc[i].off; l1[i] = c->h_m[i]; }
      assemble_features(c, c->rsK, g.max_m, c->qrA.p, o1, l1, 0, N);
      if (nn) {
        for (int i = 0; i < N; ++i) o2[i] = c->h_qrdesc[N + i].off;
        assemble_features(c, c->rsKb, g.max_m, c->qrA.p, o2, l1, 0, N);
      }
      c->h_offAm.assign(N + 1, 0);
      c->h_offCD.assign(N + 1, 0);
      for (int i = 0; i < N; ++i) {
        c->h_offAm[i + 1] = c->h_offAm[i] + (long long)c->h_nG[i] * M;
        c->h_offCD[i + 1] = c->h_offCD[i] + (long long)c->h_nD[i] * M;
      }
      c->Am.alloc(std::max(c->h_offAm[N], 1ll));
      std::vector<int> ldA(c->h_nG.begin(), c->h_nG.end());
      assemble_features(c, c->rsA, g.max_nG, c->Am.p, std::vector<long long>(c->h_offAm.begin(), c->h_offAm.end() - 1),
                        ldA, 0, N);
      if (nn) {
        c->CD.alloc(std::max(c->h_offCD[N], 1ll));
        std::vector<int> ldC(c->h_nD.begin(), c->h_nD.end());
        assemble_features(c, c->rsAb, g.max_nD, c->CD.p,
                          std::vector<long long>(c->h_offCD.begin(), c->h_offCD.end() - 1), ldC, 0, N);
      }
      // unit columns: K_c column M+t has a 1 at interface row n_I+n_B+t; Kbar column
      // M+t has a 1 at flux row n_I+n_B+n_P+t
      std::vector<long long> pos;
      for (int b = 0; b < nmat; ++b) {
        const int i = b % N;
        const QRDesc& d = c->h_qrdesc[b];
        const SubInfo& sb = g.subs[i];
        const int r0 = b < N ? sb.n_I + sb.n_B : sb.n_I + sb.n_B + sb.n_P;
        const int cnt = b < N ? sb.n_G() : sb.n_D;
        for (int t = 0; t < cnt; ++t) pos.push_back(d.off + (long long)(M + t) * d.ld + r0 + t);
      }
      if (!pos.empty()) {
        const long long* dp = c->arena.put(pos, s);
        k_set_units<<<ceil_div((long long)pos.size(), kBlock), kBlock, 0, s>>>(dp, (long long)pos.size(), c->qrA.p);
        HIPCHK(hipGetLastError());
      }
    }
    c->mark(1);
    // ---- blocked Householder QR of all matrices: 16-column panels, WY updates on MFMA
    {
      const int rpt = rows_per_thread(g.max_m);
      c->npanel = ceil_div(M, kNB);
      c->Tbuf.alloc((size_t)nmat * c->npanel * kNB * kNB);
      for (int p = 0; p < c->npanel; ++p) {
        const int k = p * kNB;
        launch_qr_panel16<double>(ceil_div(g.max_m, kPanelThreads), dim3(nmat), s, c->qrdesc.p, c->qrA.p, c->tau.p, c->Tbuf.p, k, p, c->npanel);
        const int c0 = k + std::min(kNB, M - k);
        const int ntile = ceil_div(c->max_ncols - c0, kUC);
        if (ntile > 0) {
          k_qr_wy<double><<<dim3(nmat, ntile), kBlock, 0, s>>>(c->qrdesc.p, c->qrA.p, c->Tbuf.p, k, p, c->npanel,
                                                               c->qrA.p, c->qr_coff.p, c->qr_ldc.p, c->qr_cn.p, c0, 1);
          HIPCHK(hipGetLastError());
        }
      }
    }
    c->mark(2);
    // ---- Q_G^T copy (M x n_G, ld M), then E = R^{-1} Q_G^T in place, Xbar = Rbar^{-1} Qbar_D^T in place
    {
      c->h_offQG.assign(N + 1, 0);
      for (int i = 0; i < N; ++i) c->h_offQG[i + 1] = c->h_offQG[i] + (long long)M * c->h_nG[i];
      c->QG.alloc(std::max(c->h_offQG[N], 1ll));
      std::vector<CopyDesc> cp;
      for (int i = 0; i < N; ++i) {
        const QRDesc& d = c->h_qrdesc[i];
        if (c->h_nG[i] == 0) continue;
        cp.push_back(CopyDesc{d.off + (long long)M * d.ld, c->h_offQG[i], d.ld, M, M, c->h_nG[i], 0, 0});
      }
      copy_batch<double>(c, cp, c->qrA.p, c->QG.p);
      // triangular solves on the appended columns
      std::vector<long long> xoff(nmat);
      std::vector<int> ldx(nmat), xn(nmat);
      int maxx = 0;
      for (int b = 0; b < nmat; ++b) {
        const QRDesc& d = c->h_qrdesc[b];
        xoff[b] = d.off + (long long)M * d.ld;
        ldx[b] = d.ld;
        xn[b] = d.ncols - M;
        maxx = std::max(maxx, xn[b]);
      }
      if (maxx > 0) {
        const long long* dxo = c->arena.put(xoff, s);
        const int* dld = c->arena.put(ldx, s);
        const int* dxn = c->arena.put(xn, s);
        const size_t smt = (size_t)M * kTRSMC * sizeof(double);
        if (smt > 65536) HIPCHK(hipFuncSetAttribute((const void*)k_trsm<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smt));
        k_trsm<double><<<dim3(nmat, ceil_div(maxx, kTRSMC)), kBlock, smt, s>>>(c->qrdesc.p, c->qrA.p, c->qrA.p, dxo,
                                                                               dld, dxn, 0);
        HIPCHK(hipGetLastError());
      }
    }
    // ---- local interface operators
    {
      c->h_offG.assign(N + 1, 0);
      c->h_offN.assign(N + 1, 0);
      for (int i = 0; i < N; ++i) {
        c->h_offG[i + 1] = c->h_offG[i] + (long long)c->h_nG[i] * c->h_nG[i];
        c->h_offN[i + 1] = c->h_offN[i] + (long long)c->h_nD[i] * c->h_nD[i];
      }
      const size_t nGt = std::max(c->h_offG[N], 1ll), nNt = std::max(c->h_offN[N], 1ll);
      c->Gm.alloc(nGt); c->Lm.alloc(nGt); c->LTm.alloc(nGt);
      c->Nm.alloc(nNt); c->NTm.alloc(nNt);
      c->Gm.zero(s); c->Lm.zero(s); c->LTm.zero(s); c->Nm.zero(s); c->NTm.zero(s);
      c->offG.upload(std::vector<long long>(c->h_offG.begin(), c->h_offG.end() - 1), s);
      c->offN.upload(std::vector<long long>(c->h_offN.begin(), c->h_offN.end() - 1), s);
      std::vector<GemmDesc> gG, gL, gN;
      std::vector<CopyDesc> tL, tN;
      for (int i = 0; i < N; ++i) {
        const int ng = c->h_nG[i], nd = c->h_nD[i];
        const QRDesc& d = c->h_qrdesc[i];
        if (ng == 0) continue;
        // G = -(Q_G^T)^T (Q_G^T) (+ I below)
        gG.push_back(GemmDesc{c->h_offQG[i], c->h_offQG[i], c->h_offG[i], M, M, ng, ng, ng, M});
        // L = A_m E
        gL.push_back(GemmDesc{c->h_offAm[i], d.off + (long long)M * d.ld, c->h_offG[i], ng, d.ld, ng, ng, ng, M});
        tL.push_back(CopyDesc{c->h_offG[i], c->h_offG[i], ng, ng, ng, ng, 1, 0});
        if (nn && nd > 0) {
          const QRDesc& db = c->h_qrdesc[N + i];
          gN.push_back(GemmDesc{c->h_offCD[i], db.off + (long long)M * db.ld, c->h_offN[i], nd, db.ld, nd, nd, nd, M});
          tN.push_back(CopyDesc{c->h_offN[i], c->h_offN[i], nd, nd, nd, nd, 1, 0});
        }
      }
      gemm_batch<double>(c, gG, c->QG.p, c->QG.p, c->Gm.p, 1, -1.0, 0.0);
      {
        std::vector<long long> o;
        std::vector<int> n;
        for (int i = 0; i < N; ++i) if (c->h_nG[i]) { o.push_back(c->h_offG[i]); n.push_back(c->h_nG[i]); }
        if (!o.empty()) {
          const long long* dO = c->arena.put(o, s);
          const int* dn = c->arena.put(n, s);
          k_add_diag<<<(unsigned)o.size(), kBlock, 0, s>>>(dO, dn, c->Gm.p, 1.0);
          HIPCHK(hipGetLastError());
        }
      }
      // A_m and E live in different buffers: run the GEMM with A = Am, B = qrA
      if (!gL.empty()) {
        int mm = 0, nn2 = 0;
        for (auto& q : gL) { mm = std::max(mm, q.m); nn2 = std::max(nn2, q.n); }
        const GemmDesc* dd = c->arena.put(gL, s);
        k_gemm<double, double><<<dim3(ceil_div(mm, 16), ceil_div(nn2, 16), (unsigned)gL.size()), kBlock, 0, s>>>(
            dd, c->Am.p, c->qrA.p, c->Lm.p, 0, 1.0, 0.0);
        HIPCHK(hipGetLastError());
      }
      copy_batch<double>(c, tL, c->Lm.p, c->LTm.p);
      if (!gN.empty()) {
        int mm = 0, nn2 = 0;
        for (auto& q : gN) { mm = std::max(mm, q.m); nn2 = std::max(nn2, q.n); }
        const GemmDesc* dd = c->arena.put(gN, s);
        k_gemm<double, double><<<dim3(ceil_div(mm, 16), ceil_div(nn2, 16), (unsigned)gN.size()), kBlock, 0, s>>>(
            dd, c->CD.p, c->qrA.p, c->Nm.p, 0, 1.0, 0.0);
        HIPCHK(hipGetLastError());
        copy_batch<double>(c, tN, c->Nm.p, c->NTm.p);
      }
    }
    c->mark(3);
    // ---- coarse problem: D_PiPi, S_Pi = sum G_PiPi + D^T D, Cholesky, inverse, X1
    if (c->nP > 0) {
      const int n = c->nP;
      const size_t nn2 = (size_t)n * n;
      c->Dpp.alloc(nn2); c->Gs.alloc(nn2); c->Spi.alloc(nn2); c->Sfac.alloc(nn2); c->Sinv.alloc(nn2);
      c->Zm.alloc(nn2); c->Ztm.alloc(nn2); c->Wm.alloc(nn2); c->X1.alloc(4 * nn2);
      c->Dpp.zero(s); c->Gs.zero(s);
      k_coarse_assemble<double><<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, c->pi_own_ptr.p, c->pi_own_slot.p,
                                                                       c->pi_slot_sub.p, c->pi_off.p, c->pi_l2g.p,
                                                                       c->offG.p, c->nG_dev.p, c->Gm.p, c->Lm.p,
                                                                       c->Dpp.p, c->Gs.p);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(c->Spi.p, c->Gs.p, nn2 * sizeof(double), hipMemcpyDeviceToDevice, s));
      gemm_batch<double>(c, {GemmDesc{0, 0, 0, n, n, n, n, n, n}}, c->Dpp.p, c->Dpp.p, c->Spi.p, 1, 1.0, 1.0);
      HIPCHK(hipMemcpyAsync(c->Sfac.p, c->Spi.p, nn2 * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemsetAsync(c->flags.p, 0, 8 * sizeof(unsigned), s));
      k_cholesky<<<1, kBlock, 0, s>>>(c->Sfac.p, n, c->flags.p);
      HIPCHK(hipGetLastError());
      const size_t smi = (size_t)n * 4 * sizeof(double);
      if (smi > 160 * 1024) c->fail(DDELM_E_SHAPE, "coarse problem too large for the inverse kernel");
      if (smi > 65536) HIPCHK(hipFuncSetAttribute((const void*)k_chol_inverse, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smi));
      k_chol_inverse<<<ceil_div(n, 4), kBlock, smi, s>>>(c->Sfac.p, n, c->Sinv.p);
      HIPCHK(hipGetLastError());
      // Z = D Sinv, Zt = Z^T, W = D Zt, X1
      gemm_batch<double>(c, {GemmDesc{0, 0, 0, n, n, n, n, n, n}}, c->Dpp.p, c->Sinv.p, c->Zm.p, 0, 1.0, 0.0);
      copy_batch<double>(c, {CopyDesc{0, 0, n, n, n, n, 1, 0}}, c->Zm.p, c->Ztm.p);
      gemm_batch<double>(c, {GemmDesc{0, 0, 0, n, n, n, n, n, n}}, c->Dpp.p, c->Ztm.p, c->Wm.p, 0, 1.0, 0.0);
      k_assemble_X1<<<std::min(ceil_div(4ll * nn2, kBlock), 4096), kBlock, 0, s>>>(n, c->Sinv.p, c->Zm.p, c->Wm.p,
                                                                                   c->X1.p);
      HIPCHK(hipGetLastError());
    } else {
      c->X1.alloc(1);
    }
    c->mark(4);
    // offsets used by every solve
    c->offm_d.upload(std::vector<long long>(c->h_offm.begin(), c->h_offm.end() - 1), s);
    c->offB_d.upload(std::vector<long long>(c->h_offB.begin(), c->h_offB.end() - 1), s);
    c->offQG_d.upload(std::vector<long long>(c->h_offQG.begin(), c->h_offQG.end() - 1), s);
    c->offAm_d.upload(std::vector<long long>(c->h_offAm.begin(), c->h_offAm.end() - 1), s);
    unsigned fl[8];
    HIPCHK(hipMemcpyAsync(fl, c->flags.p, sizeof(fl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (fl[0] & 2u) c->fail(DDELM_E_CHOLESKY, "S_Pi is not positive definite");
    for (int k = 0; k < 4; ++k) c->phase_ms[k] = c->span(k, k + 1);
    c->factored = true;
  });
}

ddelm_status ddelm_solve(ddelm_ctx c, int nrhs, const double* f_I, const double* g_B, double* coef, double* mu_pi,
                         double* mu_dl, ddelm_stats* stats) {
  if (!c) return DDELM_E_ARG;
  int iters = 0;
  double relres = 0.0;
  bool noconv = false;
  ddelm_status st = run_guarded(c, [&]() {
    if (!c->factored) c->fail(DDELM_E_STATE, "ddelm_solve called before ddelm_factor");
    if (nrhs < 1 || nrhs > c->opt.max_nrhs) c->fail(DDELM_E_ARG, "nrhs out of range");
    if (!f_I || !coef || (!g_B && c->geo.sum_nB > 0)) c->fail(DDELM_E_ARG, "null array");
    hipStream_t s = c->stream;
    const int N = c->N, M = c->M;
    alloc_solve_workspace(c, nrhs);
    auto t0 = std::chrono::steady_clock::now();
    c->arena.reset();
    c->mark(5);
    const DBuf<long long>& offm_d = c->offm_d;
    const DBuf<long long>& offB_d = c->offB_d;
    // ---- f, Q^T f, projections, K^+ f, fluxes
    k_rhs_assemble<<<dim3(N, nrhs), kBlock, 0, s>>>(N, c->n_int, c->sizes_dev.p, offm_d.p, offB_d.p, c->summ,
                                                     c->geo.sum_nB, f_I, g_B, c->F.p);
    HIPCHK(hipGetLastError());
    const int rpt = rows_per_thread(c->geo.max_m);
    for (int p = 0; p < c->npanel; ++p) {
      k_qr_wy<double><<<dim3(N, ceil_div(nrhs, kUC)), kBlock, 0, s>>>(c->qrdesc.p, c->qrA.p, c->Tbuf.p, p * kNB, p,
                                                                      c->npanel, c->F.p, c->f_off.p, c->f_ld.p,
                                                                      c->f_cn.p, 0, 1);
      HIPCHK(hipGetLastError());
    }
    (void)rpt;
    const DBuf<long long>& offQG_d = c->offQG_d;
    const DBuf<long long>& offAm_d = c->offAm_d;
    k_rhs_proj<<<dim3(N, nrhs), kBlock, M * sizeof(double), s>>>(M, c->sizes_dev.p, c->pi_off.p, c->dl_off.p,
                                                                  offQG_d.p, c->QG.p, offm_d.p, c->summ, c->F.p,
                                                                  c->sumP, c->sumD, c->rho_loc.p, c->s_loc.p);
    HIPCHK(hipGetLastError());
    {
      const size_t smt = (size_t)M * kTRSMC * sizeof(double);
      const int* cnM = c->arena.put(std::vector<int>(N, nrhs), s);
      k_trsm<double><<<dim3(N, ceil_div(nrhs, kTRSMC)), kBlock, smt, s>>>(c->qrdesc.p, c->qrA.p, c->F.p, c->f_off.p,
                                                                          c->f_ld.p, cnM, 0);
      HIPCHK(hipGetLastError());
      k_rhs_flux<<<dim3(N, nrhs), kBlock, M * sizeof(double), s>>>(M, c->sizes_dev.p, c->pi_off.p, c->dl_off.p,
                                                                    offAm_d.p, c->Am.p, offm_d.p, c->summ, c->F.p,
                                                                    c->sumP, c->sumD, c->psi_loc.p, c->l_loc.p);
      HIPCHK(hipGetLastError());
    }
    // ---- b of eq. nn-mixed
    OpArgs<double> a = op_args(c, nrhs);
    run_phases_after_stage1(c, a, nrhs, nullptr);
    if (c->nD > 0) {
      k_ph_sum_w<double><<<dim3(ceil_div(c->nD, kBlock), nrhs), kBlock, 0, s>>>(a, c->cg_b.p);
      HIPCHK(hipGetLastError());
    }
    if (c->nP > 0) {
      k_save_pif<<<ceil_div(c->nP * nrhs, kBlock), kBlock, 0, s>>>(c->nP, nrhs, c->c1.p, c->pif.p);
      HIPCHK(hipGetLastError());
    }
    c->mark(6);
    HIPCHK(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    // ---- CG
    if (c->nD > 0) {
      int mode = c->opt.cg_mode == 0 ? (nrhs <= 16 ? 2 : 1) : c->opt.cg_mode;
      if (mode == 2) cg_persistent(c, nrhs);
      else cg_multilaunch(c, nrhs);
      std::vector<double> sc((size_t)nrhs * 8);
      unsigned fl[8];
      HIPCHK(hipMemcpyAsync(sc.data(), c->cg_scal.p, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(fl, c->flags.p, sizeof(fl), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (fl[0] & 1u) c->fail(DDELM_E_HIP, "device grid barrier wait expired");
      for (int r = 0; r < nrhs; ++r) {
        iters = std::max(iters, (int)sc[8 * r + 6]);
        const double rr = sc[8 * r], bb = sc[8 * r + 1];
        if (!(rr == rr)) c->fail(DDELM_E_NONFINITE, "NaN in CG");
        relres = std::max(relres, bb > 0 ? std::sqrt(rr / bb) : 0.0);
        if (sc[8 * r + 5] == 0.0) noconv = true;
      }
    } else {
      HIPCHK(hipStreamSynchronize(s));
    }
    c->mark(7);
    auto t2 = std::chrono::steady_clock::now();
    // ---- recovery: mu_Pi = pi_f - [S^-1 (rho + D^T psi)](mu_D); c = c_f0 + E mu
    if (c->nP > 0) {
      if (c->nD > 0) {
        const size_t sm = local_smem(c);
        k_ph_local_v<double><<<dim3(N, nrhs), kBlock, sm, s>>>(a, c->cg_x.p);
        k_ph_coarse1<double><<<dim3(ceil_div(2 * c->nP, kBlock), nrhs), kBlock, sm, s>>>(a);
        HIPCHK(hipGetLastError());
      } else {
        fill(s, c->c1.p, (long long)nrhs * 2 * c->nP, 0.0);
      }
      k_mu_pi<<<ceil_div(c->nP * nrhs, kBlock), kBlock, 0, s>>>(c->nP, nrhs, c->pif.p, c->c1.p, c->pif.p);
      HIPCHK(hipGetLastError());
    }
    k_recover<<<dim3(N, nrhs), kBlock, (size_t)std::max(c->geo.max_nG, 1) * sizeof(double), s>>>(
        M, c->nP, c->nD, c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->pi_l2g.p, c->dl_l2g.p, c->qrdesc.p, c->qrA.p,
        offm_d.p, c->summ, c->F.p, c->pif.p, c->cg_x.p, N, coef);
    HIPCHK(hipGetLastError());
    if (mu_pi && c->nP > 0)
      HIPCHK(hipMemcpyAsync(mu_pi, c->pif.p, (size_t)nrhs * c->nP * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (mu_dl && c->nD > 0)
      HIPCHK(hipMemcpyAsync(mu_dl, c->cg_x.p, (size_t)nrhs * c->nD * sizeof(double), hipMemcpyDeviceToDevice, s));
    c->mark(8);
    HIPCHK(hipStreamSynchronize(s));
    auto t3 = std::chrono::steady_clock::now();
    c->phase_ms[4] = c->span(5, 6);
    c->phase_ms[5] = c->span(6, 7);
    c->phase_ms[6] = c->span(7, 8);
    if (stats) {
      stats->iters = iters;
      stats->refine_steps = 0;
      stats->rel_res = relres;
      stats->ms_rhs = std::chrono::duration<double, std::milli>(t1 - t0).count();
      stats->ms_cg = std::chrono::duration<double, std::milli>(t2 - t1).count();
      stats->ms_recover = std::chrono::duration<double, std::milli>(t3 - t2).count();
    }
  });
  if (st == DDELM_OK && noconv) return DDELM_WARN_NOCONV;
  return st;
}

ddelm_status ddelm_evaluate(ddelm_ctx c, int nrhs, const double* coef, long long npts, const double* x, double* u,
                            double* grad) {
  if (!c) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    if (nrhs < 1 || npts < 0 || !coef || (npts > 0 && (!x || !u))) c->fail(DDELM_E_ARG, "bad evaluate arguments");
    const Geometry& g = c->geo;
    for (int r = 0; r < nrhs && npts > 0; ++r) {
      k_evaluate<<<ceil_div(npts, kBlock), kBlock, 0, c->stream>>>(g.nx, g.ny, c->M, c->N, g.lo[0], g.lo[1], g.h[0],
                                                                  g.h[1], c->W.p, c->b.p, coef, npts, x, u, grad, r);
      HIPCHK(hipGetLastError());
    }
  });
}

ddelm_status ddelm_get_sizes(ddelm_ctx c, ddelm_sizes* o) {
  if (!c || !o) return DDELM_E_ARG;
  if (c->N == 0) return DDELM_E_STATE;
  o->N = c->N; o->M = c->M; o->n_pi = c->nP; o->n_dl = c->nD; o->n_int = c->n_int;
  o->max_m = c->geo.max_m; o->sum_nB = c->geo.sum_nB; o->sum_nG = (long long)c->sumP + c->sumD;
  return DDELM_OK;
}

ddelm_status ddelm_get_counts(ddelm_ctx c, int* n_B, int* n_P, int* n_D, int* m) {
  if (!c) return DDELM_E_ARG;
  if (c->N == 0) return DDELM_E_STATE;
  for (int i = 0; i < c->N; ++i) {
    if (n_B) n_B[i] = c->h_nB[i];
    if (n_P) n_P[i] = c->h_nP[i];
    if (n_D) n_D[i] = c->h_nD[i];
    if (m) m[i] = c->h_m[i];
  }
  return DDELM_OK;
}

ddelm_status ddelm_get_indexing(ddelm_ctx c, int* pi_glob, int* dl_glob) {
  if (!c) return DDELM_E_ARG;
  if (c->N == 0) return DDELM_E_STATE;
  if (pi_glob) std::copy(c->geo.pi_loc2glob.begin(), c->geo.pi_loc2glob.end(), pi_glob);
  if (dl_glob) std::copy(c->geo.dl_loc2glob.begin(), c->geo.dl_loc2glob.end(), dl_glob);
  return DDELM_OK;
}

ddelm_status ddelm_get_boundary_points(ddelm_ctx c, double* x_B) {
  if (!c || !x_B) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    std::vector<double> h;
    for (auto& sb : c->geo.subs) h.insert(h.end(), sb.xB.begin(), sb.xB.end());
    if (!h.empty()) {
      HIPCHK(hipMemcpyAsync(x_B, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    }
  });
}

ddelm_status ddelm_get_interface_points(ddelm_ctx c, double* x_pi, double* x_dl) {
  if (!c) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    if (x_pi && c->nP)
      HIPCHK(hipMemcpyAsync(x_pi, c->geo.x_pi.data(), c->geo.x_pi.size() * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
    if (x_dl && c->nD)
      HIPCHK(hipMemcpyAsync(x_dl, c->geo.x_dl.data(), c->geo.x_dl.size() * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

ddelm_status ddelm_get_local_matrix(ddelm_ctx c, int which, int sub, double* out, int* rows, int* cols) {
  if (!c || !rows || !cols) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    if (which != 8 && (sub < 0 || sub >= c->N)) c->fail(DDELM_E_ARG, "sub out of range");
    const int M = c->M;
    int R = 0, C = 0;
    switch (which) {
      case 0: case 2: R = c->h_m[sub]; C = M; break;
      case 1: R = c->h_nG[sub]; C = M; break;
      case 3: R = c->h_nD[sub]; C = M; break;
      case 4: R = M; C = M; break;
      case 5: case 6: R = C = c->h_nG[sub]; break;
      case 7: R = C = c->h_nD[sub]; break;
      case 8: R = C = c->nP; break;
      default: c->fail(DDELM_E_ARG, "unknown matrix id");
    }
    *rows = R; *cols = C;
    if (!out || R == 0 || C == 0) return;
    hipStream_t s = c->stream;
    HIPCHK(hipStreamSynchronize(s));
    c->arena.reset();
    DBuf<double> tmp;
    tmp.alloc((size_t)R * C);
    tmp.zero(s);
    const double* src = nullptr;
    long long soff = 0;
    int ld = R;
    if (which <= 3) {
      const RowSetDev& rs = which == 0 ? c->rsK : which == 1 ? c->rsA : which == 2 ? c->rsKb : c->rsAb;
      std::vector<long long> o(c->N, 0);
      std::vector<int> l(c->N, R);
      assemble_features(c, rs, R, tmp.p, o, l, sub, 1);
      src = tmp.p; soff = 0; ld = R;
      // column-major R x C -> row-major output
      copy_batch<double>(c, {CopyDesc{0, 0, R, C, R, C, 1, 0}}, src, out);
      HIPCHK(hipStreamSynchronize(s));
      return;
    }
    if (!c->factored) c->fail(DDELM_E_STATE, "matrix needs ddelm_factor");
    if (which == 4) {
      const QRDesc& d = c->h_qrdesc[sub];
      copy_batch<double>(c, {CopyDesc{d.off, 0, d.ld, C, R, C, 1, 0}}, c->qrA.p, out);
      HIPCHK(hipStreamSynchronize(s));
      return;
    }
    if (which == 5) { src = c->Gm.p; soff = c->h_offG[sub]; }
    if (which == 6) { src = c->Lm.p; soff = c->h_offG[sub]; }
    if (which == 7) {
      if (!c->use_nn) c->fail(DDELM_E_STATE, "no Neumann-Neumann operator with theta = 0");
      src = c->Nm.p; soff = c->h_offN[sub];
    }
    if (which == 8) src = c->Spi.p;
    copy_batch<double>(c, {CopyDesc{soff, 0, R, R, R, C, 1, 0}}, src, out);
    HIPCHK(hipStreamSynchronize(s));
  });
}

ddelm_status ddelm_get_phase_times(ddelm_ctx c, double* ms) {
  if (!c || !ms) return DDELM_E_ARG;
  for (int k = 0; k < 8; ++k) ms[k] = c->phase_ms[k];
  return DDELM_OK;
}

const char* ddelm_last_error(ddelm_ctx c) { return c ? c->err.c_str() : "null context"; }

void ddelm_destroy(ddelm_ctx c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  delete c;
}

}  // extern "C"
