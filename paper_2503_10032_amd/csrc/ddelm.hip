// C ABI of the DDELM-NN library: context, setup, factorisation, solve and
// evaluation on one gfx950 GPU.  See include/ddelm.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdint>
#include <map>
#include <memory>
#include <tuple>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ddelm.h"
#include "geometry.hpp"
#include "kernels_setup.hpp"
#include "kernels_solve.hpp"
#include "kernels_cg.hpp"
#include "kernels_qr.hpp"
#include "kernels_rhs.hpp"
#include "kernels_adj.hpp"
#include "kernel_entries.hpp"

using namespace ddelm;

// Device array behind ddelm_solve_noalloc: the workspace of an allocation-free
// solve is carved out of it (one copy per GPU, alive until the process ends).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

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

// ---- process-wide resources kept between contexts
// Device memory freed by a destroyed context (whose stream has drained) is
// kept in an idle list per device and handed to later allocations of a
// similar size, so a context set up after another one of similar size
// allocates nothing from the driver.  Memory freed while its context is
// alive goes to that context's own list: only the same context reuses it,
// and since all of a context's work is ordered on its stream (the side
// stream of the QR joins it before anything after the QR is queued), a
// block handed out again is only touched by work queued after every earlier
// use.  Side streams, events and pinned staging buffers of destroyed
// contexts are kept idle as well.  ddelm_release_cached_memory returns the
// idle part to the runtime; nothing is released at exit.
struct BlockList {
  std::multimap<size_t, void*> free;          // capacity in bytes -> block
  // smallest block of at least `bytes` that does not waste much of itself
  void* take(size_t bytes, size_t& cap) {
    auto it = free.lower_bound(bytes);
    if (it == free.end() || it->first > 2 * bytes + (size_t(1) << 20)) return nullptr;
    cap = it->first;
    void* p = it->second;
    free.erase(it);
    return p;
  }
  void put(void* p, size_t cap) { free.emplace(cap, p); }
};

struct Resources {
  std::mutex mu;
  std::vector<BlockList> idle;                          // per device
  std::vector<std::pair<int, hipStream_t>> streams;     // idle side streams (device, stream)
  std::vector<std::pair<int, hipEvent_t>> events_t;     // idle events with timing
  std::vector<std::pair<int, hipEvent_t>> events_n;     // idle events without timing
  struct Staging { int dev; size_t cap; char* d; char* h; };
  std::vector<Staging> staging;                         // idle descriptor arenas
  BlockList& dev_list(int dev) {
    if ((int)idle.size() <= dev) idle.resize(dev + 1);
    return idle[dev];
  }
};
Resources& res() {
  static Resources* r = new Resources();
  return *r;
}

hipEvent_t take_event(int dev, bool timing) {
  {
    Resources& R = res();
    std::lock_guard<std::mutex> lk(R.mu);
    auto& v = timing ? R.events_t : R.events_n;
    for (size_t k = v.size(); k-- > 0;)
      if (v[k].first == dev) {
        hipEvent_t e = v[k].second;
        v.erase(v.begin() + k);
        return e;
      }
  }
  hipEvent_t e;
  HIPCHK(hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming));
  return e;
}
void give_event(int dev, bool timing, hipEvent_t e) {
  Resources& R = res();
  std::lock_guard<std::mutex> lk(R.mu);
  (timing ? R.events_t : R.events_n).push_back({dev, e});
}
hipStream_t take_stream(int dev) {
  {
    Resources& R = res();
    std::lock_guard<std::mutex> lk(R.mu);
    for (size_t k = R.streams.size(); k-- > 0;)
      if (R.streams[k].first == dev) {
        hipStream_t st = R.streams[k].second;
        R.streams.erase(R.streams.begin() + k);
        return st;
      }
  }
  hipStream_t st;
  HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));   // default priority
  return st;
}

// free list of the context whose API call is running on this thread
struct CtxBlocks {
  int dev = 0;
  BlockList list;
};
thread_local CtxBlocks* tl_blocks = nullptr;
thread_local hipStream_t tl_stream = nullptr;    // stream of the context whose call is running
struct BlocksScope {
  CtxBlocks* prev;
  explicit BlocksScope(CtxBlocks* b) : prev(tl_blocks) { tl_blocks = b; }
  ~BlocksScope() { tl_blocks = prev; }
};
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(tl_stream) { tl_stream = s; }
  ~StreamScope() { tl_stream = prev; }
};

// Debugging aid: with DDELM_DEBUG_POISON=1 in the environment every device
// block handed to a buffer is first filled with 0xFF bytes (a NaN in float
// and double), so a kernel that reads memory nobody wrote shows up as
// non-finite results instead of silently reading zeros or stale values.
bool poison_enabled() {
  const char* e = getenv("DDELM_DEBUG_POISON");
  return e && e[0] == '1';
}

void release_idle_memory_locked(Resources& R) {
  for (BlockList& l : R.idle) {
    for (auto& kv : l.free) (void)hipFree(kv.second);
    l.free.clear();
  }
}

void* dev_alloc(size_t bytes, size_t& cap) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  bytes = (bytes + 255) & ~size_t(255);
  if (tl_blocks && tl_blocks->dev == dev)
    if (void* p = tl_blocks->list.take(bytes, cap)) return p;
  Resources& R = res();
  {
    std::lock_guard<std::mutex> lk(R.mu);
    if (void* p = R.dev_list(dev).take(bytes, cap)) return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(R.mu);
      release_idle_memory_locked(R);
    }
    e = hipMalloc(&p, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw StatusError{DDELM_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  cap = bytes;
  return p;
}

void dev_free(void* p, size_t cap) {
  if (!p) return;
  if (tl_blocks) tl_blocks->list.put(p, cap);
  else (void)hipFree(p);      // outside any context call: free for good (synchronises)
}

// Host-to-device copy through the pinned staging buffer of the running call's
// context (asynchronous, the host does not wait); false when there is none
// or it is full, and the caller copies from pageable memory instead.
bool stage_upload(void* dst, const void* src, size_t bytes, hipStream_t s);

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  size_t cap = 0;     // bytes of the block behind p
  void alloc(size_t count) {
    free();
    n = count;
    if (count == 0) return;
    try {
      p = (T*)dev_alloc(count * sizeof(T), cap);
      if (poison_enabled()) HIPCHK(hipMemsetAsync(p, 0xFF, cap, tl_stream));
    } catch (...) {
      p = nullptr;
      n = 0;
      throw;
    }
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    alloc(h.size());
    if (h.empty() || stage_upload(p, h.data(), h.size() * sizeof(T), s)) return;
    HIPCHK(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void zero(hipStream_t s) {
    if (n) HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
  void free() {
    dev_free(p, cap);
    p = nullptr;
    n = 0;
    cap = 0;
  }
  ~DBuf() { free(); }
};

// Several buffers cleared by one kernel launch instead of one fill each.
struct ZeroBatch {
  std::vector<std::pair<unsigned*, long long>> v;
  template <typename T>
  ZeroBatch& add(DBuf<T>& b) {
    static_assert(sizeof(T) % 4 == 0, "cleared as 32-bit words");
    if (b.n) v.push_back({reinterpret_cast<unsigned*>(b.p), (long long)(b.n * sizeof(T) / 4)});
    return *this;
  }
  void launch(hipStream_t s) {
    for (size_t k0 = 0; k0 < v.size(); k0 += kZeroMax) {
      ZeroList z{};
      long long most = 0;
      const int cnt = (int)std::min(v.size() - k0, (size_t)kZeroMax);
      for (int k = 0; k < cnt; ++k) {
        z.p[k] = v[k0 + k].first;
        z.n[k] = v[k0 + k].second;
        most = std::max(most, z.n[k]);
      }
      const unsigned gx = (unsigned)std::max<long long>(1, std::min<long long>((most + kBlock - 1) / kBlock, 256));
      k_zero_many<<<dim3(gx, cnt), kBlock, 0, s>>>(z);
      HIPCHK(hipGetLastError());
    }
    v.clear();
  }
};

// Device copies of small per-call descriptor arrays: one device buffer and one
// pinned host staging buffer, filled by a bump pointer and reset at the start
// of every API call (the previous call has drained the stream).
struct Arena {
  char* dev = nullptr;
  char* host = nullptr;
  size_t cap = 0, used = 0;
  int device = 0;
  void ensure(size_t c) {
    if (c <= cap) return;
    release();
    HIPCHK(hipGetDevice(&device));
    {
      // an idle arena of a destroyed context, if one is large enough
      Resources& R = res();
      std::lock_guard<std::mutex> lk(R.mu);
      for (size_t k = 0; k < R.staging.size(); ++k) {
        const Resources::Staging& a = R.staging[k];
        if (a.dev == device && a.cap >= c) {
          dev = a.d; host = a.h; cap = a.cap;
          R.staging.erase(R.staging.begin() + k);
          return;
        }
      }
    }
    HIPCHK(hipMalloc((void**)&dev, c));
    HIPCHK(hipHostMalloc((void**)&host, c, hipHostMallocDefault));
    cap = c;
  }
  // the copies out of the staging buffer may still be queued: free for good
  void release() {
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    dev = host = nullptr;
    cap = used = 0;
  }
  // after the context's stream has drained: keep the buffers for the next context
  void retire() {
    if (dev) {
      Resources& R = res();
      std::lock_guard<std::mutex> lk(R.mu);
      R.staging.push_back({device, cap, dev, host});
    }
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
  // copy `bytes` from src to the device address dst through the pinned buffer
  bool stage(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t off = (used + 255) & ~size_t(255);
    if (!host || off + bytes > cap) return false;
    std::memcpy(host + off, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, host + off, bytes, hipMemcpyHostToDevice, s));
    used = off + bytes;
    return true;
  }
  ~Arena() { release(); }
};

// Pinned staging of table uploads for the context whose call is running
// (reset with the descriptor arena, after the stream has drained).
thread_local Arena* tl_upload = nullptr;
struct UploadScope {
  Arena* prev;
  explicit UploadScope(Arena* a) : prev(tl_upload) { tl_upload = a; }
  ~UploadScope() { tl_upload = prev; }
};
bool stage_upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  return tl_upload && tl_upload->stage(dst, src, bytes, s);
}

__host__ __device__ inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Mixed-precision refinement stops once a step shrinks the correction by less
// than this factor: the iteration then sits near its float32 fixed point and
// further steps cost a full inner solve each for little change.
constexpr double kRefineStall = 0.5;

struct RowSetDev {
  int lead = 0;
  DBuf<int> row0, ptr;
  DBuf<Term> terms;
  // rows with more than kLongTerms terms: (subdomain, local row) pairs by
  // subdomain; first[i] = first pair of subdomain i
  std::vector<int> h_long, h_long_first;
  DBuf<int> long_rows;
  void upload(const RowSet& r, hipStream_t s) {
    lead = r.lead;
    row0.upload(r.row0, s);
    ptr.upload(r.ptr, s);
    terms.upload(r.terms, s);
    const int N = (int)r.row0.size() - 1;
    h_long.clear();
    h_long_first.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) {
      h_long_first[i] = (int)h_long.size() / 2;
      for (int row = r.row0[i]; row < r.row0[i + 1]; ++row)
        if (r.ptr[row + 1] - r.ptr[row] > kLongTerms) {
          h_long.push_back(i);
          h_long.push_back(r.lead + row - r.row0[i]);
        }
    }
    h_long_first[N] = (int)h_long.size() / 2;
    long_rows.upload(h_long, s);
  }
};

// Local factors and operators in the storage type T of the local solves.
template <typename T>
struct LocalBufs {
  DBuf<T> qrA, tau, Tbuf, Tbig;        // QR matrices (K_c^i | E_G, Kbar^i | E_flux), tau, panel and block T
  DBuf<T> topA, tau1, Tbuf1, Tbig1;    // two-stage QR: features of K_c^i, factored in their first t_i rows
  DBuf<T> Am, CD;                      // A_m^i (n_G x M), Abar^i (n_D x M)
  DBuf<T> QG;                          // Q_G^T (M x n_G) per subdomain
  DBuf<T> Gm, Lm, LTm, Nm, NTm;        // local interface operators
  DBuf<T> F;                           // [nrhs][sum m] local right-hand sides
};

}  // namespace

struct ddelm_ctx_s {
  hipStream_t stream = nullptr;
  CtxBlocks* blocks = new CtxBlocks();   // device memory freed while the context lives
  hipStream_t side = nullptr;          // second stream of the QR look-ahead (created on first use)
  std::vector<hipEvent_t> sync_ev;     // ordering events between the two streams
  ddelm_options opt;
  Geometry geo;
  int N = 0, M = 0, n_int = 0;
  int nP = 0, nD = 0, sumP = 0, sumD = 0;
  bool factored = false;
  bool use_nn = true;     // theta != 0: Kbar factored and P applied
  bool mixed = false;     // float32 Householder QR + float64 refinement of the coupled system
  bool f32cg = false;     // float32 local operators in the CG (mixed, or precision 2)
  bool noalloc = false;   // inside ddelm_solve_noalloc: no event creation, no tuning runs
  std::string err;
  int device = 0;
  int num_cu = 0;

  // problem copies
  DBuf<double> W, b, geom, x_int;
  // coefficient of -div(rho grad u) (ddelm_set_coefficient); empty: rho = 1
  DBuf<double> rho_int, rho_iface;
  bool has_rho = false;
  RowSetDev rsK, rsA, rsKb, rsAb;
  // sizes per subdomain
  std::vector<int> h_m, h_nG, h_nD, h_nP, h_nB;
  std::vector<long long> h_offB;     // offsets into g_B
  std::vector<long long> h_offm;     // offsets into packed row space (sum m)
  long long summ = 0;
  // QR layout: 2N matrices (K_c then Kbar)
  DBuf<QRDesc> qrdesc;
  std::vector<QRDesc> h_qrdesc;
  bool two_stage = false;              // QR of the shared interior and boundary rows first
  DBuf<QRDesc> topdesc;
  std::vector<QRDesc> h_topdesc;
  DBuf<long long> top_coff;
  DBuf<int> top_ldc, top_cn;
  int max_ncols = 0;
  int npanel = 0, nblock = 0;
  DBuf<long long> qr_coff;
  DBuf<int> qr_ldc, qr_cn;
  std::vector<long long> h_offAm, h_offCD, h_offQG, h_offG, h_offN, h_offK;
  DBuf<long long> offG, offN;
  LocalBufs<double> l64;
  LocalBufs<float> l32;
  template <typename T>
  LocalBufs<T>& lb();
  // float64 K_c^i features kept for the refinement residuals (mixed precision)
  DBuf<double> K64;
  DBuf<long long> offK_d;
  double kappa_est = 0.0;              // max |R_jj| / min |R_jj| over the factored matrices
  // coarse (always float64)
  DBuf<double> Spi, Sfac, Sinv, Dpp, Gs, Zm, Ztm, Wm, X1, X1t;
  DBuf<unsigned> flags;                // [0] barrier expired (1) / Cholesky (2)
  DBuf<unsigned> chk;                  // setup: lowest subdomain with an interior point outside it
  // indexing on device
  DBuf<int> pi_off, dl_off, pi_l2g, dl_l2g, pi_own_ptr, pi_own_slot, dl_own_ptr, dl_own_slot, pi_slot_sub;
  DBuf<int> nG_dev;
  // solve workspaces
  int cap_nrhs = 0;
  DBuf<long long> f_off;               // per subdomain offset into F
  DBuf<int> f_ld, f_cn;
  DBuf<double> s_loc, l_loc, rho_loc, psi_loc, lam_loc, y_loc, z_loc, t_loc, nu_loc, w_loc, c1, c2, pif;
  DBuf<double> cg_x, cg_r, cg_p, cg_p1, cg_w, cg_b, cg_part, cg_scal, mu_slot, e_slot;
  DBuf<double> cg_r1, cg_s1;    // second r and s buffers of the persistent CG
  DBuf<double> cg_u, cg_c;             // distributed coarse phases: gathered right-hand side, X1 times it
  DBuf<double> cg_b0, cg_xs, cg_sx, cg_nrm;   // interface solve: b, accumulated x, S_theta x, norms
  DBuf<double> cg_rsl, cg_ssl, cg_psl; // persistent CG with one unit per subdomain: r, s, p at the slots
  const double* cg_ref = nullptr;      // per-RHS squared norm the CG stopping test is relative to
  int cg_blocks = 0, cg_slices = 0, cg_dist = 0;   // launch shape of the last persistent CG
  // refinement workspaces (mixed precision)
  DBuf<double> F64, fGP, fGD, aP, aD, hPb, hDb, dcoef, dmup, dmud, nrm_part;
  DBuf<double> ref_muP, ref_muD;       // refined mu_Pi, mu_Delta
  DBuf<double> fGP0, fGD0, hP0, hD0;   // interface rows and flux rows of a general right-hand side
  // adjoint workspaces
  int adj_cap = 0;
  DBuf<double> adj_yP, adj_yD, adj_zD, adj_mloc, adj_eloc, adj_etaD, adj_lbar;   // slot vectors
  DBuf<double> adj_gP, adj_u, adj_c2, adj_nu, adj_pbar;                          // coarse / interface
  DBuf<double> adj_fb, adj_hP, adj_hD;                                           // result (f, h cotangents)
  DBuf<double> adj_fw, adj_hwP, adj_hwD, adj_zc, adj_zP, adj_zDg, adj_fbGP, adj_fbGD;   // refinement
  DBuf<unsigned> bar;
  DBuf<int> sizes_dev;                 // per subdomain M, n_I, n_B, m, n_G
  Arena arena;
  Arena upload;     // pinned staging of table uploads (its device half is unused)
  DBuf<long long> offm_d, offB_d, offQG_d, offAm_d;
  // phase timing (HIP events on the stream)
  hipEvent_t ev[10] = {};
  double phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  void mark(int k) {
    if (noalloc) return;          // phase times are not taken in allocation-free calls
    if (!ev[k]) ev[k] = take_event(device, true);
    HIPCHK(hipEventRecord(ev[k], stream));
  }
  double span(int a, int b) {
    if (noalloc) return 0.0;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[a], ev[b]));
    return (double)ms;
  }
  // Called by ddelm_destroy once the context's stream has drained: the side
  // stream is drained here, then the buffers' memory goes to the context's
  // free list (member destructors; ddelm_destroy moves it to the idle list)
  // and the staging arena, events and side stream to the idle lists.
  ~ddelm_ctx_s() {
    for (auto& e : ev)
      if (e) give_event(device, true, e);
    for (auto& e : sync_ev)
      if (e) give_event(device, false, e);
    if (side) {
      (void)hipStreamSynchronize(side);
      Resources& R = res();
      std::lock_guard<std::mutex> lk(R.mu);
      R.streams.push_back({device, side});
    }
    arena.retire();
    upload.retire();
  }
  // event k of the cross-stream ordering pool (timing disabled)
  hipEvent_t sev(size_t k) {
    while (sync_ev.size() <= k) sync_ev.push_back(take_event(device, false));
    return sync_ev[k];
  }
  hipStream_t side_stream() {
    if (!side) side = take_stream(device);
    return side;
  }

  void fail(ddelm_status st, const std::string& m) { throw StatusError{st, m}; }
};

template <>
LocalBufs<double>& ddelm_ctx_s::lb<double>() { return l64; }
template <>
LocalBufs<float>& ddelm_ctx_s::lb<float>() { return l32; }

namespace {

template <typename F>
ddelm_status run_guarded(ddelm_ctx c, F&& fn) {
  BlocksScope scope(c ? c->blocks : nullptr);
  StreamScope sscope(c ? c->stream : nullptr);
  UploadScope uscope(c ? &c->upload : nullptr);
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
void launch_qr_panel16(int rows, dim3 grid, hipStream_t s, const QRDesc* d, T* A, T* tau, T* Tb, int k, int panel,
                       int npanel) {
  // up to 256 rows: one row per thread of a 256-thread workgroup (fewer waves
  // in each column's reduction, more matrices per compute unit); else
  // ceil(rows / 512) rows per thread of 512 threads
  if (rows <= 256) {
    launch_qr_panel16_rpt<T, 1, 256>(grid, s, d, A, tau, Tb, k, panel, npanel);
    HIPCHK(hipGetLastError());
    return;
  }
  switch (ceil_div(rows, kPanelThreads)) {
#define CASE(R) case R: launch_qr_panel16_rpt<T, R, kPanelThreads>(grid, s, d, A, tau, Tb, k, panel, npanel); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
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
  const int nx = ceil_div(mm, kGT), ny = ceil_div(nn, kGT), nmat = (int)h.size();
  k_gemm_mfma<T, T, T><<<(nmat >= 8 ? ceil_div(nmat, 8) * 8 : nmat) * nx * ny, kBlock, 0, c->stream>>>(d, A, B, C, transA, alpha, beta, nx, ny,
                                                                           nmat);
  HIPCHK(hipGetLastError());
}

// C (TC) = alpha op(A) B + beta C with A and B of different storage types
template <typename TA, typename TB, typename TC>
void gemm_batch_mixed(ddelm_ctx c, const std::vector<GemmDesc>& h, const TA* A, const TB* B, TC* C, int transA,
                      double alpha, double beta) {
  if (h.empty()) return;
  int mm = 0, nn = 0;
  for (auto& g : h) { mm = std::max(mm, g.m); nn = std::max(nn, g.n); }
  if (mm == 0 || nn == 0) return;
  const GemmDesc* d = c->arena.put(h, c->stream);
  const int nx = ceil_div(mm, kGT), ny = ceil_div(nn, kGT), nmat = (int)h.size();
  k_gemm_mfma<TA, TB, TC><<<(nmat >= 8 ? ceil_div(nmat, 8) * 8 : nmat) * nx * ny, kBlock, 0, c->stream>>>(d, A, B, C, transA, alpha, beta, nx, ny,
                                                                           nmat);
  HIPCHK(hipGetLastError());
}

template <typename TS, typename TD>
void copy_batch(ddelm_ctx c, const std::vector<CopyDesc>& h, const TS* S, TD* D) {
  if (h.empty()) return;
  long long mx = 0;
  int mc = 0;
  for (auto& cd : h) {
    mx = std::max(mx, (long long)cd.rows * cd.cols);
    mc = std::max(mc, cd.cols);
  }
  if (mx == 0) return;
  const CopyDesc* d = c->arena.put(h, c->stream);
  dim3 grid(std::min(mc, 1024), (unsigned)h.size());   // a column per workgroup and step
  k_copy2d<TS, TD><<<grid, kBlock, 0, c->stream>>>(d, S, D);
  HIPCHK(hipGetLastError());
}

void fill(hipStream_t s, double* p, long long n, double v) {
  if (n <= 0) return;
  k_fill<<<std::min(ceil_div(n, kBlock), 4096), kBlock, 0, s>>>(p, n, v);
  HIPCHK(hipGetLastError());
}

template <typename TS, typename TD>
void convert(hipStream_t s, const TS* src, TD* dst, long long n) {
  if (n <= 0) return;
  k_convert<TS, TD><<<std::min(ceil_div(n, kBlock), 4096), kBlock, 0, s>>>(src, dst, n);
  HIPCHK(hipGetLastError());
}

// feature assembly into column-major blocks
template <typename T>
void assemble_features(ddelm_ctx c, const RowSetDev& rs, int max_rows, T* out, const std::vector<long long>& off,
                       const std::vector<int>& ld, int sub0, int nsub, const int* first_row = nullptr) {
  if (max_rows == 0 || nsub == 0) return;
  FeatArgs a;
  a.lead = rs.lead; a.xint = c->x_int.p;
  a.row0 = rs.row0.p; a.ptr = rs.ptr.p; a.terms = rs.terms.p;
  a.W = c->W.p; a.bias = c->b.p; a.geom = c->geom.p;
  a.off = c->arena.put(off, c->stream); a.ld = c->arena.put(ld, c->stream); a.M = c->M; a.sub0 = sub0;
  a.rho_int = c->has_rho ? c->rho_int.p : nullptr;
  a.rho_iface = c->has_rho ? c->rho_iface.p : nullptr;
  a.first_row = first_row;
  dim3 grid(ceil_div(max_rows, 64), ceil_div(c->M, kWaves * kFeatCols), nsub);
  k_features<T><<<grid, kBlock, 0, c->stream>>>(a, out);
  HIPCHK(hipGetLastError());
  const int l0 = rs.h_long_first[sub0], l1 = rs.h_long_first[sub0 + nsub];
  if (l1 > l0) {
    k_features_long<T><<<dim3(l1 - l0, ceil_div(c->M, 4)), kBlock, 0, c->stream>>>(a, rs.long_rows.p + 2 * l0, out);
    HIPCHK(hipGetLastError());
  }
}

template <typename T>
OpArgs<T> op_args(ddelm_ctx c, int nrhs) {
  OpArgs<T> a;
  LocalBufs<T>& L = c->lb<T>();
  a.N = c->N; a.nP = c->nP; a.nD = c->nD; a.nrhs = nrhs;
  a.sumP = c->sumP; a.sumD = c->sumD; a.theta = c->use_nn ? c->opt.theta : 0.0;
  a.pi_off = c->pi_off.p; a.dl_off = c->dl_off.p; a.pi_l2g = c->pi_l2g.p; a.dl_l2g = c->dl_l2g.p;
  a.pi_own_ptr = c->pi_own_ptr.p; a.pi_own_slot = c->pi_own_slot.p;
  a.dl_own_ptr = c->dl_own_ptr.p; a.dl_own_slot = c->dl_own_slot.p;
  a.offG = c->offG.p; a.offN = c->offN.p;
  a.Gm = L.Gm.p; a.Lm = L.Lm.p; a.LTm = L.LTm.p; a.Nm = L.Nm.p; a.NTm = L.NTm.p;
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

// Right-hand sides per workgroup for the kernels that stage a block of them
// in LDS (per_rhs doubles each, the matrix read once per block): the largest
// power of two up to 16 (and up to nrhs) whose block fits in 56 KiB.
inline int rhs_group(int nrhs, size_t per_rhs) {
  int P = 1;
  while (P < 16 && P < nrhs && per_rhs * 2 * P * sizeof(double) <= ((size_t)56 << 10)) P *= 2;
  return P;
}
// f(std::integral_constant<int, P>()) for P in {1, 2, 4, 8, 16}
template <typename Fn>
void with_rhs_group(int P, Fn&& f) {
  switch (P) {
    case 1: f(std::integral_constant<int, 1>()); break;
    case 2: f(std::integral_constant<int, 2>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 8: f(std::integral_constant<int, 8>()); break;
    default: f(std::integral_constant<int, 16>()); break;
  }
}


// The per-subdomain local stages (kernels_solve.hpp) on groups of P
// right-hand sides: v -> G, L rows; -N lambda; -N^T (P lambda); eta -> L^T
// rows.  Each stages its gathered vectors as [point][P] in LDS.
template <typename T>
void launch_local_v(ddelm_ctx c, const OpArgs<T>& a, const double* v, int nrhs, hipStream_t s) {
  const size_t per = (size_t)std::max(c->geo.max_nG, 1);
  with_rhs_group(rhs_group(nrhs, per), [&](auto kp) {
    constexpr int P = decltype(kp)::value;
    k_ph_local_v<T, P><<<dim3(c->N, ceil_div(nrhs, P)), kBlock, per * P * sizeof(double), s>>>(a, v, nrhs);
  });
  HIPCHK(hipGetLastError());
}
template <typename T>
void launch_local_N(ddelm_ctx c, const OpArgs<T>& a, int transposed, int nrhs, hipStream_t s) {
  const size_t per = (size_t)std::max(c->geo.max_nD, 1);
  with_rhs_group(rhs_group(nrhs, per), [&](auto kp) {
    constexpr int P = decltype(kp)::value;
    const dim3 g(c->N, ceil_div(nrhs, P));
    if (transposed) k_ph_P2<T, P><<<g, kBlock, per * P * sizeof(double), s>>>(a, nrhs);
    else k_ph_P1<T, P><<<g, kBlock, per * P * sizeof(double), s>>>(a, nrhs);
  });
  HIPCHK(hipGetLastError());
}
template <typename T>
void launch_local_eta(ddelm_ctx c, const OpArgs<T>& a, int nrhs, hipStream_t s) {
  const size_t per = (size_t)std::max(c->geo.max_nD, 1);
  with_rhs_group(rhs_group(nrhs, per), [&](auto kp) {
    constexpr int P = decltype(kp)::value;
    k_ph_eta<T, P><<<dim3(c->N, ceil_div(nrhs, P)), kBlock, per * P * sizeof(double), s>>>(a, nrhs);
  });
  HIPCHK(hipGetLastError());
}

// --------------------------------------------------------------- solve workspaces

// The solve workspace for nrhs right-hand sides: every buffer with its
// length, and whether it is cleared when it is set up.
struct WsEntry {
  DBuf<double>* buf;
  size_t n;
  bool zero;
};

std::vector<WsEntry> solve_workspace(ddelm_ctx c, int nrhs) {
  const size_t D = (size_t)nrhs * std::max(c->sumD, 1), P = (size_t)nrhs * std::max(c->sumP, 1);
  const size_t C = (size_t)nrhs * std::max(2 * c->nP, 1);
  const size_t nPr = (size_t)nrhs * std::max(c->nP, 1), V = (size_t)nrhs * std::max(c->nD, 1);
  std::vector<WsEntry> w;
  w.push_back({&c->l64.F, (size_t)nrhs * c->summ, false});
  for (DBuf<double>* b : {&c->s_loc, &c->l_loc, &c->lam_loc, &c->y_loc, &c->z_loc, &c->t_loc, &c->w_loc})
    w.push_back({b, D, true});
  for (DBuf<double>* b : {&c->rho_loc, &c->psi_loc, &c->nu_loc}) w.push_back({b, P, true});
  w.push_back({&c->c1, C, true});
  w.push_back({&c->c2, C, true});
  w.push_back({&c->cg_u, C, false});
  w.push_back({&c->cg_c, C, false});
  w.push_back({&c->pif, nPr, true});
  for (DBuf<double>* b : {&c->cg_x, &c->cg_r, &c->cg_p, &c->cg_p1, &c->cg_w, &c->cg_b, &c->cg_r1, &c->cg_s1,
                          &c->cg_b0, &c->cg_xs, &c->cg_sx})
    w.push_back({b, V, false});
  w.push_back({&c->cg_nrm, (size_t)2 * nrhs, false});
  for (DBuf<double>* b : {&c->cg_rsl, &c->cg_ssl, &c->cg_psl}) w.push_back({b, D, false});
  w.push_back({&c->mu_slot, P, true});
  w.push_back({&c->e_slot, P, true});
  w.push_back({&c->cg_part, (size_t)3 * nrhs * 4096, false});
  w.push_back({&c->cg_scal, (size_t)nrhs * 8, false});
  w.push_back({&c->fGP, P, true});
  w.push_back({&c->fGD, D, true});
  w.push_back({&c->fGP0, P, true});
  w.push_back({&c->fGD0, D, true});
  w.push_back({&c->hP0, nPr, true});
  w.push_back({&c->hD0, V, true});
  if (c->mixed) {
    w.push_back({&c->F64, (size_t)nrhs * c->summ, false});
    w.push_back({&c->aP, P, true});
    w.push_back({&c->aD, D, true});
    w.push_back({&c->hPb, nPr, true});
    w.push_back({&c->hDb, V, true});
    w.push_back({&c->dcoef, (size_t)nrhs * c->N * c->M, false});
    w.push_back({&c->dmup, nPr, true});
    w.push_back({&c->dmud, V, true});
    w.push_back({&c->nrm_part, (size_t)nrhs * 2 * 256, false});
    w.push_back({&c->ref_muP, nPr, true});
    w.push_back({&c->ref_muD, V, true});
  }
  return w;
}

void alloc_solve_workspace(ddelm_ctx c, int nrhs) {
  if (nrhs <= c->cap_nrhs) return;
  hipStream_t s = c->stream;
  ZeroBatch zb;
  for (const WsEntry& e : solve_workspace(c, nrhs)) {
    e.buf->alloc(e.n);
    if (e.zero) zb.add(*e.buf);
  }
  zb.launch(s);
  std::vector<long long> foff(c->N);
  std::vector<int> fld(c->N, (int)c->summ), fcn(c->N, nrhs);
  for (int i = 0; i < c->N; ++i) foff[i] = c->h_offm[i];
  c->f_off.upload(foff, s);
  c->f_ld.upload(fld, s);
  c->f_cn.upload(fcn, s);
  c->cap_nrhs = nrhs;
  HIPCHK(hipStreamSynchronize(s));
}

// Allocation-free solves: the workspace of one call is carved out of a
// file-scope device array instead of the context's own buffers.  Each GPU
// holds its copy of the array until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for that device
// (taken by ddelm_setup with the device current), never through its name.
// Every call on a device shares that device's array, so calls that overlap
// on one GPU race; the buffers that must start at zero are cleared by a
// kernel at every call.
struct ScratchAddrs {
  std::mutex mu;
  std::vector<void*> ptr;     // per device: address of `scratch` on that device
};
ScratchAddrs& scratch_addrs() {
  static ScratchAddrs* s = new ScratchAddrs();
  return *s;
}
void* scratch_on(int dev) {
  ScratchAddrs& S = scratch_addrs();
  std::lock_guard<std::mutex> lk(S.mu);
  return dev < (int)S.ptr.size() ? S.ptr[dev] : nullptr;
}

// Binds the solve workspace of nrhs right-hand sides (and the per-subdomain
// offset tables, through the descriptor arena) to the scratch array of the
// context's device for the duration of one call; the context's own buffers
// are restored when it goes out of scope.
struct ScratchBinding {
  ddelm_ctx c;
  struct Saved {
    DBuf<double>* b;
    double* p;
    size_t n, cap;
  };
  std::vector<Saved> saved;
  long long* f_off_p = nullptr;
  int* f_ld_p = nullptr;
  int* f_cn_p = nullptr;
  size_t f_off_n = 0, f_ld_n = 0, f_cn_n = 0, f_off_cap = 0, f_ld_cap = 0, f_cn_cap = 0;
  int cap_nrhs = 0;
  ScratchBinding(ddelm_ctx ctx, int nrhs) : c(ctx) {
    char* base = (char*)scratch_on(c->device);
    if (!base) c->fail(DDELM_E_STATE, "no scratch address for this device (context not set up on it)");
    const std::vector<WsEntry> ws = solve_workspace(c, nrhs);
    size_t off = 0;
    for (const WsEntry& e : ws) off = ((off + 255) & ~size_t(255)) + e.n * sizeof(double);
    if (off > kScratchBytes)
      c->fail(DDELM_E_SHAPE, "allocation-free solve needs " + std::to_string(off) + " bytes of scratch, above the " +
                                 std::to_string(kScratchBytes) + " available");
    // the offset tables go through the descriptor arena (which may refuse);
    // nothing of the context is touched before that has succeeded
    std::vector<long long> foff(c->N);
    for (int i = 0; i < c->N; ++i) foff[i] = c->h_offm[i];
    long long* a_off = c->arena.put(foff, c->stream);
    int* a_ld = c->arena.put(std::vector<int>(c->N, (int)c->summ), c->stream);
    int* a_cn = c->arena.put(std::vector<int>(c->N, nrhs), c->stream);
    cap_nrhs = c->cap_nrhs;
    f_off_p = c->f_off.p; f_off_n = c->f_off.n; f_off_cap = c->f_off.cap;
    f_ld_p = c->f_ld.p; f_ld_n = c->f_ld.n; f_ld_cap = c->f_ld.cap;
    f_cn_p = c->f_cn.p; f_cn_n = c->f_cn.n; f_cn_cap = c->f_cn.cap;
    c->f_off.p = a_off; c->f_off.n = c->N; c->f_off.cap = 0;
    c->f_ld.p = a_ld; c->f_ld.n = c->N; c->f_ld.cap = 0;
    c->f_cn.p = a_cn; c->f_cn.n = c->N; c->f_cn.cap = 0;
    c->cap_nrhs = nrhs;
    off = 0;
    ZeroBatch zb;
    for (const WsEntry& e : ws) {
      off = (off + 255) & ~size_t(255);
      saved.push_back({e.buf, e.buf->p, e.buf->n, e.buf->cap});
      e.buf->p = (double*)(base + off);
      e.buf->n = e.n;
      e.buf->cap = 0;
      off += e.n * sizeof(double);
      if (e.zero) zb.add(*e.buf);
    }
    try {
      zb.launch(c->stream);
    } catch (...) {
      restore();       // a throwing constructor runs no destructor
      throw;
    }
  }
  ~ScratchBinding() { restore(); }
  void restore() {
    for (const Saved& v : saved) {
      v.b->p = v.p;
      v.b->n = v.n;
      v.b->cap = v.cap;
    }
    c->f_off.p = f_off_p; c->f_off.n = f_off_n; c->f_off.cap = f_off_cap;
    c->f_ld.p = f_ld_p; c->f_ld.n = f_ld_n; c->f_ld.cap = f_ld_cap;
    c->f_cn.p = f_cn_p; c->f_cn.n = f_cn_n; c->f_cn.cap = f_cn_cap;
    c->cap_nrhs = cap_nrhs;
    saved.clear();
  }
};

// --------------------------------------------------------------- operator phases after the first stage
template <typename T>
void run_phases_after_stage1(ddelm_ctx c, OpArgs<T>& a, int nrhs, const double* hP) {
  hipStream_t s = c->stream;
  const size_t sm = local_smem(c);
  const dim3 gl(c->N, nrhs);
  if (c->nP > 0) {
    OpArgs<T> ah = a;
    ah.hP = hP;
    k_ph_coarse1<T><<<dim3(ceil_div(2 * c->nP, kBlock), nrhs), kBlock, sm, s>>>(ah);
    HIPCHK(hipGetLastError());
  }
  k_ph_lam<T><<<gl, kBlock, 0, s>>>(a);
  HIPCHK(hipGetLastError());
  if (a.theta != 0.0) {
    launch_local_N<T>(c, a, 0, nrhs, s);
    launch_local_N<T>(c, a, 1, nrhs, s);
  }
  launch_local_eta<T>(c, a, nrhs, s);
  if (c->nP > 0) {
    k_ph_coarse2<T><<<dim3(ceil_div(2 * c->nP, kBlock), nrhs), kBlock, sm, s>>>(a);
    HIPCHK(hipGetLastError());
  }
  k_ph_w<T><<<gl, kBlock, 0, s>>>(a);
  HIPCHK(hipGetLastError());
}

CGState cg_state(ddelm_ctx c, int nrhs, int nblk, double tol) {
  CGState s;
  s.x = c->cg_x.p; s.r = c->cg_r.p; s.p = c->cg_p.p; s.w = c->cg_w.p;
  s.part = c->cg_part.p; s.scal = c->cg_scal.p;
  s.n = c->nD; s.nrhs = nrhs; s.nblk = nblk;
  s.tol = tol; s.maxit = c->opt.maxit;
  s.bref = c->cg_ref;
  return s;
}

template <typename T>
void cg_multilaunch(ddelm_ctx c, int nrhs, double tol) {
  hipStream_t s = c->stream;
  const int nblk = std::max(1, std::min(256, ceil_div(c->nD, kBlock)));
  CGState st = cg_state(c, nrhs, nblk, tol);
  OpArgs<T> a = op_args<T>(c, nrhs);
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
      launch_local_v<T>(c, a, st.p, nrhs, s);
      run_phases_after_stage1<T>(c, a, nrhs, nullptr);
      k_cg_wdot<T><<<dim3(nblk, nrhs), kBlock, 0, s>>>(a, st);
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
}

// Launch configuration of the persistent CG: row slices per subdomain and
// redundant or distributed coarse phases.
struct CgConfig {
  int S = 1;
  int dist = 0;
};

template <typename T, int NR>
void launch_fused(ddelm_ctx c, int nrhs, double tol, const CgConfig& cfg, int maxit) {
  hipStream_t s = c->stream;
  const Geometry& g = c->geo;
  FusedArgs<T> f;
  f.a = op_args<T>(c, nrhs);
  const int S = cfg.S;
  f.S = S;
  f.nrhs = nrhs;
  f.tol = tol;
  f.maxit = maxit;
  f.bref = c->cg_ref;
  f.x = c->cg_x.p; f.r = c->cg_r.p; f.r1 = c->cg_r1.p; f.p0 = c->cg_p.p; f.p1 = c->cg_p1.p;
  f.s0 = c->cg_w.p; f.s1 = c->cg_s1.p;
  f.part = c->cg_part.p; f.mu_slot = c->mu_slot.p; f.e_slot = c->e_slot.p; f.scal = c->cg_scal.p;
  f.rsl = c->cg_rsl.p; f.ssl = c->cg_ssl.p; f.psl = c->cg_psl.p;
  f.err = c->flags.p;
  // LDS: gathered vectors (xs), product rows (ys), the partial sums of the
  // non-MFMA products (fewer than 8 right-hand sides only) and the coarse
  // right-hand side of the redundant coarse phases (not needed when they are
  // distributed); the less LDS, the more workgroups per compute unit.
  const int xs = std::max(g.max_nD, 1) * NR;
  const int ys = 2 * std::max(g.max_nG, 1) * NR;
  const int part = NR >= 8 ? 0 : kBlock * 2 * NR;
  const int cu = cfg.dist ? 0 : std::max(2 * c->nP, 1);
  f.lds_ys = xs;
  f.lds_part = xs + ys;
  f.lds_cu = xs + ys + part;
  // the distributed coarse rows stage whole coarse right-hand sides (2 nP
  // values each, at least one) in the same LDS, from its start
  // (and the corner columns of L, G and L^T for a slice, 2 x 4 x n_D values, from its start)
  const int area = std::max(cfg.dist ? std::max(xs + ys + part + cu, 2 * c->nP) : xs + ys + part + cu,
                            8 * std::max(g.max_nD, 1));
  f.lds_total = (area + 1) & ~1;     // the int tables after it stay 16-byte aligned
  f.dist = cfg.dist;
  f.X1t = c->X1t.p;
  f.ug = c->cg_u.p;
  f.cg1 = c->cg_c.p;
  const size_t smem0 = sizeof(double) * (size_t)f.lds_total;
  if (smem0 > 160 * 1024) c->fail(DDELM_E_SHAPE, "CG workspace exceeds the LDS of one compute unit");
  // index tables (owner slots of the units' Delta points, of all Pi points)
  int pi_owners = 0;
  for (int k = 0; k < c->nP; ++k) pi_owners = std::max(pi_owners, g.pi_own_ptr[k + 1] - g.pi_own_ptr[k]);
  const int tab_nd = std::max(g.max_nD, 1);
  const int tab_pi = (!f.dist && pi_owners <= kMaxOwn) ? 1 : 0;
  const size_t tab_bytes = sizeof(int) * ((size_t)kTabUnits * tab_nd * (1 + kMaxOwn) + (tab_pi ? (size_t)kMaxOwn * c->nP : 0));
  const bool tab_fits = smem0 + tab_bytes <= 160 * 1024;
  size_t smem = smem0 + (tab_fits ? tab_bytes : 0);
  const void* fn = cg_fused_kernel<T, NR>();
  if (smem > 65536) HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  int per_cu = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, smem));
  if (per_cu < 1) c->fail(DDELM_E_SHAPE, "CG kernel cannot be resident");
  int nb = std::min(c->num_cu * std::min(per_cu, 2), c->N * S);
  if (const char* env = getenv("DDELM_CG_BLOCKS")) nb = std::max(1, std::min(nb, atoi(env)));
  nb = std::max(1, std::min(nb, 4096));
  const int units_per_block = ceil_div(c->N * S, nb);
  f.tab_units = (tab_fits && units_per_block <= kTabUnits) ? units_per_block : 0;
  f.tab_nd = tab_nd;
  f.tab_pi = f.tab_units ? tab_pi : 0;
  if (const char* env = getenv("DDELM_CG_TABLES"))
    if (atoi(env) == 0) f.tab_units = f.tab_pi = 0;
  f.flags = c->bar.p;
  HIPCHK(hipMemcpyAsync(f.r, c->cg_b.p, (size_t)nrhs * c->nD * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(c->bar.p, 0, (size_t)nb * kFlagStride * sizeof(unsigned), s));
  void* args[] = {(void*)&f};
  HIPCHK(hipLaunchCooperativeKernel(fn, dim3(nb), dim3(kBlock), args, smem, s));
  c->cg_blocks = nb;
  c->cg_slices = S;
  c->cg_dist = f.dist;
}

// Autotuner of the CG launch.  The first solve of a problem shape in the
// process times a few iterations of every candidate configuration on the
// actual operator and right-hand side (tolerance 0, so each runs the same
// number of iterations) and keeps the fastest; later solves of the same shape
// reuse it.  Candidates: 1, 2 or 4 row slices per subdomain, and redundant or
// distributed coarse phases where n_Pi * nrhs makes both plausible.
// DDELM_CG_SLICES / DDELM_CG_COARSE fix a choice, DDELM_AUTOTUNE=0 turns the
// tuner off (then a size heuristic decides).
struct CgKey {
  int tsize, nr, N, nP, nD, maxG, maxD, nrhs;
  bool operator<(const CgKey& o) const {
    return std::tie(tsize, nr, N, nP, nD, maxG, maxD, nrhs) <
           std::tie(o.tsize, o.nr, o.N, o.nP, o.nD, o.maxG, o.maxD, o.nrhs);
  }
};
std::map<CgKey, CgConfig>& cg_tuned() {
  static std::map<CgKey, CgConfig>* m = new std::map<CgKey, CgConfig>();
  return *m;
}
constexpr int kTuneIters = 8;

template <typename T, int NR>
CgConfig cg_choose(ddelm_ctx c, int nrhs) {
  // heuristic: slices so that small problems still spread over the chip;
  // distributed coarse phases when every unit gathering the whole coarse
  // right-hand side would cost more than the extra synchronisations
  CgConfig h;
  h.S = std::max(1, std::min(4, 128 / std::max(c->N, 1)));
  h.dist = (long long)c->nP * nrhs > 512 ? 1 : 0;
  const char* es = getenv("DDELM_CG_SLICES");
  const char* ed = getenv("DDELM_CG_COARSE");
  const char* ea = getenv("DDELM_AUTOTUNE");
  if (es) h.S = std::max(1, std::min(8, atoi(es)));
  if (ed) h.dist = atoi(ed) != 0 ? 1 : 0;
  if ((es && ed) || (ea && atoi(ea) == 0)) return h;
  const CgKey key{(int)sizeof(T), NR, c->N, c->nP, c->nD, c->geo.max_nG, c->geo.max_nD, nrhs};
  {
    Resources& R = res();
    std::lock_guard<std::mutex> lk(R.mu);
    auto it = cg_tuned().find(key);
    if (it != cg_tuned().end()) return it->second;
  }
  if (c->noalloc) return h;      // no timing runs (they take events) inside an allocation-free call
  std::vector<CgConfig> cand;
  for (int S : {1, 2, 4}) {
    if (es && S != h.S) continue;
    if ((long long)c->N * S > 8192) continue;
    const long long np_r = (long long)c->nP * nrhs;
    for (int d : {0, 1}) {
      if (ed && d != h.dist) continue;
      if (!ed && d != h.dist && (np_r < 64 || np_r > 8192)) continue;   // only the heuristic's choice is plausible
      cand.push_back({S, d});
    }
  }
  hipStream_t s = c->stream;
  hipEvent_t t0 = take_event(c->device, true), t1 = take_event(c->device, true);
  CgConfig best = h;
  float best_ms = 1e30f;
  launch_fused<T, NR>(c, nrhs, 0.0, cand.front(), kTuneIters);    // warm-up (code load, first touch)
  for (const CgConfig& cf : cand) {
    HIPCHK(hipEventRecord(t0, s));
    launch_fused<T, NR>(c, nrhs, 0.0, cf, kTuneIters);
    HIPCHK(hipEventRecord(t1, s));
    HIPCHK(hipEventSynchronize(t1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    if (ms < best_ms) {
      best_ms = ms;
      best = cf;
    }
  }
  give_event(c->device, true, t0);
  give_event(c->device, true, t1);
  Resources& R = res();
  std::lock_guard<std::mutex> lk(R.mu);
  cg_tuned()[key] = best;
  return best;
}

template <typename T, int NR>
void cg_run(ddelm_ctx c, int nrhs, double tol) {
  const CgConfig cfg = cg_choose<T, NR>(c, nrhs);
  launch_fused<T, NR>(c, nrhs, tol, cfg, c->opt.maxit);
}

template <typename T>
void cg_persistent(ddelm_ctx c, int nrhs, double tol) {
  if (nrhs <= 1) cg_run<T, 1>(c, nrhs, tol);
  else if (nrhs <= 2) cg_run<T, 2>(c, nrhs, tol);
  else if (nrhs <= 4) cg_run<T, 4>(c, nrhs, tol);
  else if (nrhs <= 8) cg_run<T, 8>(c, nrhs, tol);
  else if (nrhs <= 16) cg_run<T, 16>(c, nrhs, tol);
  else c->fail(DDELM_E_ARG, "the persistent CG handles at most 16 right-hand sides");
}

// --------------------------------------------------------------- factorisation
// A batch of matrices to factor and apply: descriptors (host and device),
// the storage, and per matrix the column offset / leading dimension / column
// count seen by the block-reflector updates.
template <typename T>
struct QRSet {
  const QRDesc* desc = nullptr;
  const std::vector<QRDesc>* h = nullptr;
  const long long* coff = nullptr;
  const int* ldc = nullptr;
  const int* cn = nullptr;
  int nmat = 0, max_ncols = 0;
  T* A = nullptr;
  DBuf<T>* tau = nullptr;
  DBuf<T>* Tbuf = nullptr;
  DBuf<T>* Tbig = nullptr;
};

// Blocked Householder QR of every matrix of the set: 16-column panels
// updating their 64-column block, then one 64-wide block reflector per block
// for the trailing matrix; all products on MFMA.  tau must be allocated;
// Tbuf and Tbig are allocated here.
template <typename T>
void qr_all(ddelm_ctx c, const QRSet<T>& q) {
  hipStream_t s = c->stream;
  const int M = c->M;
  const int nmat = q.nmat;
  {
    c->npanel = ceil_div(M, kNB);
    c->nblock = ceil_div(M, kBB);
    q.Tbuf->alloc((size_t)nmat * c->npanel * kNB * kNB);
    q.Tbig->alloc((size_t)nmat * c->nblock * kBB * kBB);
    // Look-ahead: after block b is factored, its block reflector is applied
    // first to the columns of block b+1 (on the main stream, which then
    // factors block b+1) and to the columns beyond on a second stream, so
    // the panels of block b+1 run beside the bulk of block b's update.
    // Events: T[b] (block b factored, main), R[b] (block b's far update done,
    // side).  The near update of block b waits for R[b-1], which updated the
    // same columns before it; the two updates of one block touch disjoint
    // columns and read only that block's reflectors and T factor.
    const int nmat8 = ceil_div(nmat, 8) * 8;
    // block-reflector updates address a matrix by 32-bit byte offsets when
    // every matrix of the set is under 2^31 bytes
    bool off32 = true;
    for (const QRDesc& d : *q.h) off32 = off32 && (long long)d.ld * d.ncols * (long long)sizeof(T) < (1LL << 31);
    auto update = [&](int kb, int blk, int ntile, hipStream_t st, const int* cend, int cfirst) {
      if (off32)
        k_qr_wy64<T, kBC, true><<<nmat8 * ntile, kBlock, 0, st>>>(q.desc, q.A, q.Tbig->p, kb, blk,
                                                                  c->nblock, nmat, ntile, q.A, q.coff, q.ldc, cend,
                                                                  cfirst, 1);
      else
        k_qr_wy64<T><<<nmat8 * ntile, kBlock, 0, st>>>(q.desc, q.A, q.Tbig->p, kb, blk, c->nblock, nmat, ntile,
                                                       q.A, q.coff, q.ldc, cend, cfirst, 1);
    };
    hipStream_t s2 = c->side_stream();
    HIPCHK(hipEventRecord(c->sev(0), s));
    HIPCHK(hipStreamWaitEvent(s2, c->sev(0), 0));
    auto evT = [&](int b) { return c->sev(1 + 2 * (size_t)b); };
    auto evR = [&](int b) { return c->sev(2 + 2 * (size_t)b); };
    // column ends of every block (cnb) and of every near update (cnn), one upload
    std::vector<int> cn_all((size_t)2 * c->nblock * nmat);
    for (int blk = 0; blk < c->nblock; ++blk) {
      const int kb = blk * kBB, bw = std::min(kBB, M - kb);
      std::fill_n(cn_all.begin() + (size_t)2 * blk * nmat, nmat, kb + bw);
      std::fill_n(cn_all.begin() + (size_t)(2 * blk + 1) * nmat, nmat, std::min(kb + bw + kBB, M));
    }
    const int* cn_dev = c->arena.put(cn_all, s);
    // rows a panel touches: all from its first column on, or (zero band)
    // its own 16 and those from zhi on
    int panel_rows = 0;
    for (const QRDesc& d : *q.h) panel_rows = std::max(panel_rows, d.zhi > 0 ? std::min(d.m, d.m - d.zhi + kNB) : d.m);
    for (int blk = 0; blk < c->nblock; ++blk) {
      const int kb = blk * kBB, bw = std::min(kBB, M - kb);
      const int* cnb = cn_dev + (size_t)2 * blk * nmat;
      for (int k = kb; k < kb + bw; k += kNB) {
        const int p = k / kNB;
        launch_qr_panel16<T>(panel_rows, dim3(nmat), s, q.desc, q.A, q.tau->p, q.Tbuf->p, k, p,
                             c->npanel);
        const int c0 = k + std::min(kNB, M - k);
        if (c0 < kb + bw) {
          const dim3 grid(nmat, ceil_div(kb + bw - c0, kUC));
          if (off32)
            k_qr_wy<T, true><<<grid, kBlock, 0, s>>>(q.desc, q.A, q.Tbuf->p, k, p, c->npanel, q.A, q.coff, q.ldc,
                                                     cnb, c0, 1);
          else
            k_qr_wy<T><<<grid, kBlock, 0, s>>>(q.desc, q.A, q.Tbuf->p, k, p, c->npanel, q.A, q.coff, q.ldc, cnb, c0,
                                               1);
          HIPCHK(hipGetLastError());
        }
      }
      k_qr_tmerge<T><<<nmat, kBlock, 0, s>>>(q.desc, q.A, q.Tbuf->p, q.Tbig->p, kb, blk, c->npanel, c->nblock);
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(evT(blk), s));
      const int c0 = kb + bw;                                    // first trailing column
      const int c1 = std::min(c0 + kBB, M);                      // end of the next block
      // near update: the next block's columns, on the main stream
      if (c1 > c0) {
        if (blk > 0) HIPCHK(hipStreamWaitEvent(s, evR(blk - 1), 0));
        const int* cnn = cn_dev + (size_t)(2 * blk + 1) * nmat;   // = c1
        const int ntn = ceil_div(c1 - c0, kBC);
        update(kb, blk, ntn, s, cnn, c0);
        HIPCHK(hipGetLastError());
      }
      // far update: every column after the next block (and the appended unit
      // columns), on the side stream
      const int ntf = ceil_div(q.max_ncols - c1, kBC);
      HIPCHK(hipStreamWaitEvent(s2, evT(blk), 0));
      if (ntf > 0) {
        update(kb, blk, ntf, s2, q.cn, c1);
        HIPCHK(hipGetLastError());
      }
      HIPCHK(hipEventRecord(evR(blk), s2));
    }
    HIPCHK(hipStreamWaitEvent(s, evR(c->nblock - 1), 0));
  }
}

template <typename T>
void factor_impl(ddelm_ctx c) {
  hipStream_t s = c->stream;
  const int N = c->N, M = c->M;
  const Geometry& g = c->geo;
  const bool nn = c->use_nn;
  const int nmat = nn ? 2 * N : N;
  LocalBufs<T>& L = c->lb<T>();
  // ---- two-stage QR.  The interior and boundary rows (the first t_i =
  // n_I + n_B rows) of K_c^i and Kbar^i are the same, so their QR
  // T_i = Q1 [R1; 0] is done once; K_c^i and Kbar^i then only need the QR
  // of the (M + n_G) x M matrix [R1; G], G their interface rows, and
  // Q = diag(Q1, I) Q2.  The rows of Q at the interface (the transformed unit
  // columns) and R come from the second stage alone.  Used when every
  // subdomain has t_i >= M (otherwise one QR of the whole matrix).
  bool two = nn;
  for (int i = 0; i < N; ++i) two = two && c->h_m[i] - c->h_nG[i] >= M;
  if (const char* env = getenv("DDELM_QR_TWO_STAGE"))
    if (atoi(env) == 0) two = false;
  c->two_stage = two;
  // ---- layout of the QR matrices: K_c^i: m x (M + n_G), Kbar^i: m x (M + n_D)
  // (two-stage: (M + n_G) rows each)
  c->h_qrdesc.assign(nmat, QRDesc());
  long long off = 0, toff = 0;
  c->max_ncols = 0;
  for (int b = 0; b < nmat; ++b) {
    const int i = b % N;
    QRDesc d;
    const int rows = two ? M + c->h_nG[i] : c->h_m[i];
    d.off = off; d.m = rows; d.ld = rows;
    d.ncols = M + (b < N ? c->h_nG[i] : c->h_nD[i]);
    d.nrefl = M; d.tau = toff;
    d.zhi = two ? M : 0;   // [R1; G]: R1 is upper triangular
    c->h_qrdesc[b] = d;
    off += (long long)d.ld * d.ncols;
    toff += M;
    c->max_ncols = std::max(c->max_ncols, d.ncols);
  }
  L.qrA.alloc(off);
  L.tau.alloc(toff);
  c->qrdesc.upload(c->h_qrdesc, s);
  if (!two) {
    long long most = 0;
    for (const QRDesc& d : c->h_qrdesc) most = std::max(most, (long long)d.ld * (d.ncols - d.nrefl));
    if (most > 0) {
      k_zero_appended<T><<<dim3(std::min(ceil_div(most, kBlock), 64), nmat), kBlock, 0, s>>>(c->qrdesc.p, L.qrA.p);
      HIPCHK(hipGetLastError());
    }
  }
  {
    std::vector<long long> coff(nmat);
    std::vector<int> ldc(nmat), cn(nmat);
    for (int b = 0; b < nmat; ++b) { coff[b] = c->h_qrdesc[b].off; ldc[b] = c->h_qrdesc[b].ld; cn[b] = c->h_qrdesc[b].ncols; }
    c->qr_coff.upload(coff, s); c->qr_ldc.upload(ldc, s); c->qr_cn.upload(cn, s);
  }
  // stage one: the full features of K_c^i (ld m_i) hold T_i in their first t_i rows
  DBuf<T> kbfull;
  if (two) {
    c->h_topdesc.assign(N, QRDesc());
    long long o = 0;
    for (int i = 0; i < N; ++i) {
      QRDesc d;
      d.off = o; d.m = c->h_m[i] - c->h_nG[i]; d.ld = c->h_m[i];
      d.ncols = M; d.nrefl = M; d.tau = (long long)i * M; d.zhi = 0;
      c->h_topdesc[i] = d;
      o += (long long)c->h_m[i] * M;
    }
    L.topA.alloc(o);
    L.tau1.alloc((size_t)N * M);
    kbfull.alloc(o);
    c->topdesc.upload(c->h_topdesc, s);
    std::vector<long long> coff(N);
    std::vector<int> ldc(N), cn(N, M);
    for (int i = 0; i < N; ++i) { coff[i] = c->h_topdesc[i].off; ldc[i] = c->h_topdesc[i].ld; }
    c->top_coff.upload(coff, s); c->top_ldc.upload(ldc, s); c->top_cn.upload(cn, s);
  } else {
    L.topA.free(); L.tau1.free(); L.Tbuf1.free(); L.Tbig1.free();
  }
  c->mark(0);
  // ---- features
  {
    std::vector<long long> o1(N), o2(N);
    std::vector<int> l1(N);
    for (int i = 0; i < N; ++i) {
      o1[i] = two ? c->h_topdesc[i].off : c->h_qrdesc[i].off;
      o2[i] = two ? c->h_topdesc[i].off : c->h_qrdesc[N + i].off;
      l1[i] = c->h_m[i];
    }
    c->h_offAm.assign(N + 1, 0);
    c->h_offCD.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) {
      c->h_offAm[i + 1] = c->h_offAm[i] + (long long)c->h_nG[i] * M;
      c->h_offCD[i + 1] = c->h_offCD[i] + (long long)c->h_nD[i] * M;
    }
    const std::vector<long long> oAm(c->h_offAm.begin(), c->h_offAm.end() - 1);
    const std::vector<int> ldA(c->h_nG.begin(), c->h_nG.end());
    L.Am.alloc(std::max(c->h_offAm[N], 1ll));
    assemble_features<T>(c, c->rsK, g.max_m, two ? L.topA.p : L.qrA.p, o1, l1, 0, N);
    assemble_features<T>(c, c->rsA, g.max_nG, L.Am.p, oAm, ldA, 0, N);
    if (nn) {
      // two-stage: only the interface rows of Kbar^i (its other rows are those of K_c^i)
      const int* kb_first = nullptr;
      if (two) {
        std::vector<int> fr(N);
        for (int i = 0; i < N; ++i) fr[i] = c->h_m[i] - c->h_nG[i];
        kb_first = c->arena.put(fr, s);
      }
      assemble_features<T>(c, c->rsKb, g.max_m, two ? kbfull.p : L.qrA.p, o2, l1, 0, N, kb_first);
      std::vector<int> ldC(c->h_nD.begin(), c->h_nD.end());
      const std::vector<long long> oCD(c->h_offCD.begin(), c->h_offCD.end() - 1);
      L.CD.alloc(std::max(c->h_offCD[N], 1ll));
      assemble_features<T>(c, c->rsAb, g.max_nD, L.CD.p, oCD, ldC, 0, N);
    }
    if (!two) {
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
        k_set_units<T><<<ceil_div((long long)pos.size(), kBlock), kBlock, 0, s>>>(dp, (long long)pos.size(), L.qrA.p);
        HIPCHK(hipGetLastError());
      }
    }
  }
  c->mark(1);
  // Mixed precision: the Householder QR (the bulk of the flops) runs in
  // float32 on the f32 matrix cores.  Its factors are then widened to
  // float64, and everything downstream (triangular solves, local interface
  // operators, coarse problem, right-hand sides, recovery) runs in float64
  // arithmetic on them; only the CG keeps float32 copies of the local
  // interface operators.  The K_c^i features stay in float64 for the
  // refinement residuals.
  if (c->mixed) {
    c->h_offK.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) c->h_offK[i + 1] = c->h_offK[i] + (long long)c->h_m[i] * M;
    c->K64.alloc(c->h_offK[N]);
    std::vector<CopyDesc> cp;
    for (int i = 0; i < N; ++i) {
      const long long src = two ? c->h_topdesc[i].off : c->h_qrdesc[i].off;
      cp.push_back(CopyDesc{src, c->h_offK[i], c->h_m[i], c->h_m[i], c->h_m[i], M, 0, 0});
    }
    copy_batch<double, double>(c, cp, two ? L.topA.p : L.qrA.p, c->K64.p);
    c->offK_d.upload(std::vector<long long>(c->h_offK.begin(), c->h_offK.end() - 1), s);
  }
  // one QR stage over a set of matrices, in float64 or (mixed) in float32 and widened
  auto run_qr = [&](QRSet<T> q64) {
    if (!c->mixed) {
      qr_all<T>(c, q64);
      return;
    }
    const size_t nA = q64.A == L.qrA.p ? L.qrA.n : L.topA.n;
    DBuf<float> A32, tau32, Tbuf32, Tbig32;
    A32.alloc(nA);
    tau32.alloc(q64.tau->n);
    convert<double, float>(s, q64.A, A32.p, (long long)nA);
    QRSet<float> q32;
    q32.desc = q64.desc; q32.h = q64.h; q32.coff = q64.coff; q32.ldc = q64.ldc; q32.cn = q64.cn;
    q32.nmat = q64.nmat; q32.max_ncols = q64.max_ncols;
    q32.A = A32.p; q32.tau = &tau32; q32.Tbuf = &Tbuf32; q32.Tbig = &Tbig32;
    qr_all<float>(c, q32);
    convert<float, double>(s, A32.p, q64.A, (long long)nA);
    convert<float, double>(s, tau32.p, q64.tau->p, (long long)tau32.n);
    q64.Tbig->alloc(Tbig32.n);
    convert<float, double>(s, Tbig32.p, q64.Tbig->p, (long long)Tbig32.n);
  };
  if (two) {
    QRSet<T> q1;
    q1.desc = c->topdesc.p; q1.h = &c->h_topdesc; q1.coff = c->top_coff.p; q1.ldc = c->top_ldc.p; q1.cn = c->top_cn.p;
    q1.nmat = N; q1.max_ncols = M;
    q1.A = L.topA.p; q1.tau = &L.tau1; q1.Tbuf = &L.Tbuf1; q1.Tbig = &L.Tbig1;
    run_qr(q1);
    // the reduced matrices [R1 0; G E] of K_c^i and Kbar^i
    std::vector<int> uoff(nmat);
    for (int b = 0; b < nmat; ++b) uoff[b] = b < N ? 0 : c->h_nP[b % N];
    const int* duoff = c->arena.put(uoff, s);
    int most = 0;   // columns of the widest matrix
    for (const QRDesc& d : c->h_qrdesc) most = std::max(most, d.ncols);
    k_stage2_assemble<T><<<dim3((unsigned)std::min(most, 64), nmat), kBlock, 0, s>>>(
        c->qrdesc.p, c->topdesc.p, N, M, duoff, L.topA.p, kbfull.p, L.qrA.p);
    HIPCHK(hipGetLastError());
    kbfull.free();
  }
  {
    QRSet<T> q2;
    q2.desc = c->qrdesc.p; q2.h = &c->h_qrdesc; q2.coff = c->qr_coff.p; q2.ldc = c->qr_ldc.p; q2.cn = c->qr_cn.p;
    q2.nmat = nmat; q2.max_ncols = c->max_ncols;
    q2.A = L.qrA.p; q2.tau = &L.tau; q2.Tbuf = &L.Tbuf; q2.Tbig = &L.Tbig;
    run_qr(q2);
  }
  c->mark(2);
  // ---- condition estimates of the triangular factors (reported in the solve statistics)
  DBuf<double> kap;
  kap.alloc(nmat);
  k_diag_ratio<T><<<nmat, kBlock, 0, s>>>(c->qrdesc.p, L.qrA.p, kap.p);
  HIPCHK(hipGetLastError());
  std::vector<double> h_kap(nmat);
  HIPCHK(hipMemcpyAsync(h_kap.data(), kap.p, nmat * sizeof(double), hipMemcpyDeviceToHost, s));
  // ---- Q_G^T copy (M x n_G, ld M), then E = R^{-1} Q_G^T and Xbar = Rbar^{-1} Qbar_D^T in place
  {
    c->h_offQG.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) c->h_offQG[i + 1] = c->h_offQG[i] + (long long)M * c->h_nG[i];
    L.QG.alloc(std::max(c->h_offQG[N], 1ll));
    std::vector<CopyDesc> cp;
    for (int i = 0; i < N; ++i) {
      const QRDesc& d = c->h_qrdesc[i];
      if (c->h_nG[i] == 0) continue;
      cp.push_back(CopyDesc{d.off + (long long)M * d.ld, c->h_offQG[i], d.ld, M, M, c->h_nG[i], 0, 0});
    }
    copy_batch<T, T>(c, cp, L.qrA.p, L.QG.p);
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
      const size_t smt = (size_t)M * kTRSMC * sizeof(T);
      if (smt > 65536)
        HIPCHK(hipFuncSetAttribute((const void*)k_trsm<T, kTRSMC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)smt));
      const int nt = ceil_div(maxx, kTRSMC);
      k_trsm<T, kTRSMC><<<ceil_div(nmat, 8) * 8 * nt, kBlock, smt, s>>>(c->qrdesc.p, L.qrA.p, L.qrA.p, dxo, dld, dxn,
                                                                       0, nmat, nt);
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
    L.Gm.alloc(nGt); L.Lm.alloc(nGt); L.LTm.alloc(nGt);
    L.Nm.alloc(nNt); L.NTm.alloc(nNt);
    ZeroBatch().add(L.Gm).add(L.Lm).add(L.LTm).add(L.Nm).add(L.NTm).launch(s);
    c->offG.upload(std::vector<long long>(c->h_offG.begin(), c->h_offG.end() - 1), s);
    c->offN.upload(std::vector<long long>(c->h_offN.begin(), c->h_offN.end() - 1), s);
    std::vector<GemmDesc> gG, gL, gN;
    std::vector<CopyDesc> tL, tN;
    for (int i = 0; i < N; ++i) {
      const int ng = c->h_nG[i], nd = c->h_nD[i];
      const QRDesc& d = c->h_qrdesc[i];
      if (ng == 0) continue;
      gG.push_back(GemmDesc{c->h_offQG[i], c->h_offQG[i], c->h_offG[i], M, M, ng, ng, ng, M});
      gL.push_back(GemmDesc{c->h_offAm[i], d.off + (long long)M * d.ld, c->h_offG[i], ng, d.ld, ng, ng, ng, M});
      tL.push_back(CopyDesc{c->h_offG[i], c->h_offG[i], ng, ng, ng, ng, 1, 0});
      if (nn && nd > 0) {
        const QRDesc& db = c->h_qrdesc[N + i];
        gN.push_back(GemmDesc{c->h_offCD[i], db.off + (long long)M * db.ld, c->h_offN[i], nd, db.ld, nd, nd, nd, M});
        tN.push_back(CopyDesc{c->h_offN[i], c->h_offN[i], nd, nd, nd, nd, 1, 0});
      }
    }
    gemm_batch<T>(c, gG, L.QG.p, L.QG.p, L.Gm.p, 1, -1.0, 0.0);
    {
      std::vector<long long> o;
      std::vector<int> n;
      for (int i = 0; i < N; ++i) if (c->h_nG[i]) { o.push_back(c->h_offG[i]); n.push_back(c->h_nG[i]); }
      if (!o.empty()) {
        const long long* dO = c->arena.put(o, s);
        const int* dn = c->arena.put(n, s);
        k_add_diag_t<T><<<(unsigned)o.size(), kBlock, 0, s>>>(dO, dn, L.Gm.p, T(1));
        HIPCHK(hipGetLastError());
      }
    }
    gemm_batch<T>(c, gL, L.Am.p, L.qrA.p, L.Lm.p, 0, 1.0, 0.0);
    copy_batch<T, T>(c, tL, L.Lm.p, L.LTm.p);
    if (!gN.empty()) {
      gemm_batch<T>(c, gN, L.CD.p, L.qrA.p, L.Nm.p, 0, 1.0, 0.0);
      copy_batch<T, T>(c, tN, L.Nm.p, L.NTm.p);
    }
    if (c->f32cg) {
      // float32 copies of the local interface operators for the CG
      LocalBufs<float>& L32 = c->l32;
      DBuf<T>* src[5] = {&L.Gm, &L.Lm, &L.LTm, &L.Nm, &L.NTm};
      DBuf<float>* dst[5] = {&L32.Gm, &L32.Lm, &L32.LTm, &L32.Nm, &L32.NTm};
      for (int k = 0; k < 5; ++k) {
        dst[k]->alloc(src[k]->n);
        convert<T, float>(s, src[k]->p, dst[k]->p, (long long)src[k]->n);
      }
    }
  }
  c->mark(3);
  // ---- coarse problem (float64): D_PiPi, S_Pi = sum G_PiPi + D^T D, Cholesky, inverse, X1
  if (c->nP > 0) {
    const int n = c->nP;
    const size_t nn2 = (size_t)n * n;
    c->Dpp.alloc(nn2); c->Gs.alloc(nn2); c->Spi.alloc(nn2); c->Sfac.alloc(nn2); c->Sinv.alloc(nn2);
    c->Zm.alloc(nn2); c->Ztm.alloc(nn2); c->Wm.alloc(nn2); c->X1.alloc(4 * nn2);
    c->Dpp.zero(s); c->Gs.zero(s);
    k_coarse_assemble<T><<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, c->pi_own_ptr.p, c->pi_own_slot.p, c->pi_slot_sub.p,
                                                                c->pi_off.p, c->pi_l2g.p, c->offG.p, c->nG_dev.p,
                                                                L.Gm.p, L.Lm.p, c->Dpp.p, c->Gs.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->Spi.p, c->Gs.p, nn2 * sizeof(double), hipMemcpyDeviceToDevice, s));
    gemm_batch<double>(c, {GemmDesc{0, 0, 0, n, n, n, n, n, n}}, c->Dpp.p, c->Dpp.p, c->Spi.p, 1, 1.0, 1.0);
    HIPCHK(hipMemcpyAsync(c->Sfac.p, c->Spi.p, nn2 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(c->flags.p, 0, 8 * sizeof(unsigned), s));
    {
      DBuf<double> lt;   // L21^T of the current block column
      lt.alloc((size_t)kCB * n);
      for (int k0 = 0; k0 < n; k0 += kCB) {
        const int nbk = std::min(kCB, n - k0), m = n - k0 - nbk;
        k_chol_diag<<<1, kBlock, 0, s>>>(c->Sfac.p, n, k0, nbk, c->flags.p);
        HIPCHK(hipGetLastError());
        if (m == 0) break;
        k_chol_panel<<<ceil_div(m, kBlock), kBlock, 0, s>>>(c->Sfac.p, n, k0, nbk);
        HIPCHK(hipGetLastError());
        copy_batch<double, double>(c, {CopyDesc{(long long)k0 * n + k0 + nbk, 0, n, nbk, m, nbk, 1, 0}}, c->Sfac.p,
                                   lt.p);
        gemm_batch<double>(c, {GemmDesc{(long long)k0 * n + k0 + nbk, 0, (long long)(k0 + nbk) * n + k0 + nbk, n, nbk,
                                        n, m, m, nbk}},
                           c->Sfac.p, lt.p, c->Sfac.p, 0, -1.0, 1.0);
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    const size_t smi = (size_t)n * 4 * sizeof(double);
    if (smi + sizeof(double) * kIB * (kIB + 1) > 160 * 1024)
      c->fail(DDELM_E_SHAPE, "coarse problem too large for the inverse kernel");
    if (smi > 65536) HIPCHK(hipFuncSetAttribute((const void*)k_chol_inverse, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smi));
    k_chol_inverse<<<ceil_div(n, 4), kBlock, smi, s>>>(c->Sfac.p, n, c->Sinv.p);
    HIPCHK(hipGetLastError());
    gemm_batch<double>(c, {GemmDesc{0, 0, 0, n, n, n, n, n, n}}, c->Dpp.p, c->Sinv.p, c->Zm.p, 0, 1.0, 0.0);
    copy_batch<double, double>(c, {CopyDesc{0, 0, n, n, n, n, 1, 0}}, c->Zm.p, c->Ztm.p);
    gemm_batch<double>(c, {GemmDesc{0, 0, 0, n, n, n, n, n, n}}, c->Dpp.p, c->Ztm.p, c->Wm.p, 0, 1.0, 0.0);
    k_assemble_X1<<<std::min(ceil_div(4ll * nn2, kBlock), 4096), kBlock, 0, s>>>(n, c->Sinv.p, c->Zm.p, c->Wm.p,
                                                                                 c->X1.p);
    HIPCHK(hipGetLastError());
    c->X1t.alloc(4 * nn2);
    copy_batch<double, double>(c, {CopyDesc{0, 0, 2 * n, 2 * n, 2 * n, 2 * n, 1, 0}}, c->X1.p, c->X1t.p);
  } else {
    c->X1.alloc(1);
    c->X1t.alloc(1);
  }
  c->mark(4);
  c->offm_d.upload(std::vector<long long>(c->h_offm.begin(), c->h_offm.end() - 1), s);
  c->offB_d.upload(std::vector<long long>(c->h_offB.begin(), c->h_offB.end() - 1), s);
  c->offQG_d.upload(std::vector<long long>(c->h_offQG.begin(), c->h_offQG.end() - 1), s);
  c->offAm_d.upload(std::vector<long long>(c->h_offAm.begin(), c->h_offAm.end() - 1), s);
  unsigned fl[8];
  HIPCHK(hipMemcpyAsync(fl, c->flags.p, sizeof(fl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (fl[0] & 2u) c->fail(DDELM_E_CHOLESKY, "S_Pi is not positive definite");
  c->kappa_est = 0.0;
  for (double v : h_kap) c->kappa_est = std::max(c->kappa_est, v);
  for (int k = 0; k < 4; ++k) c->phase_ms[k] = c->span(k, k + 1);
}

// --------------------------------------------------------------- one DDELM-NN solve on prepared local RHS
//
// F (type T, [nrhs][sum m]) holds f^i for every subdomain; fGP/fGD are its
// interface rows in slot order (null when zero); hP/hD the flux right-hand
// side (null when zero).  Writes coef (overwrite or accumulate), mu_pi, mu_dl.
struct CoreOut {
  int iters = 0;
  double relres = 0.0;
  bool noconv = false;
  double true_rel = 0.0;     // float64 residual of the interface system after the solve
  double start_rel = 0.0;    // ... at the starting point (warm start), else 0
  int restarts = 0;
  double ms_rhs = 0, ms_cg = 0, ms_rec = 0;
};

// CG on eq. nn-mixed for the right-hand sides in cg_b (solution in cg_x)
template <typename T>
void run_cg(ddelm_ctx c, int nrhs, double tol, CoreOut& res) {
  if (c->nD == 0) return;
  hipStream_t s = c->stream;
  const int mode = c->opt.cg_mode == 0 ? (nrhs <= 16 ? 2 : 1) : c->opt.cg_mode;
  if (mode == 2) cg_persistent<T>(c, nrhs, tol);
  else cg_multilaunch<T>(c, nrhs, tol);
  std::vector<double> sc((size_t)nrhs * 8);
  unsigned fl[8];
  HIPCHK(hipMemcpyAsync(sc.data(), c->cg_scal.p, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(fl, c->flags.p, sizeof(fl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (fl[0] & 1u) c->fail(DDELM_E_HIP, "device grid barrier wait expired");
  for (int r = 0; r < nrhs; ++r) {
    res.iters = std::max(res.iters, (int)sc[8 * r + 6]);
    const double rr = sc[8 * r], bb = sc[8 * r + 1];
    if (!(rr == rr)) c->fail(DDELM_E_NONFINITE, "NaN in CG");
    res.relres = std::max(res.relres, bb > 0 ? std::sqrt(rr / bb) : 0.0);
    if (sc[8 * r + 5] == 0.0) res.noconv = true;
  }
}

// out = S_theta v ([nrhs][nD]) with the float64 local operators: the operator
// phases of the CG, launched one by one (they reuse the solve workspace; the
// recovery recomputes what it needs from mu_Delta).
void apply_s_theta64(ddelm_ctx c, int nrhs, const double* v, double* out) {
  hipStream_t s = c->stream;
  OpArgs<double> a = op_args<double>(c, nrhs);
  launch_local_v<double>(c, a, v, nrhs, s);
  run_phases_after_stage1<double>(c, a, nrhs, nullptr);
  k_ph_sum_w<double><<<dim3(ceil_div(c->nD, kBlock), nrhs), kBlock, 0, s>>>(a, out);
  HIPCHK(hipGetLastError());
}

constexpr int kMaxRestarts = 3;         // float64 CG: restarts against recurrence drift
constexpr int kMaxRefineRestarts = 12;  // float32 CG operators: each restart is one refinement step

// S_theta mu = b (b in cg_b, mu returned in cg_x) from the starting point x0
// (null: zero).  The CG (local operators of storage type TC) runs on the
// residual b - S_theta x0 and stops at tol relative to ||b||; then the
// residual is formed again with the float64 operators and, while it exceeds
// tol ||b|| (recurrence drift; float32 operators), the CG is restarted on it.
template <typename TC>
void interface_solve(ddelm_ctx c, int nrhs, double tol, const double* x0, CoreOut& res) {
  if (c->nD == 0) return;
  hipStream_t s = c->stream;
  const long long nv = (long long)nrhs * c->nD;
  const size_t vb = (size_t)nv * sizeof(double);
  HIPCHK(hipMemcpyAsync(c->cg_b0.p, c->cg_b.p, vb, hipMemcpyDeviceToDevice, s));
  std::vector<double> nrm((size_t)2 * nrhs);
  if (x0) {
    HIPCHK(hipMemcpyAsync(c->cg_xs.p, x0, vb, hipMemcpyDeviceToDevice, s));
    apply_s_theta64(c, nrhs, c->cg_xs.p, c->cg_sx.p);
    k_resid_norms<<<nrhs, kBlock, 0, s>>>(c->nD, c->cg_b0.p, c->cg_sx.p, c->cg_b.p, c->cg_nrm.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(nrm.data(), c->cg_nrm.p, nrm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r)
      if (nrm[nrhs + r] > 0.0) res.start_rel = std::max(res.start_rel, std::sqrt(nrm[r] / nrm[nrhs + r]));
  } else {
    k_resid_norms<<<nrhs, kBlock, 0, s>>>(c->nD, c->cg_b0.p, nullptr, nullptr, c->cg_nrm.p);
  }
  HIPCHK(hipGetLastError());
  struct RefScope {
    ddelm_ctx c;
    ~RefScope() { c->cg_ref = nullptr; }
  } ref_scope{c};
  c->cg_ref = c->cg_nrm.p + nrhs;    // ||b||^2 per right-hand side
  bool have_x = x0 != nullptr;
  for (int k = 0;; ++k) {
    CoreOut part;
    run_cg<TC>(c, nrhs, tol, part);
    res.iters += part.iters;
    res.relres = part.relres;
    res.noconv = res.noconv || part.noconv;
    if (have_x) {
      k_add_to<<<std::min(ceil_div(nv, kBlock), 1024), kBlock, 0, s>>>(nv, c->cg_x.p, c->cg_xs.p);
      HIPCHK(hipGetLastError());
    } else {
      HIPCHK(hipMemcpyAsync(c->cg_xs.p, c->cg_x.p, vb, hipMemcpyDeviceToDevice, s));
    }
    have_x = true;
    apply_s_theta64(c, nrhs, c->cg_xs.p, c->cg_sx.p);
    k_resid_norms<<<nrhs, kBlock, 0, s>>>(c->nD, c->cg_b0.p, c->cg_sx.p, c->cg_b.p, c->cg_nrm.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(nrm.data(), c->cg_nrm.p, nrm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      const double rr = nrm[r], bb = nrm[nrhs + r];
      if (!(rr == rr)) c->fail(DDELM_E_NONFINITE, "NaN in the interface residual");
      worst = std::max(worst, bb > 0.0 ? std::sqrt(rr / bb) : 0.0);
    }
    res.true_rel = worst;
    if (worst <= tol || k == (c->f32cg ? kMaxRefineRestarts : kMaxRestarts) || part.noconv) break;
    res.restarts += 1;
  }
  HIPCHK(hipMemcpyAsync(c->cg_x.p, c->cg_xs.p, vb, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->cg_b.p, c->cg_b0.p, vb, hipMemcpyDeviceToDevice, s));
}

// Q^T or Q applied to the first nrhs columns of the local right-hand sides
// of every K_c^i: for up to 4 columns one launch applies all blocks (columns
// in LDS), otherwise one 64-column-tile launch per block.
template <typename T, int NR>
void launch_apply_narrow(ddelm_ctx c, const QRDesc* desc, const T* A, const T* Tbig, int nrhs, int transT,
                         hipStream_t s) {
  LocalBufs<T>& L = c->lb<T>();
  const size_t smem = (size_t)std::max(c->geo.max_m, 1) * NR * sizeof(T);
  const void* fn = (const void*)k_qr_apply_narrow<T, NR>;
  if (smem > 65536) HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  k_qr_apply_narrow<T, NR><<<c->N, an_threads(NR), smem, s>>>(desc, A, Tbig, c->nblock, L.F.p, c->f_off.p,
                                                              c->f_ld.p, nrhs, transT);
  HIPCHK(hipGetLastError());
}

// Q^T (transT = 1) or Q (transT = 0) of one set of N matrices applied to the
// local vectors F (rows 0..d.m-1 of every subdomain's block).
template <typename T>
void apply_q_set(ddelm_ctx c, const QRDesc* desc, const T* A, const T* Tbig, int nrhs, int transT, hipStream_t s) {
  if (nrhs <= 1) return launch_apply_narrow<T, 1>(c, desc, A, Tbig, nrhs, transT, s);
  if (nrhs <= 2) return launch_apply_narrow<T, 2>(c, desc, A, Tbig, nrhs, transT, s);
  if (nrhs <= 4) return launch_apply_narrow<T, 4>(c, desc, A, Tbig, nrhs, transT, s);
  LocalBufs<T>& L = c->lb<T>();
  const int N = c->N;
  const int* cnR = c->arena.put(std::vector<int>(N, nrhs), s);
  // 32-bit byte offsets when a subdomain's block of F (nrhs columns of
  // leading dimension summ) and every QR matrix are under 2^31 bytes
  bool off32 = (long long)c->summ * nrhs * (long long)sizeof(T) < (1LL << 31);
  for (const QRDesc& d : c->h_qrdesc) off32 = off32 && (long long)d.ld * d.ncols * (long long)sizeof(T) < (1LL << 31);
  for (const QRDesc& d : c->h_topdesc) off32 = off32 && (long long)d.ld * d.ncols * (long long)sizeof(T) < (1LL << 31);
  for (int q = 0; q < c->nblock; ++q) {
    const int blk = transT ? q : c->nblock - 1 - q;
    const int ntile = nrhs <= 16 ? 1 : ceil_div(nrhs, kBC);
    const dim3 grid(ceil_div(N, 8) * 8 * ntile);
    auto args = std::make_tuple(desc, A, Tbig, blk * kBB, blk, c->nblock, N, ntile, L.F.p, (const long long*)c->f_off.p,
                                (const int*)c->f_ld.p, cnR, 0, transT);
    auto launch = [&](auto kern) {
      std::apply([&](auto... a) { kern<<<grid, kBlock, 0, s>>>(a...); }, args);
    };
    if (nrhs <= 16)   // one 16-column tile per matrix
      off32 ? launch(k_qr_wy64<T, 16, true>) : launch(k_qr_wy64<T, 16>);
    else
      off32 ? launch(k_qr_wy64<T, kBC, true>) : launch(k_qr_wy64<T>);
    HIPCHK(hipGetLastError());
  }
}

// Q^T (transT = 1) or Q (transT = 0) of every K_c^i applied to the local
// vectors F.  Two-stage factors: Q = diag(Q1, I) Q2 in the full row order
// once the interface rows are moved next to the first M rows: Q^T is Q1^T on
// the first t_i rows, the interface rows moved up to row M, then Q2^T; Q is
// the reverse (the rows M..t_i-1 of the first stage's vector are zero).
template <typename T>
void apply_q_local(ddelm_ctx c, int nrhs, int transT, hipStream_t s) {
  LocalBufs<T>& L = c->lb<T>();
  if (!c->two_stage) return apply_q_set<T>(c, c->qrdesc.p, L.qrA.p, L.Tbig.p, nrhs, transT, s);
  const size_t sm = sizeof(double) * (size_t)std::max(c->geo.max_nG, 1);
  if (transT) {
    apply_q_set<T>(c, c->topdesc.p, L.topA.p, L.Tbig1.p, nrhs, 1, s);
    k_move_rows<T><<<dim3(c->N, nrhs), kBlock, sm, s>>>(c->M, c->sizes_dev.p, c->offm_d.p, c->summ, L.F.p, 0);
    HIPCHK(hipGetLastError());
    apply_q_set<T>(c, c->qrdesc.p, L.qrA.p, L.Tbig.p, nrhs, 1, s);
  } else {
    apply_q_set<T>(c, c->qrdesc.p, L.qrA.p, L.Tbig.p, nrhs, 0, s);
    k_move_rows<T><<<dim3(c->N, nrhs), kBlock, sm, s>>>(c->M, c->sizes_dev.p, c->offm_d.p, c->summ, L.F.p, 1);
    HIPCHK(hipGetLastError());
    apply_q_set<T>(c, c->topdesc.p, L.topA.p, L.Tbig1.p, nrhs, 0, s);
  }
}

template <typename T>
CoreOut solve_core(ddelm_ctx c, int nrhs, const double* fGP, const double* fGD, const double* hP, const double* hD,
                   double tol, double* coef, int accumulate, double* mu_pi_out, double* mu_dl_out,
                   const double* x0 = nullptr) {
  CoreOut res;
  hipStream_t s = c->stream;
  const int N = c->N, M = c->M;
  LocalBufs<T>& L = c->lb<T>();
  auto t0 = std::chrono::steady_clock::now();
  c->mark(5);
  // ---- Q^T f (block reflectors), projections, K^+ f, fluxes
  apply_q_local<T>(c, nrhs, 1, s);
  const int PM = rhs_group(nrhs, M);   // right-hand sides per workgroup with M values each in LDS
  with_rhs_group(PM, [&](auto kp) {
    constexpr int P = decltype(kp)::value;
    k_rhs_proj<T, P><<<dim3(N, ceil_div(nrhs, P)), kBlock, (size_t)M * P * sizeof(double), s>>>(
        M, nrhs, c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->offQG_d.p, L.QG.p, c->offm_d.p, c->summ, L.F.p, c->sumP,
        c->sumD, fGP, fGD, c->rho_loc.p, c->s_loc.p);
  });
  HIPCHK(hipGetLastError());
  {
    const size_t smt = (size_t)M * kTRSMC * sizeof(T);
    const int* cnM = c->arena.put(std::vector<int>(N, nrhs), s);
    const int nt = ceil_div(nrhs, kTRSMC);
    k_trsm<T, kTRSMC><<<ceil_div(N, 8) * 8 * nt, kBlock, smt, s>>>(c->qrdesc.p, L.qrA.p, L.F.p, c->f_off.p,
                                                                   c->f_ld.p, cnM, 0, N, nt);
    HIPCHK(hipGetLastError());

    with_rhs_group(PM, [&](auto kp) {
      constexpr int P = decltype(kp)::value;
      k_rhs_flux<T, T, P><<<dim3(N, ceil_div(nrhs, P)), kBlock, (size_t)M * P * sizeof(double), s>>>(
          M, c->nD, nrhs, c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->dl_l2g.p, c->dl_own_ptr.p, c->dl_own_slot.p,
          c->offAm_d.p, L.Am.p, c->offm_d.p, c->summ, L.F.p, c->sumP, c->sumD, hD, c->psi_loc.p, c->l_loc.p);
    });
    HIPCHK(hipGetLastError());
  }
  // ---- b of eq. nn-mixed
  OpArgs<T> a = op_args<T>(c, nrhs);
  run_phases_after_stage1<T>(c, a, nrhs, hP);
  if (c->nD > 0) {
    k_ph_sum_w<T><<<dim3(ceil_div(c->nD, kBlock), nrhs), kBlock, 0, s>>>(a, c->cg_b.p);
    HIPCHK(hipGetLastError());
  }
  if (c->nP > 0) {
    k_save_pif<<<ceil_div(c->nP * nrhs, kBlock), kBlock, 0, s>>>(c->nP, nrhs, c->c1.p, c->pif.p);
    HIPCHK(hipGetLastError());
  }
  c->mark(6);
  HIPCHK(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  // ---- CG (float32 local operators in mixed precision)
  if (c->f32cg) interface_solve<float>(c, nrhs, tol, x0, res);
  else interface_solve<T>(c, nrhs, tol, x0, res);
  c->mark(7);
  auto t2 = std::chrono::steady_clock::now();
  // ---- recovery: mu_Pi = pi_f - [S^-1 (rho + D^T psi)](mu_D); c = c_f0 + E mu
  if (c->nP > 0) {
    if (c->nD > 0) {
      const size_t sm = local_smem(c);
      launch_local_v<T>(c, a, c->cg_x.p, nrhs, s);
      k_ph_coarse1<T><<<dim3(ceil_div(2 * c->nP, kBlock), nrhs), kBlock, sm, s>>>(a);
      HIPCHK(hipGetLastError());
    } else {
      fill(s, c->c1.p, (long long)nrhs * 2 * c->nP, 0.0);
    }
    k_mu_pi<<<ceil_div(c->nP * nrhs, kBlock), kBlock, 0, s>>>(c->nP, nrhs, c->pif.p, c->c1.p, c->pif.p);
    HIPCHK(hipGetLastError());
  }
  {
    const int mg = std::max(c->geo.max_nG, 1);
    with_rhs_group(rhs_group(nrhs, mg), [&](auto kp) {
      constexpr int P = decltype(kp)::value;
      k_recover<T, P><<<dim3(N, ceil_div(nrhs, P)), kBlock, (size_t)mg * P * sizeof(double), s>>>(
          M, c->nP, c->nD, nrhs, c->pi_off.p, c->dl_off.p, c->pi_l2g.p, c->dl_l2g.p, c->qrdesc.p, L.qrA.p, c->offm_d.p,
          c->summ, L.F.p, c->pif.p, c->cg_x.p, N, coef, accumulate);
    });
    HIPCHK(hipGetLastError());
  }
  if (mu_pi_out && c->nP > 0)
    HIPCHK(hipMemcpyAsync(mu_pi_out, c->pif.p, (size_t)nrhs * c->nP * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (mu_dl_out && c->nD > 0)
    HIPCHK(hipMemcpyAsync(mu_dl_out, c->cg_x.p, (size_t)nrhs * c->nD * sizeof(double), hipMemcpyDeviceToDevice, s));
  c->mark(8);
  HIPCHK(hipStreamSynchronize(s));
  auto t3 = std::chrono::steady_clock::now();
  c->phase_ms[4] += c->span(5, 6);
  c->phase_ms[5] += c->span(6, 7);
  c->phase_ms[6] += c->span(7, 8);
  res.ms_rhs = std::chrono::duration<double, std::milli>(t1 - t0).count();
  res.ms_cg = std::chrono::duration<double, std::milli>(t2 - t1).count();
  res.ms_rec = std::chrono::duration<double, std::milli>(t3 - t2).count();
  return res;
}

// sums over rhs of |dx|^2 and |x|^2 after x += dx (host result per rhs)
void axpy_norms(ddelm_ctx c, const double* dx, double* x, int n, int nrhs, std::vector<double>& dn,
                std::vector<double>& xn) {
  dn.assign(nrhs, 0.0);
  xn.assign(nrhs, 0.0);
  if (n <= 0) return;
  const int nblk = std::max(1, std::min(256, ceil_div(n, kBlock)));
  k_axpy_norms<<<dim3(nblk, nrhs), kBlock, 0, c->stream>>>(dx, x, n, nblk, c->nrm_part.p);
  HIPCHK(hipGetLastError());
  std::vector<double> h((size_t)nrhs * nblk * 2);
  HIPCHK(hipMemcpyAsync(h.data(), c->nrm_part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int r = 0; r < nrhs; ++r)
    for (int b = 0; b < nblk; ++b) {
      dn[r] += h[((size_t)r * nblk + b) * 2];
      xn[r] += h[((size_t)r * nblk + b) * 2 + 1];
    }
}

// --------------------------------------------------------------- adjoint of the solve

void alloc_adjoint_workspace(ddelm_ctx c, int nrhs) {
  if (nrhs <= c->adj_cap) return;
  const size_t D = (size_t)nrhs * std::max(c->sumD, 1), P = (size_t)nrhs * std::max(c->sumP, 1);
  const size_t nP = (size_t)nrhs * std::max(c->nP, 1), nD = (size_t)nrhs * std::max(c->nD, 1);
  const size_t C2 = (size_t)nrhs * std::max(2 * c->nP, 1);
  for (DBuf<double>* b : {&c->adj_yP, &c->adj_mloc, &c->adj_eloc}) b->alloc(P);
  for (DBuf<double>* b : {&c->adj_yD, &c->adj_zD, &c->adj_etaD, &c->adj_lbar}) b->alloc(D);
  c->adj_gP.alloc(nP);
  c->adj_nu.alloc(nP);
  c->adj_u.alloc(C2);
  c->adj_c2.alloc(C2);
  c->adj_pbar.alloc((size_t)nrhs * std::max(c->sumP + c->sumD, 1));
  c->adj_fb.alloc((size_t)nrhs * c->summ);
  c->adj_hP.alloc(nP);
  c->adj_hD.alloc(nD);
  for (DBuf<double>* b : {&c->adj_yP, &c->adj_yD, &c->adj_zD, &c->adj_mloc, &c->adj_eloc, &c->adj_etaD,
                          &c->adj_lbar, &c->adj_gP, &c->adj_nu, &c->adj_u, &c->adj_c2, &c->adj_hP, &c->adj_hD})
    b->zero(c->stream);
  if (c->mixed) {
    c->adj_fw.alloc((size_t)nrhs * c->summ);
    c->adj_hwP.alloc(nP);
    c->adj_hwD.alloc(nD);
    c->adj_zc.alloc((size_t)nrhs * c->N * c->M);
    c->adj_zP.alloc(nP);
    c->adj_zDg.alloc(nD);
    c->adj_fbGP.alloc(P);
    c->adj_fbGD.alloc(D);
    for (DBuf<double>* b : {&c->adj_hwP, &c->adj_hwD, &c->adj_zP, &c->adj_zDg, &c->adj_fbGP, &c->adj_fbGD})
      b->zero(c->stream);
  }
  c->adj_cap = nrhs;
}

// One transposed DDELM-NN solve with the factors of type T: from the
// cotangents (cbar [nrhs][N][M], mubP [nrhs][nP], mubD [nrhs][nD]; the last
// two may be null) of (c, mu_Pi, mu_Delta) to those of the local right-hand
// side (fbar [nrhs][sum m], all rows) and of the flux rows (hbP, hbD).
// fbGP / fbGD (optional) receive the interface rows of fbar in slot order.
template <typename T>
CoreOut adjoint_core(ddelm_ctx c, int nrhs, const double* cbar, const double* mubP, const double* mubD, double tol,
                     double* fbar, double* hbP, double* hbD, double* fbGP, double* fbGD) {
  CoreOut res;
  hipStream_t s = c->stream;
  const int N = c->N, M = c->M, nP = c->nP, nD = c->nD;
  const int sumG = c->sumP + c->sumD;
  LocalBufs<T>& L = c->lb<T>();
  OpArgs<T> a = op_args<T>(c, nrhs);
  const size_t sm = local_smem(c);
  const size_t smG = sizeof(double) * (size_t)std::max(c->geo.max_nG, 1);
  const dim3 gl(N, nrhs);
  const dim3 gP(ceil_div(std::max(nP, 1), kBlock), nrhs), gP2(ceil_div(std::max(2 * nP, 1), kBlock), nrhs);
  const dim3 gD(ceil_div(std::max(nD, 1), kBlock), nrhs);
  auto t0 = std::chrono::steady_clock::now();
  c->mark(5);
  // ---- transpose of the recovery c = cf0 + E mu, mu_Pi = mu1 - (X1 u')[:nP]
  k_adj_Et<T><<<gl, kBlock, (size_t)M * sizeof(double), s>>>(M, N, c->pi_off.p, c->dl_off.p, c->qrdesc.p, L.qrA.p,
                                                              cbar, c->sumP, c->sumD, c->adj_yP.p, c->adj_yD.p);
  HIPCHK(hipGetLastError());
  if (nP > 0) {
    k_owner_sum<<<gP, kBlock, 0, s>>>(nP, c->pi_own_ptr.p, c->pi_own_slot.p, c->adj_yP.p, c->sumP, mubP, c->adj_gP.p,
                                      nP, 0);
    k_x1t<<<gP2, kBlock, 0, s>>>(c->X1.p, 2 * nP, 0, nP, c->adj_gP.p, nP, 2 * nP, -1.0, c->adj_u.p, 2 * nP);
    HIPCHK(hipGetLastError());
  }
  if (nD > 0) {
    k_adj_rec<T><<<gl, kBlock, 0, s>>>(a, c->adj_yD.p, c->adj_u.p, c->adj_zD.p);
    k_owner_sum<<<gD, kBlock, 0, s>>>(nD, c->dl_own_ptr.p, c->dl_own_slot.p, c->adj_zD.p, c->sumD, mubD, c->cg_b.p,
                                      nD, 0);
    HIPCHK(hipGetLastError());
  }
  c->mark(6);
  HIPCHK(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  // ---- the transposed interface system: S_theta is symmetric, so the same CG
  if (c->f32cg) interface_solve<float>(c, nrhs, tol, nullptr, res);
  else interface_solve<T>(c, nrhs, tol, nullptr, res);
  c->mark(7);
  auto t2 = std::chrono::steady_clock::now();
  // ---- transpose of the right-hand-side map
  k_adj_A1<T><<<gl, kBlock, sm, s>>>(a, c->cg_x.p, c->adj_mloc.p, c->adj_eloc.p, c->adj_etaD.p);
  HIPCHK(hipGetLastError());
  if (nP > 0) {
    k_owner_sum<<<gP, kBlock, 0, s>>>(nP, c->pi_own_ptr.p, c->pi_own_slot.p, c->adj_mloc.p, c->sumP, nullptr,
                                      c->adj_c2.p, 2 * nP, 0);
    k_owner_sum<<<gP, kBlock, 0, s>>>(nP, c->pi_own_ptr.p, c->pi_own_slot.p, c->adj_eloc.p, c->sumP, nullptr,
                                      c->adj_c2.p, 2 * nP, nP);
    k_x1t<<<gP, kBlock, 0, s>>>(c->X1.p, 2 * nP, 0, 2 * nP, c->adj_c2.p, 2 * nP, nP, 1.0, c->adj_nu.p, nP);
    HIPCHK(hipGetLastError());
  }
  if (nD > 0) {
    k_adj_A2<T><<<gl, kBlock, 0, s>>>(a, c->adj_etaD.p, c->adj_nu.p);
    if (a.theta != 0.0) {
      launch_local_N<T>(c, a, 0, nrhs, s);
      launch_local_N<T>(c, a, 1, nrhs, s);
    }
    k_adj_A3<T><<<gl, kBlock, sm, s>>>(a, c->adj_lbar.p, c->adj_mloc.p);
    k_adj_hD<T><<<gD, kBlock, 0, s>>>(a, hbD);
    HIPCHK(hipGetLastError());
  }
  if (nP > 0) {
    // [mu1_bar; e1_bar] (e1_bar is already in the second half), then u = X1^T [mu1_bar; e1_bar]
    k_owner_sum<<<gP, kBlock, 0, s>>>(nP, c->pi_own_ptr.p, c->pi_own_slot.p, c->adj_mloc.p, c->sumP, c->adj_gP.p,
                                      c->adj_c2.p, 2 * nP, 0);
    k_x1t<<<gP2, kBlock, 0, s>>>(c->X1.p, 2 * nP, 0, 2 * nP, c->adj_c2.p, 2 * nP, 2 * nP, 1.0, c->adj_u.p, 2 * nP);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy2DAsync(hbP, nP * sizeof(double), c->adj_u.p + nP, 2 * nP * sizeof(double), nP * sizeof(double),
                            nrhs, hipMemcpyDeviceToDevice, s));
  }
  // ---- local stage: f_bar_i = Q [R^{-T} cf0_bar + Q_G^T pbar; 0] - pbar on the interface rows
  k_adj_F<T, T><<<gl, kBlock, smG, s>>>(M, N, nP, nD, c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->pi_l2g.p,
                                          c->dl_l2g.p, c->offAm_d.p, L.Am.p, cbar, c->adj_u.p, c->adj_lbar.p,
                                          c->cg_x.p, c->sumD, c->offm_d.p, c->summ, L.F.p, c->adj_pbar.p, sumG);
  HIPCHK(hipGetLastError());
  const int* cnM = c->arena.put(std::vector<int>(N, nrhs), s);
  const int nt = ceil_div(nrhs, kTRSMC);
  k_trsm<T, kTRSMC><<<ceil_div(N, 8) * 8 * nt, kBlock, (size_t)M * kTRSMC * sizeof(T), s>>>(
      c->qrdesc.p, L.qrA.p, L.F.p, c->f_off.p, c->f_ld.p, cnM, 1, N, nt);
  k_adj_alpha<T><<<gl, kBlock, smG, s>>>(M, c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->offQG_d.p, L.QG.p,
                                         c->adj_pbar.p, sumG, c->offm_d.p, c->summ, L.F.p);
  HIPCHK(hipGetLastError());
  apply_q_local<T>(c, nrhs, 0, s);
  k_adj_fout<T><<<gl, kBlock, 0, s>>>(c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->offm_d.p, c->summ, L.F.p,
                                      c->adj_pbar.p, sumG, c->sumP, c->sumD, fbar, fbGP, fbGD);
  HIPCHK(hipGetLastError());
  c->mark(8);
  HIPCHK(hipStreamSynchronize(s));
  auto t3 = std::chrono::steady_clock::now();
  c->phase_ms[4] += c->span(5, 6) + c->span(7, 8);
  c->phase_ms[5] += c->span(6, 7);
  res.ms_rhs = std::chrono::duration<double, std::milli>(t1 - t0).count();
  res.ms_cg = std::chrono::duration<double, std::milli>(t2 - t1).count();
  res.ms_rec = std::chrono::duration<double, std::milli>(t3 - t2).count();
  return res;
}

// Shared body of ddelm_solve_adjoint and ddelm_solve_adjoint_general.
ddelm_status adjoint_any(ddelm_ctx c, int nrhs, const double* cbar, const double* mubP, const double* mubD,
                         double* f_I_bar, double* g_B_bar, double* f_loc_bar, double* h_bar, ddelm_stats* stats) {
  if (!c) return DDELM_E_ARG;
  bool noconv = false;
  ddelm_stats st{};
  ddelm_status code = run_guarded(c, [&]() {
    if (!c->factored) c->fail(DDELM_E_STATE, "adjoint solve called before ddelm_factor");
    if (nrhs < 1 || nrhs > c->opt.max_nrhs) c->fail(DDELM_E_ARG, "nrhs out of range");
    if (!cbar) c->fail(DDELM_E_ARG, "coef_bar is null");
    hipStream_t s = c->stream;
    const int N = c->N, nP = c->nP, nD = c->nD;
    alloc_solve_workspace(c, nrhs);
    alloc_adjoint_workspace(c, nrhs);
    HIPCHK(hipStreamSynchronize(s));
    c->arena.reset();
    c->upload.reset();
    c->phase_ms[4] = c->phase_ms[5] = c->phase_ms[6] = 0.0;
    auto acc = [&](const CoreOut& o) {
      st.iters += o.iters;
      st.rel_res = o.relres;
      st.cg_restarts += o.restarts;
      st.true_rel_res = o.true_rel;
      st.ms_rhs += o.ms_rhs;
      st.ms_cg += o.ms_cg;
      st.ms_recover += o.ms_rec;
      noconv = noconv || o.noconv;
    };
    if (!c->mixed) {
      acc(adjoint_core<double>(c, nrhs, cbar, mubP, mubD, c->opt.tol, c->adj_fb.p, c->adj_hP.p, c->adj_hD.p, nullptr,
                               nullptr));
      noconv = noconv || st.true_rel_res > c->opt.tol;
    } else {
      // float32 transposed solves, refined on the float64 transposed residual:
      // z = (cbar, mubar) - Op^T y, y += adjoint(z).  This removes the part of
      // the float32 error that the transposed residual sees and stalls after
      // one or two steps: the rest lies along the difference between the
      // float32 range of Q_i and the range of K_c^i, which Op^T does not see.
      const long long nc = (long long)nrhs * N * c->M;
      HIPCHK(hipMemcpyAsync(c->adj_zc.p, cbar, nc * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (nP) {
        if (mubP)
          HIPCHK(hipMemcpyAsync(c->adj_zP.p, mubP, (size_t)nrhs * nP * sizeof(double), hipMemcpyDeviceToDevice, s));
        else
          fill(s, c->adj_zP.p, (long long)nrhs * nP, 0.0);
      }
      if (nD) {
        if (mubD)
          HIPCHK(hipMemcpyAsync(c->adj_zDg.p, mubD, (size_t)nrhs * nD * sizeof(double), hipMemcpyDeviceToDevice, s));
        else
          fill(s, c->adj_zDg.p, (long long)nrhs * nD, 0.0);
      }
      fill(s, c->adj_fb.p, (long long)nrhs * c->summ, 0.0);
      if (nP) fill(s, c->adj_hP.p, (long long)nrhs * nP, 0.0);
      if (nD) fill(s, c->adj_hD.p, (long long)nrhs * nD, 0.0);
      size_t shm = 0;
      for (int i = 0; i < N; ++i) shm = std::max(shm, (size_t)(c->h_m[i] + c->h_nG[i]));
      shm *= sizeof(double);
      double prev_worst = 0.0;
      for (int step = 0; step <= c->opt.refine_maxit; ++step) {
        acc(adjoint_core<double>(c, nrhs, c->adj_zc.p, nP ? c->adj_zP.p : nullptr, nD ? c->adj_zDg.p : nullptr,
                                c->opt.inner_tol, c->adj_fw.p, c->adj_hwP.p, c->adj_hwD.p, c->adj_fbGP.p,
                                c->adj_fbGD.p));
        if (step > 0) st.refine_steps += 1;
        std::vector<double> dn, xn, dpn, xpn, ddn, xdn;
        axpy_norms(c, c->adj_fw.p, c->adj_fb.p, (int)c->summ, nrhs, dn, xn);
        axpy_norms(c, c->adj_hwP.p, c->adj_hP.p, nP, nrhs, dpn, xpn);
        axpy_norms(c, c->adj_hwD.p, c->adj_hD.p, nD, nrhs, ddn, xdn);
        double worst = 0.0;
        for (int r = 0; r < nrhs; ++r) {
          const double num = dn[r] + (nP ? dpn[r] : 0.0) + (nD ? ddn[r] : 0.0);
          const double den = xn[r] + (nP ? xpn[r] : 0.0) + (nD ? xdn[r] : 0.0);
          worst = std::max(worst, den > 0 ? std::sqrt(num / den) : std::sqrt(num));
        }
        if (step > 0) st.refine_corr = worst;
        if ((step > 0 && (worst <= c->opt.refine_tol || worst > kRefineStall * prev_worst)) ||
            step == c->opt.refine_maxit)
          break;
        prev_worst = worst;
        k_adj_resid<<<dim3(N, nrhs), kBlock, shm, s>>>(
            c->M, nP, nD, c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->pi_l2g.p, c->dl_l2g.p, c->offK_d.p, c->K64.p,
            c->offAm_d.p, c->l64.Am.p, c->offm_d.p, c->summ, c->adj_fw.p, nP ? c->adj_hwP.p : nullptr,
            nD ? c->adj_hwD.p : nullptr, N, c->adj_zc.p);
        HIPCHK(hipGetLastError());
        if (nP)
          k_owner_sum<<<dim3(ceil_div(nP, kBlock), nrhs), kBlock, 0, s>>>(
              nP, c->pi_own_ptr.p, c->pi_own_slot.p, c->adj_fbGP.p, c->sumP, c->adj_zP.p, c->adj_zP.p, nP, 0);
        if (nD)
          k_owner_sum<<<dim3(ceil_div(nD, kBlock), nrhs), kBlock, 0, s>>>(
              nD, c->dl_own_ptr.p, c->dl_own_slot.p, c->adj_fbGD.p, c->sumD, c->adj_zDg.p, c->adj_zDg.p, nD, 0);
        HIPCHK(hipGetLastError());
      }
    }
    // ---- outputs
    if (f_loc_bar)
      HIPCHK(hipMemcpyAsync(f_loc_bar, c->adj_fb.p, (size_t)nrhs * c->summ * sizeof(double), hipMemcpyDeviceToDevice,
                            s));
    if (h_bar) {
      const int nG = nP + nD;
      if (nP)
        HIPCHK(hipMemcpy2DAsync(h_bar, nG * sizeof(double), c->adj_hP.p, nP * sizeof(double), nP * sizeof(double),
                                nrhs, hipMemcpyDeviceToDevice, s));
      if (nD)
        HIPCHK(hipMemcpy2DAsync(h_bar + nP, nG * sizeof(double), c->adj_hD.p, nD * sizeof(double),
                                nD * sizeof(double), nrhs, hipMemcpyDeviceToDevice, s));
    }
    if (f_I_bar) {
      k_adj_out<<<dim3(N, nrhs), kBlock, 0, s>>>(N, c->n_int, c->sizes_dev.p, c->offm_d.p, c->offB_d.p, c->summ,
                                                 c->geo.sum_nB, c->adj_fb.p, f_I_bar, g_B_bar);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
  });
  st.cg_blocks = c->cg_blocks;
  st.cg_slices = c->cg_slices;
  st.cg_coarse_dist = c->cg_dist;
  st.kappa_est_max = c->kappa_est;
  if (c->mixed) st.true_rel_res = std::nan("");
  if (stats) *stats = st;
  if (code == DDELM_OK && noconv) return DDELM_WARN_NOCONV;
  return code;
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
  o->inner_tol = 1e-3;
}

ddelm_status ddelm_setup(ddelm_ctx* out, const ddelm_problem* prob, const ddelm_options* opt, void* stream) {
  if (!out || !prob) return DDELM_E_ARG;
  *out = nullptr;
  ddelm_ctx c = new ddelm_ctx_s();
  c->stream = (hipStream_t)stream;
  ddelm_status st = run_guarded(c, [&]() {
    if (opt) c->opt = *opt;
    else ddelm_default_options(&c->opt);
    const ddelm_options& o = c->opt;
    if (!(o.theta >= 0.0 && o.theta <= 1.0)) c->fail(DDELM_E_ARG, "theta must lie in [0, 1]");
    if (o.coarse < 0 || o.coarse > 4) c->fail(DDELM_E_ARG, "coarse must be 0, 1, 2, 3 or 4");
    if (o.coarse == 0 && o.theta != 0.0)
      c->fail(DDELM_E_ARG, "theta must be 0 without a coarse space (Kbar needs Dirichlet corner rows)");
    if (o.precision < 0 || o.precision > 2) c->fail(DDELM_E_ARG, "precision must be 0, 1 or 2");
    if (o.precision == 1 && !(o.refine_maxit >= 0 && o.refine_tol > 0.0 && o.inner_tol > 0.0 && o.inner_tol < 1.0))
      c->fail(DDELM_E_ARG, "refinement options out of range");
    c->mixed = o.precision == 1;
    c->f32cg = o.precision >= 1;
    if (!(o.tol > 0.0 && o.tol < 1.0)) c->fail(DDELM_E_ARG, "tol must lie in (0, 1)");
    if (o.maxit < 1) c->fail(DDELM_E_ARG, "maxit must be >= 1");
    if (o.max_nrhs < 1 || o.max_nrhs > 64) c->fail(DDELM_E_ARG, "max_nrhs must lie in [1, 64]");
    if (o.cg_mode < 0 || o.cg_mode > 2) c->fail(DDELM_E_ARG, "cg_mode must be 0, 1 or 2");
    if (prob->M < 1 || prob->M > 1024) c->fail(DDELM_E_SHAPE, "M must lie in [1, 1024]");
    if (!prob->edge_s || !prob->x_int || !prob->W || !prob->b) c->fail(DDELM_E_ARG, "null array in problem");
    if (prob->n_extra < 0 || (prob->n_extra > 0 && !prob->extra_s)) c->fail(DDELM_E_ARG, "bad extra_s");
    HIPCHK(hipGetDevice(&c->device));
    c->blocks->dev = c->device;
    {
      // address of this device's copy of `scratch` (once per device)
      ScratchAddrs& S = scratch_addrs();
      std::lock_guard<std::mutex> lk(S.mu);
      if ((int)S.ptr.size() <= c->device) S.ptr.resize(c->device + 1, nullptr);
      if (!S.ptr[c->device]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        S.ptr[c->device] = ptr;
      }
    }
    HIPCHK(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    const int N = prob->nx * prob->ny;
    if (prob->nx < 1 || prob->ny < 1 || (long long)prob->nx * prob->ny > (1 << 20))
      c->fail(DDELM_E_SHAPE, "nx, ny out of range");
    if (prob->n_int < 1) c->fail(DDELM_E_SHAPE, "n_int must be >= 1");
    c->N = N; c->M = prob->M; c->n_int = prob->n_int;
    std::string e = c->geo.build(prob->nx, prob->ny, prob->lo, prob->hi, prob->p, prob->edge_s, prob->n_extra,
                                 prob->extra_s, prob->n_int, o.coarse);
    if (!e.empty()) c->fail(DDELM_E_SHAPE, e);
    Geometry& g = c->geo;
    c->nP = g.n_pi; c->nD = g.n_dl;
    c->sumP = g.pi_off[N]; c->sumD = g.dl_off[N];
    c->use_nn = o.theta != 0.0 && o.coarse > 0;
    if (g.max_m > kBlock * 12) c->fail(DDELM_E_SHAPE, "local row count above 3072");
    if (g.max_nG > 4096) c->fail(DDELM_E_SHAPE, "too many interface points per subdomain");
    for (int k = 0; k < g.n_dl; ++k)
      if (g.dl_own_ptr[k + 1] - g.dl_own_ptr[k] > kMaxOwn) c->fail(DDELM_E_SHAPE, "Delta point with more than 4 owners");
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
    {
      // pinned staging for the table uploads below (the host does not wait for them)
      size_t need = (size_t)1 << 20;
      for (const RowSet* r : {&g.rowsK, &g.rowsA, &g.rowsKb, &g.rowsAb})
        need += sizeof(int) * (r->row0.size() + 3 * r->ptr.size()) + sizeof(Term) * r->terms.size();
      need += sizeof(double) * 8 * (size_t)N +
              sizeof(int) * (16 * (size_t)N + g.pi_loc2glob.size() + g.dl_loc2glob.size() + g.pi_own_slot.size() +
                             g.dl_own_slot.size() + g.pi_own_ptr.size() + g.dl_own_ptr.size() + (size_t)c->sumP);
      c->upload.ensure(need);
    }
    // problem copies
    c->W.alloc((size_t)N * c->M * 2);
    HIPCHK(hipMemcpyAsync(c->W.p, prob->W, c->W.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    c->b.alloc((size_t)N * c->M);
    HIPCHK(hipMemcpyAsync(c->b.p, prob->b, c->b.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    c->x_int.alloc((size_t)N * prob->n_int * 2);
    HIPCHK(hipMemcpyAsync(c->x_int.p, prob->x_int, c->x_int.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<double> geom(8 * (size_t)N);   // centre and half widths, then the closed boxes
    for (int i = 0; i < N; ++i) {
      geom[4 * i] = g.subs[i].cx; geom[4 * i + 1] = g.subs[i].cy;
      geom[4 * i + 2] = g.subs[i].hx; geom[4 * i + 3] = g.subs[i].hy;
      g.box(i, &geom[4 * ((size_t)N + i)]);
    }
    c->geom.upload(geom, s);
    // interior points inside their subdomains, checked on the device (read back at the end of setup)
    c->chk.alloc(1);
    HIPCHK(hipMemsetAsync(c->chk.p, 0xFF, sizeof(unsigned), s));
    {
      const long long npt = (long long)N * prob->n_int;
      const unsigned nblk = (unsigned)std::min<long long>(ceil_div(npt, (long long)kBlock), 1024);
      k_check_interior<<<nblk, kBlock, 0, s>>>(c->x_int.p, c->geom.p + 4 * (size_t)N, N, prob->n_int, c->chk.p);
      HIPCHK(hipGetLastError());
    }
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
    unsigned first_bad = 0;
    HIPCHK(hipMemcpyAsync(&first_bad, c->chk.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (first_bad != 0xFFFFFFFFu)
      c->fail(DDELM_E_SHAPE, "interior point outside its subdomain (subdomain " + std::to_string(first_bad) + ")");
  });
  if (st != DDELM_OK) {
    // keep the context only to report the error through ddelm_last_error
    *out = c;
    return st;
  }
  *out = c;
  return DDELM_OK;
}

ddelm_status ddelm_set_coefficient(ddelm_ctx c, const double* rho_I, const double* rho_pi, const double* rho_dl) {
  if (!c) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    hipStream_t s = c->stream;
    HIPCHK(hipStreamSynchronize(s));
    c->factored = false;
    if (!rho_I && !rho_pi && !rho_dl) {      // back to rho = 1
      c->has_rho = false;
      return;
    }
    if (!rho_I || !rho_dl || (c->nP > 0 && !rho_pi)) c->fail(DDELM_E_ARG, "null coefficient array");
    const size_t nI = (size_t)c->N * c->n_int * 3, nG = (size_t)c->nP + c->nD;
    // validated on the host: a set-up time copy of a few values per point
    std::vector<double> hI(nI), hG(nG);
    HIPCHK(hipMemcpy(hI.data(), rho_I, nI * sizeof(double), hipMemcpyDeviceToHost));
    if (c->nP > 0) HIPCHK(hipMemcpy(hG.data(), rho_pi, c->nP * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hG.data() + c->nP, rho_dl, c->nD * sizeof(double), hipMemcpyDeviceToHost));
    for (double v : hI)
      if (!std::isfinite(v)) c->fail(DDELM_E_NONFINITE, "non-finite coefficient value");
    for (double v : hG)
      if (!std::isfinite(v)) c->fail(DDELM_E_NONFINITE, "non-finite coefficient value");
    for (size_t k = 0; k < nI; k += 3)
      if (!(hI[k] > 0.0)) c->fail(DDELM_E_ARG, "coefficient rho must be positive at the interior points");
    for (double v : hG)
      if (!(v > 0.0)) c->fail(DDELM_E_ARG, "coefficient rho must be positive at the interface points");
    c->has_rho = false;
    c->rho_int.upload(hI, s);
    c->rho_iface.upload(hG, s);
    HIPCHK(hipStreamSynchronize(s));
    c->has_rho = true;
  });
}

ddelm_status ddelm_factor(ddelm_ctx c) {
  if (!c) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset();
    c->upload.reset();
    c->factored = false;
    factor_impl<double>(c);
    c->factored = true;
  });
}

}  // extern "C"

namespace {

// Shared body of ddelm_solve (f_I, g_B given) and ddelm_solve_general (f_loc, h given).
ddelm_status solve_any(ddelm_ctx c, int nrhs, const double* f_I, const double* g_B, const double* f_loc,
                       const double* h, const double* mu0, double* coef, double* mu_pi, double* mu_dl,
                       ddelm_stats* stats, bool noalloc = false) {
  if (!c) return DDELM_E_ARG;
  bool noconv = false;
  ddelm_stats st{};
  const bool general = f_loc != nullptr;
  ddelm_status code = run_guarded(c, [&]() {
    if (!c->factored) c->fail(DDELM_E_STATE, "solve called before ddelm_factor");
    if (nrhs < 1 || nrhs > c->opt.max_nrhs) c->fail(DDELM_E_ARG, "nrhs out of range");
    if (!coef || (!general && (!f_I || (!g_B && c->geo.sum_nB > 0)))) c->fail(DDELM_E_ARG, "null array");
    hipStream_t s = c->stream;
    const int N = c->N;
    if (!noalloc) alloc_solve_workspace(c, nrhs);
    HIPCHK(hipStreamSynchronize(s));
    c->arena.reset();
    c->upload.reset();
    struct NoAllocScope {
      ddelm_ctx c;
      ~NoAllocScope() { c->noalloc = false; }
    } na_scope{c};
    std::unique_ptr<ScratchBinding> bound;
    if (noalloc) {
      c->noalloc = true;
      bound.reset(new ScratchBinding(c, nrhs));
    }
    c->phase_ms[4] = c->phase_ms[5] = c->phase_ms[6] = 0.0;
    auto acc = [&](const CoreOut& o) {
      st.iters += o.iters;
      st.rel_res = o.relres;
      st.cg_restarts += o.restarts;
      st.ms_rhs += o.ms_rhs;
      st.ms_cg += o.ms_cg;
      st.ms_recover += o.ms_rec;
      noconv = noconv || o.noconv;
    };
    // flux right-hand side of a general solve, split into the Pi and Delta blocks
    const double* h0P = nullptr;
    const double* h0D = nullptr;
    if (general && h) {
      const int nG = c->nP + c->nD;
      if (c->nP) {
        HIPCHK(hipMemcpy2DAsync(c->hP0.p, c->nP * sizeof(double), h, nG * sizeof(double), c->nP * sizeof(double), nrhs,
                                hipMemcpyDeviceToDevice, s));
        h0P = c->hP0.p;
      }
      if (c->nD) {
        HIPCHK(hipMemcpy2DAsync(c->hD0.p, c->nD * sizeof(double), h + c->nP, nG * sizeof(double),
                                c->nD * sizeof(double), nrhs, hipMemcpyDeviceToDevice, s));
        h0D = c->hD0.p;
      }
    }
    const double* f0P = general ? c->fGP0.p : nullptr;
    const double* f0D = general ? c->fGD0.p : nullptr;
    // local right-hand sides (float64; mixed precision keeps a copy for the residuals)
    double* F64 = c->mixed ? c->F64.p : nullptr;
    if (general)
      k_rhs_split<double><<<dim3(N, nrhs), kBlock, 0, s>>>(c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->offm_d.p,
                                                           c->summ, c->sumP, c->sumD, f_loc, c->l64.F.p, F64,
                                                           c->fGP0.p, c->fGD0.p);
    else
      k_rhs_assemble<double><<<dim3(N, nrhs), kBlock, 0, s>>>(N, c->n_int, c->sizes_dev.p, c->offm_d.p, c->offB_d.p,
                                                              c->summ, c->geo.sum_nB, f_I, g_B, c->l64.F.p, F64);
    HIPCHK(hipGetLastError());
    const double* x0 = (mu0 && c->nD > 0) ? mu0 : nullptr;
    if (!c->mixed) {
      const CoreOut o = solve_core<double>(c, nrhs, f0P, f0D, h0P, h0D, c->opt.tol, coef, 0, mu_pi, mu_dl, x0);
      acc(o);
      st.true_rel_res = o.true_rel;
      st.start_rel_res = o.start_rel;
      noconv = noconv || o.true_rel > c->opt.tol;
    } else {
      // The float32-QR solve, refined on the float64 residual of the coupled
      // system [f - K_c c - B mu; h - A_m c] of eq. ddelm: each correction is
      // the same solve applied to that residual.
      DBuf<double>& muP = c->ref_muP;
      DBuf<double>& muD = c->ref_muD;
      const CoreOut o0 = solve_core<double>(c, nrhs, f0P, f0D, h0P, h0D, c->opt.inner_tol, coef, 0, muP.p, muD.p,
                                            x0);
      acc(o0);
      st.start_rel_res = o0.start_rel;
      const int P = rhs_group(nrhs, c->M);   // right-hand sides per residual workgroup
      const size_t shm = (size_t)c->M * P * sizeof(double);
      double prev_worst = 0.0, worst = 0.0;
      for (int step = 0; step < c->opt.refine_maxit; ++step) {
        with_rhs_group(P, [&](auto kp) {
          constexpr int PP = decltype(kp)::value;
          k_residual<PP><<<dim3(N, ceil_div(nrhs, PP)), kBlock, shm, s>>>(
              c->M, c->nP, c->nD, nrhs, c->sizes_dev.p, c->pi_off.p, c->dl_off.p, c->pi_l2g.p, c->dl_l2g.p,
              c->offK_d.p, c->K64.p, c->offAm_d.p, c->l64.Am.p, c->offm_d.p, c->summ, c->F64.p, coef, muP.p, muD.p, N,
              c->sumP, c->sumD, c->l64.F.p, c->fGP.p, c->fGD.p, c->aP.p, c->aD.p);
        });
        HIPCHK(hipGetLastError());
        if (c->nP + c->nD > 0) {
          k_flux_residual<<<dim3(ceil_div(c->nP + c->nD, kBlock), nrhs), kBlock, 0, s>>>(
              c->nP, c->nD, c->sumP, c->sumD, c->pi_own_ptr.p, c->pi_own_slot.p, c->dl_own_ptr.p, c->dl_own_slot.p,
              c->aP.p, c->aD.p, h0P, h0D, c->hPb.p, c->hDb.p);
          HIPCHK(hipGetLastError());
        }
        acc(solve_core<double>(c, nrhs, c->fGP.p, c->fGD.p, c->nP ? c->hPb.p : nullptr, c->nD ? c->hDb.p : nullptr,
                               c->opt.inner_tol, coef, 1, c->dmup.p, c->dmud.p));
        st.refine_steps += 1;
        std::vector<double> dn, xn, dpn, xpn;
        axpy_norms(c, c->dmud.p, muD.p, c->nD, nrhs, dn, xn);
        axpy_norms(c, c->dmup.p, muP.p, c->nP, nrhs, dpn, xpn);
        worst = 0.0;
        for (int r = 0; r < nrhs; ++r) {
          const double num = dn[r] + dpn[r], den = xn[r] + xpn[r];
          worst = std::max(worst, den > 0 ? std::sqrt(num / den) : std::sqrt(num));
        }
        // stop at the tolerance, or when the refinement stalls: the correction
        // shrank by less than kRefineStall, so the iteration sits at its fixed point
        if (worst <= c->opt.refine_tol || (step > 0 && worst > kRefineStall * prev_worst)) break;
        prev_worst = worst;
      }
      st.refine_corr = c->opt.refine_maxit > 0 ? worst : 0.0;
      st.true_rel_res = std::nan("");
      noconv = noconv || (c->opt.refine_maxit > 0 && worst > c->opt.refine_tol);
      if (mu_pi && c->nP > 0)
        HIPCHK(hipMemcpyAsync(mu_pi, muP.p, (size_t)nrhs * c->nP * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (mu_dl && c->nD > 0)
        HIPCHK(hipMemcpyAsync(mu_dl, muD.p, (size_t)nrhs * c->nD * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
  });
  st.cg_blocks = c->cg_blocks;
  st.cg_slices = c->cg_slices;
  st.cg_coarse_dist = c->cg_dist;
  st.kappa_est_max = c->kappa_est;
  if (stats) *stats = st;
  if (code == DDELM_OK && noconv) return DDELM_WARN_NOCONV;
  return code;
}

}  // namespace

extern "C" {

ddelm_status ddelm_solve(ddelm_ctx c, int nrhs, const double* f_I, const double* g_B, const double* mu0,
                         double* coef, double* mu_pi, double* mu_dl, ddelm_stats* stats) {
  if (!f_I) {
    if (c) c->err = "f_I is null";
    return DDELM_E_ARG;
  }
  return solve_any(c, nrhs, f_I, g_B, nullptr, nullptr, mu0, coef, mu_pi, mu_dl, stats);
}

ddelm_status ddelm_solve_noalloc(ddelm_ctx c, int nrhs, const double* f_I, const double* g_B, double* coef,
                                 double* mu_pi, double* mu_dl, ddelm_stats* stats) {
  if (!f_I) {
    if (c) c->err = "f_I is null";
    return DDELM_E_ARG;
  }
  return solve_any(c, nrhs, f_I, g_B, nullptr, nullptr, nullptr, coef, mu_pi, mu_dl, stats, true);
}

ddelm_status ddelm_solve_general(ddelm_ctx c, int nrhs, const double* f_loc, const double* h, double* coef,
                                 double* mu_pi, double* mu_dl, ddelm_stats* stats) {
  if (!f_loc) {
    if (c) c->err = "f_loc is null";
    return DDELM_E_ARG;
  }
  return solve_any(c, nrhs, nullptr, nullptr, f_loc, h, nullptr, coef, mu_pi, mu_dl, stats);
}

// From this many points on, ddelm_evaluate bins them by subdomain and runs on the matrix cores.
constexpr long long kEvalBinMin = 4096;

ddelm_status ddelm_evaluate(ddelm_ctx c, int nrhs, const double* coef, long long npts, const double* x, double* u,
                            double* grad) {
  if (!c) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    if (nrhs < 1 || npts < 0 || !coef || (npts > 0 && (!x || !u))) c->fail(DDELM_E_ARG, "bad evaluate arguments");
    const Geometry& g = c->geo;
    if (npts >= kEvalBinMin) {
      // many points: bin them by subdomain, then tiles of 16 points on f64 MFMA
      hipStream_t s = c->stream;
      const int N = c->N, M = c->M;
      if (npts > INT32_MAX) c->fail(DDELM_E_SHAPE, "too many evaluation points");
      const int ngroups = ceil_div(nrhs, 16);
      DBuf<int> cnt, cursor, perm;
      DBuf<double> coefT;
      cnt.alloc(N);
      cursor.alloc(N);
      perm.alloc((size_t)npts);
      coefT.alloc((size_t)ngroups * N * M * 16);
      ZeroBatch().add(cnt).add(cursor).launch(s);
      const unsigned pb = (unsigned)ceil_div(npts, (long long)kBlock);
      k_bin_count<<<pb, kBlock, 0, s>>>(g.nx, g.ny, g.lo[0], g.lo[1], g.h[0], g.h[1], npts, x, cnt.p);
      HIPCHK(hipGetLastError());
      std::vector<int> hc(N);
      HIPCHK(hipMemcpyAsync(hc.data(), cnt.p, N * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::vector<long long> hoff(N + 1, 0), htoff(N + 1, 0);
      for (int i = 0; i < N; ++i) {
        hoff[i + 1] = hoff[i] + hc[i];
        htoff[i + 1] = htoff[i] + ceil_div((long long)hc[i], 16ll);
      }
      c->arena.reset();
      const long long* doff = c->arena.put(hoff, s);
      const long long* dtoff = c->arena.put(htoff, s);
      k_bin_scatter<<<pb, kBlock, 0, s>>>(g.nx, g.ny, g.lo[0], g.lo[1], g.h[0], g.h[1], npts, x, doff, cursor.p,
                                          perm.p);
      HIPCHK(hipGetLastError());
      k_coef_transpose<<<(unsigned)std::min<long long>(ceil_div((long long)coefT.n, (long long)kBlock), 8192), kBlock, 0, s>>>(
          N, M, nrhs, ngroups, coef, coefT.p);
      HIPCHK(hipGetLastError());
      const long long ntiles = htoff[N];
      const dim3 grid((unsigned)ceil_div(ntiles, (long long)kWaves), (unsigned)ngroups);
      if (grad)
        k_evaluate_mfma<true><<<grid, kBlock, 0, s>>>(g.nx, M, N, g.lo[0], g.lo[1], g.h[0], g.h[1], c->W.p, c->b.p,
                                                      coefT.p, doff, dtoff, ntiles, perm.p, npts, x, u, grad, nrhs);
      else
        k_evaluate_mfma<false><<<grid, kBlock, 0, s>>>(g.nx, M, N, g.lo[0], g.lo[1], g.h[0], g.h[1], c->W.p, c->b.p,
                                                       coefT.p, doff, dtoff, ntiles, perm.p, npts, x, u, grad, nrhs);
      HIPCHK(hipGetLastError());
    } else if (npts > 0) {
      // right-hand sides per thread: all of them up to 16 (one tanh per point and neuron), else groups of 16
      auto launch = [&](auto nrb, auto with_grad) {
        constexpr int NRB = decltype(nrb)::value;
        constexpr bool GRAD = decltype(with_grad)::value;
        k_evaluate<NRB, GRAD><<<dim3(ceil_div(npts, kBlock), ceil_div(nrhs, NRB)), kBlock, 0, c->stream>>>(
            g.nx, g.ny, c->M, c->N, g.lo[0], g.lo[1], g.h[0], g.h[1], c->W.p, c->b.p, coef, npts, x, u, grad, nrhs);
      };
      using One = std::integral_constant<int, 1>;
      using Eight = std::integral_constant<int, 8>;
      using Sixteen = std::integral_constant<int, 16>;
      using Yes = std::true_type;
      using No = std::false_type;
      if (nrhs == 1) grad ? launch(One(), Yes()) : launch(One(), No());
      else if (nrhs <= 8) grad ? launch(Eight(), Yes()) : launch(Eight(), No());
      else grad ? launch(Sixteen(), Yes()) : launch(Sixteen(), No());
      HIPCHK(hipGetLastError());
    }
  });
}

ddelm_status ddelm_solve_adjoint(ddelm_ctx c, int nrhs, const double* coef_bar, double* f_I_bar, double* g_B_bar,
                                 ddelm_stats* stats) {
  if (!f_I_bar) {
    if (c) c->err = "f_I_bar is null";
    return DDELM_E_ARG;
  }
  return adjoint_any(c, nrhs, coef_bar, nullptr, nullptr, f_I_bar, g_B_bar, nullptr, nullptr, stats);
}

ddelm_status ddelm_solve_adjoint_general(ddelm_ctx c, int nrhs, const double* coef_bar, const double* mu_pi_bar,
                                         const double* mu_dl_bar, double* f_loc_bar, double* h_bar,
                                         ddelm_stats* stats) {
  if (!f_loc_bar) {
    if (c) c->err = "f_loc_bar is null";
    return DDELM_E_ARG;
  }
  return adjoint_any(c, nrhs, coef_bar, mu_pi_bar, mu_dl_bar, nullptr, nullptr, f_loc_bar, h_bar, stats);
}

ddelm_status ddelm_evaluate_adjoint(ddelm_ctx c, int nrhs, long long npts, const double* x, const double* u_bar,
                                    const double* grad_bar, double* coef_bar) {
  if (!c) return DDELM_E_ARG;
  return run_guarded(c, [&]() {
    if (c->N == 0) c->fail(DDELM_E_STATE, "setup did not complete");
    if (nrhs < 1 || nrhs > 65535 || npts < 0 || !coef_bar || (npts > 0 && (!x || !u_bar)))
      c->fail(DDELM_E_ARG, "bad evaluate_adjoint arguments");
    const Geometry& g = c->geo;
    k_eval_adj<<<dim3(c->N, ceil_div(c->M, kBlock), nrhs), kBlock, 0, c->stream>>>(
        g.nx, g.ny, c->M, c->N, g.lo[0], g.lo[1], g.h[0], g.h[1], c->W.p, c->b.p, npts, x, u_bar, grad_bar, coef_bar);
    HIPCHK(hipGetLastError());
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

}  // extern "C"

namespace {
template <typename T>
void local_matrix_factored(ddelm_ctx c, int which, int sub, int R, int C, double* out) {
  LocalBufs<T>& L = c->lb<T>();
  if (which == 4) {
    const QRDesc& d = c->h_qrdesc[sub];
    copy_batch<T, double>(c, {CopyDesc{d.off, 0, d.ld, C, R, C, 1, 0}}, L.qrA.p, out);
    return;
  }
  const T* src = nullptr;
  long long soff = 0;
  if (which == 5) { src = L.Gm.p; soff = c->h_offG[sub]; }
  if (which == 6) { src = L.Lm.p; soff = c->h_offG[sub]; }
  if (which == 7) {
    if (!c->use_nn) c->fail(DDELM_E_STATE, "no Neumann-Neumann operator with theta = 0");
    src = L.Nm.p; soff = c->h_offN[sub];
  }
  copy_batch<T, double>(c, {CopyDesc{soff, 0, R, C, R, C, 1, 0}}, src, out);
}
}  // namespace

extern "C" {

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
    c->upload.reset();
    if (which <= 3) {
      DBuf<double> tmp;
      tmp.alloc((size_t)R * C);
      tmp.zero(s);
      const RowSetDev& rs = which == 0 ? c->rsK : which == 1 ? c->rsA : which == 2 ? c->rsKb : c->rsAb;
      std::vector<long long> o(c->N, 0);
      std::vector<int> l(c->N, R);
      assemble_features<double>(c, rs, R, tmp.p, o, l, sub, 1);
      copy_batch<double, double>(c, {CopyDesc{0, 0, R, C, R, C, 1, 0}}, tmp.p, out);
      HIPCHK(hipStreamSynchronize(s));
      return;
    }
    if (!c->factored) c->fail(DDELM_E_STATE, "matrix needs ddelm_factor");
    if (which == 8) {
      copy_batch<double, double>(c, {CopyDesc{0, 0, R, C, R, C, 1, 0}}, c->Spi.p, out);
    } else {
      local_matrix_factored<double>(c, which, sub, R, C, out);
    }
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
  CtxBlocks* blocks = c->blocks;
  {
    BlocksScope scope(blocks);     // the buffers' destructors put their memory on this list
    delete c;                      // (drains the side stream first)
  }
  Resources& R = res();
  std::lock_guard<std::mutex> lk(R.mu);
  BlockList& l = R.dev_list(blocks->dev);
  for (auto& kv : blocks->list.free) l.put(kv.second, kv.first);
  delete blocks;
}

ddelm_status ddelm_release_cached_memory(void) {
  Resources& R = res();
  std::lock_guard<std::mutex> lk(R.mu);
  ddelm_status st = DDELM_OK;
  release_idle_memory_locked(R);
  for (auto& e : R.events_t) (void)hipEventDestroy(e.second);
  for (auto& e : R.events_n) (void)hipEventDestroy(e.second);
  for (auto& x : R.streams) (void)hipStreamDestroy(x.second);
  for (auto& a : R.staging) {
    (void)hipFree(a.d);
    (void)hipHostFree(a.h);
  }
  R.events_t.clear();
  R.events_n.clear();
  R.streams.clear();
  R.staging.clear();
  return st;
}

}  // extern "C"
