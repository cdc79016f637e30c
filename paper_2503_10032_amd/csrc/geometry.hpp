// Host-side interface indexing for a uniform 2-D partition.
//
// Builds, for every subdomain, the collocation rows of the local matrices
// as lists of "terms" (point, normal, weight, operator), the split of the
// interface into Pi (subdomain corners inside the domain) and Delta, the
// global numbering of both, and the owner lists used by the gather/sum
// kernels.  Integer lattice keys decide which points are shared, so the
// split is exact.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ddelm {

enum TermOp : int { OP_VALUE = 0, OP_NEG_LAPLACE = 1, OP_FLUX = 2 };

struct Term {          // one contribution  wgt * op(phi)(x)  to a matrix row
  double x, y;         // global coordinates
  double nx, ny;       // normal (used by OP_FLUX)
  double wgt;
  int op;
  int iface;           // OP_FLUX: global interface index of the point (the #Pi
                       // points first, then #Delta), where a coefficient
                       // rho of the flux rho dphi/dn is looked up; else 0
};

struct SubInfo {
  int ix, iy;
  double cx, cy;       // centre
  double hx, hy;       // half widths
  int n_I, n_B, n_P, n_D;
  int m() const { return n_I + n_B + n_P + n_D; }
  int n_G() const { return n_P + n_D; }
  std::vector<double> xB;       // [n_B][2]
  std::vector<int> pi_glob;     // [n_P] sorted
  std::vector<int> dl_glob;     // [n_D] sorted
  std::vector<double> xG;       // [n_G][2] (Pi block then Delta block)
};

// Row descriptors of one family of local matrices, all subdomains
// concatenated.  The first `lead` rows of every subdomain are its interior
// collocation rows, -Laplace(phi) at the given interior points, which are not
// stored as terms; row lead + r of subdomain i has terms
// [ptr[row0_i + r], ptr[row0_i + r + 1]).
struct RowSet {
  int lead = 0;                 // implicit interior rows per subdomain
  std::vector<int> row0;        // [N+1] first stored row of each subdomain
  std::vector<int> ptr;         // [stored rows+1]
  std::vector<Term> terms;
  void begin_sub() { row0.push_back((int)ptr.size() - 1); }
  void add_row(std::initializer_list<Term> ts) {
    for (const Term& t : ts) terms.push_back(t);
    ptr.push_back((int)terms.size());
  }
  void add_row(const std::vector<Term>& ts) {
    for (const Term& t : ts) terms.push_back(t);
    ptr.push_back((int)terms.size());
  }
};

struct Geometry {
  int threads = 0;     // host threads for the row sets (0: up to 8, by problem size)
  int nx = 0, ny = 0, N = 0, p = 0, coarse = 2;
  double lo[2], hi[2], h[2];
  int n_pi = 0, n_dl = 0, n_edges = 0;
  std::vector<double> s, s_extra;
  std::vector<SubInfo> subs;
  // row sets: K (K_c or K), A (A_m or A) rows at local Gamma, Kbar, Abar
  RowSet rowsK, rowsA, rowsKb, rowsAb;
  // owner lists (CSR over global points; entries = local slot index into
  // the concatenated per-subdomain Pi / Delta slot arrays, by subdomain order)
  std::vector<int> pi_own_ptr, pi_own_slot;   // [n_pi+1], [sum n_P]
  std::vector<int> dl_own_ptr, dl_own_slot;   // [n_dl+1], [sum n_D]
  std::vector<int> pi_off, dl_off;            // [N+1] slot offsets per subdomain
  std::vector<int> pi_loc2glob, dl_loc2glob;  // [sum n_P], [sum n_D]
  std::vector<double> x_pi, x_dl;             // [n_pi][2], [n_dl][2]
  int max_m = 0, max_nG = 0, max_nD = 0, max_nP = 0;
  long long sum_nB = 0;

  // Returns an empty string on success, else an error message.
  std::string build(int nx, int ny, const double* lo, const double* hi, int p, const double* edge_s,
                    int n_extra, const double* extra_s, int n_int, int coarse);
  // closed box [x0, x1] x [y0, y1] of subdomain i (the lattice lines, as the rows use them)
  void box(int i, double* b) const {
    const int ix = i % nx, iy = i / nx;
    b[0] = lo[0] + ix * h[0]; b[1] = lo[0] + (ix + 1) * h[0];
    b[2] = lo[1] + iy * h[1]; b[3] = lo[1] + (iy + 1) * h[1];
  }
};

}  // namespace ddelm
