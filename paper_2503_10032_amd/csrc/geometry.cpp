// Host-side interface indexing for a uniform 2-D partition (see geometry.hpp).
//
// Layout rules (paper sec. 2.2.1 for the point sets, sec. 3 for the Pi/Delta
// split, sec. 3.2 for the change of variables and the mean-flux rows):
//  * every side of a subdomain carries p points at parameters s_k; the ends
//    of a side are subdomain corners (lattice vertices);
//  * points on the domain boundary are boundary points, with g rows;
//  * corners inside the domain are Pi; all other interface points are Delta;
//  * K_c Delta row at parameter s on a side with ends a (s=0), b (s=1):
//      phi(x) - (1-s) phi(x_a) [a in Pi] - s phi(x_b) [b in Pi]
//    i.e. the rows of (T^i)^{-1} C phi, T^i built from linear hats;
//  * A_m corner row: for each interface side through the corner, the mean
//    outward flux over the side's points except its far end.
#include "geometry.hpp"

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdint>
#include <set>
#include <thread>
#include <tuple>

namespace ddelm {

namespace {

enum Side { BOTTOM = 0, RIGHT = 1, TOP = 2, LEFT = 3 };
const double kNormal[4][2] = {{0.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}, {-1.0, 0.0}};

struct SideDesc {
  bool on_boundary;
  int v0x, v0y, v1x, v1y;   // lattice ends at s = 0 and s = 1
  int edge;                 // global interior edge index, -1 on the boundary
};

}  // namespace

std::string Geometry::build(int nx_, int ny_, const double* lo_, const double* hi_, int p_,
                            const double* edge_s, int n_extra, const double* extra_s, int n_int, int coarse_) {
  nx = nx_; ny = ny_; N = nx * ny; p = p_; coarse = coarse_;
  if (nx < 1 || ny < 1) return "nx, ny must be >= 1";
  if ((long long)nx * ny > (1 << 20)) return "too many subdomains";
  if (p < 3 || p > 4096) return "p must be in [3, 4096]";
  if (n_int < 1) return "n_int must be >= 1";
  if (coarse < 0 || coarse > 4) return "coarse must be 0, 1, 2, 3 or 4";
  for (int a = 0; a < 2; ++a) {
    if (!(lo_[a] < hi_[a])) return "lo must be < hi";
    lo[a] = lo_[a]; hi[a] = hi_[a];
  }
  h[0] = (hi[0] - lo[0]) / nx;
  h[1] = (hi[1] - lo[1]) / ny;
  s.assign(edge_s, edge_s + p);
  if (s[0] != 0.0 || s[p - 1] != 1.0) return "edge_s must start at 0 and end at 1";
  for (int k = 1; k < p; ++k)
    if (!(s[k] > s[k - 1])) return "edge_s must be strictly increasing";
  s_extra.assign(extra_s, extra_s + n_extra);
  for (double e : s_extra)
    if (!(e > 0.0 && e < 1.0)) return "extra_s entries must lie in (0,1)";

  const int n_vedges = (nx - 1) * ny, n_hedges = (ny - 1) * nx;
  n_edges = n_vedges + n_hedges;
  const int n_cross = (nx - 1) * (ny - 1);
  n_pi = coarse > 0 ? n_cross : 0;
  n_dl = n_edges * (p - 2) + (coarse == 0 ? n_cross : 0);

  auto vx = [&](int jx) { return lo[0] + jx * h[0]; };
  auto vy = [&](int jy) { return lo[1] + jy * h[1]; };
  auto on_bnd = [&](int jx, int jy) { return jx == 0 || jx == nx || jy == 0 || jy == ny; };
  auto cross = [&](int jx, int jy) { return (jy - 1) * (nx - 1) + (jx - 1); };

  auto side_desc = [&](int ix, int iy, int sd) {
    SideDesc d;
    switch (sd) {
      case BOTTOM:
        d.on_boundary = iy == 0; d.v0x = ix; d.v0y = iy; d.v1x = ix + 1; d.v1y = iy;
        d.edge = d.on_boundary ? -1 : n_vedges + (iy - 1) * nx + ix;
        break;
      case TOP:
        d.on_boundary = iy + 1 == ny; d.v0x = ix; d.v0y = iy + 1; d.v1x = ix + 1; d.v1y = iy + 1;
        d.edge = d.on_boundary ? -1 : n_vedges + iy * nx + ix;
        break;
      case LEFT:
        d.on_boundary = ix == 0; d.v0x = ix; d.v0y = iy; d.v1x = ix; d.v1y = iy + 1;
        d.edge = d.on_boundary ? -1 : iy * (nx - 1) + (ix - 1);
        break;
      default:  // RIGHT
        d.on_boundary = ix + 1 == nx; d.v0x = ix + 1; d.v0y = iy; d.v1x = ix + 1; d.v1y = iy + 1;
        d.edge = d.on_boundary ? -1 : iy * (nx - 1) + ix;
        break;
    }
    return d;
  };
  // coordinates of the point at parameter t on side sd of subdomain (ix, iy)
  auto side_point = [&](int ix, int iy, int sd, double t, double* out) {
    switch (sd) {
      case BOTTOM: out[0] = lo[0] + (ix + t) * h[0]; out[1] = lo[1] + iy * h[1]; break;
      case TOP:    out[0] = lo[0] + (ix + t) * h[0]; out[1] = lo[1] + (iy + 1) * h[1]; break;
      case LEFT:   out[0] = lo[0] + ix * h[0];       out[1] = lo[1] + (iy + t) * h[1]; break;
      default:     out[0] = lo[0] + (ix + 1) * h[0]; out[1] = lo[1] + (iy + t) * h[1]; break;
    }
  };

  subs.assign(N, SubInfo());
  rowsK = RowSet(); rowsA = RowSet(); rowsKb = RowSet(); rowsAb = RowSet();
  rowsK.lead = rowsKb.lead = n_int;   // interior rows come straight from x_int

  // Rows of subdomains [i0, i1) appended to rs[0..3] (K, A, Kbar, Abar).  A
  // subdomain's rows depend only on its own position, so ranges of
  // subdomains are built independently and concatenated in order.
  auto build_range = [&](int i0, int i1, RowSet* rs) {
    RowSet& rK = rs[0];
    RowSet& rA = rs[1];
    RowSet& rKb = rs[2];
    RowSet& rAb = rs[3];
    {
      const size_t side_rows = (size_t)(i1 - i0) * (4 * (size_t)p + 4 * s_extra.size() + 8);
      for (int k = 0; k < 4; ++k) {
        rs[k].ptr.reserve(side_rows + 1);
        rs[k].row0.reserve(i1 - i0 + 1);
        rs[k].terms.reserve(2 * side_rows);
      }
      rA.terms.reserve(side_rows + (size_t)(i1 - i0) * 8 * p);
    }
    for (int k = 0; k < 4; ++k) rs[k].ptr.push_back(0);
    std::vector<Term> ft, ct;   // terms of one corner flux row / one continuity row
    ft.reserve(8 * (size_t)p);
    ct.reserve(3);
    for (int i = i0; i < i1; ++i) {
      const int ix = i % nx, iy = i / nx;
      SubInfo& sb = subs[i];
      sb.ix = ix; sb.iy = iy;
      sb.cx = lo[0] + (ix + 0.5) * h[0];
      sb.cy = lo[1] + (iy + 0.5) * h[1];
      sb.hx = 0.5 * h[0];
      sb.hy = 0.5 * h[1];
      sb.n_I = n_int;
      SideDesc sds[4];
      for (int sd = 0; sd < 4; ++sd) sds[sd] = side_desc(ix, iy, sd);
      // ---- boundary points
      std::set<std::tuple<int, int, int>> seen;   // (kind, a, b): kind 0 vertex (jx,jy), 1 side point
      sb.xB.clear();
      for (int sd = 0; sd < 4; ++sd) {
        if (!sds[sd].on_boundary) continue;
        for (int k = 0; k < p; ++k) {
          std::tuple<int, int, int> key;
          if (k == 0) key = {0, sds[sd].v0x, sds[sd].v0y};
          else if (k == p - 1) key = {0, sds[sd].v1x, sds[sd].v1y};
          else key = {1, sd, k};
          if (!seen.insert(key).second) continue;
          double xy[2];
          side_point(ix, iy, sd, s[k], xy);
          sb.xB.push_back(xy[0]); sb.xB.push_back(xy[1]);
        }
      }
      for (int sd = 0; sd < 4; ++sd) {
        if (!sds[sd].on_boundary) continue;
        for (double t : s_extra) {
          double xy[2];
          side_point(ix, iy, sd, t, xy);
          sb.xB.push_back(xy[0]); sb.xB.push_back(xy[1]);
        }
      }
      sb.n_B = (int)sb.xB.size() / 2;
      // ---- interface points: (global index, x, y, kind, side, k, vertex)
      struct GP { int g; double x, y; int side; int k; int vjx, vjy; };
      std::vector<GP> pis, dls;
      const int corners[4][2] = {{ix, iy}, {ix + 1, iy}, {ix, iy + 1}, {ix + 1, iy + 1}};
      for (auto& c : corners) {
        if (on_bnd(c[0], c[1])) continue;
        GP gp{0, vx(c[0]), vy(c[1]), -1, -1, c[0], c[1]};
        if (coarse > 0) { gp.g = cross(c[0], c[1]); pis.push_back(gp); }
        else { gp.g = n_edges * (p - 2) + cross(c[0], c[1]); dls.push_back(gp); }
      }
      for (int sd = 0; sd < 4; ++sd) {
        if (sds[sd].on_boundary) continue;
        for (int k = 1; k <= p - 2; ++k) {
          double xy[2];
          side_point(ix, iy, sd, s[k], xy);
          dls.push_back(GP{sds[sd].edge * (p - 2) + (k - 1), xy[0], xy[1], sd, k, -1, -1});
        }
      }
      auto byg = [](const GP& a, const GP& b) { return a.g < b.g; };
      std::sort(pis.begin(), pis.end(), byg);
      std::sort(dls.begin(), dls.end(), byg);
      sb.n_P = (int)pis.size();
      sb.n_D = (int)dls.size();
      sb.pi_glob.clear(); sb.dl_glob.clear(); sb.xG.clear();
      for (auto& g : pis) { sb.pi_glob.push_back(g.g); sb.xG.push_back(g.x); sb.xG.push_back(g.y); }
      for (auto& g : dls) { sb.dl_glob.push_back(g.g); sb.xG.push_back(g.x); sb.xG.push_back(g.y); }
      auto is_pi = [&](int jx, int jy) { return coarse > 0 && !on_bnd(jx, jy); };
      // normal of a vertex row: sum over this subdomain's interface sides through it
      auto vertex_normal = [&](int jx, int jy, double* n) {
        n[0] = n[1] = 0.0;
        for (int sd = 0; sd < 4; ++sd) {
          if (sds[sd].on_boundary) continue;
          bool inc = (sds[sd].v0x == jx && sds[sd].v0y == jy) || (sds[sd].v1x == jx && sds[sd].v1y == jy);
          if (inc) { n[0] += kNormal[sd][0]; n[1] += kNormal[sd][1]; }
        }
      };
      // ---- rows
      for (int k = 0; k < 4; ++k) rs[k].begin_sub();
      for (int k = 0; k < sb.n_B; ++k) {
        Term t{sb.xB[2 * k], sb.xB[2 * k + 1], 0, 0, 1.0, OP_VALUE, 0};
        rK.add_row({t});
        rKb.add_row({t});
      }
      for (auto& g : pis) {
        Term t{g.x, g.y, 0, 0, 1.0, OP_VALUE, 0};
        rK.add_row({t});
        rKb.add_row({t});
        // flux row at a corner
        ft.clear();
        if (coarse == 2 || coarse == 4) {      // mean-flux corner rows (A_m)
          for (int sd = 0; sd < 4; ++sd) {
            if (sds[sd].on_boundary) continue;
            const bool at0 = sds[sd].v0x == g.vjx && sds[sd].v0y == g.vjy;
            const bool at1 = sds[sd].v1x == g.vjx && sds[sd].v1y == g.vjy;
            if (!at0 && !at1) continue;
            const int k0 = at0 ? 0 : 1, k1 = at0 ? p - 2 : p - 1;   // far end excluded
            for (int k = k0; k <= k1; ++k) {
              double xy[2];
              side_point(ix, iy, sd, s[k], xy);
              // the corner itself (k = 0 or p - 1) is a Pi point, the rest Delta points of the edge
              const int gi = (k == 0 || k == p - 1) ? g.g : n_pi + sds[sd].edge * (p - 2) + (k - 1);
              ft.push_back(Term{xy[0], xy[1], kNormal[sd][0], kNormal[sd][1], 1.0 / (p - 1), OP_FLUX, gi});
            }
          }
        } else {
          double n[2];
          vertex_normal(g.vjx, g.vjy, n);
          ft.push_back(Term{g.x, g.y, n[0], n[1], 1.0, OP_FLUX, g.g});
        }
        rA.add_row(ft);
      }
      for (auto& g : dls) {
        double n[2];
        if (g.side >= 0) { n[0] = kNormal[g.side][0]; n[1] = kNormal[g.side][1]; }
        else vertex_normal(g.vjx, g.vjy, n);
        // continuity row
        ct.assign(1, Term{g.x, g.y, 0, 0, 1.0, OP_VALUE, 0});
        if ((coarse == 2 || coarse == 3) && g.side >= 0) {   // change of variables (K_c)
          const SideDesc& d = sds[g.side];
          const double sk = s[g.k];
          if (is_pi(d.v0x, d.v0y)) ct.push_back(Term{vx(d.v0x), vy(d.v0y), 0, 0, -(1.0 - sk), OP_VALUE, 0});
          if (is_pi(d.v1x, d.v1y)) ct.push_back(Term{vx(d.v1x), vy(d.v1y), 0, 0, -sk, OP_VALUE, 0});
        }
        rK.add_row(ct);
        rA.add_row({Term{g.x, g.y, n[0], n[1], 1.0, OP_FLUX, n_pi + g.g}});
        rKb.add_row({Term{g.x, g.y, n[0], n[1], 1.0, OP_FLUX, n_pi + g.g}});
        rAb.add_row({Term{g.x, g.y, 0, 0, 1.0, OP_VALUE, 0}});
      }
    }
  };
  RowSet* fin[4] = {&rowsK, &rowsA, &rowsKb, &rowsAb};
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nthr = threads > 0 ? std::min(threads, N)
                               : (int)std::min<long long>(std::min(8u, hw), std::max(1, N / 64));
  if (nthr <= 1) {
    RowSet part[4];
    build_range(0, N, part);
    for (int k = 0; k < 4; ++k) {
      fin[k]->row0 = std::move(part[k].row0);
      fin[k]->ptr = std::move(part[k].ptr);
      fin[k]->terms = std::move(part[k].terms);
    }
  } else {
    std::vector<RowSet> part((size_t)4 * nthr);
    std::vector<int> first(nthr + 1);
    for (int t = 0; t <= nthr; ++t) first[t] = (int)((long long)N * t / nthr);
    std::vector<char> failed(nthr, 0);
    {
      std::vector<std::thread> th;
      for (int t = 0; t < nthr; ++t)
        th.emplace_back([&, t]() {
          try {
            build_range(first[t], first[t + 1], &part[(size_t)4 * t]);
          } catch (...) {
            failed[t] = 1;
          }
        });
      for (auto& x : th) x.join();
    }
    for (int t = 0; t < nthr; ++t)
      if (failed[t]) return "out of host memory building the row sets";
    // concatenate: ranges in order, row indices and term offsets shifted
    std::vector<long long> roff((size_t)4 * (nthr + 1), 0), toff((size_t)4 * (nthr + 1), 0);
    for (int k = 0; k < 4; ++k)
      for (int t = 0; t < nthr; ++t) {
        const RowSet& r = part[(size_t)4 * t + k];
        roff[(size_t)4 * (t + 1) + k] = roff[(size_t)4 * t + k] + (long long)r.ptr.size() - 1;
        toff[(size_t)4 * (t + 1) + k] = toff[(size_t)4 * t + k] + (long long)r.terms.size();
      }
    for (int k = 0; k < 4; ++k) {
      if (toff[(size_t)4 * nthr + k] > INT32_MAX) return "row sets too large";
      fin[k]->ptr.assign((size_t)roff[(size_t)4 * nthr + k] + 1, 0);
      fin[k]->terms.resize((size_t)toff[(size_t)4 * nthr + k]);
      fin[k]->row0.assign(N, 0);
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nthr; ++t)
      th.emplace_back([&, t]() {
        for (int k = 0; k < 4; ++k) {
          const RowSet& r = part[(size_t)4 * t + k];
          const int ro = (int)roff[(size_t)4 * t + k], to = (int)toff[(size_t)4 * t + k];
          std::copy(r.terms.begin(), r.terms.end(), fin[k]->terms.begin() + to);
          for (size_t j = 1; j < r.ptr.size(); ++j) fin[k]->ptr[ro + j] = r.ptr[j] + to;
          for (size_t q = 0; q < r.row0.size(); ++q) fin[k]->row0[first[t] + q] = r.row0[q] + ro;
        }
      });
    for (auto& x : th) x.join();
  }
  for (RowSet* r : fin) r->row0.push_back((int)r->ptr.size() - 1);

  // ---- slot offsets, owner lists, global coordinates
  pi_off.assign(N + 1, 0);
  dl_off.assign(N + 1, 0);
  max_m = max_nG = max_nD = max_nP = 0;
  sum_nB = 0;
  for (int i = 0; i < N; ++i) {
    pi_off[i + 1] = pi_off[i] + subs[i].n_P;
    dl_off[i + 1] = dl_off[i] + subs[i].n_D;
    max_m = std::max(max_m, subs[i].m());
    max_nG = std::max(max_nG, subs[i].n_G());
    max_nD = std::max(max_nD, subs[i].n_D);
    max_nP = std::max(max_nP, subs[i].n_P);
    sum_nB += subs[i].n_B;
  }
  pi_loc2glob.assign(pi_off[N], 0);
  dl_loc2glob.assign(dl_off[N], 0);
  // owner lists in CSR form by counting: slots of a point in subdomain order
  pi_own_ptr.assign(n_pi + 1, 0);
  dl_own_ptr.assign(n_dl + 1, 0);
  x_pi.assign(2 * (size_t)n_pi, 0.0);
  x_dl.assign(2 * (size_t)n_dl, 0.0);
  for (int i = 0; i < N; ++i) {
    const SubInfo& sb = subs[i];
    for (int a = 0; a < sb.n_P; ++a) {
      const int g = sb.pi_glob[a];
      pi_loc2glob[pi_off[i] + a] = g;
      if (pi_own_ptr[g + 1]++ == 0) { x_pi[2 * g] = sb.xG[2 * a]; x_pi[2 * g + 1] = sb.xG[2 * a + 1]; }
    }
    for (int a = 0; a < sb.n_D; ++a) {
      const int g = sb.dl_glob[a];
      dl_loc2glob[dl_off[i] + a] = g;
      if (dl_own_ptr[g + 1]++ == 0) {
        x_dl[2 * g] = sb.xG[2 * (sb.n_P + a)];
        x_dl[2 * g + 1] = sb.xG[2 * (sb.n_P + a) + 1];
      }
    }
  }
  for (int g = 0; g < n_pi; ++g) {
    if (pi_own_ptr[g + 1] == 0) return "internal: Pi point without owner";
    pi_own_ptr[g + 1] += pi_own_ptr[g];
  }
  for (int g = 0; g < n_dl; ++g) {
    if (dl_own_ptr[g + 1] < 2) return "internal: Delta point with fewer than two owners";
    dl_own_ptr[g + 1] += dl_own_ptr[g];
  }
  pi_own_slot.assign(pi_own_ptr[n_pi], 0);
  dl_own_slot.assign(dl_own_ptr[n_dl], 0);
  std::vector<int> pcur(pi_own_ptr.begin(), pi_own_ptr.end() - 1), dcur(dl_own_ptr.begin(), dl_own_ptr.end() - 1);
  for (int i = 0; i < N; ++i) {
    const SubInfo& sb = subs[i];
    for (int a = 0; a < sb.n_P; ++a) pi_own_slot[pcur[sb.pi_glob[a]]++] = pi_off[i] + a;
    for (int a = 0; a < sb.n_D; ++a) dl_own_slot[dcur[sb.dl_glob[a]]++] = dl_off[i] + a;
  }
  return "";
}

}  // namespace ddelm
