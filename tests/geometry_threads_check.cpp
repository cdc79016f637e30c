// Host check: the row sets and owner tables of Geometry::build are the same
// whether they are built by one thread or by several (ranges of subdomains
// built independently and concatenated).  Exit status 0 when all agree.
#include "geometry.hpp"

#include <cstdio>
#include <cstring>
#include <vector>

namespace {
bool same_rows(const ddelm::RowSet& a, const ddelm::RowSet& b) {
  if (a.lead != b.lead || a.row0 != b.row0 || a.ptr != b.ptr || a.terms.size() != b.terms.size()) return false;
  return a.terms.empty() || std::memcmp(a.terms.data(), b.terms.data(), a.terms.size() * sizeof(ddelm::Term)) == 0;
}
bool same(const ddelm::Geometry& g, const ddelm::Geometry& o) {
  if (!(same_rows(g.rowsK, o.rowsK) && same_rows(g.rowsA, o.rowsA) && same_rows(g.rowsKb, o.rowsKb) &&
        same_rows(g.rowsAb, o.rowsAb)))
    return false;
  if (g.pi_own_ptr != o.pi_own_ptr || g.pi_own_slot != o.pi_own_slot || g.dl_own_ptr != o.dl_own_ptr ||
      g.dl_own_slot != o.dl_own_slot || g.pi_off != o.pi_off || g.dl_off != o.dl_off ||
      g.pi_loc2glob != o.pi_loc2glob || g.dl_loc2glob != o.dl_loc2glob || g.x_pi != o.x_pi || g.x_dl != o.x_dl)
    return false;
  if (g.max_m != o.max_m || g.max_nG != o.max_nG || g.sum_nB != o.sum_nB) return false;
  for (int i = 0; i < g.N; ++i) {
    const ddelm::SubInfo &a = g.subs[i], &b = o.subs[i];
    if (a.xB != b.xB || a.xG != b.xG || a.pi_glob != b.pi_glob || a.dl_glob != b.dl_glob || a.n_B != b.n_B ||
        a.n_P != b.n_P || a.n_D != b.n_D || a.cx != b.cx || a.cy != b.cy)
      return false;
  }
  return true;
}
}  // namespace

int main() {
  struct Case { int nx, ny, p, n_extra, coarse; };
  const Case cases[] = {{32, 32, 40, 39, 2}, {2, 2, 16, 0, 2}, {8, 8, 32, 0, 1}, {16, 16, 20, 0, 3},
                        {4, 3, 9, 4, 0},     {3, 3, 12, 11, 4}, {40, 7, 10, 0, 2}, {1, 1, 5, 0, 2},
                        {17, 9, 7, 3, 4},    {5, 13, 6, 2, 2}};
  int bad = 0;
  for (const Case& c : cases) {
    std::vector<double> s(c.p), ex(c.n_extra);
    for (int k = 0; k < c.p; ++k) s[k] = (double)k / (c.p - 1);
    s[c.p - 1] = 1.0;
    for (int k = 0; k < c.n_extra; ++k) ex[k] = (k + 0.5) / c.n_extra;
    const double lo[2] = {0.0, 0.0}, hi[2] = {1.0, 1.0};
    ddelm::Geometry ref;
    ref.threads = 1;
    const std::string e1 = ref.build(c.nx, c.ny, lo, hi, c.p, s.data(), c.n_extra, ex.data(), 25, c.coarse);
    for (int t : {2, 3, 8, 0}) {
      ddelm::Geometry g;
      g.threads = t;
      const std::string e2 = g.build(c.nx, c.ny, lo, hi, c.p, s.data(), c.n_extra, ex.data(), 25, c.coarse);
      const bool ok = e1 == e2 && same(g, ref);
      if (!ok) {
        std::printf("DIFFERENT: %dx%d p=%d extra=%d coarse=%d threads=%d\n", c.nx, c.ny, c.p, c.n_extra, c.coarse, t);
        ++bad;
      }
    }
  }
  std::printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
