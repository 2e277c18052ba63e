// Host construction of the closest point method band (Section 2.1):
// tube-radius active set, ghost shell of the 7-point stencil, tensor-product
// Lagrange extension rows. Compiled with -ffp-contract=off so that the
// floating-point decisions (distance test, stencil placement) are the plain
// IEEE evaluation of the stated formulas.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "cpm_internal.h"

namespace cpm {
namespace {

struct Grid {
  double lo[3];
  double h;
  int64_t n[3];
  int64_t lin(int64_t i, int64_t j, int64_t k) const { return (i * n[1] + j) * n[2] + k; }
  void split(int64_t L, int64_t* ijk) const {
    ijk[2] = L % n[2];
    int64_t q = L / n[2];
    ijk[1] = q % n[1];
    ijk[0] = q / n[1];
  }
  double coord(int a, int64_t i) const { return lo[a] + (double)i * h; }
  bool inside(int64_t i, int64_t j, int64_t k) const {
    return i >= 0 && i < n[0] && j >= 0 && j < n[1] && k >= 0 && k < n[2];
  }
};

// First stencil index along one axis and the local coordinate s = t - base.
// Odd degree: the closest point lies in the central cell; even degree: the
// central node is the nearest node.
inline int64_t stencil_base(double cpa, double lo, double h, int p, double* s) {
  double t = (cpa - lo) / h;
  int64_t b = (p & 1) ? (int64_t)std::floor(t) - (p - 1) / 2 : (int64_t)std::floor(t + 0.5) - p / 2;
  *s = t - (double)b;
  return b;
}

// Lagrange basis on the nodes 0..p: l_m(s) = prod_{q != m} (s - q) / prod_{q != m} (m - q).
inline void lagrange(double s, int p, double* w) {
  for (int m = 0; m <= p; ++m) {
    double num = 1.0, den = 1.0;
    for (int q = 0; q <= p; ++q) {
      if (q == m) continue;
      num *= (s - (double)q);
      den *= (double)(m - q);
    }
    w[m] = num / den;
  }
}

struct CpCache {
  std::unordered_map<int64_t, int64_t> at;
  std::vector<double> cp, nrm;
  void put(int64_t L, const double* c, const double* nr) {
    auto it = at.find(L);
    if (it != at.end()) return;
    at.emplace(L, (int64_t)(cp.size() / 3));
    cp.insert(cp.end(), c, c + 3);
    nrm.insert(nrm.end(), nr, nr + 3);
  }
};

}  // namespace

int build_band(Band& b, cpm_cp_fn fn, void* user, const double lo[3], const double hi[3],
               double h, int p, double band_factor, std::string& err) {
  if (!fn) { err = "build_band: null closest-point callback"; return CPM_EINVAL; }
  if (p != 2 && p != 3) { err = "build_band: degree must be 2 or 3"; return CPM_EINVAL; }
  if (!(h > 0) || !std::isfinite(h)) { err = "build_band: h must be positive and finite"; return CPM_EINVAL; }
  Grid g;
  g.h = h;
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] > lo[a])) {
      err = "build_band: need finite lo < hi";
      return CPM_EINVAL;
    }
    g.lo[a] = lo[a];
    double na = std::floor((hi[a] - lo[a]) / h + 0.5) + 1.0;
    if (na > 2.0e6) { err = "build_band: grid too large"; return CPM_EINVAL; }
    g.n[a] = (int64_t)na;
  }
  const double rho2 = band_factor > 0 ? band_factor * band_factor : 0.75 * (double)((p + 1) * (p + 1));
  const double r2 = rho2 * (h * h);
  const double rc = std::sqrt(r2) + 2.5 * h;  // closest points cached for possible ghosts
  const double rc2 = rc * rc;

  CpCache cache;
  std::vector<int64_t> act;
  {
    const int64_t slab = g.n[1] * g.n[2];
    std::vector<double> X((size_t)slab * 3), C((size_t)slab * 3), N((size_t)slab * 3);
    for (int64_t i = 0; i < g.n[0]; ++i) {
      const double x0 = g.coord(0, i);
      for (int64_t j = 0; j < g.n[1]; ++j) {
        const double x1 = g.coord(1, j);
        for (int64_t k = 0; k < g.n[2]; ++k) {
          double* x = &X[(size_t)(j * g.n[2] + k) * 3];
          x[0] = x0;
          x[1] = x1;
          x[2] = g.coord(2, k);
        }
      }
      if (fn(user, slab, X.data(), C.data(), N.data()) != 0) {
        err = "build_band: closest-point callback failed";
        return CPM_ECALLBACK;
      }
      for (int64_t q = 0; q < slab; ++q) {
        const double* x = &X[(size_t)q * 3];
        const double* c = &C[(size_t)q * 3];
        if (!std::isfinite(c[0]) || !std::isfinite(c[1]) || !std::isfinite(c[2])) continue;
        const double d0 = x[0] - c[0], d1 = x[1] - c[1], d2 = x[2] - c[2];
        const double dd = (d0 * d0 + d1 * d1) + d2 * d2;
        const int64_t L = i * slab + q;
        if (dd <= r2) act.push_back(L);
        if (dd <= rc2) cache.put(L, c, &N[(size_t)q * 3]);
      }
    }
  }

  // Closest points of nodes outside the cache, queried in one batch.
  auto fetch = [&](const std::vector<int64_t>& Ls) -> int {
    std::vector<double> X, C, N;
    std::vector<int64_t> need;
    for (int64_t L : Ls)
      if (!cache.at.count(L)) need.push_back(L);
    if (need.empty()) return CPM_OK;
    X.resize(need.size() * 3);
    C.resize(need.size() * 3);
    N.resize(need.size() * 3);
    for (size_t q = 0; q < need.size(); ++q) {
      int64_t ijk[3];
      g.split(need[q], ijk);
      for (int a = 0; a < 3; ++a) X[q * 3 + a] = g.coord(a, ijk[a]);
    }
    if (fn(user, (int64_t)need.size(), X.data(), C.data(), N.data()) != 0) {
      err = "build_band: closest-point callback failed";
      return CPM_ECALLBACK;
    }
    for (size_t q = 0; q < need.size(); ++q) cache.put(need[q], &C[q * 3], &N[q * 3]);
    return CPM_OK;
  };

  static const int OFF[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  std::vector<int64_t> ghost;
  for (;;) {
    std::unordered_map<int64_t, char> is_act;
    is_act.reserve(act.size() * 2);
    for (int64_t L : act) is_act.emplace(L, 1);
    ghost.clear();
    for (int64_t L : act) {
      int64_t ijk[3];
      g.split(L, ijk);
      for (int q = 0; q < 6; ++q) {
        const int64_t a = ijk[0] + OFF[q][0], bb = ijk[1] + OFF[q][1], cc = ijk[2] + OFF[q][2];
        if (!g.inside(a, bb, cc)) { err = "build_band: ghost node outside the grid box"; return CPM_EINVAL; }
        const int64_t M = g.lin(a, bb, cc);
        if (!is_act.count(M)) ghost.push_back(M);
      }
    }
    std::sort(ghost.begin(), ghost.end());
    ghost.erase(std::unique(ghost.begin(), ghost.end()), ghost.end());
    int rc_ = fetch(ghost);
    if (rc_ != CPM_OK) return rc_;
    std::vector<int64_t> missing;
    auto check_row = [&](int64_t L) -> int {
      const double* c = &cache.cp[(size_t)cache.at.at(L) * 3];
      if (!std::isfinite(c[0]) || !std::isfinite(c[1]) || !std::isfinite(c[2])) {
        err = "build_band: closest point undefined at a band node";
        return CPM_EINVAL;
      }
      int64_t bs[3];
      double s;
      for (int a = 0; a < 3; ++a) bs[a] = stencil_base(c[a], g.lo[a], g.h, p, &s);
      for (int a = 0; a <= p; ++a)
        for (int bb = 0; bb <= p; ++bb)
          for (int cc = 0; cc <= p; ++cc) {
            const int64_t I = bs[0] + a, J = bs[1] + bb, K = bs[2] + cc;
            if (!g.inside(I, J, K)) { err = "build_band: interpolation stencil leaves the grid box"; return CPM_EINVAL; }
            const int64_t M = g.lin(I, J, K);
            if (!is_act.count(M)) missing.push_back(M);
          }
      return CPM_OK;
    };
    for (int64_t L : act)
      if ((rc_ = check_row(L)) != CPM_OK) return rc_;
    for (int64_t L : ghost)
      if ((rc_ = check_row(L)) != CPM_OK) return rc_;
    if (missing.empty()) break;
    std::sort(missing.begin(), missing.end());
    missing.erase(std::unique(missing.begin(), missing.end()), missing.end());
    if ((rc_ = fetch(missing)) != CPM_OK) return rc_;
    std::vector<int64_t> merged;
    std::merge(act.begin(), act.end(), missing.begin(), missing.end(), std::back_inserter(merged));
    act.swap(merged);
  }
  if (act.empty()) { err = "build_band: no grid node lies within the tube radius"; return CPM_EINVAL; }
  if (act.size() + ghost.size() >= (size_t)INT32_MAX) { err = "build_band: band too large"; return CPM_EINVAL; }

  Band nb;
  for (int a = 0; a < 3; ++a) { nb.lo[a] = g.lo[a]; nb.n[a] = g.n[a]; }
  nb.h = h;
  nb.p = p;
  nb.n_act = (int64_t)act.size();
  nb.n_ghost = (int64_t)ghost.size();
  const int64_t NT = nb.total();
  nb.lin.reserve(NT);
  nb.lin.insert(nb.lin.end(), act.begin(), act.end());
  nb.lin.insert(nb.lin.end(), ghost.begin(), ghost.end());
  std::unordered_map<int64_t, int32_t> index;
  index.reserve(NT * 2);
  for (int64_t q = 0; q < NT; ++q) index.emplace(nb.lin[q], (int32_t)q);

  const int P1 = p + 1;
  nb.ijk.resize(NT * 3);
  nb.xyz.resize(NT * 3);
  nb.cp.resize(NT * 3);
  nb.nrm.resize(NT * 3);
  nb.base.resize(NT * 3);
  nb.wts.resize(NT * 3 * P1);
  nb.lines.resize(NT * P1 * P1);
  for (int64_t q = 0; q < NT; ++q) {
    int64_t ijk[3];
    g.split(nb.lin[q], ijk);
    const int64_t ci = cache.at.at(nb.lin[q]);
    double s[3];
    int64_t bs[3];
    for (int a = 0; a < 3; ++a) {
      nb.ijk[q * 3 + a] = (int32_t)ijk[a];
      nb.xyz[q * 3 + a] = g.coord(a, ijk[a]);
      nb.cp[q * 3 + a] = cache.cp[ci * 3 + a];
      nb.nrm[q * 3 + a] = cache.nrm[ci * 3 + a];
      bs[a] = stencil_base(nb.cp[q * 3 + a], g.lo[a], g.h, p, &s[a]);
      nb.base[q * 3 + a] = (int32_t)bs[a];
      lagrange(s[a], p, &nb.wts[(q * 3 + a) * P1]);
    }
    for (int a = 0; a < P1; ++a)
      for (int bb = 0; bb < P1; ++bb) {
        const int64_t L0 = g.lin(bs[0] + a, bs[1] + bb, bs[2]);
        const int32_t first = index.at(L0);
        for (int cc = 1; cc < P1; ++cc)
          if (first + cc >= nb.n_act || nb.lin[first + cc] != L0 + cc) {
            err = "build_band: internal error, stencil line not contiguous";
            return CPM_EINVAL;
          }
        nb.lines[(q * P1 + a) * P1 + bb] = first;
      }
  }
  nb.nbr.resize(nb.n_act * 6);
  for (int64_t q = 0; q < nb.n_act; ++q) {
    for (int d = 0; d < 6; ++d) {
      const int64_t M = g.lin(nb.ijk[q * 3] + OFF[d][0], nb.ijk[q * 3 + 1] + OFF[d][1],
                              nb.ijk[q * 3 + 2] + OFF[d][2]);
      nb.nbr[q * 6 + d] = index.at(M);
    }
  }
  b = std::move(nb);
  return CPM_OK;
}

}  // namespace cpm
