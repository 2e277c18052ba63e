// Host construction of the overlapping decomposition (Sections 3, 4, 5):
// disjoint coordinate partitions, breadth-first overlap layers, local ghost and
// transmission-node sets, the subsurface closest points of eq. locCP, the
// conormal term of eq. naConorm and the cross-point weights of Section 5.2.2.
// Compiled with -ffp-contract=off (see setup_band.cpp).
#include <algorithm>
#include <cmath>
#include <thread>

#include "cpm_internal.h"

namespace cpm {
namespace {

// Recursive coordinate bisection on grid indices: split along the axis of
// largest index extent (ties x < y < z), nodes ordered by (index on that
// axis, L); the left floor(n/2) parts receive floor(|S| W_l / W) nodes.
void rcb(const Band& b, std::vector<int32_t>& idx, int first, int n, const double* w,
         std::vector<int32_t>& part) {
  if (n == 1) {
    for (int32_t q : idx) part[q] = first;
    return;
  }
  int32_t mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  for (int32_t q : idx)
    for (int a = 0; a < 3; ++a) {
      mn[a] = std::min(mn[a], b.ijk[(size_t)q * 3 + a]);
      mx[a] = std::max(mx[a], b.ijk[(size_t)q * 3 + a]);
    }
  int axis = 0;
  for (int a = 1; a < 3; ++a)
    if (mx[a] - mn[a] > mx[axis] - mn[axis]) axis = a;
  std::sort(idx.begin(), idx.end(), [&](int32_t u, int32_t v) {
    const int32_t cu = b.ijk[(size_t)u * 3 + axis], cv = b.ijk[(size_t)v * 3 + axis];
    if (cu != cv) return cu < cv;
    return b.lin[u] < b.lin[v];
  });
  const int nl = n / 2;
  size_t cut;
  if (!w) {
    cut = (idx.size() * (size_t)nl) / (size_t)n;
  } else {
    double wl = 0.0, wt = 0.0;
    for (int q = first; q < first + nl; ++q) wl += w[q];
    for (int q = first; q < first + n; ++q) wt += w[q];
    cut = (size_t)std::floor((double)idx.size() * wl / wt);
  }
  std::vector<int32_t> left(idx.begin(), idx.begin() + cut), right(idx.begin() + cut, idx.end());
  idx.clear();
  idx.shrink_to_fit();
  rcb(b, left, first, nl, w, part);
  rcb(b, right, first + nl, n - nl, w, part);
}

// Recursive graph bisection of the 6-neighbour graph of the actives: as rcb,
// but nodes are ordered by breadth-first distance inside the subgraph induced
// by the current set, from a pseudo-peripheral node (a sweep from the lowest
// band index finds the farthest node, lowest index on ties; a second sweep
// starts there), ties by band index; unreachable nodes come last. idx is
// sorted by band index on entry; pos is a scratch map band index -> position
// (-1 outside the set).
void bfs_dist(const Band& b, const std::vector<int32_t>& idx, const std::vector<int32_t>& pos, int start,
              std::vector<int32_t>& dist) {
  const int64_t na = b.n_act;
  dist.assign(idx.size(), -1);
  std::vector<int32_t> queue;
  queue.reserve(idx.size());
  dist[start] = 0;
  queue.push_back(start);
  for (size_t h = 0; h < queue.size(); ++h) {
    const int32_t u = queue[h];
    const int32_t q = idx[u];
    for (int e = 0; e < 6; ++e) {
      const int32_t y = b.nbr[(size_t)q * 6 + e];
      if (y >= na) continue;
      const int32_t v = pos[y];
      if (v < 0 || dist[v] >= 0) continue;
      dist[v] = dist[u] + 1;
      queue.push_back(v);
    }
  }
}

void graph_bisect(const Band& b, std::vector<int32_t>& idx, int first, int n, const double* w,
                  std::vector<int32_t>& pos, std::vector<int32_t>& part) {
  if (n == 1) {
    for (int32_t q : idx) part[q] = first;
    return;
  }
  for (size_t u = 0; u < idx.size(); ++u) pos[idx[u]] = (int32_t)u;
  std::vector<int32_t> dist;
  bfs_dist(b, idx, pos, 0, dist);
  int far = 0;
  for (size_t u = 1; u < idx.size(); ++u)
    if (dist[u] > dist[far]) far = (int)u;
  bfs_dist(b, idx, pos, far, dist);
  for (int32_t q : idx) pos[q] = -1;
  const int32_t unreached = (int32_t)b.n_act + 1;
  std::vector<int32_t> order(idx.size());
  for (size_t u = 0; u < idx.size(); ++u) order[u] = (int32_t)u;
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const int32_t dx = dist[x] < 0 ? unreached : dist[x], dy = dist[y] < 0 ? unreached : dist[y];
    if (dx != dy) return dx < dy;
    return idx[x] < idx[y];
  });
  const int nl = n / 2;
  size_t cut;
  if (!w) {
    cut = (idx.size() * (size_t)nl) / (size_t)n;
  } else {
    double wl = 0.0, wt = 0.0;
    for (int q = first; q < first + nl; ++q) wl += w[q];
    for (int q = first; q < first + n; ++q) wt += w[q];
    cut = (size_t)std::floor((double)idx.size() * wl / wt);
  }
  std::vector<int32_t> left, right;
  left.reserve(cut);
  right.reserve(idx.size() - cut);
  for (size_t u = 0; u < idx.size(); ++u) (u < cut ? left : right).push_back(idx[order[u]]);
  idx.clear();
  idx.shrink_to_fit();
  std::sort(left.begin(), left.end());
  std::sort(right.begin(), right.end());
  // Pieces of the right group cut off from its largest connected piece (ties:
  // the piece holding the lowest band index) join the left group.
  if (!right.empty()) {
    for (size_t u = 0; u < right.size(); ++u) pos[right[u]] = (int32_t)u;
    std::vector<int32_t> comp(right.size(), -1), csize;
    int ncomp = 0;
    std::vector<int32_t> queue;
    for (size_t s0 = 0; s0 < right.size(); ++s0) {
      if (comp[s0] >= 0) continue;
      comp[s0] = ncomp;
      queue.assign(1, (int32_t)s0);
      for (size_t hq = 0; hq < queue.size(); ++hq) {
        const int32_t q = right[queue[hq]];
        for (int e = 0; e < 6; ++e) {
          const int32_t y = b.nbr[(size_t)q * 6 + e];
          if (y >= b.n_act) continue;
          const int32_t v = pos[y];
          if (v < 0 || comp[v] >= 0) continue;
          comp[v] = ncomp;
          queue.push_back(v);
        }
      }
      csize.push_back((int32_t)queue.size());
      ++ncomp;
    }
    for (int32_t q : right) pos[q] = -1;
    if (ncomp > 1) {
      int keep = 0;  // components are numbered in order of their lowest member
      for (int c = 1; c < ncomp; ++c)
        if (csize[c] > csize[keep]) keep = c;
      std::vector<int32_t> r2;
      for (size_t u = 0; u < right.size(); ++u) (comp[u] == keep ? r2 : left).push_back(right[u]);
      right.swap(r2);
      std::sort(left.begin(), left.end());
    }
  }
  graph_bisect(b, left, first, nl, w, pos, part);
  graph_bisect(b, right, first + nl, n - nl, w, pos, part);
}

// Interface alignment (Section 3.2): `passes` rounds in which every node with
// an active FD neighbour in another part moves, all at once, to the part of
// the grid node nearest to its closest point.
int align_interfaces(const Band& b, std::vector<int32_t>& part, int passes, std::string& err) {
  const int64_t na = b.n_act;
  std::vector<int32_t> xbar(na);
  for (int64_t q = 0; q < na; ++q) {
    int64_t g[3];
    for (int a = 0; a < 3; ++a) {
      const double t = (b.cp[q * 3 + a] - b.lo[a]) / b.h;
      g[a] = (int64_t)std::floor(t + 0.5);
    }
    const int64_t L = (g[0] * b.n[1] + g[1]) * b.n[2] + g[2];
    const auto it = std::lower_bound(b.lin.begin(), b.lin.begin() + na, L);
    if (it == b.lin.begin() + na || *it != L) {
      err = "partition: a closest point's nearest grid node is not active";
      return CPM_EINVAL;
    }
    xbar[q] = (int32_t)(it - b.lin.begin());
  }
  std::vector<int32_t> next(na);
  for (int pass = 0; pass < passes; ++pass) {
    for (int64_t q = 0; q < na; ++q) {
      bool iface = false;
      for (int e = 0; e < 6; ++e) {
        const int32_t y = b.nbr[q * 6 + e];
        if (y < na && part[y] != part[q]) iface = true;
      }
      next[q] = iface ? part[xbar[q]] : part[q];
    }
    part.swap(next);
  }
  return CPM_OK;
}

void sort_unique(std::vector<int32_t>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}


// Reverse Cuthill-McKee order of the local unknowns [Sigma_j ; B_j] (B_j only
// for ORAS) on the symmetrised pattern of A_j (eq. localOP): a Sigma row holds
// its own node and the interpolation stencils of its neighbours' extension rows
// (a transmission neighbour contributes the stencil of its Robin row, at x*(b),
// eq. robfo; for RAS an active neighbour outside Sigma_j contributes nothing); a
// B row holds its node and the stencil at x*(b). Breadth-first from the
// lowest-degree node of each component, neighbours visited in increasing
// degree (ties: lower local index), the whole order reversed. Stencil nodes
// whose interpolation weight is exactly zero (a closest point on a grid
// plane) are not entries. `lpos` is an all -1 scratch of N_T entries and is
// left that way.
std::vector<int32_t> rcm_order(const Band& b, const Sub& sd, bool oras, std::vector<int32_t>& lpos,
                               std::vector<int32_t>& reach) {
  const int64_t na = b.n_act;
  const int P1 = b.p + 1, P2 = P1 * P1;
  const int m = (int)sd.sigma.size();
  const int n = m + (oras ? (int)sd.bnd.size() : 0);
  for (int q = 0; q < m; ++q) lpos[sd.sigma[q]] = q;
  if (oras)
    for (int q = 0; q < n - m; ++q) lpos[sd.bnd[q]] = m + q;
  // pattern rows without the diagonal, duplicates removed
  std::vector<int32_t> stamp(n, -1), off(n + 1, 0), col;
  col.reserve((size_t)n * 96);
  auto add_ext = [&](int row, int32_t node) {
    const double* w = &b.wts[(size_t)node * 3 * P1];  // x, y, z weights
    for (int a = 0; a < P2; ++a) {
      const int32_t first = b.lines[(size_t)node * P2 + a];
      const double wab = w[a / P1] * w[P1 + a % P1];
      for (int c = 0; c < P1; ++c) {
        const int32_t q = lpos[first + c];
        if (wab * w[2 * P1 + c] != 0.0 && q >= 0 && q != row && stamp[q] != row) {
          stamp[q] = row;
          col.push_back(q);
        }
      }
    }
  };
  for (int r = 0; r < n; ++r) {
    if (r < m) {
      const int32_t x = sd.sigma[r];
      for (int e = 0; e < 6; ++e) {
        const int32_t y = b.nbr[(size_t)x * 6 + e];
        if (y < na) {
          const int32_t q = lpos[y];
          if (q >= m) add_ext(r, sd.xstar[q - m]);
          else if (q >= 0) add_ext(r, y);
        } else {
          add_ext(r, y);
        }
      }
    } else {
      add_ext(r, sd.xstar[r - m]);
    }
    off[r + 1] = (int32_t)col.size();
  }
  for (int q = 0; q < m; ++q) lpos[sd.sigma[q]] = -1;
  if (oras)
    for (int q = 0; q < n - m; ++q) lpos[sd.bnd[q]] = -1;
  // symmetrise: rows of the transpose, then the union of both per node
  std::vector<int32_t> toff(n + 1, 0), tcol(col.size());
  for (int32_t q : col) toff[q + 1]++;
  for (int r = 0; r < n; ++r) toff[r + 1] += toff[r];
  {
    std::vector<int32_t> fill(toff.begin(), toff.end() - 1);
    for (int r = 0; r < n; ++r)
      for (int32_t e = off[r]; e < off[r + 1]; ++e) tcol[fill[col[e]]++] = r;
  }
  std::vector<int32_t> soff(n + 1, 0), scol;
  scol.reserve(col.size() * 2);
  std::fill(stamp.begin(), stamp.end(), -1);
  for (int r = 0; r < n; ++r) {
    for (int32_t e = off[r]; e < off[r + 1]; ++e) {
      stamp[col[e]] = r;
      scol.push_back(col[e]);
    }
    for (int32_t e = toff[r]; e < toff[r + 1]; ++e)
      if (stamp[tcol[e]] != r) {
        stamp[tcol[e]] = r;
        scol.push_back(tcol[e]);
      }
    soff[r + 1] = (int32_t)scol.size();
  }
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<uint8_t> seen(n, 0);
  auto deg = [&](int32_t q) { return soff[q + 1] - soff[q]; };
  auto by_degree = [&](int32_t x, int32_t y) { return deg(x) != deg(y) ? deg(x) < deg(y) : x < y; };
  std::vector<int32_t> fresh;
  while ((int)order.size() < n) {
    int32_t start = -1;
    for (int q = 0; q < n; ++q)
      if (!seen[q] && (start < 0 || deg(q) < deg(start))) start = q;
    seen[start] = 1;
    order.push_back(start);
    for (size_t h = order.size() - 1; h < order.size(); ++h) {
      const int32_t v = order[h];
      fresh.clear();
      for (int32_t e = soff[v]; e < soff[v + 1]; ++e)
        if (!seen[scol[e]]) {
          seen[scol[e]] = 1;
          fresh.push_back(scol[e]);
        }
      std::sort(fresh.begin(), fresh.end(), by_degree);
      order.insert(order.end(), fresh.begin(), fresh.end());
    }
  }
  std::reverse(order.begin(), order.end());
  // first nonzero column of each row in elimination order (diagonal included),
  // then reach[c] = 1 + the last position p with first[p] <= c
  std::vector<int32_t> at(n), first(n);
  for (int p = 0; p < n; ++p) at[order[p]] = p;
  for (int r = 0; r < n; ++r) {
    int32_t f = at[r];
    for (int32_t e = off[r]; e < off[r + 1]; ++e) f = std::min(f, at[col[e]]);
    first[at[r]] = f;
  }
  reach.assign(n, 0);
  for (int p = 0; p < n; ++p) reach[first[p]] = std::max(reach[first[p]], p + 1);
  for (int c = 1; c < n; ++c) reach[c] = std::max(reach[c], reach[c - 1]);
  return order;
}

}  // namespace

int build_decomposition(const Band& b, Decomp& d, int method, int n_sub, const double* weights,
                        int overlap, int kind, double alpha, double alpha_cross,
                        std::string& err) {
  const int64_t na = b.n_act;
  if (kind != CPM_RAS && kind != CPM_ORAS) { err = "partition: kind must be RAS or ORAS"; return CPM_EINVAL; }
  if (overlap < 0 || (kind == CPM_ORAS && overlap < 1)) { err = "partition: overlap must be >= 1 for ORAS, >= 0 for RAS"; return CPM_EINVAL; }
  if (kind == CPM_ORAS && !(alpha > 0 && std::isfinite(alpha))) { err = "partition: ORAS needs a positive finite alpha"; return CPM_EINVAL; }
  if (!(alpha_cross >= 0) || !std::isfinite(alpha_cross)) { err = "partition: alpha_cross must be >= 0"; return CPM_EINVAL; }
  if (n_sub < 1 || n_sub > na) { err = "partition: n_sub out of range"; return CPM_EINVAL; }
  const bool align = (method & CPM_PART_ALIGN) != 0;
  method &= ~CPM_PART_ALIGN;
  if (method == CPM_PART_OCTANT && n_sub != 8) { err = "partition: octant partition has 8 parts"; return CPM_EINVAL; }
  if (method != CPM_PART_OCTANT && method != CPM_PART_RCB && method != CPM_PART_GRAPH) {
    err = "partition: unknown method";
    return CPM_EINVAL;
  }
  if (weights)
    for (int q = 0; q < n_sub; ++q)
      if (!(weights[q] > 0) || !std::isfinite(weights[q])) { err = "partition: weights must be positive"; return CPM_EINVAL; }

  Decomp nd;
  nd.n_sub = n_sub;
  nd.kind = kind;
  nd.overlap = overlap;
  nd.alpha = alpha;
  nd.alpha_cross = alpha_cross;
  nd.part.assign(na, -1);
  if (method == CPM_PART_OCTANT) {
    for (int64_t q = 0; q < na; ++q) {
      const int32_t* x = &b.ijk[q * 3];
      nd.part[q] = 4 * (x[0] >= b.n[0] / 2) + 2 * (x[1] >= b.n[1] / 2) + (x[2] >= b.n[2] / 2);
    }
  } else if (method == CPM_PART_RCB) {
    std::vector<int32_t> idx(na);
    for (int64_t q = 0; q < na; ++q) idx[q] = (int32_t)q;
    rcb(b, idx, 0, n_sub, weights, nd.part);
  } else {
    std::vector<int32_t> idx(na), pos(na, -1);
    for (int64_t q = 0; q < na; ++q) idx[q] = (int32_t)q;
    graph_bisect(b, idx, 0, n_sub, weights, pos, nd.part);
  }
  if (align) {
    const int rc = align_interfaces(b, nd.part, b.p + 1, err);
    if (rc != CPM_OK) return rc;
  }
  std::vector<int64_t> count(n_sub, 0);
  for (int32_t q : nd.part) count[q]++;
  for (int j = 0; j < n_sub; ++j)
    if (count[j] == 0) { err = "partition: a part is empty"; return CPM_EINVAL; }

  // Cross points: active nodes whose active neighbours lie in >= 2 other parts.
  nd.cross.assign(na, 0);
  for (int64_t q = 0; q < na; ++q) {
    int32_t seen[6];
    int ns = 0;
    for (int e = 0; e < 6; ++e) {
      const int32_t y = b.nbr[q * 6 + e];
      if (y >= na) continue;
      const int32_t py = nd.part[y];
      if (py == nd.part[q]) continue;
      bool dup = false;
      for (int s = 0; s < ns; ++s) dup |= (seen[s] == py);
      if (!dup) seen[ns++] = py;
    }
    nd.cross[q] = ns >= 2;
  }
  // Grid nodes within 2 N_O grid units (inclusive) of a cross point.
  std::vector<uint8_t> near_cross;
  if (kind == CPM_ORAS && alpha_cross > 0) {
    near_cross.assign((size_t)(b.n[0] * b.n[1] * b.n[2]), 0);
    const int R = 2 * overlap;
    for (int64_t q = 0; q < na; ++q) {
      if (!nd.cross[q]) continue;
      const int32_t* x = &b.ijk[q * 3];
      for (int di = -R; di <= R; ++di)
        for (int dj = -R; dj <= R; ++dj)
          for (int dk = -R; dk <= R; ++dk) {
            if (di * di + dj * dj + dk * dk > R * R) continue;
            const int64_t I = x[0] + di, J = x[1] + dj, K = x[2] + dk;
            if (I < 0 || J < 0 || K < 0 || I >= b.n[0] || J >= b.n[1] || K >= b.n[2]) continue;
            near_cross[(size_t)((I * b.n[1] + J) * b.n[2] + K)] = 1;
          }
    }
  }

  std::vector<std::vector<int32_t>> members(n_sub);
  for (int64_t q = 0; q < na; ++q) members[nd.part[q]].push_back((int32_t)q);
  nd.subs.resize(n_sub);
  const int P1 = b.p + 1, NS = P1 * P1 * P1;
  std::vector<int> fail(n_sub, 0);

  auto build_one = [&](int j, std::vector<uint8_t>& mark, std::vector<int32_t>& lpos) {
    Sub& sd = nd.subs[j];
    sd.tilde = members[j];
    // Breadth-first overlap layers inside the active set.
    std::vector<int32_t> sigma = sd.tilde, front = sd.tilde;
    for (int32_t q : sigma) mark[q] = 1;
    for (int layer = 0; layer < overlap; ++layer) {
      std::vector<int32_t> next;
      for (int32_t q : front)
        for (int e = 0; e < 6; ++e) {
          const int32_t y = b.nbr[(size_t)q * 6 + e];
          if (y < na && !mark[y]) {
            mark[y] = 1;
            next.push_back(y);
          }
        }
      sigma.insert(sigma.end(), next.begin(), next.end());
      front.swap(next);
    }
    sort_unique(front);
    sd.fin = front;
    sort_unique(sigma);
    sd.sigma = sigma;
    // Local ghosts and transmission nodes.
    std::vector<int32_t> bnd;
    for (int32_t q : sd.sigma)
      for (int e = 0; e < 6; ++e) {
        const int32_t y = b.nbr[(size_t)q * 6 + e];
        if (y >= na) sd.ghost.push_back(y);
        else if (!mark[y]) bnd.push_back(y);
      }
    sort_unique(sd.ghost);
    auto add_cols = [&](int32_t row) {
      for (int a = 0; a < P1 * P1; ++a) {
        const int32_t first = b.lines[(size_t)row * P1 * P1 + a];
        for (int c = 0; c < P1; ++c)
          if (!mark[first + c]) bnd.push_back(first + c);
      }
    };
    for (int32_t q : sd.sigma) add_cols(q);
    for (int32_t q : sd.ghost) add_cols(q);
    sort_unique(bnd);
    sd.bnd = bnd;
    (void)NS;
    for (int32_t q : sd.sigma) mark[q] = 0;
    if (kind != CPM_ORAS) {
      sd.order = rcm_order(b, sd, false, lpos, sd.reach);
      return;
    }
    const size_t nbd = sd.bnd.size();
    sd.xstar.resize(nbd);
    sd.s.resize(nbd);
    sd.alpha.resize(nbd);
    if (nbd && sd.fin.empty()) { fail[j] = 1; return; }
    for (size_t q = 0; q < nbd; ++q) {
      const int32_t bn = sd.bnd[q];
      const double* xb = &b.xyz[(size_t)bn * 3];
      double best = INFINITY;
      int32_t arg = -1;
      for (int32_t f : sd.fin) {  // ascending band index: the first minimum is kept
        const double* c = &b.cp[(size_t)f * 3];
        const double d0 = xb[0] - c[0], d1 = xb[1] - c[1], d2 = xb[2] - c[2];
        const double dd = (d0 * d0 + d1 * d1) + d2 * d2;
        if (dd < best) { best = dd; arg = f; }
      }
      sd.xstar[q] = arg;
      const double* y = &b.cp[(size_t)arg * 3];
      const double* nr = &b.nrm[(size_t)arg * 3];
      const double d0 = xb[0] - y[0], d1 = xb[1] - y[1], d2 = xb[2] - y[2];
      const double dn = (d0 * nr[0] + d1 * nr[1]) + d2 * nr[2];
      const double t0 = d0 - dn * nr[0], t1 = d1 - dn * nr[1], t2 = d2 - dn * nr[2];
      sd.s[q] = std::sqrt((t0 * t0 + t1 * t1) + t2 * t2);
      sd.alpha[q] = alpha;
      if (!near_cross.empty()) {
        const int32_t* x = &b.ijk[(size_t)bn * 3];
        if (near_cross[(size_t)(((int64_t)x[0] * b.n[1] + x[1]) * b.n[2] + x[2])]) sd.alpha[q] = alpha_cross;
      }
    }
    sd.order = rcm_order(b, sd, true, lpos, sd.reach);
  };

  const int nth = std::max(1, std::min<int>(n_sub, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back([&, t]() {
      std::vector<uint8_t> mark(na, 0);
      std::vector<int32_t> lpos(b.total(), -1);
      for (int j = t; j < n_sub; j += nth) build_one(j, mark, lpos);
    });
  for (auto& th : pool) th.join();
  for (int j = 0; j < n_sub; ++j)
    if (fail[j]) { err = "partition: subdomain has transmission nodes but no final overlap layer"; return CPM_EINVAL; }
  d = std::move(nd);
  return CPM_OK;
}

}  // namespace cpm
