// Host-side hierarchy of the DH^2 matrix (Section 2): see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <set>

namespace dh2 {

namespace {

inline double norm3(double a, double b, double c) { return std::sqrt(a * a + b * b + c * c); }

struct TreeBuilder {
  const double* V;
  const int32_t* T;
  std::vector<double> cen;          // [n][3] centroids
  std::vector<double> vlo, vhi;     // [n][3] vertex boxes per triangle
  Plan* p;
  int leafsize;

  int64_t build(std::vector<int64_t>& ids, int32_t level, int64_t parent) {
    const int64_t me = (int64_t)p->cl.size();
    p->cl.emplace_back();
    {
      Cluster& c = p->cl.back();
      c.size = (int64_t)ids.size();
      c.level = level;
      c.parent = parent;
      for (int d = 0; d < 3; ++d) {
        double lo = vlo[3 * ids[0] + d], hi = vhi[3 * ids[0] + d];
        for (int64_t i : ids) {
          lo = std::min(lo, vlo[3 * i + d]);
          hi = std::max(hi, vhi[3 * i + d]);
        }
        c.lo[d] = lo;
        c.hi[d] = hi;
      }
      c.diam = norm3(c.hi[0] - c.lo[0], c.hi[1] - c.lo[1], c.hi[2] - c.lo[2]);
    }
    if ((int64_t)ids.size() <= leafsize) {
      p->cl[me].first = (int64_t)p->perm.size();
      p->perm.insert(p->perm.end(), ids.begin(), ids.end());
      return me;
    }
    // bisection of the centroid box along its longest side (first axis on ties)
    double clo[3], chi[3], ext[3];
    for (int d = 0; d < 3; ++d) {
      clo[d] = chi[d] = cen[3 * ids[0] + d];
      for (int64_t i : ids) {
        clo[d] = std::min(clo[d], cen[3 * i + d]);
        chi[d] = std::max(chi[d], cen[3 * i + d]);
      }
      ext[d] = chi[d] - clo[d];
    }
    int d = 0;
    for (int a = 1; a < 3; ++a)
      if (ext[a] > ext[d]) d = a;
    std::vector<int64_t> a, b;
    if (ext[d] > 0.0) {
      const double mid = 0.5 * (clo[d] + chi[d]);
      for (int64_t i : ids) (cen[3 * i + d] < mid ? a : b).push_back(i);
    } else {
      const size_t h = (ids.size() + 1) / 2;
      a.assign(ids.begin(), ids.begin() + h);
      b.assign(ids.begin() + h, ids.end());
    }
    std::vector<int64_t>().swap(ids);
    const int64_t start = (int64_t)p->perm.size();
    int64_t c0 = build(a, level + 1, me);
    int64_t c1 = build(b, level + 1, me);
    Cluster& c = p->cl[me];
    c.first = start;
    c.child[0] = c0;
    c.child[1] = c1;
    c.nchild = 2;
    return me;
  }
};

std::vector<double> direction_grid(int m) {
  std::vector<double> out((size_t)6 * m * m * 3);
  size_t k = 0;
  for (int f = 0; f < 6; ++f) {
    const int ax = f / 2;
    const double sgn = (f % 2 == 0) ? 1.0 : -1.0;
    int u = -1, w = -1;
    for (int a = 0; a < 3; ++a)
      if (a != ax) (u < 0 ? u : w) = a;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double c[3] = {0.0, 0.0, 0.0};
        c[ax] = sgn;
        c[u] = -1.0 + (double)(2 * i + 1) / (double)m;
        c[w] = -1.0 + (double)(2 * j + 1) / (double)m;
        const double r = norm3(c[0], c[1], c[2]);
        out[3 * k + 0] = c[0] / r;
        out[3 * k + 1] = c[1] / r;
        out[3 * k + 2] = c[2] / r;
        ++k;
      }
  }
  return out;
}

// nearest direction: squared distance summed x, y, z; lowest index within 1e-12 of the minimum
int32_t nearest(const double u[3], const std::vector<double>& D) {
  const size_t nd = D.size() / 3;
  std::vector<double> key(nd);
  double mn = INFINITY;
  for (size_t i = 0; i < nd; ++i) {
    const double dx = u[0] - D[3 * i], dy = u[1] - D[3 * i + 1], dz = u[2] - D[3 * i + 2];
    key[i] = dx * dx + dy * dy + dz * dz;
    mn = std::min(mn, key[i]);
  }
  for (size_t i = 0; i < nd; ++i)
    if (key[i] <= mn + 1e-12) return (int32_t)i;
  return 0;
}

struct BlockBuilder {
  Plan* p;
  void visit(int64_t t, int64_t s) {
    const Cluster& a = p->cl[t];
    const Cluster& b = p->cl[s];
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double g = std::max(std::max(0.0, b.lo[d] - a.hi[d]), a.lo[d] - b.hi[d]);
      acc += g * g;
    }
    const double dist = std::sqrt(acc);
    const double md = std::max(a.diam, b.diam);
    const double md2 = std::max(a.diam * a.diam, b.diam * b.diam);
    if (md <= p->eta * dist && p->kappa * md2 <= p->eta * dist) {
      int32_t c = 0;
      if (p->dir_m[a.level] != 0) {
        double dd[3];
        for (int d = 0; d < 3; ++d) dd[d] = 0.5 * (a.lo[d] + a.hi[d]) - 0.5 * (b.lo[d] + b.hi[d]);
        const double r = norm3(dd[0], dd[1], dd[2]);
        const double u[3] = {dd[0] / r, dd[1] / r, dd[2] / r};
        c = nearest(u, p->dirs[a.level]);
      }
      p->adm.push_back({t, s, c});
    } else if (a.leaf() || b.leaf()) {
      p->near.push_back({t, s});
    } else {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) visit(a.child[i], b.child[j]);
    }
  }
};

}  // namespace

int64_t Plan::slot_of(int64_t t, int32_t c) const {
  const auto& v = cl_slots[t];
  auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(c, (int64_t)-1));
  if (it == v.end() || it->first != c) return -1;
  return it->second;
}

std::string build_plan(const double* vertices, int64_t nv, const int32_t* triangles, int64_t n,
                       double kappa, int order, double eta, int leafsize, double eta1, Plan& p) {
  p = Plan();
  p.n = n;
  p.kappa = kappa;
  p.eta = eta;
  p.eta1 = eta1;
  p.order = order;
  p.leafsize = leafsize;
  p.k = order * order * order;
  (void)nv;

  // ---- cluster tree
  TreeBuilder tb;
  tb.V = vertices;
  tb.T = triangles;
  tb.p = &p;
  tb.leafsize = leafsize;
  tb.cen.resize(3 * n);
  tb.vlo.resize(3 * n);
  tb.vhi.resize(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double* a = vertices + 3 * (int64_t)triangles[3 * i + 0];
    const double* b = vertices + 3 * (int64_t)triangles[3 * i + 1];
    const double* c = vertices + 3 * (int64_t)triangles[3 * i + 2];
    for (int d = 0; d < 3; ++d) {
      tb.cen[3 * i + d] = ((a[d] + b[d]) + c[d]) / 3.0;
      tb.vlo[3 * i + d] = std::min(std::min(a[d], b[d]), c[d]);
      tb.vhi[3 * i + d] = std::max(std::max(a[d], b[d]), c[d]);
    }
  }
  {
    std::vector<int64_t> ids(n);
    for (int64_t i = 0; i < n; ++i) ids[i] = i;
    p.perm.reserve(n);
    tb.build(ids, 0, -1);
  }
  p.depth = 0;
  for (const auto& c : p.cl) p.depth = std::max(p.depth, c.level);

  // ---- directions (Remark on the construction of directions)
  p.dirs.resize(p.depth + 1);
  p.dir_m.assign(p.depth + 1, 0);
  for (int l = 0; l <= p.depth; ++l) {
    double dl = 0.0;
    for (const auto& c : p.cl)
      if (c.level == l) dl = std::max(dl, c.diam);
    if (kappa * dl <= eta1) {
      p.dirs[l] = {0.0, 0.0, 0.0};
      p.dir_m[l] = 0;
    } else {
      const int m = (int)std::ceil(std::sqrt(2.0) * kappa * dl / eta1);
      p.dirs[l] = direction_grid(m);
      p.dir_m[l] = m;
    }
  }
  p.sd.resize(p.depth);
  for (int l = 0; l < p.depth; ++l) {
    const size_t nd = p.dirs[l].size() / 3;
    p.sd[l].resize(nd);
    for (size_t c = 0; c < nd; ++c) p.sd[l][c] = nearest(&p.dirs[l][3 * c], p.dirs[l + 1]);
  }

  // ---- block tree
  BlockBuilder bb{&p};
  bb.visit(0, 0);

  // ---- slots: downward closure of the row and column occurrences
  const int64_t nc = (int64_t)p.cl.size();
  std::vector<std::set<int32_t>> rows(nc), cols(nc);
  for (const auto& b : p.adm) {
    rows[b.t].insert(b.c);
    cols[b.s].insert(b.c);
  }
  for (int64_t t = 0; t < nc; ++t) {  // preorder: parents before children
    const Cluster& c = p.cl[t];
    for (int i = 0; i < c.nchild; ++i) {
      for (int32_t d : rows[t]) rows[c.child[i]].insert(p.sd[c.level][d]);
      for (int32_t d : cols[t]) cols[c.child[i]].insert(p.sd[c.level][d]);
    }
  }
  std::vector<int64_t> lorder(nc);
  for (int64_t t = 0; t < nc; ++t) lorder[t] = t;
  std::stable_sort(lorder.begin(), lorder.end(),
                   [&](int64_t a, int64_t b) { return p.cl[a].level < p.cl[b].level; });
  p.cl_slots.assign(nc, {});
  for (int64_t t : lorder) {
    std::set<int32_t> all(rows[t]);
    all.insert(cols[t].begin(), cols[t].end());
    for (int32_t d : all) {
      const int64_t id = (int64_t)p.slots.size();
      p.slots.push_back({t, d});
      p.slot_row.push_back(rows[t].count(d) ? 1 : 0);
      p.slot_col.push_back(cols[t].count(d) ? 1 : 0);
      p.cl_slots[t].push_back({d, id});
    }
  }
  // ---- row / column block lists per slot
  const int64_t ns = (int64_t)p.slots.size();
  std::vector<std::vector<int64_t>> rl(ns), cll(ns);
  for (int64_t b = 0; b < (int64_t)p.adm.size(); ++b) {
    rl[p.slot_of(p.adm[b].t, p.adm[b].c)].push_back(b);
    cll[p.slot_of(p.adm[b].s, p.adm[b].c)].push_back(b);
  }
  p.row_ptr.assign(ns + 1, 0);
  p.col_ptr.assign(ns + 1, 0);
  for (int64_t q = 0; q < ns; ++q) {
    std::stable_sort(rl[q].begin(), rl[q].end(),
                     [&](int64_t a, int64_t b) { return p.adm[a].s < p.adm[b].s; });
    std::stable_sort(cll[q].begin(), cll[q].end(),
                     [&](int64_t a, int64_t b) { return p.adm[a].t < p.adm[b].t; });
    p.row_ptr[q + 1] = p.row_ptr[q] + (int64_t)rl[q].size();
    p.col_ptr[q + 1] = p.col_ptr[q] + (int64_t)cll[q].size();
    p.row_blk.insert(p.row_blk.end(), rl[q].begin(), rl[q].end());
    p.col_blk.insert(p.col_blk.end(), cll[q].begin(), cll[q].end());
  }
  return std::string();
}

}  // namespace dh2
