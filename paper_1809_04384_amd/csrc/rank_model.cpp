// Features of the learned rank predictor (host, from the hierarchy).
#include "rank_model.hpp"

#include <algorithm>
#include <cmath>

namespace dh2 {

void rank_features(const Plan& p, double tol, bool row, std::vector<float>& out) {
  const int64_t ns = (int64_t)p.slots.size();
  out.assign((size_t)ns * kRankFeatures, 0.0f);
  const std::vector<int64_t>& ptr = row ? p.row_ptr : p.col_ptr;
  const std::vector<int64_t>& blk = row ? p.row_blk : p.col_blk;
  // blocks of the ancestor lists, top-down: a slot inherits the totals of the
  // father's slots whose son direction is its direction (slots are sorted by level)
  std::vector<double> anc(ns, 0.0);
  for (int64_t q = 0; q < ns; ++q) {
    const Slot& s = p.slots[q];
    const int64_t tp = p.cl[s.t].parent;
    if (tp < 0) continue;
    for (const auto& pr : p.cl_slots[tp])
      if (p.son_dir(tp, pr.first) == s.c) anc[q] += anc[pr.second] + (double)(ptr[pr.second + 1] - ptr[pr.second]);
  }
  const double ltol = std::max(-16.0, std::log10(std::max(tol, 1e-300)));
  for (int64_t q = 0; q < ns; ++q) {
    const Slot& s = p.slots[q];
    const Cluster& c = p.cl[s.t];
    const double* d = p.dir(s.t, s.c);
    double lo = 1e300, hi = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double w = c.hi[a] - c.lo[a];
      lo = std::min(lo, w);
      hi = std::max(hi, w);
    }
    double other = 0.0;
    for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) {
      const AdmBlock& b = p.adm[blk[e]];
      other += (double)p.cl[row ? b.s : b.t].size;
    }
    float* f = &out[(size_t)q * kRankFeatures];
    f[0] = (float)std::log2((double)c.size);
    f[1] = (float)((double)c.level / std::max(1, p.depth));
    f[2] = (float)(p.kappa * c.diam);
    f[3] = (float)ltol;
    f[4] = (float)p.order;
    f[5] = (d[0] != 0.0 || d[1] != 0.0 || d[2] != 0.0) ? 1.0f : 0.0f;
    f[6] = (float)std::log2(1.0 + (double)(ptr[q + 1] - ptr[q]));
    f[7] = (float)std::log2(1.0 + anc[q]);
    f[8] = c.leaf() ? 1.0f : 0.0f;
    f[9] = (float)(hi > 0.0 ? lo / hi : 1.0);
    f[10] = (float)std::log2(1.0 + other);
    f[11] = (float)p.eta;
  }
}

}  // namespace dh2
