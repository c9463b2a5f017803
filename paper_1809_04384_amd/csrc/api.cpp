// C ABI (include/dh2.h) and host orchestration of the DH^2 build and matvec.
//
// Build phases (Boerm & Boerst, arXiv 1809.04384):
//   structure      cluster tree, directions, block tree           (Section 2; plan.cpp)
//   near field     dense inadmissible leaves                       (Definition of DH^2 matrices)
//   interpolation  leaf bases V_tc and transfers E_{t'c}           (Section 2, eq. (nested_apx))
//   basis weights  R_tc with V_tc = P_tc R_tc, bottom-up           (eq. (basis_weights_def))
//   block weights  omega_b = |R_tc S_b R_sc^*|_F                   (block-relative error control, Section 5)
//   total weights  Zhat_tc, top-down, rows and columns             (eq. (recomp_weight_full))
//   truncation     SVD -> Q_tc / F_{t'c}, ranks, C_tc, bottom-up   (Section 3.2, eq. (C_tc))
//   projection     Stilde_b = C_tc S_b C_{W,sc}^*                  (Lemma 'Projections')
// The couplings S_b are never stored: they are regenerated on the device in
// batches wherever a phase needs them.  All device work runs on the handle's
// stream; the host only builds descriptor lists and reads back the ranks of
// each level (they size the next level's products).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <set>
#include <atomic>
#include <thread>
#include <string>
#include <vector>

#include "../../include/dh2.h"
#include "kernels.hpp"
#include "matvec.hpp"
#include "plan.hpp"
#include "rank_model.hpp"
#include "scratch.hpp"

using namespace dh2;

namespace {

thread_local std::string g_err;

struct Fail {
  dh2_status st;
  std::string msg;
};

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw Fail{e_ == hipErrorOutOfMemory ? DH2_ERR_OOM : DH2_ERR_DEVICE,               \
                 std::string(#x) + " failed: " + hipGetErrorString(e_)};                 \
  } while (0)

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2) P'^2) on [-1,1], halved
  }
}

QuadTab make_quad() {
  QuadTab q{};
  // 7-point rule of Radon (degree 5): centroid and two orbits (a,a,1-2a)
  const double s15 = std::sqrt(15.0);
  const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
  const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
  const double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a, a, 1 - 2 * a}, {a, 1 - 2 * a, a},
                            {1 - 2 * a, a, a},         {b, b, 1 - 2 * b}, {b, 1 - 2 * b, b},
                            {1 - 2 * b, b, b}};
  const double ws[7] = {9.0 / 40.0, wa, wa, wa, wb, wb, wb};
  for (int i = 0; i < 7; ++i) {
    for (int d = 0; d < 3; ++d) q.b7[i][d] = pts[i][d];
    q.w7[i] = ws[i];
  }
  // 16-point rule: 4 x 4 Gauss-Legendre on the square, Duffy-collapsed
  double u[4], wu[4];
  gauss_legendre01(4, u, wu);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * i + j;
      q.b16[k][0] = 1.0 - u[i];
      q.b16[k][1] = u[i] * (1.0 - u[j]);
      q.b16[k][2] = u[i] * u[j];
      q.w16[k] = 2.0 * wu[i] * wu[j] * u[i];
    }
  // the paper's rule of order 3: 3 x 3 Gauss-Legendre, Duffy-collapsed
  double u3[3], wu3[3];
  gauss_legendre01(3, u3, wu3);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int k = 3 * i + j;
      q.b9[k][0] = 1.0 - u3[i];
      q.b9[k][1] = u3[i] * (1.0 - u3[j]);
      q.b9[k][2] = u3[i] * u3[j];
      q.w9[k] = 2.0 * wu3[i] * wu3[j] * u3[i];
    }
  return q;
}

ChebTab make_cheb(int m) {
  ChebTab c{};
  c.m = m;
  for (int j = 0; j < m; ++j) c.node[j] = std::cos((2 * j + 1) * M_PI / (2.0 * m));
  for (int j = 0; j < m; ++j) {
    double den = 1.0;
    for (int l = 0; l < m; ++l)
      if (l != j) den *= (c.node[j] - c.node[l]);
    c.inv_den[j] = 1.0 / den;
  }
  return c;
}

}  // namespace

// ---------------------------------------------------------------------------
struct dh2_plan_s {
  Plan plan;
};

struct dh2_problem {
  Plan plan;
  int precision = DH2_FP64;
  hipStream_t stream = nullptr;
  int max_nrhs = 16;
  double tol = 0;
  int norm_mode = 0;
  int rank_mode = 0;       // DH2_RANKS_EXACT / DH2_RANKS_LEARNED
  int sketch_rank = 0;     // fixed predicted rank of every slot (0 = the predictor's)
  int autotune = 0;        // dh2_options.autotune
  int weights_mode = 0;    // dh2_options.weights
  int quadrature = 0;      // dh2_options.quadrature
  int mv_var[4] = {0, 0, 0, 0};  // block-row pipeline shape: near / coupling, nrhs <= 16 / > 16
  int device = 0;
  size_t ws_bytes = 0;
  std::vector<void*> allocs;
  dh2_stats stats{};

  // device data kept after the build
  int64_t* perm_d = nullptr;
  double* box_d = nullptr;
  double* dirs_d = nullptr;
  std::vector<int64_t> dir_off;        // first global direction index of each level
  void* near_d = nullptr;              // near-field blocks
  std::vector<int64_t> near_off;
  void* V_d = nullptr;                 // leaf bases (FP64)
  std::vector<int64_t> V_off;          // per slot (-1 if none)
  void* E_d = nullptr;                 // transfers (FP64), per slot 2 k x k
  std::vector<int64_t> E_off;
  std::vector<int32_t> rank_row, rank_col;  // -1 if not in the set
  std::vector<int32_t> pred_row, pred_col;  // learned-rank form: predicted ranks
  std::vector<std::vector<double>> sig_row, sig_col;
  std::vector<double> omega;
  z64* R_d = nullptr;                  // basis weights, per slot k x k (rows rR)
  z64* Zr_d = nullptr;                 // total weights (rows, columns), per slot k x k
  z64* Zc_d = nullptr;
  std::vector<int32_t> rR, rZr, rZc;
  ChebTab cheb{};
  // compressed representation
  std::vector<z64*> Qr_ptr, Qc_ptr;   // Qhat per slot (m x rank, column-major)
  std::vector<int32_t> Qr_m, Qc_m;
  void* St_d = nullptr;  std::vector<int64_t> St_off;   // Stilde_b (element type of the handle)
  int64_t St_total = 0;
  std::vector<void*> Qr32, Qc32;      // FP32 handles: complex64 copies of Qhat used by the matvec
  // matvec schedule.  A view holds the device addresses one product uses: the
  // descriptor lists and the staging buffers they point into (gathered X Xp,
  // its row-major copy XT, Y in cluster order Yp, the row-major slot vectors
  // xhT).  `own` points into the handle's staging arena; `scr` holds the same
  // descriptors relocated into the library's static scratch array (the
  // allocation-free product), when the arena fits there.
  struct MvView {
    MvOut* outs = nullptr;
    MvTerm* terms = nullptr;
    MfRow* near_rows = nullptr;
    MfRow* coup_rows = nullptr;
    SlotT* xh_tr = nullptr;
    void* Xp = nullptr;
    void* XT = nullptr;
    void* Yp = nullptr;
    void* xhT = nullptr;
  };
  MvView mv_own, mv_scr;
  bool has_scr = false;
  char* stage_d = nullptr;               // staging arena of the handle's own products
  size_t stage_bytes = 0;
  struct Phase { int64_t out_begin, out_end; int group; };
  std::vector<Phase> mv_phases;     // groups: 1 forward, 2 coupling, 3 backward, 5 leaf output

  int64_t n_coup_rows = 0;

  NearSeg* near_segs_d = nullptr;
  int64_t n_near_rows = 0;
  // matrix-core block rows (every right-hand-side count): one per leaf
  // (segments near_segs_d) and one per row slot (segments coup_mf_segs_d)
  XcdSplit near_split{}, coup_split{};  // per-XCD ranges of the two row lists
  NearSeg* coup_mf_segs_d = nullptr;
  void* zero16_d = nullptr;             // 16 zero elements, never written after the build
  int64_t n_xh_tr = 0;
  int64_t n_xh_rows = 0;            // rows of the row-major slot vectors xhT
  int64_t near_matvec_bytes = 0;    // matrix bytes streamed by the near-field kernel

  // Stream-ordered allocations on the handle's stream: a release does not wait
  // for the whole device (builds of other handles on other streams go on)
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    HIPCHK(hipMallocAsync(&p, count * sizeof(T), stream));
    allocs.push_back(p);
    return (T*)p;
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) {
      (void)hipFreeAsync(p, stream);
      allocs.erase(it);
    }
  }
  // host bytes of pending asynchronous uploads, kept alive until the next sync()
  std::vector<std::vector<char>> pending_host;

  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    if (!v.empty()) {
      pending_host.emplace_back((const char*)v.data(), (const char*)v.data() + v.size() * sizeof(T));
      HIPCHK(hipMemcpyAsync(p, pending_host.back().data(), v.size() * sizeof(T),
                            hipMemcpyHostToDevice, stream));
    }
    return p;
  }
  bool own_stream = false;               // created by dh2_build_many, destroyed with the handle
  ~dh2_problem() {
    // Products may still run on streams other than the handle's (per-call
    // streams of dh2_matvec_stream, branches of a batch graph): wait for the
    // whole device before the memory goes back to the pool.
    (void)hipDeviceSynchronize();
    for (void* p : allocs) (void)hipFreeAsync(p, stream);
    if (stream) (void)hipStreamSynchronize(stream);
    else (void)hipDeviceSynchronize();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  void sync() {
    HIPCHK(hipStreamSynchronize(stream));
    pending_host.clear();
  }
  void check_launch() { HIPCHK(hipGetLastError()); }
};

namespace {

// ---- matvec schedule (begin) ----
// Order of the rows of a block-row launch (k_mv_rows_mfma: XCD x runs the
// list entries [off[x], off[x + 1]) in order): the rows, longest first, are
// dealt to the 8 XCDs in snake order (the last partial round forward), so the
// per-XCD counts and totals are balanced and each XCD starts with its longest
// rows.  Returns the row indices in list order and fills the split.  (Rows in
// cluster order cut into 8 equal-work ranges, so that neighbouring clusters
// share right-hand-side rows in one XCD's L2, ran the near field at n = 131k
// in 10.8 ms against 9.3 ms.)
std::vector<int64_t> xcd_balanced_order(const std::vector<double>& work, XcdSplit& split) {
  const int64_t n = (int64_t)work.size();
  std::vector<int64_t> by(n);
  std::iota(by.begin(), by.end(), (int64_t)0);
  std::stable_sort(by.begin(), by.end(), [&](int64_t a, int64_t b) { return work[a] > work[b]; });
  std::vector<std::vector<int64_t>> share(8);
  const int64_t full = n / 8 * 8;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t r = i / 8, pos = i % 8;
    const int64_t x = (i < full && (r & 1)) ? 7 - pos : pos;
    share[x].push_back(by[i]);
  }
  std::vector<int64_t> out;
  out.reserve(n);
  split.width = 0;
  for (int x = 0; x < 8; ++x) {
    split.off[x] = (int32_t)out.size();
    split.width = std::max(split.width, (int32_t)share[x].size());
    out.insert(out.end(), share[x].begin(), share[x].end());
  }
  split.off[8] = (int32_t)out.size();
  return out;
}

// ---- matvec schedule (end) ----

typedef z64 C64;

// slot-level bookkeeping used during the build
struct SlotInfo {
  int64_t t;
  int32_t c, level;
  bool leaf;
  int64_t child_slot[2] = {-1, -1};
  int32_t nrows;              // #t
  int64_t row0;               // first cluster-order position
};

struct Builder {
  dh2_problem& h;
  Plan& p;
  int k;
  int64_t ns;
  ChebTab ct;
  std::vector<SlotInfo> si;
  std::vector<int32_t> rR;                 // rows of R per slot
  C64* R_d = nullptr;                      // per slot k x k: the compacted R of an unpivoted
                                           // Householder QR, zero left of its diagonal (GemmDesc.tri)
  C64* Zr_d = nullptr;                     // per slot k x k (row pass)
  C64* Zc_d = nullptr;                     // per slot k x k (column pass)
  std::vector<int32_t> rZr, rZc;
  std::vector<C64*> Cr_ptr, Cc_ptr;                    // C_tc rank x k per slot
  std::vector<void*> keep_rc;                          // their allocations (freed after the build)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t* cnt_d = nullptr;                            // per slot: rows of a compacted fold

  // read the compacted row counts of the given slots
  void read_counts(const std::vector<int64_t>& qs, std::vector<int32_t>& dst) {
    h.sync();
    if (qs.empty()) return;
    std::vector<int32_t> all(ns);
    HIPCHK(hipMemcpy(all.data(), cnt_d, ns * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t q : qs) dst[q] = all[q];
  }
  std::vector<int64_t> slot_by_level_begin;            // slots sorted by level

  Builder(dh2_problem& hh) : h(hh), p(hh.plan) {}

  C64* Rp(int64_t q) { return R_d + (size_t)q * k * k; }
  // leaf slots narrower than k keep projected total weights (see total_weights)
  bool projected(int64_t q) const { return si[q].leaf && si[q].nrows < k; }
  C64* Zp(bool row, int64_t q) { return (row ? Zr_d : Zc_d) + (size_t)q * k * k; }
  int64_t gdir(int64_t t, int32_t c) { return h.dir_off[p.cl[t].level] + c; }
  int child_index(int64_t t) {
    const Cluster& par = p.cl[p.cl[t].parent];
    return par.child[0] == t ? 0 : 1;
  }
  C64* Ep(int64_t parent_slot, int ci) { return (C64*)h.E_d + h.E_off[parent_slot] + (size_t)ci * k * k; }

  template <class T>
  T* upload_tmp(const std::vector<T>& v, std::vector<void*>& tmp) {
    T* d = h.upload(v);
    tmp.push_back(d);
    return d;
  }
  // Batched GEMMs launched with grids of exactly their tiles: descriptors are
  // grouped by (row tiles, column tiles) of 32, one launch per group, so no
  // workgroup is started for a tile outside its product.
  // Batched complex products, grouped by tile counts.  force64: on the FP64
  // kernel whatever the handle's precision.
  // Flops of one product: 8 per complex multiply-add; a Hermitian product
  // (upper) counts its upper triangle, a trapezoidal operand (tri) the
  // products outside its zeros: sum over the rows i (columns n) of K - i
  // (K - n).  At most one tri bit is set per descriptor.
  static double gemm_desc_flops(const GemmDesc& g) {
    if (g.upper) return 4.0 * g.N * (g.N + 1.0) * g.K;
    auto trap = [](double rows, double K) {     // sum over i < min(rows, K) of K - i
      const double r = std::min(rows, K);
      return r * K - r * (r - 1.0) / 2.0;
    };
    if (g.tri & 1) return 8.0 * g.N * trap(g.M, g.K);
    if (g.tri & 2) return 8.0 * g.M * trap(g.N, g.K);
    return 8.0 * g.M * g.N * g.K;
  }
  void gemm(const std::vector<GemmDesc>& gd, std::vector<void*>& tmp, bool force64 = false) {
    if (gd.empty()) return;
    auto key = [](const GemmDesc& g) {
      return std::min((g.M + 31) / 32, 16) * 17 + std::min((g.N + 31) / 32, 16);
    };
    std::vector<GemmDesc> v;
    v.reserve(gd.size());
    for (const GemmDesc& g : gd)
      if (g.M > 0 && g.N > 0) v.push_back(g);
    if (v.empty()) return;
    std::stable_sort(v.begin(), v.end(), [&](const GemmDesc& a, const GemmDesc& b) { return key(a) < key(b); });
    for (const GemmDesc& g : v) h.stats.gemm_flops += gemm_desc_flops(g);
    const GemmDesc* d = upload_tmp(v, tmp);
    size_t i0 = 0;
    while (i0 < v.size()) {
      const int kk = key(v[i0]);
      size_t i1 = i0;
      int maxM = 0, maxN = 0;
      while (i1 < v.size() && key(v[i1]) == kk) {
        maxM = std::max(maxM, v[i1].M);
        maxN = std::max(maxN, v[i1].N);
        ++i1;
      }
      h.stats.gemm_launches += (int64_t)((i1 - i0 + 65534) / 65535);
      if (force64)
        launch_gemm<double>(d + i0, (int64_t)(i1 - i0), maxM, maxN, h.stream);
      else if (h.precision == DH2_BF16X3)
        launch_gemm_bf16x3(d + i0, (int64_t)(i1 - i0), maxM, maxN, h.stream);
      else if (h.precision == DH2_FP32)
        launch_gemm_f32(d + i0, (int64_t)(i1 - i0), maxM, maxN, h.stream);
      else
        launch_gemm<double>(d + i0, (int64_t)(i1 - i0), maxM, maxN, h.stream);
      i0 = i1;
    }
  }
  // QR flops of fold tasks (see dh2_stats.qr_flops); pieces indexed by the tasks
  void count_folds(const std::vector<FoldTask>& ts, const std::vector<FoldPiece>& ps) {
    for (const FoldTask& t : ts) {
      double M = 0;
      for (int32_t e = t.piece_begin; e < t.piece_end; ++e) M += ps[e].rows;
      const double n = t.n;
      double f = 8.0 * M * n * n;
      if (t.init_zero) {
        const double r = std::min(M, n);
        f -= 8.0 / 3.0 * r * r * r;
      }
      h.stats.qr_flops += f;
    }
  }
  int64_t n_coupling_gen = 0;   // S_b generated during the build
  int64_t n_coupling_fused = 0; // of which inside products (k_gemm_coupling, never stored)
  void free_tmp(std::vector<void*>& tmp) {
    h.sync();
    for (void* x : tmp) h.release(x);
    tmp.clear();
  }
  // Release without waiting: the frees are stream-ordered after the batch's
  // kernels, so the host may prepare the next batch while they run; every
  // few batches the stream is synchronised to drop the host copies of the
  // uploaded descriptors.
  void free_tmp_async(std::vector<void*>& tmp, int64_t batch_index) {
    for (void* x : tmp) h.release(x);
    tmp.clear();
    if (batch_index % 8 == 7) h.sync();
  }

  // ------------------------------------------------------------------
  void setup_slots() {
    k = p.k;
    ns = (int64_t)p.slots.size();
    ct = make_cheb(p.order);
    si.resize(ns);
    for (int64_t q = 0; q < ns; ++q) {
      const Slot& s = p.slots[q];
      const Cluster& c = p.cl[s.t];
      si[q].t = s.t;
      si[q].c = s.c;
      si[q].level = c.level;
      si[q].leaf = c.leaf();
      si[q].nrows = (int32_t)c.size;
      si[q].row0 = c.first;
      if (!c.leaf())
        for (int i = 0; i < 2; ++i) si[q].child_slot[i] = p.slot_of(c.child[i], p.son_dir(s.t, s.c));
    }
  }

  // parents (inherited contributions) of slot q within a set (row or column flags)
  std::vector<int64_t> parents_of(int64_t q, const std::vector<uint8_t>& flag) {
    std::vector<int64_t> out;
    const int64_t t = si[q].t;
    const int64_t tp = p.cl[t].parent;
    if (tp < 0) return out;
    for (const auto& pr : p.cl_slots[tp]) {
      const int32_t cp = pr.first;
      if (p.son_dir(tp, cp) == si[q].c && flag[pr.second]) out.push_back(pr.second);
    }
    return out;
  }

  // ------------------------------------------------------------------
  void interpolation() {
    // leaf bases
    std::vector<LeafDesc> ld;
    h.V_off.assign(ns, -1);
    int64_t voff = 0;
    for (int64_t q = 0; q < ns; ++q)
      if (si[q].leaf) {
        h.V_off[q] = voff;
        ld.push_back({si[q].row0, si[q].nrows, (int32_t)si[q].t, gdir(si[q].t, si[q].c), voff});
        voff += (int64_t)si[q].nrows * k;
      }
    h.V_d = h.alloc<C64>(voff);
    std::vector<void*> tmp;
    launch_leaf_basis<double>(upload_tmp(ld, tmp), (int64_t)ld.size(), ct, p.kappa, x7, w7, nq_far, h.box_d,
                              h.dirs_d, h.V_d, h.stream);
    h.check_launch();
    // transfers
    std::vector<TransDesc> td;
    h.E_off.assign(ns, -1);
    int64_t eoff = 0;
    for (int64_t q = 0; q < ns; ++q)
      if (!si[q].leaf) {
        h.E_off[q] = eoff;
        const Cluster& c = p.cl[si[q].t];
        for (int i = 0; i < 2; ++i) {
          td.push_back({(int32_t)c.child[i], (int32_t)si[q].t, gdir(si[q].t, si[q].c),
                        h.dir_off[c.level + 1] + p.son_dir(si[q].t, si[q].c), eoff});
          eoff += (int64_t)k * k;
        }
      }
    h.E_d = h.alloc<C64>(eoff);
    launch_transfer<double>(upload_tmp(td, tmp), (int64_t)td.size(), ct, p.kappa, h.box_d, h.dirs_d,
                            h.E_d, h.stream);
    h.check_launch();
    free_tmp(tmp);
  }

  const double* x7 = nullptr;   // far rule: points and weights per triangle (nq_far each)
  const double* w7 = nullptr;
  int nq_far = 7;

  // ------------------------------------------------------------------
  // basis weights, bottom-up (eq. (basis_weights_def))
  void basis_weights() {
    rR.assign(ns, 0);
    R_d = h.alloc<C64>((size_t)ns * k * k);
    for (int l = p.depth; l >= 0; --l) {
      std::vector<int64_t> qs;
      for (int64_t q = 0; q < ns; ++q)
        if (si[q].level == l) qs.push_back(q);
      size_t i0 = 0;
      while (i0 < qs.size()) {
        std::vector<GemmDesc> gd;
        std::vector<FoldPiece> pieces;
        std::vector<FoldTask> tasks;
        size_t used = 0;
        size_t i1 = i0;
        for (; i1 < qs.size(); ++i1) {
          const int64_t q = qs[i1];
          if (!si[q].leaf && used + (size_t)2 * k * k * sizeof(C64) > ws_bytes && i1 > i0) break;
          FoldTask tk{};
          tk.R = Rp(q);
          tk.n = k;
          tk.ldr = k;
          tk.init_zero = 1;
          tk.compact = 1;
          tk.count = cnt_d + q;
          tk.piece_begin = (int32_t)pieces.size();
          if (si[q].leaf) {
            pieces.push_back({(C64*)h.V_d + h.V_off[q], si[q].nrows, si[q].nrows});
          } else {
            int rows = 0;
            for (int i = 0; i < 2; ++i) {
              const int64_t cq = si[q].child_slot[i];
              const int r = rR[cq];
              C64* dst = (C64*)(ws + used);
              used += (size_t)std::max(r, 1) * k * sizeof(C64);
              if (r > 0) {
                GemmDesc g{};
                g.A = Rp(cq); g.lda = k; g.M = r; g.K = k; g.tri = 1;
                g.B = Ep(q, i); g.ldb = k; g.N = k;
                g.C = dst; g.ldc = r;
                g.alpha_re = 1.0;
                gd.push_back(g);
                pieces.push_back({dst, r, r});
              }
              rows += r;
            }
            (void)rows;
          }
          tk.piece_end = (int32_t)pieces.size();
          tasks.push_back(tk);
        }
        std::vector<void*> tmp;
        gemm(gd, tmp);
        count_folds(tasks, pieces);
        ++h.stats.batches_basis_weights;
        launch_fold<double>(upload_tmp(tasks, tmp), (int64_t)tasks.size(), upload_tmp(pieces, tmp), k,
                            h.stream);
        h.check_launch();
        free_tmp(tmp);
        i0 = i1;
      }
      read_counts(qs, rR);
    }
  }

  // generate S_b for a list of blocks into the workspace at dst
  void gen_couplings(const std::vector<int64_t>& blocks, C64* dst, std::vector<void*>& tmp) {
    std::vector<CoupDesc> cd(blocks.size());
    for (size_t i = 0; i < blocks.size(); ++i) {
      const AdmBlock& b = p.adm[blocks[i]];
      cd[i] = {(int32_t)b.t, (int32_t)b.s, gdir(b.t, b.c)};
    }
    n_coupling_gen += (int64_t)cd.size();
    launch_coupling<double>(upload_tmp(cd, tmp), (int64_t)cd.size(), ct, p.kappa, h.box_d, h.dirs_d,
                            dst, h.stream);
    h.check_launch();
  }
  // Products with S_b evaluated inside them (k_gemm_coupling), in each form's
  // own product arithmetic (FP64, FP32 or split-BF16x3 matrix cores).
  bool fuse_couplings() const { return true; }
  CoupGemmDesc coup_desc(int64_t b, const C64* A, int lda, int M, int conj, int tri, C64* C, int ldc,
                         double alpha) {
    const AdmBlock& ab = p.adm[b];
    CoupGemmDesc c{};
    c.A = A; c.lda = lda; c.M = M;
    c.t = (int32_t)ab.t; c.s = (int32_t)ab.s; c.dir = gdir(ab.t, ab.c);
    c.conj = conj; c.tri = tri;
    c.C = C; c.ldc = ldc;
    c.alpha = alpha;
    return c;
  }
  // Grouped by row count: products with M <= 32 and <= 64 get the kernel
  // with 32- and 64-row chunks, the rest 128-row chunks.
  void gemm_coupling(const std::vector<CoupGemmDesc>& cd, std::vector<void*>& tmp) {
    if (cd.empty()) return;
    std::vector<CoupGemmDesc> grp[3];
    for (const CoupGemmDesc& c : cd) {
      if (c.M <= 0) continue;
      GemmDesc g{};
      g.M = c.M; g.N = k; g.K = k; g.tri = c.tri;
      h.stats.gemm_flops += gemm_desc_flops(g);
      const int gi = c.M <= 32 ? 0 : (c.M <= 64 ? 1 : 2);
      const int64_t chunks = gi < 2 ? 1 : (c.M + 127) / 128;   // S_b is evaluated once per chunk
      n_coupling_gen += chunks;
      n_coupling_fused += chunks;
      grp[gi].push_back(c);
    }
    for (int gi = 0; gi < 3; ++gi) {
      if (grp[gi].empty()) continue;
      h.stats.gemm_launches += (int64_t)((grp[gi].size() + 65534) / 65535);
      launch_gemm_coupling(upload_tmp(grp[gi], tmp), (int64_t)grp[gi].size(), 1 << gi, ct, p.kappa, h.box_d,
                           h.dirs_d, h.precision == DH2_FP32 ? 1 : (h.precision == DH2_BF16X3 ? 2 : 0), h.stream);
    }
    h.check_launch();
  }

  // ------------------------------------------------------------------
  // block weights omega_b = |R_tc S_b R_sc^*|_F, or its spectral norm
  void block_weights() {
    const int64_t nb = (int64_t)p.adm.size();
    double* om_d = h.alloc<double>(nb);
    const size_t per = (size_t)3 * k * k * sizeof(C64);
    const int64_t batch = std::max<int64_t>(1, (int64_t)(ws_bytes / per));
    for (int64_t b0 = 0; b0 < nb; b0 += batch) {
      const int64_t b1 = std::min(nb, b0 + batch);
      std::vector<int64_t> blocks;
      for (int64_t b = b0; b < b1; ++b) blocks.push_back(b);
      C64* S = (C64*)ws;
      C64* T1 = S + (size_t)(b1 - b0) * k * k;
      C64* T2 = T1 + (size_t)(b1 - b0) * k * k;
      std::vector<void*> tmp;
      ++h.stats.batches_block_weights;
      gen_couplings(blocks, S, tmp);
      std::vector<GemmDesc> g1, g2;
      std::vector<FrobDesc> fd;
      for (int64_t b = b0; b < b1; ++b) {
        const AdmBlock& a = p.adm[b];
        const int64_t qt = p.slot_of(a.t, a.c), qs = p.slot_of(a.s, a.c);
        const int rt = rR[qt], rs = rR[qs];
        const size_t i = (size_t)(b - b0);
        GemmDesc g{};
        g.A = Rp(qt); g.lda = k; g.M = rt; g.K = k; g.tri = 1;
        g.B = S + i * k * k; g.ldb = k; g.N = k;
        g.C = T1 + i * k * k; g.ldc = std::max(rt, 1);
        g.alpha_re = 1.0;
        g1.push_back(g);
        GemmDesc g2d{};
        g2d.A = T1 + i * k * k; g2d.lda = std::max(rt, 1); g2d.M = rt; g2d.K = k;
        g2d.B = Rp(qs); g2d.ldb = k; g2d.N = rs; g2d.opB = 2; g2d.tri = 2;
        g2d.C = T2 + i * k * k; g2d.ldc = std::max(rt, 1);
        g2d.alpha_re = 1.0;
        g2.push_back(g2d);
        fd.push_back({T2 + i * k * k, rt, rs, std::max(rt, 1), 0, b});
      }
      gemm(g1, tmp);
      gemm(g2, tmp);
      if (h.norm_mode == 0)
        launch_frob<double>(upload_tmp(fd, tmp), (int64_t)fd.size(), om_d, h.stream);
      else
        spectral_weights(blocks, S, T1, T2, om_d, tmp);
      h.check_launch();
      free_tmp(tmp);
    }
    h.omega.resize(nb);
    if (nb) HIPCHK(hipMemcpy(h.omega.data(), om_d, nb * sizeof(double), hipMemcpyDeviceToHost));
    h.release(om_d);
  }

  // omega_b = |M_b|_2 for M_b = R_tc S_b R_sc^* (rt x rs, column-major in T2 with
  // leading dimension max(rt, 1)), the i-th block of the list at position i.  The Gram matrix of the
  // smaller side is squared kSpecSquarings times, each time after an exact
  // power-of-two normalisation, so Gs ~ G^(2^j); a column of Gs then spans the
  // dominant eigenvector up to (lambda_2 / lambda_1)^(2^j) and its Rayleigh
  // quotient gives |M_b|_2 (k_spec_final).  S and T1 hold the two ping-pong
  // copies of the Gram power.
  static constexpr int kSpecSquarings = 10;
  void spectral_weights(const std::vector<int64_t>& blocks, C64* S, C64* T1, C64* T2, double* om_d,
                        std::vector<void*>& tmp) {
    const size_t kk = (size_t)k * k;
    std::vector<GemmDesc> gram, sq[2];
    std::vector<FrobDesc> sc[2];
    std::vector<SpecDesc> sd;
    for (size_t i = 0; i < blocks.size(); ++i) {
      const int64_t b = blocks[i];
      const AdmBlock& a = p.adm[b];
      const int rt = rR[p.slot_of(a.t, a.c)], rs = rR[p.slot_of(a.s, a.c)];
      const int side = rs <= rt ? 0 : 1;
      const int pp = side == 0 ? rs : rt;
      const int ldm = std::max(rt, 1), ldg = std::max(pp, 1);
      C64* M = T2 + i * kk;
      C64* G[2] = {S + i * kk, T1 + i * kk};
      if (rt > 0 && rs > 0) {
        GemmDesc g{};
        g.A = M; g.lda = ldm;
        g.B = M; g.ldb = ldm;
        if (side == 0) {            // M^* M
          g.opA = 2; g.M = rs; g.K = rt; g.N = rs;
        } else {                    // M M^*
          g.opB = 2; g.M = rt; g.K = rs; g.N = rt;
        }
        g.C = G[0]; g.ldc = ldg;
        g.alpha_re = 1.0;
        gram.push_back(g);
        for (int j = 0; j < 2; ++j) {
          sc[j].push_back({G[j], pp, pp, ldg, 0, 0});
          GemmDesc q{};
          q.A = G[j]; q.lda = ldg; q.M = pp; q.K = pp;
          q.B = G[j]; q.ldb = ldg; q.N = pp;
          q.C = G[1 - j]; q.ldc = ldg;
          q.alpha_re = 1.0;
          sq[j].push_back(q);
        }
      }
      sd.push_back({G[kSpecSquarings % 2], M, rt > 0 && rs > 0 ? pp : 0, ldg, rt, rs, ldm, side, b});
    }
    gemm(gram, tmp);
    const FrobDesc* scd[2] = {upload_tmp(sc[0], tmp), upload_tmp(sc[1], tmp)};
    for (int j = 0; j < kSpecSquarings; ++j) {
      launch_scale_pow2(scd[j % 2], (int64_t)sc[j % 2].size(), h.stream);
      gemm(sq[j % 2], tmp);
    }
    launch_spec_final(upload_tmp(sd, tmp), (int64_t)sd.size(), om_d, h.stream);
  }

  // ------------------------------------------------------------------
  // total weights, top-down (eq. (recomp_weight_full)).  row = true: rows of
  // Z_tc^* are omega_b^{-1} R_sc S_b^* (blocks of row(t,c)) and Zhat_{t+c+} E_{tc+}^*
  // (inherited); row = false: the same for G^* with omega_b^{-1} R_tc S_b.
  // A leaf's Zhat enters nothing but its own truncation, and only through
  // V_tc Zhat^H, whose Gram matrix is (Z^* V^H)^H (Z^* V^H): every stacked row
  // of a leaf slot with #t < k is multiplied by V_tc^H before the fold, which
  // then factors an M x #t matrix instead of an M x k one.  The slot keeps that #t x #t
  // factor ("projected total weight", rows rZ) in place of Zhat; the
  // truncation's SVD of V Zhat^H is its SVD (same singular values and left
  // singular vectors).
  // Stacked rows of the total-weight passes: a piece (block or inherited
  // rows) of a slot, and a batch item (pieces [e0, e1) of slot a of the level).
  struct PieceSrc { int64_t q; int64_t blockid; int64_t parent; int rows; };
  struct Item { size_t a; size_t e0, e1; };

  // Gram form of the block and total weights: used when the handle asks for
  // it and the tolerance is at least kGramMinTol (the Gram matrix holds the squares of
  // the singular values, so those below about 1e-8 of the largest lose their
  // relative accuracy; the rank rule then looks at singular values of at
  // least tol times the largest).
  static constexpr double kGramMinTol = 1e-7;
  bool use_gram() const { return h.weights_mode == DH2_WEIGHTS_GRAM && h.tol >= kGramMinTol; }

  // ------------------------------------------------------------------
  // Gram form of the block and total weights (dh2_options.weights = GRAM).
  // The total weight of a slot enters the truncation only through
  // Zhat^H Zhat, the Gram matrix of its stacked rows, and a Gram matrix is a
  // sum: G_tc = sum over the blocks b of row (t, c) of omega_b^-2
  // (R_sc S_b^H)^H (R_sc S_b^H), plus E G_{t+c+} E^H for the inherited rows
  // (the same for the column side with R_tc S_b).  The block part needs no
  // parent, so it is accumulated before the top-down pass, in two passes over
  // the blocks: in column-slot order (the block weights: R_tc S_b, then
  // omega_b from R_tc S_b R_sc^H, then the column Gram matrices of those same
  // rows scaled by omega_b^-1) and in row-slot order (R_sc S_b^H / omega_b and
  // the row Gram matrices).  In each pass the rows of a batch are formed into
  // per-slot segments of consecutive blocks, and the segments' Gram matrices
  // are formed on the FP64 matrix cores and added to their slots'.  The
  // top-down pass then adds the inherited rows Zhat_{t+c+} E^H level by level,
  // projects leaf slots narrower than k (V G V^H), and factors every Gram
  // matrix by pivoted Cholesky (Zhat = R).  S_b is generated twice for block
  // and total weights (instead of three times), and R_tc S_b formed once.
  static constexpr int64_t kSegRows = 1024;

  // Stacked rows of one slot side for the blocks of a batch (in slot order):
  // the row products into segments of at most kSegRows rows (a run of one
  // slot's blocks, longer runs cut), and one Gram product per segment, all in
  // one launch: a slot with a single segment in the batch adds it to its
  // Gram matrix directly, the segments of a slot with several go to
  // temporaries that k_gram_sum then adds.  col: column side (R_tc S_b,
  // addresses written into colpiece / colld per block), else row side
  // (R_sc S_b^H / omega_b).  scale_later: the rows get their omega_b^-1 by a
  // separate pass once omega_b is known (rw, ss).  S: the batch's stored
  // couplings, or nullptr to form them inside the products (cpieces).
  struct GramRows {
    std::vector<GemmDesc> pieces, gram;
    std::vector<CoupGemmDesc> cpieces;     // the pieces with S_b formed inside (S == nullptr)
    std::vector<GramSumTask> sums;
    std::vector<const void*> srcs;
    std::vector<RowWeightTask> rw;
    std::vector<SegScaleTask> ss;
  };
  GramRows stack_rows(bool col, const std::vector<int64_t>& blocks, C64* S, C64* P, double* Wt, bool scale_later,
                      std::vector<C64*>* colpiece, std::vector<int32_t>* colld, std::vector<void*>& tmp) {
    const size_t kk = (size_t)k * k;
    GramRows out;
    std::vector<size_t> temp_of;    // Gram product writing each temporary
    size_t poff = 0;
    size_t e = 0;
    while (e < blocks.size()) {
      const AdmBlock& a0 = p.adm[blocks[e]];
      const int64_t q = col ? p.slot_of(a0.s, a0.c) : p.slot_of(a0.t, a0.c);
      size_t end = e;
      while (end < blocks.size()) {
        const AdmBlock& ab = p.adm[blocks[end]];
        if ((col ? p.slot_of(ab.s, ab.c) : p.slot_of(ab.t, ab.c)) != q) break;
        ++end;
      }
      std::vector<GemmDesc> segs;
      while (e < end) {
        // one segment: blocks [e, f) of this slot
        size_t f = e;
        int64_t rows = 0;
        while (f < end) {
          const AdmBlock& ab = p.adm[blocks[f]];
          const int r = col ? rR[p.slot_of(ab.t, ab.c)] : rR[p.slot_of(ab.s, ab.c)];
          const int rr = (col || h.omega[blocks[f]] > 0.0) ? r : 0;
          if (f > e && rows + rr > kSegRows) break;
          rows += rr;
          ++f;
        }
        C64* base = P + poff;
        double* wbase = scale_later ? Wt + poff / k : nullptr;
        poff += (size_t)rows * k;
        int64_t roff = 0;
        for (size_t g = e; g < f; ++g) {
          const int64_t b = blocks[g];
          const AdmBlock& ab = p.adm[b];
          const int64_t other = col ? p.slot_of(ab.t, ab.c) : p.slot_of(ab.s, ab.c);
          const int r = rR[other];
          if (r <= 0 || (!col && !(h.omega[b] > 0.0))) continue;
          const double alpha = col ? 1.0 : 1.0 / h.omega[b];
          if (S) {
            GemmDesc d{};
            d.A = Rp(other); d.lda = k; d.M = r; d.K = k; d.tri = 1;
            d.B = S + (size_t)g * kk; d.ldb = k; d.N = k; d.opB = col ? 0 : 2;
            d.C = base + roff; d.ldc = (int32_t)rows;
            d.alpha_re = alpha;
            out.pieces.push_back(d);
          } else {
            out.cpieces.push_back(coup_desc(b, Rp(other), k, r, col ? 0 : 1, 1, base + roff, (int32_t)rows, alpha));
          }
          if (colpiece) {
            (*colpiece)[g] = base + roff;
            (*colld)[g] = (int32_t)rows;
          }
          if (scale_later) out.rw.push_back(RowWeightTask{(int64_t)(wbase - Wt) + roff, r, 0, b});
          roff += r;
        }
        if (rows > 0) {
          if (scale_later) out.ss.push_back(SegScaleTask{base, wbase, (int32_t)rows, k});
          GemmDesc d{};
          d.A = base; d.lda = (int32_t)rows; d.opA = 2;
          d.B = base; d.ldb = (int32_t)rows;
          d.M = k; d.N = k; d.K = (int32_t)rows;
          d.upper = projected(q) ? 0 : 1;       // leaf projections need the whole matrix
          d.alpha_re = 1.0;
          segs.push_back(d);
        }
        e = f;
      }
      if (segs.size() == 1) {
        segs[0].C = Zp(!col, q);
        segs[0].ldc = k;
        segs[0].accumulate = 1;
        out.gram.push_back(segs[0]);
      } else if (segs.size() > 1) {
        const int32_t s0 = (int32_t)out.srcs.size();
        for (GemmDesc& d : segs) {
          // temporary number srcs.size(); its address is set once all are counted
          temp_of.push_back(out.gram.size());
          d.ldc = k;
          out.gram.push_back(d);
          out.srcs.push_back(nullptr);
        }
        // the k x k Gram matrix (a narrow leaf's is projected in the top-down pass)
        out.sums.push_back(GramSumTask{Zp(!col, q), k, k, s0, (int32_t)out.srcs.size(), 0,
                                       projected(q) ? 1 : 0});
      }
    }
    if (!temp_of.empty()) {
      C64* T = h.alloc<C64>(temp_of.size() * kk);
      tmp.push_back(T);
      for (size_t i = 0; i < temp_of.size(); ++i) {
        out.gram[temp_of[i]].C = T + i * kk;
        out.srcs[i] = T + i * kk;
      }
    }
    return out;
  }
  // the Gram products of stack_rows and the sums of the split slots
  void add_grams(const GramRows& gr, std::vector<void*>& tmp) {
    gemm(gr.gram, tmp, true);
    if (!gr.sums.empty())
      launch_gram_sum(upload_tmp(gr.sums, tmp), (int64_t)gr.sums.size(),
                      (const void* const*)upload_tmp(gr.srcs, tmp), h.stream);
  }

  void weights_gram() {
    const int64_t nb = (int64_t)p.adm.size();
    const size_t kk = (size_t)k * k;
    double* om_d = h.alloc<double>(nb);
    Zr_d = h.alloc<C64>((size_t)ns * kk);
    Zc_d = h.alloc<C64>((size_t)ns * kk);
    HIPCHK(hipMemsetAsync(Zr_d, 0, (size_t)ns * kk * sizeof(C64), h.stream));
    HIPCHK(hipMemsetAsync(Zc_d, 0, (size_t)ns * kk * sizeof(C64), h.stream));
    rZr.assign(ns, 0);
    rZc.assign(ns, 0);
    // pass 1, blocks in column-slot order.  Per block: S_b, scratch of the
    // spectral norm, R_tc S_b R_sc^H, the rows R_tc S_b (at most k x k) and
    // their k scale factors.
    // The spectral norm needs S_b itself (and S, T1 as scratch); the Frobenius
    // norm needs only the rows R_tc S_b, formed with S_b inside the product.
    {
      const bool fused = fuse_couplings() && h.norm_mode == 0;
      const size_t per = (fused ? 2 : 4) * kk * sizeof(C64) + (size_t)k * sizeof(double);
      if (per > ws_bytes) throw Fail{DH2_ERR_OOM, "workspace too small for one block of the Gram weights"};
      const int64_t batch = std::max<int64_t>(1, (int64_t)(ws_bytes / per));
      for (int64_t b0 = 0; b0 < nb; b0 += batch) {
        const int64_t b1 = std::min(nb, b0 + batch);
        const size_t nbat = (size_t)(b1 - b0);
        std::vector<int64_t> blocks(p.col_blk.begin() + b0, p.col_blk.begin() + b1);
        C64* S = fused ? nullptr : (C64*)ws;
        C64* T1 = fused ? nullptr : S + nbat * kk;
        C64* T2 = fused ? (C64*)ws : T1 + nbat * kk;
        C64* P = T2 + nbat * kk;
        double* Wt = (double*)(P + nbat * kk);
        std::vector<void*> tmp;
        ++h.stats.batches_block_weights;
        if (!fused) gen_couplings(blocks, S, tmp);
        std::vector<C64*> colpiece(nbat, nullptr);
        std::vector<int32_t> colld(nbat, 0);
        GramRows gr = stack_rows(true, blocks, S, P, Wt, true, &colpiece, &colld, tmp);
        std::vector<GemmDesc> g2;
        std::vector<FrobDesc> fd;
        for (size_t i = 0; i < nbat; ++i) {
          const AdmBlock& a = p.adm[blocks[i]];
          const int rt = rR[p.slot_of(a.t, a.c)], rs = rR[p.slot_of(a.s, a.c)];
          if (colpiece[i]) {
            GemmDesc d{};
            d.A = colpiece[i]; d.lda = colld[i]; d.M = rt; d.K = k;
            d.B = Rp(p.slot_of(a.s, a.c)); d.ldb = k; d.N = rs; d.opB = 2; d.tri = 2;
            d.C = T2 + i * kk; d.ldc = std::max(rt, 1);
            d.alpha_re = 1.0;
            g2.push_back(d);
          }
          fd.push_back({T2 + i * kk, colpiece[i] ? rt : 0, rs, std::max(rt, 1), 0, blocks[i]});
        }
        gemm(gr.pieces, tmp);
        gemm_coupling(gr.cpieces, tmp);
        gemm(g2, tmp);
        if (h.norm_mode == 0)
          launch_frob<double>(upload_tmp(fd, tmp), (int64_t)fd.size(), om_d, h.stream);
        else
          spectral_weights(blocks, S, T1, T2, om_d, tmp);   // S and T1 are free by now
        launch_row_weights(upload_tmp(gr.rw, tmp), (int64_t)gr.rw.size(), om_d, Wt, h.stream);
        launch_scale_segments(upload_tmp(gr.ss, tmp), (int64_t)gr.ss.size(), k, h.stream);
        add_grams(gr, tmp);
        h.check_launch();
        free_tmp_async(tmp, b0 / batch);
      }
      h.sync();
      h.omega.resize(nb);
      if (nb) HIPCHK(hipMemcpy(h.omega.data(), om_d, nb * sizeof(double), hipMemcpyDeviceToHost));
      h.release(om_d);
    }
    // pass 2, blocks in row-slot order: S_b and the rows R_sc S_b^H / omega_b
    {
      const bool fused = fuse_couplings();
      const size_t per = (fused ? 1 : 2) * kk * sizeof(C64);
      const int64_t batch = std::max<int64_t>(1, (int64_t)(ws_bytes / per));
      for (int64_t b0 = 0; b0 < nb; b0 += batch) {
        const int64_t b1 = std::min(nb, b0 + batch);
        const size_t nbat = (size_t)(b1 - b0);
        std::vector<int64_t> blocks(p.row_blk.begin() + b0, p.row_blk.begin() + b1);
        C64* S = fused ? nullptr : (C64*)ws;
        C64* P = fused ? (C64*)ws : S + nbat * kk;
        std::vector<void*> tmp;
        if (!fused) gen_couplings(blocks, S, tmp);
        GramRows gr = stack_rows(false, blocks, S, P, nullptr, false, nullptr, nullptr, tmp);
        gemm(gr.pieces, tmp);
        gemm_coupling(gr.cpieces, tmp);
        add_grams(gr, tmp);
        h.check_launch();
        free_tmp_async(tmp, b0 / batch);
      }
      h.sync();
    }
  }

  // Top-down pass of the Gram form (see weights_gram) for the row (row =
  // true) or column slots: per level, the inherited rows Zhat_{t+c+} E^H of
  // every slot are formed (stacked per slot) and their Gram matrix added;
  // leaf slots narrower than k get V G V^H (#t x #t); every slot's Gram
  // matrix is factored by pivoted Cholesky in place (Zhat = R, rZ rows).
  void total_gram_topdown(bool row) {
    const std::vector<uint8_t>& flag = row ? p.slot_row : p.slot_col;
    std::vector<int32_t>& rZ = row ? rZr : rZc;
    const size_t kk = (size_t)k * k;
    // per slot at most: two parents' rows (2 k x k), V G (k x k), Cholesky scratch (k x k)
    const size_t per = 4 * kk * sizeof(C64);
    if (per > ws_bytes) throw Fail{DH2_ERR_OOM, "workspace too small for one slot of the Gram weights"};
    const int64_t chunk = std::max<int64_t>(1, (int64_t)(ws_bytes / per));
    for (int l = 0; l <= p.depth; ++l) {
      std::vector<int64_t> qs;
      for (int64_t q = 0; q < ns; ++q)
        if (si[q].level == l && flag[q]) qs.push_back(q);
      for (size_t c0 = 0; c0 < qs.size(); c0 += (size_t)chunk) {
        const size_t c1 = std::min(qs.size(), c0 + (size_t)chunk);
        std::vector<void*> tmp;
        std::vector<GemmDesc> gd, gg, v1, v2;
        std::vector<PcholTask> chol;
        C64* W = (C64*)ws;
        size_t off = 0;
        int maxnw = 0;
        for (size_t a = c0; a < c1; ++a) {
          const int64_t q = qs[a];
          int64_t rows = 0;
          std::vector<int64_t> par;
          for (int64_t pq : parents_of(q, flag))
            if (rZ[pq] > 0) {
              par.push_back(pq);
              rows += rZ[pq];
            }
          if (rows > 0) {
            if ((off + (size_t)rows * k) * sizeof(C64) > ws_bytes)
              throw Fail{DH2_ERR_OOM, "workspace too small for the inherited rows"};
            C64* base = W + off;
            off += (size_t)rows * k;
            int64_t roff = 0;
            for (int64_t pq : par) {
              GemmDesc d{};
              d.A = Zp(row, pq); d.lda = k; d.M = rZ[pq]; d.K = k;
              d.B = Ep(pq, child_index(si[q].t)); d.ldb = k; d.N = k; d.opB = 2;
              d.C = base + roff; d.ldc = (int32_t)rows;
              d.alpha_re = 1.0;
              gd.push_back(d);
              roff += rZ[pq];
            }
            GemmDesc d{};
            d.A = base; d.lda = (int32_t)rows; d.opA = 2;
            d.B = base; d.ldb = (int32_t)rows;
            d.M = k; d.N = k; d.K = (int32_t)rows;
            d.C = Zp(row, q); d.ldc = k;
            d.accumulate = 1;
            d.upper = projected(q) ? 0 : 1;
            d.alpha_re = 1.0;
            gg.push_back(d);
          }
          const int nw = projected(q) ? si[q].nrows : k;
          if (projected(q)) {
            // V G into the workspace, then V G V^H over G
            const int mq = si[q].nrows;
            C64* VG = W + off;
            off += (size_t)mq * k;
            GemmDesc d{};
            d.A = (C64*)h.V_d + h.V_off[q]; d.lda = mq; d.M = mq; d.K = k;
            d.B = Zp(row, q); d.ldb = k; d.N = k;
            d.C = VG; d.ldc = mq;
            d.alpha_re = 1.0;
            v1.push_back(d);
            GemmDesc e{};
            e.A = VG; e.lda = mq; e.M = mq; e.K = k;
            e.B = (C64*)h.V_d + h.V_off[q]; e.ldb = mq; e.N = mq; e.opB = 2;
            e.C = Zp(row, q); e.ldc = k;
            e.alpha_re = 1.0;
            v2.push_back(e);
          }
          maxnw = std::max(maxnw, nw);
          chol.push_back(PcholTask{Zp(row, q), nullptr, nw, k, cnt_d + q});
        }
        if (!pchol_fits_lds(maxnw)) {
          for (PcholTask& t : chol) {
            if ((off + kk) * sizeof(C64) > ws_bytes) throw Fail{DH2_ERR_OOM, "workspace too small for the Cholesky scratch"};
            t.scratch = W + off;
            off += kk;
          }
        }
        gemm(gd, tmp);
        gemm(gg, tmp, true);
        gemm(v1, tmp, true);
        gemm(v2, tmp, true);
        launch_pchol(upload_tmp(chol, tmp), (int64_t)chol.size(), maxnw, h.stream);
        ++(row ? h.stats.batches_total_weights_row : h.stats.batches_total_weights_col);
        h.check_launch();
        free_tmp(tmp);
      }
      read_counts(qs, rZ);
    }
  }

  void total_weights(bool row) {
    const std::vector<uint8_t>& flag = row ? p.slot_row : p.slot_col;
    const std::vector<int64_t>& ptr = row ? p.row_ptr : p.col_ptr;
    const std::vector<int64_t>& blk = row ? p.row_blk : p.col_blk;
    std::vector<int32_t>& rZ = row ? rZr : rZc;
    rZ.assign(ns, 0);
    C64*& Z = row ? Zr_d : Zc_d;
    Z = h.alloc<C64>((size_t)ns * k * k);
    // workspace partition: couplings | pieces | temporaries
    const size_t wsS = ws_bytes * 4 / 10, wsP = ws_bytes * 45 / 100;
    C64* Sbuf = (C64*)ws;
    C64* Pbuf = (C64*)(ws + wsS);
    C64* Tbuf = (C64*)(ws + wsS + wsP);
    const size_t wsT = ws_bytes - wsS - wsP;
    const int64_t maxS = std::max<int64_t>(1, (int64_t)(wsS / ((size_t)k * k * sizeof(C64))));
    const int64_t maxT = std::max<int64_t>(1, (int64_t)(wsT / ((size_t)k * k * sizeof(C64))));

    for (int l = 0; l <= p.depth; ++l) {
      std::vector<int64_t> qs;
      for (int64_t q = 0; q < ns; ++q)
        if (si[q].level == l && flag[q]) qs.push_back(q);
      // piece list of every slot of the level: (kind, index)
      std::vector<std::vector<PieceSrc>> srcs(qs.size());
      for (size_t a = 0; a < qs.size(); ++a) {
        const int64_t q = qs[a];
        for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) {
          const int64_t b = blk[e];
          if (!(h.omega[b] > 0.0)) continue;
          const AdmBlock& ab = p.adm[b];
          const int64_t other = row ? p.slot_of(ab.s, ab.c) : p.slot_of(ab.t, ab.c);
          if (rR[other] > 0) srcs[a].push_back({q, b, -1, rR[other]});
        }
        for (int64_t pq : parents_of(q, flag))
          if (rZ[pq] > 0) srcs[a].push_back({q, -1, pq, rZ[pq]});
        int64_t M = 0;
        for (auto& s : srcs[a]) M += s.rows;
        (void)M;
        rZ[q] = 0;
      }
      // batches over (slot, piece) in order
      size_t a0 = 0, e0 = 0;
      std::vector<uint8_t> started(qs.size(), 0), straddled(qs.size(), 0);
      while (a0 < qs.size()) {
        if (e0 >= srcs[a0].size()) {  // slot without pieces: rank 0, Zhat never read
          ++a0;
          e0 = 0;
          continue;
        }
        // collect a batch
        std::vector<Item> items;
        std::vector<int64_t> sblocks;
        size_t prow = 0;
        size_t a = a0, e = e0;
        while (a < qs.size()) {
          Item it{a, e, e};
          while (e < srcs[a].size()) {
            const PieceSrc& s = srcs[a][e];
            const size_t need = (size_t)s.rows * (k + (projected(qs[a]) ? si[qs[a]].nrows : 0));
            if ((s.blockid >= 0 && (int64_t)sblocks.size() >= maxS) ||
                (prow + need) * sizeof(C64) > wsP)
              break;
            if (s.blockid >= 0) sblocks.push_back(s.blockid);
            prow += need;
            ++e;
          }
          it.e1 = e;
          if (it.e1 > it.e0) items.push_back(it);
          if (e < srcs[a].size()) break;  // workspace full
          ++a;
          e = 0;
        }
        if (items.empty()) throw Fail{DH2_ERR_OOM, "workspace too small for one coupling piece"};
        ++(row ? h.stats.batches_total_weights_row : h.stats.batches_total_weights_col);
        // a slot whose rows are folded over more than one batch
        for (const Item& it : items)
          if (it.e0 > 0 || it.e1 < srcs[it.a].size())
            if (!straddled[it.a]) {
              straddled[it.a] = 1;
              ++h.stats.slots_straddled;
            }
        std::vector<void*> tmp;
        gen_couplings(sblocks, Sbuf, tmp);
        std::vector<GemmDesc> gd, gp;
        std::vector<FoldPiece> pieces;
        std::vector<std::pair<size_t, size_t>> item_pieces;  // piece range per item
        size_t sidx = 0, poff = 0;
        for (const Item& it : items) {
          const size_t pb = pieces.size();
          const int64_t qi = qs[it.a];
          const bool proj = projected(qi);
          const int mq = si[qi].nrows;
          for (size_t ee = it.e0; ee < it.e1; ++ee) {
            const PieceSrc& s = srcs[it.a][ee];
            C64* dst = Pbuf + poff;
            poff += (size_t)s.rows * k;
            GemmDesc g{};
            g.M = s.rows; g.N = k; g.K = k;
            g.C = dst; g.ldc = s.rows;
            if (s.blockid >= 0) {
              const AdmBlock& ab = p.adm[s.blockid];
              const int64_t other = row ? p.slot_of(ab.s, ab.c) : p.slot_of(ab.t, ab.c);
              g.A = Rp(other); g.lda = k; g.tri = 1;
              g.B = Sbuf + sidx * k * k; g.ldb = k; g.opB = row ? 2 : 0;
              g.alpha_re = 1.0 / h.omega[s.blockid];
              ++sidx;
            } else {
              g.A = Zp(row, s.parent); g.lda = k;
              g.B = Ep(s.parent, child_index(si[s.q].t)); g.ldb = k; g.opB = 2;
              g.alpha_re = 1.0;
            }
            gd.push_back(g);
            if (proj) {
              // the stacked row block times V_tc^H (rows x #t)
              C64* dp = Pbuf + poff;
              poff += (size_t)s.rows * mq;
              GemmDesc gq{};
              gq.A = dst; gq.lda = s.rows; gq.M = s.rows; gq.K = k;
              gq.B = (C64*)h.V_d + h.V_off[qi]; gq.ldb = mq; gq.N = mq; gq.opB = 2;
              gq.C = dp; gq.ldc = s.rows;
              gq.alpha_re = 1.0;
              gp.push_back(gq);
              pieces.push_back({dp, s.rows, s.rows});
            } else {
              pieces.push_back({dst, s.rows, s.rows});
            }
          }
          item_pieces.push_back({pb, pieces.size()});
        }
        gemm(gd, tmp);
        gemm(gp, tmp);
        h.check_launch();
        // TSQR split: fold segments of each item into temporaries when the
        // batch has few slots, merge the temporaries in a tree of 8-way folds
        // (in parallel), then fold the last ones into Zhat
        const int64_t want = 1024;
        int64_t G = std::max<int64_t>(1, (want + (int64_t)items.size() - 1) / (int64_t)items.size());
        G = std::min<int64_t>(G, std::max<int64_t>(1, (maxT * 4 / 5) / (int64_t)items.size()));
        constexpr int64_t kMerge = 8;
        std::vector<FoldTask> t1;
        std::vector<std::vector<FoldTask>> tiers;       // merge levels
        std::vector<FoldTask> t2;
        std::vector<FoldPiece> p2;
        int64_t tcount = 0;
        auto new_temp = [&]() {
          C64* Rt = Tbuf + (size_t)tcount * k * k;
          ++tcount;
          if (tcount > maxT) throw Fail{DH2_ERR_OOM, "workspace too small for the TSQR temporaries"};
          return Rt;
        };
        for (size_t ii = 0; ii < items.size(); ++ii) {
          const Item& it = items[ii];
          const int64_t q = qs[it.a];
          const int nw = projected(q) ? si[q].nrows : k;     // fold width
          const size_t pb = item_pieces[ii].first, pe = item_pieces[ii].second;
          const int64_t np = (int64_t)(pe - pb);
          const int64_t g = std::min<int64_t>(G, np);
          const int last = it.e1 >= srcs[it.a].size() ? 1 : 0;
          FoldTask fin{Zp(row, q), nw, k, 0, 0, started[it.a] ? 0 : 1, last, cnt_d + q};
          if (g <= 1) {
            fin.piece_begin = (int32_t)pb;
            fin.piece_end = (int32_t)pe;
            t2.push_back(fin);
          } else {
            // first level: g segments of the item's pieces, balanced by rows
            std::vector<int64_t> rows_prefix(np + 1, 0);
            for (int64_t e = 0; e < np; ++e) rows_prefix[e + 1] = rows_prefix[e] + pieces[pb + e].rows;
            std::vector<C64*> cur;
            size_t sb = pb;
            for (int64_t sgi = 0; sgi < g; ++sgi) {
              const int64_t target = rows_prefix[np] * (sgi + 1) / g;
              size_t se = sb;
              while (se < pe && (rows_prefix[se - pb] < target || se == sb)) ++se;
              if (sgi == g - 1) se = pe;
              if (se <= sb) continue;
              C64* Rt = new_temp();
              t1.push_back(FoldTask{Rt, nw, nw, (int32_t)sb, (int32_t)se, 1, 0, nullptr});
              cur.push_back(Rt);
              sb = se;
            }
            // merge levels: groups of kMerge temporaries (all k rows each: in
            // floating point a compacted factor may keep more nonzero rows
            // than the rows folded into it)
            size_t lvl = 0;
            while ((int64_t)cur.size() > kMerge) {
              if (tiers.size() <= lvl) tiers.emplace_back();
              std::vector<C64*> nxt;
              for (size_t a0 = 0; a0 < cur.size(); a0 += kMerge) {
                const size_t a1 = std::min(cur.size(), a0 + (size_t)kMerge);
                C64* Rt = new_temp();
                const int32_t b0 = (int32_t)(pieces.size() + p2.size());
                for (size_t a = a0; a < a1; ++a) p2.push_back({cur[a], nw, nw});
                tiers[lvl].push_back(FoldTask{Rt, nw, nw, b0, (int32_t)(pieces.size() + p2.size()), 1, 0, nullptr});
                nxt.push_back(Rt);
              }
              cur.swap(nxt);
              ++lvl;
            }
            fin.piece_begin = (int32_t)(pieces.size() + p2.size());
            for (C64* Rt : cur) p2.push_back({Rt, nw, nw});
            fin.piece_end = (int32_t)(pieces.size() + p2.size());
            t2.push_back(fin);
          }
          started[it.a] = 1;
        }
        pieces.insert(pieces.end(), p2.begin(), p2.end());
        count_folds(t1, pieces);
        for (const auto& tier : tiers) count_folds(tier, pieces);
        count_folds(t2, pieces);
        FoldPiece* pd = upload_tmp(pieces, tmp);
        // full-width (k) and projected (#t) folds in separate launches: the
        // chunk height follows the launch's largest width
        auto folds = [&](const std::vector<FoldTask>& ts) {
          std::vector<FoldTask> wide, narrow;
          int nmax = 0;
          for (const FoldTask& t : ts) {
            if (t.n == k) wide.push_back(t);
            else {
              narrow.push_back(t);
              nmax = std::max(nmax, t.n);
            }
          }
          if (!wide.empty()) launch_fold<double>(upload_tmp(wide, tmp), (int64_t)wide.size(), pd, k, h.stream);
          if (!narrow.empty())
            launch_fold<double>(upload_tmp(narrow, tmp), (int64_t)narrow.size(), pd, nmax, h.stream);
        };
        folds(t1);
        for (const auto& tier : tiers) folds(tier);
        folds(t2);
        h.check_launch();
        free_tmp(tmp);
        // advance
        const Item& last = items.back();
        a0 = last.a;
        e0 = last.e1;
        if (e0 >= srcs[a0].size()) {
          ++a0;
          e0 = 0;
        }
      }
      std::vector<int64_t> done;
      for (size_t a = 0; a < qs.size(); ++a)
        if (!srcs[a].empty()) done.push_back(qs[a]);
      read_counts(done, rZ);
    }
  }

  // ------------------------------------------------------------------
  // Learned-rank form: predicted ranks of every slot (row or column basis),
  // from the hierarchy's features and the compiled-in predictor, or the
  // handle's fixed rank when one is set (a test hook).
  std::vector<int32_t> predict_ranks(bool row) {
    std::vector<int32_t> pr(ns, 0);
    if (h.sketch_rank > 0) {
      std::fill(pr.begin(), pr.end(), h.sketch_rank);
      return pr;
    }
    const double t0 = now_ms();
    std::vector<float> f;
    rank_features(p, h.tol, row, f);
    std::vector<void*> tmp;
    float* fd = upload_tmp(f, tmp);
    int32_t* rd = h.alloc<int32_t>(ns);
    tmp.push_back(rd);
    launch_rank_mlp(fd, ns, rd, h.stream);
    h.check_launch();
    h.sync();
    HIPCHK(hipMemcpy(pr.data(), rd, ns * sizeof(int32_t), hipMemcpyDeviceToHost));
    free_tmp(tmp);
    h.stats.ms_rank_predict += now_ms() - t0;
    return pr;
  }

  // ------------------------------------------------------------------
  // truncation, bottom-up (Section 3.2): SVD of V Zhat^* (leaf) or Vhat Zhat^*
  // with Vhat = [C_{t1c1} E_{t1c}; C_{t2c2} E_{t2c}], rank by the tolerance rule,
  // Qhat = leading left singular vectors, C_tc = Qhat^* Vhat.
  //   exact path: B = Zhat Vhat^H (rZ x m), its R factor by the fold, Jacobi SVD;
  //   sketch path (learned-rank form, when the predicted rank plus the
  //   oversampling, l, is below m and rZ): A = Vhat Zhat^H (m x rZ), Y = A Omega
  //   with a Gaussian rZ x l Omega, Q = an orthonormal basis of range(Y) (Jacobi
  //   on the columns of Y), C^H = A^H Q, the discarded part A - Q C and its norm,
  //   Jacobi on the columns of C^H (left singular vectors U_C of C and sigma),
  //   the rank by the rule with the discarded norm added, Qhat = Q U_C[:, :rank].
  //   A slot whose discarded norm alone exceeds the tolerance (the predicted
  //   rank was too small) is truncated again by the exact path.
  static constexpr int kSketchOversample = 8;
  static constexpr int kSigStride = 512;
  void truncation(bool row) {
    const std::vector<uint8_t>& flag = row ? p.slot_row : p.slot_col;
    std::vector<int32_t>& rZ = row ? rZr : rZc;
    std::vector<int32_t>& rank = row ? h.rank_row : h.rank_col;
    auto& sig = row ? h.sig_row : h.sig_col;
    rank.assign(ns, -1);
    sig.assign(ns, {});
    std::vector<C64*>& Cptr = row ? Cr_ptr : Cc_ptr;
    std::vector<z64*>& Qptr = row ? h.Qr_ptr : h.Qc_ptr;
    std::vector<int32_t>& Qm = row ? h.Qr_m : h.Qc_m;
    Cptr.assign(ns, nullptr);
    Qptr.assign(ns, nullptr);
    Qm.assign(ns, 0);
    std::vector<int32_t> pred;
    if (h.rank_mode == DH2_RANKS_LEARNED) pred = predict_ranks(row);
    (row ? h.pred_row : h.pred_col) = pred;
    const size_t zs = sizeof(C64);
    for (int l = p.depth; l >= 0; --l) {
      std::vector<int64_t> qs;
      for (int64_t q = 0; q < ns; ++q)
        if (si[q].level == l && flag[q]) qs.push_back(q);
      size_t i0 = 0;
      while (i0 < qs.size()) {
        // per slot: Vhat (m x k) and the exact path's B (rZ x m), RB, U (m x m),
        // scratch 2 m^2; a sketch slot also A (m x rZ), Omega (rZ x l), Y, Q
        // (m x l), C^H (rZ x l), U_C (l x l), the Jacobi scratch of Y and C^H
        // and its discarded norm (the exact areas serve its fallback)
        struct Job {
          int64_t q;
          int m, ell;
          size_t vh, b, rb, u, sc;            // exact path
          size_t a, om, y, qq, ch, vj, sy, scc;   // sketch path
        };
        std::vector<Job> jobs;
        size_t used = 0;
        size_t i1 = i0;
        auto take = [&](size_t bytes) {
          const size_t o = used;
          used += (bytes + 255) / 256 * 256;
          return o;
        };
        for (; i1 < qs.size(); ++i1) {
          const int64_t q = qs[i1];
          Job j{};
          j.q = q;
          j.m = si[q].leaf ? si[q].nrows : rank[si[q].child_slot[0]] + rank[si[q].child_slot[1]];
          const int m = j.m, rz = rZ[q];
          j.ell = 0;
          if (!pred.empty() && m > 0 && rz > 0 && !projected(q)) {
            const int want = h.sketch_rank > 0 ? pred[q] : pred[q] + kSketchOversample;
            if (want < m && want < rz) j.ell = std::max(want, 1);
          }
          const int e = j.ell;
          size_t need = ((size_t)m * k + (size_t)rz * m + 4 * (size_t)m * m + 8) * zs + 5 * 256;
          if (e > 0)
            need += ((size_t)m * rz + (size_t)rz * e + 2 * (size_t)m * e + (size_t)rz * e + (size_t)e * e +
                     (size_t)(m + e) * e + (size_t)(rz + e) * e) * zs + 8 * 256;
          if (used + need > ws_bytes && i1 > i0) break;
          j.vh = take((size_t)m * k * zs);
          j.b = take((size_t)rz * m * zs);
          j.rb = take((size_t)m * m * zs);
          j.u = take((size_t)m * m * zs);
          j.sc = take(((size_t)2 * m * m + 8) * zs);
          if (e > 0) {
            j.a = take((size_t)m * rz * zs);
            j.om = take((size_t)rz * e * zs);
            j.y = take((size_t)m * e * zs);
            j.qq = take((size_t)m * e * zs);
            j.ch = take((size_t)rz * e * zs);
            j.vj = take((size_t)e * e * zs);
            j.sy = take((size_t)(m + e) * e * zs);
            j.scc = take((size_t)(rz + e) * e * zs);
          }
          if (used > ws_bytes) throw Fail{DH2_ERR_OOM, "workspace too small for a truncation step"};
          jobs.push_back(j);
        }
        std::vector<void*> tmp;
        const size_t nb = jobs.size();
        double* sig_d = (double*)h.alloc<double>(nb * kSigStride + 1);
        double* sigy_d = (double*)h.alloc<double>(nb * kSigStride + 1);
        int32_t* rk_d = h.alloc<int32_t>(nb + 1);
        tmp.push_back(sig_d);
        tmp.push_back(sigy_d);
        tmp.push_back(rk_d);
        std::vector<const C64*> vh_ptr(nb);
        std::vector<int> vh_ld(nb);
        std::vector<GemmDesc> g1;
        int maxm = 0;
        for (size_t b = 0; b < nb; ++b) {
          const Job& j = jobs[b];
          const int64_t q = j.q;
          const int m = j.m;
          maxm = std::max(maxm, m);
          C64* vh = (C64*)(ws + j.vh);
          if (si[q].leaf) {
            vh_ptr[b] = (C64*)h.V_d + h.V_off[q];
            vh_ld[b] = si[q].nrows;
          } else {
            int off = 0;
            for (int i = 0; i < 2; ++i) {
              const int64_t cq = si[q].child_slot[i];
              const int kc = rank[cq];
              if (kc > 0) {
                GemmDesc g{};
                g.A = Cptr[cq]; g.lda = kc; g.M = kc; g.K = k;
                g.B = Ep(q, i); g.ldb = k; g.N = k;
                g.C = vh + off; g.ldc = m;
                g.alpha_re = 1.0;
                g1.push_back(g);
              }
              off += kc;
            }
            vh_ptr[b] = vh;
            vh_ld[b] = m;
          }
        }
        if (maxm > kSigStride) throw Fail{DH2_ERR_ARG, "truncation matrix with more than 512 rows"};
        ++h.stats.batches_truncation;
        gemm(g1, tmp);
        // exact path for the given jobs: B = Zhat Vhat^H, fold, Jacobi
        auto exact = [&](const std::vector<size_t>& which) {
          std::vector<GemmDesc> g2;
          std::vector<FoldTask> ft;
          std::vector<FoldPiece> fp;
          std::vector<SvdTask> sv;
          int mm = 0;
          for (size_t b : which) {
            const Job& j = jobs[b];
            const int m = j.m, rz = rZ[j.q];
            if (m == 0 || rz == 0) continue;
            mm = std::max(mm, m);
            if (projected(j.q)) {
              // the projected total weight is already the R factor of B
              SvdTask st{};
              st.B = Zp(row, j.q); st.ldb = k;
              st.U = ws + j.u; st.ldu = m;
              st.sig = sig_d + b * kSigStride;
              st.rank = rk_d + b;
              st.scratch = ws + j.sc;
              st.m = m;
              st.norm_mode = h.norm_mode;
              st.eps = h.tol;
              sv.push_back(st);
              continue;
            }
            C64* B = (C64*)(ws + j.b);
            GemmDesc g{};
            g.A = Zp(row, j.q); g.lda = k; g.M = rz; g.K = k;
            g.B = vh_ptr[b]; g.ldb = vh_ld[b]; g.N = m; g.opB = 2;
            g.C = B; g.ldc = rz;
            g.alpha_re = 1.0;
            g2.push_back(g);
            ft.push_back(FoldTask{(C64*)(ws + j.rb), m, m, (int32_t)fp.size(), (int32_t)fp.size() + 1, 1, 0, nullptr});
            fp.push_back({B, rz, rz});
            SvdTask st{};
            st.B = ws + j.rb; st.ldb = m;
            st.U = ws + j.u; st.ldu = m;
            st.sig = sig_d + b * kSigStride;
            st.rank = rk_d + b;
            st.scratch = ws + j.sc;
            st.m = m;
            st.norm_mode = h.norm_mode;
            st.eps = h.tol;
            sv.push_back(st);
          }
          if (sv.empty()) return;
          if (!ft.empty()) {
            count_folds(ft, fp);
            gemm(g2, tmp);
            launch_fold<double>(upload_tmp(ft, tmp), (int64_t)ft.size(), upload_tmp(fp, tmp), mm, h.stream);
          }
          launch_jacobi(upload_tmp(sv, tmp), (int64_t)sv.size(), mm, mm, h.stream);
        };
        std::vector<size_t> ex, sk;
        for (size_t b = 0; b < nb; ++b) (jobs[b].ell > 0 ? sk : ex).push_back(b);
        exact(ex);
        if (!sk.empty()) {
          std::vector<GemmDesc> gA, gY, gC, gR;
          std::vector<SketchDesc> om;
          std::vector<FrobDesc> fr;
          std::vector<SvdTask> svY, svC;
          int mm = 0, mr = 0, me = 0;
          for (size_t b : sk) {
            const Job& j = jobs[b];
            const int m = j.m, rz = rZ[j.q], e = j.ell;
            mm = std::max(mm, m);
            mr = std::max(mr, rz);
            me = std::max(me, e);
            C64* A = (C64*)(ws + j.a);
            C64* Om = (C64*)(ws + j.om);
            C64* Y = (C64*)(ws + j.y);
            C64* Q = (C64*)(ws + j.qq);
            C64* CH = (C64*)(ws + j.ch);
            GemmDesc g{};
            g.A = vh_ptr[b]; g.lda = vh_ld[b]; g.M = m; g.K = k;           // A = Vhat Zhat^H
            g.B = Zp(row, j.q); g.ldb = k; g.N = rz; g.opB = 2;
            g.C = A; g.ldc = m;
            g.alpha_re = 1.0;
            gA.push_back(g);
            om.push_back({Om, rz, e, rz, 0, (int64_t)j.q * 2 + (row ? 0 : 1)});
            g = GemmDesc{};
            g.A = A; g.lda = m; g.M = m; g.K = rz;                          // Y = A Omega
            g.B = Om; g.ldb = rz; g.N = e;
            g.C = Y; g.ldc = m;
            g.alpha_re = 1.0;
            gY.push_back(g);
            SvdTask t{};
            t.B = Y; t.ldb = m; t.rows = m; t.m = e;                       // Q: basis of range(Y)
            t.W = Q; t.ldw = m;
            t.sig = sigy_d + b * kSigStride;
            t.scratch = ws + j.sy;
            t.eps = 0.0;
            svY.push_back(t);
            g = GemmDesc{};
            g.A = A; g.lda = m; g.M = rz; g.K = m; g.opA = 2;               // C^H = A^H Q
            g.B = Q; g.ldb = m; g.N = e;
            g.C = CH; g.ldc = rz;
            g.alpha_re = 1.0;
            gC.push_back(g);
            g = GemmDesc{};
            g.A = Q; g.lda = m; g.M = m; g.K = e;                           // A -= Q C
            g.B = CH; g.ldb = rz; g.N = rz; g.opB = 2;
            g.C = A; g.ldc = m;
            g.accumulate = 1;
            g.alpha_re = -1.0;
            gR.push_back(g);
            fr.push_back({A, m, rz, m, 0, (int64_t)b});
            t = SvdTask{};
            t.B = CH; t.ldb = rz; t.rows = rz; t.m = e;                    // U_C, sigma, rank
            t.U = ws + j.vj; t.ldu = e;
            t.sig = sig_d + b * kSigStride;
            t.rank = rk_d + b;
            t.scratch = ws + j.scc;
            t.norm_mode = h.norm_mode;
            t.eps = h.tol;
            t.resid = nullptr;   // set below: the discarded norm of job b
            svC.push_back(t);
          }
          h.stats.sketch_slots += (int64_t)sk.size();
          // the discarded norms, one per job (FrobDesc.index = batch position)
          double* res_d = h.alloc<double>(nb + 1);
          tmp.push_back(res_d);
          gemm(gA, tmp);
          launch_sketch_omega(upload_tmp(om, tmp), (int64_t)om.size(), 0x5EED1u, h.stream);
          gemm(gY, tmp);
          launch_jacobi(upload_tmp(svY, tmp), (int64_t)svY.size(), me, mm, h.stream);
          gemm(gC, tmp);
          gemm(gR, tmp);
          launch_frob<double>(upload_tmp(fr, tmp), (int64_t)fr.size(), res_d, h.stream);
          for (SvdTask& t : svC) {
            const size_t b = (size_t)(t.rank - rk_d);
            t.resid = res_d + b;
          }
          launch_jacobi(upload_tmp(svC, tmp), (int64_t)svC.size(), me, mr, h.stream);
        }
        h.check_launch();
        h.sync();
        std::vector<int32_t> rk(nb, 0);
        std::vector<double> sg(nb * kSigStride);
        HIPCHK(hipMemcpy(rk.data(), rk_d, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(sg.data(), sig_d, nb * kSigStride * sizeof(double), hipMemcpyDeviceToHost));
        // sketches that missed the tolerance: exact path
        std::vector<size_t> fb;
        for (size_t b : sk)
          if (rk[b] < 0) fb.push_back(b);
        if (!fb.empty()) {
          h.stats.sketch_fallbacks += (int64_t)fb.size();
          for (size_t b : fb) jobs[b].ell = 0;
          exact(fb);
          h.check_launch();
          h.sync();
          HIPCHK(hipMemcpy(rk.data(), rk_d, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
          HIPCHK(hipMemcpy(sg.data(), sig_d, nb * kSigStride * sizeof(double), hipMemcpyDeviceToHost));
        }
        // store Qhat (m x kk) and C = Qhat^* Vhat (kk x k); results are indexed by batch position
        std::vector<int> kkb(nb, 0);
        size_t qtot = 0, ctot = 0;
        for (size_t b = 0; b < nb; ++b) {
          const Job& j = jobs[b];
          const int m = j.m;
          if (m > 0 && rZ[j.q] > 0) {
            kkb[b] = rk[b];
            const int ns_sig = j.ell > 0 ? j.ell : m;
            sig[j.q].assign(sg.begin() + b * kSigStride, sg.begin() + b * kSigStride + ns_sig);
          }
          qtot += (size_t)m * kkb[b];
          ctot += (size_t)kkb[b] * k;
        }
        C64* Qb = h.alloc<C64>(std::max<size_t>(qtot, 1));
        C64* Cb = h.alloc<C64>(std::max<size_t>(ctot, 1));
        keep_rc.push_back(Cb);
        std::vector<CopyDesc> cp;
        std::vector<GemmDesc> gq, g3;
        size_t qo = 0, co = 0;
        for (size_t b = 0; b < nb; ++b) {
          const Job& j = jobs[b];
          const int64_t q = j.q;
          const int m = j.m;
          const int kk = kkb[b];
          rank[q] = kk;
          Qm[q] = m;
          Qptr[q] = Qb + qo;
          Cptr[q] = Cb + co;
          qo += (size_t)m * kk;
          co += (size_t)kk * k;
          if (kk > 0) {
            if (j.ell > 0) {
              GemmDesc g{};                                                 // Qhat = Q U_C[:, :kk]
              g.A = ws + j.qq; g.lda = m; g.M = m; g.K = j.ell;
              g.B = ws + j.vj; g.ldb = j.ell; g.N = kk;
              g.C = Qptr[q]; g.ldc = m;
              g.alpha_re = 1.0;
              gq.push_back(g);
            } else {
              cp.push_back({ws + j.u, Qptr[q], m, kk, m, m});
            }
            GemmDesc g{};
            g.A = Qptr[q]; g.lda = m; g.M = kk; g.K = m; g.opA = 2;
            g.B = vh_ptr[b]; g.ldb = vh_ld[b]; g.N = k;
            g.C = Cptr[q]; g.ldc = kk;
            g.alpha_re = 1.0;
            g3.push_back(g);
          }
        }
        if (!cp.empty()) launch_copy<double>(upload_tmp(cp, tmp), (int64_t)cp.size(), h.stream);
        gemm(gq, tmp);
        gemm(g3, tmp);
        h.check_launch();
        free_tmp(tmp);
        i0 = i1;
      }
    }
  }

  // ------------------------------------------------------------------
  // projection Stilde_b = C_tc S_b C_{W,sc}^* (Lemma 'Projections')
  void projection() {
    const int64_t nb = (int64_t)p.adm.size();
    h.St_off.assign(nb, 0);
    int64_t tot = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const AdmBlock& a = p.adm[b];
      h.St_off[b] = tot;
      tot += (int64_t)h.rank_row[p.slot_of(a.t, a.c)] * h.rank_col[p.slot_of(a.s, a.c)];
    }
    h.St_d = h.alloc<C64>((size_t)std::max<int64_t>(tot, 1));
    h.St_total = tot;
    // C_tc S_b with S_b formed inside the product (FP64), else stored first
    const bool fused = fuse_couplings();
    const size_t per = (size_t)(fused ? 1 : 2) * k * k * sizeof(C64);
    const int64_t batch = std::max<int64_t>(1, (int64_t)(ws_bytes / per));
    for (int64_t b0 = 0; b0 < nb; b0 += batch) {
      const int64_t b1 = std::min(nb, b0 + batch);
      std::vector<int64_t> blocks;
      for (int64_t b = b0; b < b1; ++b) blocks.push_back(b);
      C64* S = fused ? nullptr : (C64*)ws;
      C64* T = fused ? (C64*)ws : S + (size_t)(b1 - b0) * k * k;
      std::vector<void*> tmp;
      ++h.stats.batches_projection;
      if (!fused) gen_couplings(blocks, S, tmp);
      std::vector<GemmDesc> g1, g2;
      std::vector<CoupGemmDesc> c1;
      for (int64_t b = b0; b < b1; ++b) {
        const AdmBlock& a = p.adm[b];
        const int64_t qt = p.slot_of(a.t, a.c), qs = p.slot_of(a.s, a.c);
        const int kt = h.rank_row[qt], ks = h.rank_col[qs];
        if (kt == 0 || ks == 0) continue;
        const size_t i = (size_t)(b - b0);
        if (fused) {
          c1.push_back(coup_desc(b, Cr_ptr[qt], kt, kt, 0, 0, T + i * k * k, kt, 1.0));
        } else {
          GemmDesc g{};
          g.A = Cr_ptr[qt]; g.lda = kt; g.M = kt; g.K = k;
          g.B = S + i * k * k; g.ldb = k; g.N = k;
          g.C = T + i * k * k; g.ldc = kt;
          g.alpha_re = 1.0;
          g1.push_back(g);
        }
        GemmDesc gg{};
        gg.A = T + i * k * k; gg.lda = kt; gg.M = kt; gg.K = k;
        gg.B = Cc_ptr[qs]; gg.ldb = ks; gg.N = ks; gg.opB = 2;
        gg.C = (C64*)h.St_d + h.St_off[b]; gg.ldc = kt;
        gg.alpha_re = 1.0;
        g2.push_back(gg);
      }
      if (!g2.empty()) {
        gemm(g1, tmp);
        gemm_coupling(c1, tmp);
        gemm(g2, tmp);
      }
      h.check_launch();
      free_tmp_async(tmp, b0 / batch);
    }
    h.sync();
  }

  // ------------------------------------------------------------------
  // FP32 handles: the recompressed couplings and the new bases are rounded to
  // complex64 once, after the FP64 recompression; the FP64 couplings are freed.
  void narrow_to_fp32() {
    z32* St32 = h.alloc<z32>((size_t)std::max<int64_t>(h.St_total, 1));
    launch_narrow(h.St_d, St32, h.St_total, h.stream);
    h.check_launch();
    h.sync();
    h.release(h.St_d);
    h.St_d = St32;
    int64_t tot = 0;
    for (int64_t q = 0; q < ns; ++q) {
      if (h.rank_row[q] > 0) tot += (int64_t)h.Qr_m[q] * h.rank_row[q];
      if (h.rank_col[q] > 0) tot += (int64_t)h.Qc_m[q] * h.rank_col[q];
    }
    z32* Q32 = h.alloc<z32>((size_t)std::max<int64_t>(tot, 1));
    std::vector<NarrowDesc> nd;
    h.Qr32.assign(ns, nullptr);
    h.Qc32.assign(ns, nullptr);
    int64_t off = 0;
    for (int64_t q = 0; q < ns; ++q) {
      if (h.rank_row[q] > 0) {
        const int64_t m = (int64_t)h.Qr_m[q] * h.rank_row[q];
        h.Qr32[q] = Q32 + off;
        nd.push_back({h.Qr_ptr[q], Q32 + off, m});
        off += m;
      }
      if (h.rank_col[q] > 0) {
        const int64_t m = (int64_t)h.Qc_m[q] * h.rank_col[q];
        h.Qc32[q] = Q32 + off;
        nd.push_back({h.Qc_ptr[q], Q32 + off, m});
        off += m;
      }
    }
    if (!nd.empty()) {
      NarrowDesc* ndd = h.upload(nd);
      launch_narrow_list(ndd, (int64_t)nd.size(), h.stream);
      h.check_launch();
      h.sync();
      h.release(ndd);
    }
  }

  // ------------------------------------------------------------------
  // matvec schedule: phases of MvOut lists (see matvec.hip).  Pointers are
  // formed in elements of the handle's type (complex128 or complex64).
  // ---- matvec schedule (begin) ----
  void matvec_schedule() {
    const int nr = h.max_nrhs;
    const int64_t n = p.n;
    const bool f32 = h.precision != DH2_FP64;
    const int64_t es = f32 ? (int64_t)sizeof(z32) : (int64_t)sizeof(C64);
    auto at = [es](const void* base, int64_t e) -> char* { return (char*)base + e * es; };
    auto Qr = [&](int64_t q) -> const void* { return f32 ? h.Qr32[q] : (const void*)h.Qr_ptr[q]; };
    auto Qc = [&](int64_t q) -> const void* { return f32 ? h.Qc32[q] : (const void*)h.Qc_ptr[q]; };
    std::vector<int64_t> xo(ns, -1), yo(ns, -1), xro(ns, -1);
    int64_t xt = 0, yt = 0, xrows = 0;
    for (int64_t q = 0; q < ns; ++q) {
      if (h.rank_col[q] > 0) { xo[q] = xt; xt += (int64_t)h.rank_col[q] * nr; }
      if (h.rank_row[q] > 0) { yo[q] = yt; yt += (int64_t)h.rank_row[q] * nr; }
      if (h.rank_col[q] > 0) { xro[q] = xrows; xrows += h.rank_col[q]; }
    }
    // staging arena: Xp, XT, Yp (n x nr), slot vectors x_sc, y_tc and the
    // row-major slot vectors xhT, each 256-byte aligned
    h.n_xh_rows = xrows;
    const int64_t sizes[6] = {n * nr, n * nr, n * nr, xt, yt, xrows * nr};
    size_t offs[6], total = 0;
    for (int i = 0; i < 6; ++i) {
      offs[i] = total;
      total += ((size_t)std::max<int64_t>(sizes[i], 1) * es + 255) / 256 * 256;
    }
    h.stage_bytes = total;
    h.stage_d = h.alloc<char>(total);
    char* Xp = h.stage_d + offs[0];
    char* XT = h.stage_d + offs[1];
    char* Yp = h.stage_d + offs[2];
    char* xh = h.stage_d + offs[3];
    char* yh = h.stage_d + offs[4];
    char* xhT = h.stage_d + offs[5];
    h.mv_own.Xp = Xp;
    h.mv_own.XT = XT;
    h.mv_own.Yp = Yp;
    h.mv_own.xhT = xhT;
    std::vector<MvOut> outs;
    std::vector<MvTerm> terms;
    h.mv_phases.clear();
    int group = 1;
    auto begin_phase = [&]() { h.mv_phases.push_back({(int64_t)outs.size(), (int64_t)outs.size(), group}); };
    auto end_phase = [&]() { h.mv_phases.back().out_end = (int64_t)outs.size(); };
    // forward, leaves
    begin_phase();
    for (int64_t q = 0; q < ns; ++q)
      if (si[q].leaf && h.rank_col[q] > 0) {
        const int kq = h.rank_col[q];
        MvOut o{at(xh, xo[q]), kq, kq, (int32_t)terms.size(), 0, 0, 0};
        terms.push_back({Qc(q), at(Xp, si[q].row0), si[q].nrows, si[q].nrows, (int32_t)n, 2});
        o.term_end = (int32_t)terms.size();
        outs.push_back(o);
      }
    end_phase();
    // forward, inner clusters bottom-up
    for (int l = p.depth; l >= 0; --l) {
      begin_phase();
      for (int64_t q = 0; q < ns; ++q)
        if (si[q].level == l && !si[q].leaf && h.rank_col[q] > 0) {
          const int kq = h.rank_col[q];
          MvOut o{at(xh, xo[q]), kq, kq, (int32_t)terms.size(), 0, 0, 0};
          int off = 0;
          for (int i = 0; i < 2; ++i) {
            const int64_t cq = si[q].child_slot[i];
            const int kc = h.rank_col[cq];
            if (kc > 0)
              terms.push_back({at(Qc(q), off), at(xh, xo[cq]), kc, h.Qc_m[q], kc, 2});
            off += kc;
          }
          o.term_end = (int32_t)terms.size();
          outs.push_back(o);
        }
      end_phase();
    }
    // coupling: its own kernel, one entry per row slot.  The matrix-core form
    // reads x_sc from a row-major copy: column slot q occupies rows
    // [xro[q], xro[q] + k_q) of xhT.
    std::vector<SlotT> xtr;
    for (int64_t q = 0; q < ns; ++q)
      if (h.rank_col[q] > 0) xtr.push_back({at(xh, xo[q]), xro[q], h.rank_col[q], 0});
    h.zero16_d = h.alloc<C64>(16);
    HIPCHK(hipMemsetAsync(h.zero16_d, 0, 16 * sizeof(C64), h.stream));
    std::vector<MfRow> mrows, coup_rows, near_rows;
    std::vector<NearSeg> msegs;
    for (int64_t q = 0; q < ns; ++q)
      if (h.rank_row[q] > 0) {
        const int kq = h.rank_row[q];
        MfRow mr{at(yh, yo[q]), kq, kq, (int32_t)msegs.size(), 0};
        for (int64_t e = p.row_ptr[q]; e < p.row_ptr[q + 1]; ++e) {
          const int64_t b = p.row_blk[e];
          const AdmBlock& a = p.adm[b];
          const int64_t qs = p.slot_of(a.s, a.c);
          const int ks = h.rank_col[qs];
          if (ks > 0) msegs.push_back({at(h.St_d, h.St_off[b]), xro[qs], kq, ks});
        }
        mr.seg_end = (int32_t)msegs.size();
        mrows.push_back(mr);
      }
    h.n_coup_rows = (int64_t)mrows.size();
    {
      std::vector<double> work(mrows.size());
      for (size_t i = 0; i < mrows.size(); ++i) {
        double w = 0;
        for (int32_t e = mrows[i].seg_begin; e < mrows[i].seg_end; ++e) w += (double)msegs[e].lda * msegs[e].ncols;
        work[i] = w;
      }
      coup_rows.reserve(mrows.size());
      for (int64_t i : xcd_balanced_order(work, h.coup_split)) coup_rows.push_back(mrows[i]);
    }
    h.coup_mf_segs_d = h.upload(msegs);
    h.n_xh_tr = (int64_t)xtr.size();
    // backward, top-down: y_{t'c'} += F_{t'c} y_tc
    group = 3;
    for (int l = 1; l <= p.depth; ++l) {
      begin_phase();
      for (int64_t q = 0; q < ns; ++q)
        if (si[q].level == l && h.rank_row[q] > 0) {
          const int kq = h.rank_row[q];
          MvOut o{at(yh, yo[q]), kq, kq, (int32_t)terms.size(), 0, 1, 0};
          const int ci = child_index(si[q].t);
          for (int64_t pq : parents_of(q, p.slot_row)) {
            const int kp = h.rank_row[pq];
            if (kp <= 0) continue;
            const int off = ci == 0 ? 0 : h.rank_row[si[pq].child_slot[0]];
            terms.push_back({at(Qr(pq), off), at(yh, yo[pq]), kp, h.Qr_m[pq], kp, 0});
          }
          o.term_end = (int32_t)terms.size();
          if (o.term_end > o.term_begin) outs.push_back(o);
        }
      end_phase();
    }
    // leaf output + near field
    std::vector<std::vector<std::pair<int64_t, int64_t>>> near_of_leaf(p.cl.size());
    for (int64_t b = 0; b < (int64_t)p.near.size(); ++b) {
      const NearBlock& nbk = p.near[b];
      const Cluster& t = p.cl[nbk.t];
      // distribute the rows of t over its leaves
      std::vector<int64_t> stack{nbk.t};
      while (!stack.empty()) {
        const int64_t c = stack.back();
        stack.pop_back();
        if (p.cl[c].leaf()) near_of_leaf[c].push_back({b, p.cl[c].first - t.first});
        else
          for (int i = 0; i < 2; ++i) stack.push_back(p.cl[c].child[i]);
      }
    }
    // near field: its own kernel, one entry per leaf, writes Yp
    std::vector<NearRow> nrows;
    std::vector<NearSeg> nsegs;
    int64_t nbytes = 0;
    for (int64_t t = 0; t < (int64_t)p.cl.size(); ++t) {
      const Cluster& c = p.cl[t];
      if (!c.leaf()) continue;
      NearRow r{c.first, (int32_t)c.size, (int32_t)nsegs.size(), 0, 0};
      for (const auto& pr : near_of_leaf[t]) {
        const NearBlock& nbk = p.near[pr.first];
        const Cluster& tt = p.cl[nbk.t];
        const Cluster& ss = p.cl[nbk.s];
        nsegs.push_back({at(h.near_d, h.near_off[pr.first] + pr.second), ss.first, (int32_t)tt.size,
                         (int32_t)ss.size});
        nbytes += c.size * ss.size;
      }
      r.seg_end = (int32_t)nsegs.size();
      nrows.push_back(r);
    }
    h.near_segs_d = h.upload(nsegs);
    h.n_near_rows = (int64_t)nrows.size();
    {
      std::vector<MfRow>& mf = near_rows;
      mf.reserve(nrows.size());
      std::vector<double> work(nrows.size());
      for (size_t i = 0; i < nrows.size(); ++i) {
        double w = 0;
        for (int32_t e = nrows[i].seg_begin; e < nrows[i].seg_end; ++e) w += (double)nrows[i].nr * nsegs[e].ncols;
        work[i] = w;
      }
      for (int64_t i : xcd_balanced_order(work, h.near_split)) {
        const NearRow& r = nrows[i];
        mf.push_back({at(Yp, r.row0), (int32_t)n, r.nr, r.seg_begin, r.seg_end});
      }
    }
    h.near_matvec_bytes = nbytes * es;
    // leaf output: Y_t += Q_tc y_tc (after the near field)
    group = 5;
    begin_phase();
    for (int64_t t = 0; t < (int64_t)p.cl.size(); ++t) {
      const Cluster& c = p.cl[t];
      if (!c.leaf()) continue;
      MvOut o{at(Yp, c.first), (int32_t)c.size, (int32_t)n, (int32_t)terms.size(), 0, 1, 0};
      for (const auto& pr : p.cl_slots[t]) {
        const int64_t q = pr.second;
        if (h.rank_row[q] > 0)
          terms.push_back({Qr(q), at(yh, yo[q]), h.rank_row[q], (int32_t)c.size, h.rank_row[q], 0});
      }
      o.term_end = (int32_t)terms.size();
      if (o.term_end > o.term_begin) outs.push_back(o);
    }
    end_phase();
    h.mv_own.outs = h.upload(outs);
    h.mv_own.terms = h.upload(terms);
    h.mv_own.near_rows = h.upload(near_rows);
    h.mv_own.coup_rows = h.upload(coup_rows);
    h.mv_own.xh_tr = h.upload(xtr);
    // The same descriptors relocated into the static scratch array (device
    // address of this device's copy), for the allocation-free product: every
    // pointer into the staging arena moves by the same offset; matrix
    // pointers stay.
    size_t scr_bytes = 0;
    char* scr = (char*)scratch_region(&scr_bytes);
    h.has_scr = scr != nullptr && h.stage_bytes <= scr_bytes;
    if (h.has_scr) {
      char* const base = h.stage_d;
      const size_t len = h.stage_bytes;
      auto rel = [&](auto* ptr) {
        char* c = (char*)ptr;
        using P = decltype(ptr);
        return (c >= base && c < base + len) ? (P)(scr + (c - base)) : ptr;
      };
      for (MvOut& o : outs) o.y = rel(o.y);
      for (MvTerm& t : terms) t.x = rel(t.x);
      for (MfRow& r : near_rows) r.y = rel(r.y);
      for (MfRow& r : coup_rows) r.y = rel(r.y);
      for (SlotT& t : xtr) t.src = rel(t.src);
      h.mv_scr.outs = h.upload(outs);
      h.mv_scr.terms = h.upload(terms);
      h.mv_scr.near_rows = h.upload(near_rows);
      h.mv_scr.coup_rows = h.upload(coup_rows);
      h.mv_scr.xh_tr = h.upload(xtr);
      h.mv_scr.Xp = rel(Xp);
      h.mv_scr.XT = rel(XT);
      h.mv_scr.Yp = rel(Yp);
      h.mv_scr.xhT = rel(xhT);
    }
  }
  // ---- matvec schedule (end) ----
};

void validate(const dh2_geometry* g, double kappa, int order, double eta, int leafsize, double tol,
              double eta1) {
  if (!g) throw Fail{DH2_ERR_ARG, "geometry is NULL"};
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) throw Fail{DH2_ERR_ARG, "kappa must be finite and >= 0"};
  if (order < 1 || order > kMaxOrder) throw Fail{DH2_ERR_ARG, "order must be in [1, 8]"};
  if (!(eta > 0.0) || !std::isfinite(eta)) throw Fail{DH2_ERR_ARG, "eta must be > 0"};
  if (leafsize < 1 || leafsize > 256) throw Fail{DH2_ERR_ARG, "leafsize must be in [1, 256]"};
  if (!(tol >= 0.0) || !std::isfinite(tol)) throw Fail{DH2_ERR_ARG, "tol must be finite and >= 0"};
  if (!(eta1 > 0.0) || !std::isfinite(eta1)) throw Fail{DH2_ERR_ARG, "eta1 must be > 0"};
  if (g->n_triangles < 1 || g->n_vertices < 3 || !g->vertices || !g->triangles)
    throw Fail{DH2_ERR_GEOMETRY, "empty geometry"};
  if (g->n_triangles > (int64_t)1 << 30) throw Fail{DH2_ERR_GEOMETRY, "too many triangles"};
  for (int64_t i = 0; i < g->n_vertices * 3; ++i)
    if (!std::isfinite(g->vertices[i])) throw Fail{DH2_ERR_GEOMETRY, "non-finite vertex coordinate"};
  for (int64_t i = 0; i < g->n_triangles; ++i) {
    const int32_t* t = g->triangles + 3 * i;
    for (int v = 0; v < 3; ++v)
      if (t[v] < 0 || t[v] >= g->n_vertices)
        throw Fail{DH2_ERR_GEOMETRY, "triangle " + std::to_string(i) + " has a vertex index out of range"};
    const double* a = g->vertices + 3 * (int64_t)t[0];
    const double* b = g->vertices + 3 * (int64_t)t[1];
    const double* c = g->vertices + 3 * (int64_t)t[2];
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    if (!(cx * cx + cy * cy + cz * cz > 0.0))
      throw Fail{DH2_ERR_GEOMETRY, "triangle " + std::to_string(i) + " has zero area"};
  }
}

template <typename R>
void run_matvec_t(dh2_problem* h, const dh2_problem::MvView& v, const void* X, void* Y, int nrhs, hipEvent_t* ev,
                  hipStream_t st);

// Autotuner of the block-row products.  Each shape is timed inside whole
// products (the near-field and coupling launches see the caches and clocks
// they see in use), with the shapes interleaved over three sweeps, the first
// discarded; per phase and right-hand-side class the shape with the shortest
// best time is kept (the default unless another beats it by 3 %).
// Right-hand sides are zero (the timing does not depend on the values).
template <typename R>
void tune_block_rows_t(dh2_problem& h) {
  const hipStream_t st = h.stream;
  const int64_t n = h.plan.n;
  const size_t vb = (size_t)n * h.max_nrhs * 2 * sizeof(R);
  void* Xb = h.alloc<char>(vb);
  void* Yb = h.alloc<char>(vb);
  HIPCHK(hipMemsetAsync(Xb, 0, vb, st));
  hipEvent_t ev[8];
  for (hipEvent_t& e : ev) HIPCHK(hipEventCreate(&e));
  const int nv = mv_rows_variants();
  for (int cls = 0; cls < 2; ++cls) {
    if (cls == 1 && h.max_nrhs <= 16) {
      h.mv_var[2] = h.mv_var[0];
      h.mv_var[3] = h.mv_var[1];
      break;
    }
    const int nrhs = cls == 0 ? std::min(h.max_nrhs, 16) : h.max_nrhs;
    std::vector<float> best(2 * nv, 1e30f);
    for (int sweep = 0; sweep < 3; ++sweep)
      for (int var = 0; var < nv; ++var) {
        h.mv_var[2 * cls] = h.mv_var[2 * cls + 1] = var;
        run_matvec_t<R>(&h, h.mv_own, Xb, Yb, nrhs, ev, st);
        HIPCHK(hipEventSynchronize(ev[7]));
        if (sweep == 0) continue;
        float near = 0, coup = 0;
        HIPCHK(hipEventElapsedTime(&near, ev[4], ev[5]));
        HIPCHK(hipEventElapsedTime(&coup, ev[2], ev[3]));
        best[var] = std::min(best[var], near);
        best[nv + var] = std::min(best[nv + var], coup);
      }
    // another shape replaces the default only when it is faster by more than
    // the run-to-run spread of these timings (about 2 %)
    for (int role = 0; role < 2; ++role) {
      int arg = 0;
      for (int var = 1; var < nv; ++var)
        if (best[role * nv + var] < 0.97f * best[role * nv + arg]) arg = var;
      h.mv_var[2 * cls + role] = arg;
    }
  }
  for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
  h.release(Xb);
  h.release(Yb);
}

void tune_block_rows(dh2_problem& h) {
  if (h.precision != DH2_FP64) tune_block_rows_t<float>(h);
  else tune_block_rows_t<double>(h);
}

// Touching triangle pairs of the near field, for the paper's quadrature
// (Section 5): every ordered pair (i, j) of triangles that share a vertex (kind
// 1), an edge (2) or are identical (3), with the element offset of entry
// (pos(i), pos(j)) in the near-field storage.  Pairs in mirrored blocks are
// left out (the transposition copies them from the evaluated block).  The
// pair is integrated with the triangle of lower index in the caller's
// numbering first, its vertices ordered with the shared part first (a shared
// vertex as A, a shared edge as A -> B of both, the rest in the caller's order).
// rptr / rblk: the near blocks grouped by row cluster.
std::vector<TouchDesc> touching_pairs(const Plan& p, const dh2_geometry& g, const std::vector<int64_t>& near_off,
                                      const std::vector<uint8_t>& mirrored, const std::vector<int64_t>& rptr,
                                      const std::vector<int64_t>& rblk) {
  const int64_t n = p.n, nc = (int64_t)p.cl.size(), nv = g.n_vertices;
  const int32_t* T = g.triangles;
  std::vector<int64_t> pos(n), leaf_of(n, -1);
  for (int64_t q = 0; q < n; ++q) pos[p.perm[q]] = q;
  for (int64_t c = 0; c < nc; ++c)
    if (p.cl[c].leaf())
      for (int64_t q = p.cl[c].first; q < p.cl[c].first + p.cl[c].size; ++q) leaf_of[q] = c;
  // each row cluster's blocks by the first position of their column cluster
  std::vector<int64_t> byfirst(rblk);
  auto col_first = [&](int64_t b) { return p.cl[p.near[b].s].first; };
  for (int64_t t = 0; t < nc; ++t)
    std::sort(byfirst.begin() + rptr[t], byfirst.begin() + rptr[t + 1],
              [&](int64_t a, int64_t b) { return col_first(a) < col_first(b); });
  std::vector<int64_t> vptr(nv + 1, 0), vtri(3 * n);
  for (int64_t i = 0; i < 3 * n; ++i) ++vptr[T[i] + 1];
  for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
  {
    std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) vtri[fill[T[3 * i + a]]++] = i;
  }
  std::vector<TouchDesc> out;
  out.reserve((size_t)n * 16);
  std::vector<std::pair<int64_t, int>> cand;
  for (int64_t i = 0; i < n; ++i) {
    cand.clear();
    for (int a = 0; a < 3; ++a) {
      const int32_t v = T[3 * i + a];
      for (int64_t e = vptr[v]; e < vptr[v + 1]; ++e) {
        const int64_t j = vtri[e];
        bool found = false;
        for (auto& c : cand)
          if (c.first == j) { ++c.second; found = true; break; }
        if (!found) cand.push_back({j, 1});
      }
    }
    const int64_t pi = pos[i];
    for (const auto& c : cand) {
      const int64_t j = c.first, pj = pos[j];
      int64_t b = -1;
      for (int64_t a = leaf_of[pi]; a >= 0 && b < 0; a = p.cl[a].parent) {
        const auto lo = byfirst.begin() + rptr[a], hi = byfirst.begin() + rptr[a + 1];
        auto it = std::upper_bound(lo, hi, pj, [&](int64_t v, int64_t blk) { return v < col_first(blk); });
        if (it == lo) continue;
        const int64_t cand_b = *(it - 1);
        const Cluster& sc = p.cl[p.near[cand_b].s];
        if (pj < sc.first + sc.size) b = cand_b;
      }
      if (b < 0) throw Fail{DH2_ERR_GEOMETRY, "touching triangles outside the near field"};
      if (mirrored[b]) continue;
      const Cluster& tc = p.cl[p.near[b].t];
      const Cluster& sc = p.cl[p.near[b].s];
      TouchDesc d{};
      d.off = near_off[b] + (pi - tc.first) + (pj - sc.first) * tc.size;
      d.kind = c.second;
      const int32_t* Ta = T + 3 * std::min(i, j);
      const int32_t* Tb = T + 3 * std::max(i, j);
      auto in_b = [&](int32_t v) { return v == Tb[0] || v == Tb[1] || v == Tb[2]; };
      auto in_a = [&](int32_t v) { return v == Ta[0] || v == Ta[1] || v == Ta[2]; };
      int na = 0, nb = 0;
      for (int a = 0; a < 3; ++a)   // shared vertices first, in Ta's order
        if (in_b(Ta[a])) d.va[na++] = d.vb[nb++] = Ta[a];
      if (na != d.kind) throw Fail{DH2_ERR_GEOMETRY, "repeated vertex in a triangle"};
      for (int a = 0; a < 3; ++a) {
        if (!in_b(Ta[a])) d.va[na++] = Ta[a];
        if (!in_a(Tb[a])) d.vb[nb++] = Tb[a];
      }
      out.push_back(d);
    }
  }
  return out;
}

void build_all(dh2_problem& h, const dh2_geometry& g) {
  const double t_start = now_ms();
  Plan& p = h.plan;
  h.stats.ms_structure = 0;
  double t0 = now_ms();
  // structure (host)
  {
    std::string err = build_plan(g.vertices, g.n_vertices, g.triangles, g.n_triangles, h.plan.kappa,
                                 h.plan.order, h.plan.eta, h.plan.leafsize, h.plan.eta1, p);
    if (!err.empty()) throw Fail{DH2_ERR_ARG, err};
  }
  h.stats.ms_structure = now_ms() - t0;
  Builder bd(h);
  bd.setup_slots();
  const int k = p.k;
  const int64_t n = p.n;
  const int64_t nc = (int64_t)p.cl.size();

  // geometry, per-triangle data
  t0 = now_ms();
  std::vector<double> Vh(g.vertices, g.vertices + 3 * g.n_vertices);
  std::vector<int32_t> Th(g.triangles, g.triangles + 3 * g.n_triangles);
  double* Vd = h.upload(Vh);
  int32_t* Td = h.upload(Th);
  h.perm_d = h.upload(p.perm);
  double* x7 = h.alloc<double>((size_t)n * 21);
  double* w7 = h.alloc<double>((size_t)n * 7);
  double* x16 = h.alloc<double>((size_t)n * 48);
  double* w16 = h.alloc<double>((size_t)n * 16);
  double* x9 = h.alloc<double>((size_t)n * 27);
  double* w9 = h.alloc<double>((size_t)n * 9);
  double* selfl = h.alloc<double>((size_t)n);
  launch_tri_data(n, Vd, Td, h.perm_d, make_quad(), x7, w7, x16, w16, x9, w9, selfl, h.stream);
  h.check_launch();
  const bool paper_quad = h.quadrature == DH2_QUAD_PAPER;
  std::vector<double> box(6 * nc);
  for (int64_t t = 0; t < nc; ++t)
    for (int d = 0; d < 3; ++d) {
      box[6 * t + d] = p.cl[t].lo[d];
      box[6 * t + 3 + d] = p.cl[t].hi[d];
    }
  h.box_d = h.upload(box);
  std::vector<double> dirs;
  h.dir_off.clear();
  for (int l = 0; l <= p.depth; ++l) {
    h.dir_off.push_back((int64_t)dirs.size() / 3);
    dirs.insert(dirs.end(), p.dirs[l].begin(), p.dirs[l].end());
  }
  h.dirs_d = h.upload(dirs);

  // near field
  {
    std::vector<NearDesc> nd(p.near.size());
    h.near_off.resize(p.near.size());
    int64_t off = 0;
    for (size_t b = 0; b < p.near.size(); ++b) {
      const Cluster& t = p.cl[p.near[b].t];
      const Cluster& s = p.cl[p.near[b].s];
      nd[b] = {t.first, s.first, (int32_t)t.size, (int32_t)s.size, off};
      h.near_off[b] = off;
      off += t.size * s.size;
    }
    h.stats.near_entries = off;
    // The Galerkin matrix is symmetric: of the pair (t, s), (s, t) only the
    // block with t < s is evaluated, its mirror is its transpose.  Mirrors are
    // found through the blocks grouped by row cluster, each group sorted by
    // column cluster (a binary search per block).
    const int64_t nnear = (int64_t)p.near.size();
    std::vector<int64_t> rptr(nc + 1, 0), rblk(nnear);
    for (int64_t b = 0; b < nnear; ++b) ++rptr[p.near[b].t + 1];
    for (int64_t t = 0; t < nc; ++t) rptr[t + 1] += rptr[t];
    {
      std::vector<int64_t> fill(rptr.begin(), rptr.end() - 1);
      for (int64_t b = 0; b < nnear; ++b) rblk[fill[p.near[b].t]++] = b;
      for (int64_t t = 0; t < nc; ++t)
        std::sort(rblk.begin() + rptr[t], rblk.begin() + rptr[t + 1],
                  [&](int64_t a, int64_t c) { return p.near[a].s < p.near[c].s || (p.near[a].s == p.near[c].s && a < c); });
    }
    auto find_block = [&](int64_t t, int64_t sc) -> int64_t {   // first block (t, sc), or -1
      auto lo = std::lower_bound(rblk.begin() + rptr[t], rblk.begin() + rptr[t + 1], sc,
                                 [&](int64_t a, int64_t v) { return p.near[a].s < v; });
      return (lo != rblk.begin() + rptr[t + 1] && p.near[*lo].s == sc) ? *lo : -1;
    };
    std::vector<NearDesc> eval;
    std::vector<std::pair<int64_t, int64_t>> mirrors;      // (mirror block, evaluated block)
    for (int64_t b = 0; b < nnear; ++b) {
      const int64_t t = p.near[b].t, sc = p.near[b].s;
      if (t > sc) {
        const int64_t m = find_block(sc, t);
        if (m >= 0) {
          mirrors.push_back({b, m});
          continue;
        }
      }
      eval.push_back(nd[b]);
    }
    const int es = h.precision != DH2_FP64 ? (int)sizeof(z32) : (int)sizeof(C64);
    h.near_d = h.alloc<char>((size_t)std::max<int64_t>(off, 1) * es);
    NearDesc* ndd = h.upload(eval);
    const double* xq = paper_quad ? x9 : x16;
    const double* wq = paper_quad ? w9 : w16;
    const int nq = paper_quad ? 9 : 16;
    if (h.precision != DH2_FP64)
      launch_near<float>(ndd, (int64_t)eval.size(), p.kappa, xq, wq, selfl, h.near_d, nq, h.stream);
    else
      launch_near<double>(ndd, (int64_t)eval.size(), p.kappa, xq, wq, selfl, h.near_d, nq, h.stream);
    h.check_launch();
    // the paper's quadrature: touching pairs of the evaluated blocks take the
    // Sauter-Erichsen-Schwab rules (mirrors get them by the transposition below)
    TouchDesc* tdd = nullptr;
    if (paper_quad) {
      std::vector<uint8_t> mirrored(nnear, 0);
      for (const auto& mb : mirrors) mirrored[mb.first] = 1;
      const std::vector<TouchDesc> td = touching_pairs(p, g, h.near_off, mirrored, rptr, rblk);
      h.stats.touching_pairs = (int64_t)td.size();
      if (!td.empty()) {
        tdd = h.upload(td);
        SesTab tab{};
        gauss_legendre01(kSesOrder, tab.g, tab.gw);
        if (h.precision != DH2_FP64)
          launch_touch<float>(tdd, (int64_t)td.size(), Vd, tab, p.kappa, h.near_d, h.stream);
        else
          launch_touch<double>(tdd, (int64_t)td.size(), Vd, tab, p.kappa, h.near_d, h.stream);
        h.check_launch();
      }
    }
    std::vector<CopyDesc> cp;
    cp.reserve(mirrors.size());
    for (const auto& mb : mirrors) {
      const NearDesc& a = nd[mb.second];                  // evaluated: a.nr x a.nc
      cp.push_back({(char*)h.near_d + a.off * es, (char*)h.near_d + nd[mb.first].off * es, a.nr, a.nc,
                    a.nr, a.nc});
    }
    CopyDesc* cpd = cp.empty() ? nullptr : h.upload(cp);
    if (!cp.empty()) {
      if (h.precision != DH2_FP64) launch_transpose_blocks<float>(cpd, (int64_t)cp.size(), h.stream);
      else launch_transpose_blocks<double>(cpd, (int64_t)cp.size(), h.stream);
      h.check_launch();
    }
    h.sync();
    h.release(ndd);
    if (cpd) h.release(cpd);
    if (tdd) h.release(tdd);
  }
  h.stats.ms_near = now_ms() - t0;

  // workspace
  bd.ws_bytes = h.ws_bytes;
  bd.ws = (char*)h.alloc<char>(bd.ws_bytes);
  bd.cnt_d = h.alloc<int32_t>((size_t)std::max<int64_t>(bd.ns, 1));

  t0 = now_ms();
  bd.x7 = paper_quad ? x9 : x7;
  bd.w7 = paper_quad ? w9 : w7;
  bd.nq_far = paper_quad ? 9 : 7;
  bd.interpolation();
  h.sync();
  h.stats.ms_interp = now_ms() - t0;
  t0 = now_ms();
  bd.basis_weights();
  h.sync();
  h.stats.ms_basis_weights = now_ms() - t0;
  t0 = now_ms();
  if (bd.use_gram()) {
    // block weights and the blocks' share of the total weights in one pass
    bd.weights_gram();
    h.stats.ms_block_weights = now_ms() - t0;
    t0 = now_ms();
    bd.total_gram_topdown(true);
    bd.total_gram_topdown(false);
  } else {
    bd.block_weights();
    h.stats.ms_block_weights = now_ms() - t0;
    t0 = now_ms();
    bd.total_weights(true);
    bd.total_weights(false);
  }
  h.sync();
  h.stats.ms_total_weights = now_ms() - t0;
  t0 = now_ms();
  bd.truncation(true);
  bd.truncation(false);
  h.stats.ms_truncation = now_ms() - t0;
  t0 = now_ms();
  bd.projection();
  h.sync();
  h.stats.ms_projection = now_ms() - t0;
  h.stats.coupling_regeneration = p.adm.empty() ? 0.0 : (double)bd.n_coupling_gen / (double)p.adm.size();
  h.stats.coupling_in_products = p.adm.empty() ? 0.0 : (double)bd.n_coupling_fused / (double)p.adm.size();
  // release build-only buffers
  h.R_d = bd.R_d;
  h.Zr_d = bd.Zr_d;
  h.Zc_d = bd.Zc_d;
  h.rR = bd.rR;
  h.rZr = bd.rZr;
  h.rZc = bd.rZc;
  h.cheb = bd.ct;
  for (void* x : bd.keep_rc) h.release(x);
  h.release(bd.ws);
  h.release(bd.cnt_d);
  h.release(x7);
  h.release(w7);
  h.release(x16);
  h.release(w16);
  h.release(x9);
  h.release(w9);
  h.release(selfl);
  h.release(Vd);
  h.release(Td);
  if (h.precision != DH2_FP64) bd.narrow_to_fp32();
  bd.matvec_schedule();
  h.sync();
  if (h.autotune >= 2) {
    for (int& v : h.mv_var) v = h.autotune - 2;
  } else if (h.autotune == 1) {
    t0 = now_ms();
    tune_block_rows(h);
    h.stats.ms_autotune = now_ms() - t0;
  }
  for (int i = 0; i < 4; ++i) h.stats.mv_variant[i] = h.mv_var[i];
  h.stats.weights_gram = bd.use_gram() ? 1 : 0;
  h.stats.ms_total = now_ms() - t_start;

  // stats
  dh2_stats& s = h.stats;
  s.k = k;
  s.n = n;
  s.n_clusters = nc;
  s.n_leaves = 0;
  for (const auto& c : p.cl) s.n_leaves += c.leaf() ? 1 : 0;
  s.depth = p.depth;
  s.n_adm = (int64_t)p.adm.size();
  s.n_near = (int64_t)p.near.size();
  s.n_slots = bd.ns;
  s.n_row_slots = s.n_col_slots = 0;
  int64_t basis = 0;
  double sr = 0, sc = 0;
  s.rank_max_row = s.rank_max_col = 0;
  for (int64_t q = 0; q < bd.ns; ++q) {
    if (h.rank_row[q] >= 0) {
      ++s.n_row_slots;
      sr += h.rank_row[q];
      s.rank_max_row = std::max(s.rank_max_row, h.rank_row[q]);
      basis += (int64_t)h.Qr_m[q] * h.rank_row[q];
    }
    if (h.rank_col[q] >= 0) {
      ++s.n_col_slots;
      sc += h.rank_col[q];
      s.rank_max_col = std::max(s.rank_max_col, h.rank_col[q]);
      basis += (int64_t)h.Qc_m[q] * h.rank_col[q];
    }
  }
  s.rank_mean_row = s.n_row_slots ? sr / s.n_row_slots : 0;
  s.rank_mean_col = s.n_col_slots ? sc / s.n_col_slots : 0;
  int64_t coup = 0;
  for (const auto& a : p.adm)
    coup += (int64_t)h.rank_row[p.slot_of(a.t, a.c)] * h.rank_col[p.slot_of(a.s, a.c)];
  s.coupling_entries = coup;
  s.basis_entries = basis;
  const double e = h.precision == DH2_FP64 ? 16.0 : 8.0;
  s.matvec_bytes = e * ((double)s.near_entries + (double)coup + (double)basis);
  int64_t xsum = 0, ysum = 0;
  for (int64_t q = 0; q < bd.ns; ++q) {
    xsum += std::max(0, h.rank_col[q]);
    ysum += std::max(0, h.rank_row[q]);
  }
  s.matvec_bytes_per_rhs = e * (2.0 * n + 2.0 * (double)(xsum + ysum));
}

dh2_status fail(const Fail& f) {
  g_err = f.msg;
  return f.st;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* dh2_last_error(void) { return g_err.c_str(); }

dh2_status dh2_build(const dh2_geometry* geometry, double kappa, int order, double eta, int leafsize,
                     double tol, dh2_handle* out) {
  return dh2_build_ex(geometry, kappa, order, eta, leafsize, tol, nullptr, out);
}

dh2_status dh2_build_ex(const dh2_geometry* geometry, double kappa, int order, double eta,
                        int leafsize, double tol, const dh2_options* options, dh2_handle* out) {
  g_err.clear();
  if (!out) {
    g_err = "out is NULL";
    return DH2_ERR_ARG;
  }
  *out = nullptr;
  dh2_options opt{};
  opt.size = sizeof(opt);
  if (options) {
    if (options->size < sizeof(uint32_t) || options->size > sizeof(dh2_options)) {
      g_err = "options.size must be sizeof(dh2_options)";
      return DH2_ERR_ARG;
    }
    std::memcpy(&opt, options, options->size);
  }
  if (opt.precision != DH2_FP64 && opt.precision != DH2_FP32 && opt.precision != DH2_BF16X3) {
    g_err = "unknown precision";
    return DH2_ERR_ARG;
  }
  if (opt.norm != DH2_NORM_FROBENIUS && opt.norm != DH2_NORM_SPECTRAL) {
    g_err = "unknown norm";
    return DH2_ERR_ARG;
  }
  if (opt.rank_mode != DH2_RANKS_EXACT && opt.rank_mode != DH2_RANKS_LEARNED) {
    g_err = "unknown rank mode";
    return DH2_ERR_ARG;
  }
  if (opt.sketch_rank < 0) {
    g_err = "sketch_rank must be >= 0";
    return DH2_ERR_ARG;
  }
  if (opt.quadrature != DH2_QUAD_DEFAULT && opt.quadrature != DH2_QUAD_PAPER) {
    g_err = "quadrature must be DH2_QUAD_DEFAULT or DH2_QUAD_PAPER";
    return DH2_ERR_ARG;
  }
  if (opt.weights != DH2_WEIGHTS_HOUSEHOLDER && opt.weights != DH2_WEIGHTS_GRAM) {
    g_err = "unknown weights mode";
    return DH2_ERR_ARG;
  }
  if (opt.autotune < 0 || opt.autotune >= 2 + mv_rows_variants()) {
    g_err = "autotune must be 0, 1 or 2 + a pipeline shape in [0, " + std::to_string(mv_rows_variants()) + ")";
    return DH2_ERR_ARG;
  }
  const double eta1 = opt.eta1 > 0 ? opt.eta1 : 10.0;
  const int max_nrhs = opt.max_nrhs > 0 ? opt.max_nrhs : 16;
  const double wsgb = opt.workspace_gb > 0 ? opt.workspace_gb : 8.0;
  std::unique_ptr<dh2_problem> h;
  try {
    validate(geometry, kappa, order, eta, leafsize, tol, eta1);
    if (max_nrhs > 4096) throw Fail{DH2_ERR_ARG, "max_nrhs too large"};
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
      throw Fail{DH2_ERR_DEVICE, "no HIP device available"};
    h.reset(new dh2_problem());
    HIPCHK(hipGetDevice(&h->device));
    {
      int lds = 0;
      HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
      set_lds_limit((size_t)lds);
    }
    h->precision = opt.precision;
    h->stream = (hipStream_t)opt.stream;
    h->max_nrhs = max_nrhs;
    h->tol = tol;
    h->norm_mode = opt.norm;
    h->rank_mode = opt.rank_mode;
    h->sketch_rank = opt.sketch_rank;
    h->autotune = opt.autotune;
    h->weights_mode = opt.weights;
    h->quadrature = opt.quadrature;
    h->plan.kappa = kappa;
    h->plan.order = order;
    h->plan.eta = eta;
    h->plan.leafsize = leafsize;
    h->plan.eta1 = eta1;
    h->ws_bytes = (size_t)(wsgb * (1ull << 30));
    // small problems do not need the full workspace
    const double k = (double)order * order * order;
    const double est = (double)geometry->n_triangles * k * 16.0 * 64.0 + 64.0 * k * k * 16.0 * 64.0;
    if ((double)h->ws_bytes > est) h->ws_bytes = (size_t)est;
    h->stats.size = sizeof(dh2_stats);
    build_all(*h, *geometry);
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return DH2_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return DH2_ERR_DEVICE;
  }
  *out = h.release();
  return DH2_OK;
}

extern "C++" {
namespace {
// Runs the matvec phases on the handle's stream; with ev != NULL records
// ev[g] before group g (0 gather, 1 forward, 2 coupling, 3 backward, 4 near,
// 5 leaf output, 6 scatter) and ev[7] at the end.
// ---- matvec schedule (begin) ----
template <typename R>
void run_matvec_t(dh2_problem* h, const dh2_problem::MvView& v, const void* X, void* Y, int nrhs, hipEvent_t* ev,
                  hipStream_t st) {
  const int64_t n = h->plan.n;
  auto mark = [&](int g) {
    if (ev) HIPCHK(hipEventRecord(ev[g], st));
  };
  auto terms = [&](int g) {
    for (const auto& ph : h->mv_phases)
      if (ph.group == g && ph.out_end > ph.out_begin)
        launch_mv_terms<R>(v.outs + ph.out_begin, ph.out_end - ph.out_begin, v.terms, nrhs, st);
  };
  // every right-hand-side count runs the matrix-core block rows on row-major
  // copies (columns past nrhs read zeros)
  mark(0);
  launch_mv_permute<R>(X, v.Xp, h->perm_d, n, nrhs, 1, st);
  launch_mv_transpose<R>(v.Xp, v.XT, n, nrhs, st);
  mark(1);
  terms(1);
  launch_mv_slot_transpose<R>(v.xh_tr, h->n_xh_tr, v.xhT, nrhs, st);
  mark(2);
  const int* var = h->mv_var + (nrhs > 16 ? 2 : 0);
  launch_mv_rows_mfma<R>(v.coup_rows, h->coup_split, h->coup_mf_segs_d, v.xhT, h->zero16_d, nrhs, 1, var[1], st);
  mark(3);
  terms(3);
  mark(4);
  launch_mv_rows_mfma<R>(v.near_rows, h->near_split, h->near_segs_d, v.XT, h->zero16_d, nrhs, 0, var[0], st);
  mark(5);
  terms(5);
  mark(6);
  launch_mv_permute<R>(v.Yp, Y, h->perm_d, n, nrhs, 0, st);
  mark(7);
  HIPCHK(hipGetLastError());
}

void run_matvec(dh2_problem* h, const void* X, void* Y, int nrhs, hipEvent_t* ev, hipStream_t st,
                bool scratch = false) {
  const dh2_problem::MvView& v = scratch ? h->mv_scr : h->mv_own;
  if (h->precision != DH2_FP64) run_matvec_t<float>(h, v, X, Y, nrhs, ev, st);
  else run_matvec_t<double>(h, v, X, Y, nrhs, ev, st);
}
// ---- matvec schedule (end) ----
void run_matvec(dh2_problem* h, const void* X, void* Y, int nrhs, hipEvent_t* ev) {
  run_matvec(h, X, Y, nrhs, ev, h->stream);
}
}  // namespace
}  // extern "C++"

dh2_status dh2_matvec(dh2_handle h, const void* X, void* Y, int nrhs) {
  if (!h || !X || !Y) {
    g_err = "NULL handle or vector";
    return DH2_ERR_ARG;
  }
  if (nrhs < 1 || nrhs > h->max_nrhs) {
    g_err = "nrhs out of range [1, max_nrhs]";
    return DH2_ERR_ARG;
  }
  try {
    run_matvec(h, X, Y, nrhs, nullptr);
  } catch (const Fail& f) {
    return fail(f);
  }
  return DH2_OK;
}

dh2_status dh2_matvec_noalloc(dh2_handle h, const void* X, void* Y, int nrhs, void* stream) {
  if (!h || !X || !Y) {
    g_err = "NULL handle or vector";
    return DH2_ERR_ARG;
  }
  if (nrhs < 1 || nrhs > h->max_nrhs) {
    g_err = "nrhs out of range [1, max_nrhs]";
    return DH2_ERR_ARG;
  }
  if (!h->has_scr) {
    size_t lim = 0;
    (void)scratch_region(&lim);
    g_err = "the product's staging of this handle (" + std::to_string(h->stage_bytes >> 20) +
            " MiB for max_nrhs = " + std::to_string(h->max_nrhs) + ") exceeds the static scratch of " +
            std::to_string(lim >> 20) + " MiB (or its address lookup failed); build with a smaller max_nrhs";
    return DH2_ERR_ARG;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device) {
    (void)hipGetLastError();
    g_err = "the current device is not the handle's device";
    return DH2_ERR_ARG;
  }
  try {
    run_matvec(h, X, Y, nrhs, nullptr, (hipStream_t)stream, true);
  } catch (const Fail& f) {
    return fail(f);
  }
  return DH2_OK;
}

dh2_status dh2_matvec_stream(dh2_handle h, const void* X, void* Y, int nrhs, void* stream) {
  if (!h || !X || !Y) {
    g_err = "NULL handle or vector";
    return DH2_ERR_ARG;
  }
  if (nrhs < 1 || nrhs > h->max_nrhs) {
    g_err = "nrhs out of range [1, max_nrhs]";
    return DH2_ERR_ARG;
  }
  try {
    run_matvec(h, X, Y, nrhs, nullptr, (hipStream_t)stream);
  } catch (const Fail& f) {
    return fail(f);
  }
  return DH2_OK;
}

struct dh2_batch_s {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~dh2_batch_s() {
    // a launch of the graph may still run on the batch's stream
    if (stream) (void)hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipStream_t q : side) (void)hipStreamDestroy(q);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

dh2_status dh2_batch_create(const dh2_handle* handles, const void* const* X, void* const* Y, int nrhs,
                            int count, void* stream, dh2_batch* out) {
  g_err.clear();
  if (!out) {
    g_err = "out is NULL";
    return DH2_ERR_ARG;
  }
  *out = nullptr;
  if (!handles || !X || !Y || count < 1) {
    g_err = "NULL array or count < 1";
    return DH2_ERR_ARG;
  }
  {
    std::set<const void*> seen;
    for (int i = 0; i < count; ++i) {
      const dh2_handle h = handles[i];
      if (!h || !X[i] || !Y[i]) {
        g_err = "NULL handle or vector in the batch";
        return DH2_ERR_ARG;
      }
      if (!seen.insert(h).second) {
        g_err = "a handle appears twice in the batch";
        return DH2_ERR_ARG;
      }
      if (h->precision != handles[0]->precision) {
        g_err = "mixed precisions in one batch";
        return DH2_ERR_ARG;
      }
      if (nrhs < 1 || nrhs > h->max_nrhs) {
        g_err = "nrhs out of range [1, max_nrhs] for a handle of the batch";
        return DH2_ERR_ARG;
      }
    }
  }
  std::unique_ptr<dh2_batch_s> b(new dh2_batch_s());
  bool capturing = false;
  try {
    b->stream = (hipStream_t)stream;
    if (!b->stream) {
      HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
      b->own_stream = true;
    }
    const int nside = std::min(count, 8);
    b->side.resize(nside, nullptr);
    for (auto& q : b->side) HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    b->events.resize(nside + 1, nullptr);
    for (auto& e : b->events) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    capturing = true;
    // fork: every branch waits for the work already on the stream
    HIPCHK(hipEventRecord(b->events[nside], b->stream));
    for (int q = 0; q < nside; ++q) HIPCHK(hipStreamWaitEvent(b->side[q], b->events[nside], 0));
    for (int i = 0; i < count; ++i) run_matvec(handles[i], X[i], Y[i], nrhs, nullptr, b->side[i % nside]);
    // join
    for (int q = 0; q < nside; ++q) {
      HIPCHK(hipEventRecord(b->events[q], b->side[q]));
      HIPCHK(hipStreamWaitEvent(b->stream, b->events[q], 0));
    }
    capturing = false;
    HIPCHK(hipStreamEndCapture(b->stream, &b->graph));
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  } catch (...) {
    if (capturing) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(b->stream, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    try {
      throw;
    } catch (const Fail& f) {
      return fail(f);
    } catch (const std::bad_alloc&) {
      g_err = "host allocation failed";
      return DH2_ERR_OOM;
    } catch (const std::exception& e) {
      g_err = e.what();
      return DH2_ERR_DEVICE;
    }
  }
  *out = b.release();
  return DH2_OK;
}

dh2_status dh2_batch_run(dh2_batch b) {
  if (!b) {
    g_err = "NULL batch";
    return DH2_ERR_ARG;
  }
  try {
    HIPCHK(hipGraphLaunch(b->exec, b->stream));
    if (b->own_stream) HIPCHK(hipStreamSynchronize(b->stream));
  } catch (const Fail& f) {
    return fail(f);
  }
  return DH2_OK;
}

void dh2_batch_free(dh2_batch b) { delete b; }

dh2_status dh2_matvec_profile(dh2_handle h, const void* X, void* Y, int nrhs, double* phase_ms,
                              double* near_bytes) {
  if (!h || !X || !Y || !phase_ms) {
    g_err = "NULL argument";
    return DH2_ERR_ARG;
  }
  if (nrhs < 1 || nrhs > h->max_nrhs) {
    g_err = "nrhs out of range [1, max_nrhs]";
    return DH2_ERR_ARG;
  }
  hipEvent_t ev[8] = {};
  try {
    for (int i = 0; i < 8; ++i) HIPCHK(hipEventCreate(&ev[i]));
    run_matvec(h, X, Y, nrhs, ev);
    HIPCHK(hipEventSynchronize(ev[7]));
    for (int i = 0; i < 7; ++i) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      phase_ms[i] = ms;
    }
    if (near_bytes) *near_bytes = (double)h->near_matvec_bytes;
  } catch (const Fail& f) {
    for (int i = 0; i < 8; ++i)
      if (ev[i]) hipEventDestroy(ev[i]);
    return fail(f);
  }
  for (int i = 0; i < 8; ++i) hipEventDestroy(ev[i]);
  return DH2_OK;
}

void dh2_free(dh2_handle h) { delete h; }

dh2_status dh2_build_many(int count, const dh2_geometry* geometries, const double* kappa, const int* order,
                          const double* eta, const int* leafsize, const double* tol, const dh2_options* options,
                          int threads, dh2_handle* out) {
  g_err.clear();
  if (!out || count < 1 || !geometries || !kappa || !order || !eta || !leafsize || !tol) {
    g_err = "NULL array or count < 1";
    return DH2_ERR_ARG;
  }
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  dh2_options base{};
  base.size = sizeof(base);
  if (options) {
    if (options->size < sizeof(uint32_t) || options->size > sizeof(dh2_options)) {
      g_err = "options.size must be sizeof(dh2_options)";
      return DH2_ERR_ARG;
    }
    std::memcpy(&base, options, options->size);
  }
  const int nthr = std::max(1, std::min(count, threads > 0 ? threads : 8));
  std::vector<hipStream_t> streams(count, nullptr);
  std::vector<dh2_status> st(count, DH2_OK);
  std::vector<std::string> msg(count);
  for (int i = 0; i < count; ++i) {
    if (hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipStreamDestroy(streams[j]);
      g_err = "stream creation failed";
      return DH2_ERR_DEVICE;
    }
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::atomic<int> next{0};
  auto worker = [&]() {
    (void)hipSetDevice(dev);
    for (int i = next++; i < count; i = next++) {
      dh2_options o = base;
      o.stream = streams[i];
      st[i] = dh2_build_ex(&geometries[i], kappa[i], order[i], eta[i], leafsize[i], tol[i], &o, &out[i]);
      if (st[i] == DH2_OK) out[i]->own_stream = true;
      else msg[i] = g_err;
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthr; ++t) {
    try {
      pool.emplace_back(worker);
    } catch (...) {
      break;   // fewer threads: the calling thread takes the remaining problems
    }
  }
  worker();
  for (auto& t : pool) t.join();
  for (int i = 0; i < count; ++i) {
    if (st[i] == DH2_OK) continue;
    for (int j = 0; j < count; ++j) {
      if (out[j]) dh2_free(out[j]);   // destroys its own stream
      else (void)hipStreamDestroy(streams[j]);
      out[j] = nullptr;
    }
    g_err = "problem " + std::to_string(i) + ": " + msg[i];
    return st[i];
  }
  return DH2_OK;
}

dh2_status dh2_get_stats(dh2_handle h, dh2_stats* s) {
  if (!h || !s || s->size != sizeof(dh2_stats)) {
    g_err = "NULL handle / stats or wrong stats size";
    return DH2_ERR_ARG;
  }
  *s = h->stats;
  return DH2_OK;
}

dh2_status dh2_inspect(dh2_handle h, int what, int64_t index, double* out, int64_t* rows,
                       int64_t* cols) {
  if (!h || !rows || !cols) {
    g_err = "NULL argument";
    return DH2_ERR_ARG;
  }
  try {
    const Plan& p = h->plan;
    const int k = p.k;
    const int64_t ns = (int64_t)p.slots.size();
    const void* src = nullptr;
    int64_t r = 0, c = 0;
    std::vector<double> host;
    switch (what) {
      case DH2_INSPECT_NEAR: {
        if (index < 0 || index >= (int64_t)p.near.size()) throw Fail{DH2_ERR_ARG, "index out of range"};
        r = p.cl[p.near[index].t].size;
        c = p.cl[p.near[index].s].size;
        if (h->precision != DH2_FP64) {
          // complex64 storage, widened on the host
          if (out && r * c > 0) {
            HIPCHK(hipStreamSynchronize(h->stream));
            std::vector<z32> tmp((size_t)(r * c));
            HIPCHK(hipMemcpy(tmp.data(), (const z32*)h->near_d + h->near_off[index], tmp.size() * sizeof(z32),
                             hipMemcpyDeviceToHost));
            host.resize(2 * tmp.size());
            for (size_t i = 0; i < tmp.size(); ++i) {
              host[2 * i] = tmp[i].x;
              host[2 * i + 1] = tmp[i].y;
            }
          }
        } else {
          src = (const z64*)h->near_d + h->near_off[index];
        }
        break;
      }
      case DH2_INSPECT_LEAF_BASIS: {
        if (index < 0 || index >= ns || h->V_off[index] < 0) throw Fail{DH2_ERR_ARG, "not a leaf slot"};
        r = p.cl[p.slots[index].t].size;
        c = k;
        src = (const z64*)h->V_d + h->V_off[index];
        break;
      }
      case DH2_INSPECT_TRANSFER: {
        const int64_t q = index / 2;
        if (index < 0 || q >= ns || h->E_off[q] < 0) throw Fail{DH2_ERR_ARG, "not an inner slot"};
        r = k;
        c = k;
        src = (const z64*)h->E_d + h->E_off[q] + (index % 2) * (int64_t)k * k;
        break;
      }
      case DH2_INSPECT_RANK_PRED_ROW:
      case DH2_INSPECT_RANK_PRED_COL:
      case DH2_INSPECT_RANK_ROW:
      case DH2_INSPECT_RANK_COL: {
        const auto& rk = what == DH2_INSPECT_RANK_ROW ? h->rank_row
                         : what == DH2_INSPECT_RANK_COL ? h->rank_col
                         : what == DH2_INSPECT_RANK_PRED_ROW ? h->pred_row : h->pred_col;
        if ((int64_t)rk.size() != ns) throw Fail{DH2_ERR_ARG, "no predicted ranks (exact truncation)"};
        r = ns;
        c = 1;
        host.resize(2 * ns);
        for (int64_t q = 0; q < ns; ++q) {
          host[2 * q] = rk[q];
          host[2 * q + 1] = 0;
        }
        break;
      }
      case DH2_INSPECT_SIGMA_ROW:
      case DH2_INSPECT_SIGMA_COL: {
        if (index < 0 || index >= ns) throw Fail{DH2_ERR_ARG, "index out of range"};
        const auto& sg = (what == DH2_INSPECT_SIGMA_ROW ? h->sig_row : h->sig_col)[index];
        r = (int64_t)sg.size();
        c = 1;
        host.resize(2 * r);
        for (int64_t i = 0; i < r; ++i) {
          host[2 * i] = sg[i];
          host[2 * i + 1] = 0;
        }
        break;
      }
      case DH2_INSPECT_BASIS_WEIGHT:
      case DH2_INSPECT_TOTAL_WEIGHT_ROW:
      case DH2_INSPECT_TOTAL_WEIGHT_COL: {
        if (index < 0 || index >= ns) throw Fail{DH2_ERR_ARG, "index out of range"};
        const z64* base = what == DH2_INSPECT_BASIS_WEIGHT ? h->R_d
                          : what == DH2_INSPECT_TOTAL_WEIGHT_ROW ? h->Zr_d : h->Zc_d;
        const auto& rows = what == DH2_INSPECT_BASIS_WEIGHT ? h->rR
                           : what == DH2_INSPECT_TOTAL_WEIGHT_ROW ? h->rZr : h->rZc;
        r = rows[index];
        c = k;
        // projected total weights of leaves narrower than k (Z^* V^H): #t columns
        if (what != DH2_INSPECT_BASIS_WEIGHT) {
          const Cluster& cl = p.cl[p.slots[index].t];
          if (cl.leaf() && cl.size < k) c = cl.size;
        }
        // rows of a k x k column-major buffer: copy column by column
        if (out && r > 0) {
          HIPCHK(hipStreamSynchronize(h->stream));
          std::vector<z64> full((size_t)k * k);
          HIPCHK(hipMemcpy(full.data(), base + (size_t)index * k * k, full.size() * sizeof(z64),
                           hipMemcpyDeviceToHost));
          host.resize((size_t)2 * r * c);
          for (int64_t j = 0; j < c; ++j)
            for (int64_t i = 0; i < r; ++i) {
              host[2 * (i + j * r)] = full[i + j * k].x;
              host[2 * (i + j * r) + 1] = full[i + j * k].y;
            }
        }
        break;
      }
      case DH2_INSPECT_COUPLING: {
        if (index < 0 || index >= (int64_t)p.adm.size()) throw Fail{DH2_ERR_ARG, "index out of range"};
        r = k;
        c = k;
        if (out) {
          const AdmBlock& a = p.adm[index];
          std::vector<CoupDesc> cd{{(int32_t)a.t, (int32_t)a.s, h->dir_off[p.cl[a.t].level] + a.c}};
          CoupDesc* cdd = h->upload(cd);
          z64* S = h->alloc<z64>((size_t)k * k);
          launch_coupling<double>(cdd, 1, h->cheb, p.kappa, h->box_d, h->dirs_d, S, h->stream);
          HIPCHK(hipGetLastError());
          h->sync();
          host.resize((size_t)2 * k * k);
          HIPCHK(hipMemcpy(host.data(), S, (size_t)k * k * sizeof(z64), hipMemcpyDeviceToHost));
          h->release(S);
          h->release(cdd);
        }
        break;
      }
      case DH2_INSPECT_OMEGA: {
        r = (int64_t)h->omega.size();
        c = 1;
        host.resize(2 * r);
        for (int64_t i = 0; i < r; ++i) {
          host[2 * i] = h->omega[i];
          host[2 * i + 1] = 0;
        }
        break;
      }
      default:
        throw Fail{DH2_ERR_ARG, "unknown inspection target"};
    }
    *rows = r;
    *cols = c;
    if (out && r * c > 0) {
      if (src) {
        HIPCHK(hipStreamSynchronize(h->stream));
        HIPCHK(hipMemcpy(out, src, (size_t)r * c * 16, hipMemcpyDeviceToHost));
      } else {
        std::memcpy(out, host.data(), host.size() * sizeof(double));
      }
    }
  } catch (const Fail& f) {
    return fail(f);
  }
  return DH2_OK;
}

// ---------------------------------------------------------------------------
dh2_status dh2_plan_create(const dh2_geometry* geometry, double kappa, int order, double eta,
                           int leafsize, double eta1, dh2_plan* out) {
  g_err.clear();
  if (!out) {
    g_err = "out is NULL";
    return DH2_ERR_ARG;
  }
  *out = nullptr;
  try {
    validate(geometry, kappa, order, eta, leafsize, 0.0, eta1 > 0 ? eta1 : 10.0);
    std::unique_ptr<dh2_plan_s> p(new dh2_plan_s());
    std::string err = build_plan(geometry->vertices, geometry->n_vertices, geometry->triangles,
                                 geometry->n_triangles, kappa, order, eta, leafsize,
                                 eta1 > 0 ? eta1 : 10.0, p->plan);
    if (!err.empty()) throw Fail{DH2_ERR_ARG, err};
    *out = p.release();
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return DH2_ERR_OOM;
  }
  return DH2_OK;
}

dh2_status dh2_plan_get_sizes(dh2_plan pl, dh2_plan_sizes* s) {
  if (!pl || !s) {
    g_err = "NULL argument";
    return DH2_ERR_ARG;
  }
  const Plan& p = pl->plan;
  s->n = p.n;
  s->n_clusters = (int64_t)p.cl.size();
  s->depth = p.depth;
  s->n_adm = (int64_t)p.adm.size();
  s->n_near = (int64_t)p.near.size();
  int64_t nd = 0;
  for (const auto& d : p.dirs) nd += (int64_t)d.size() / 3;
  s->n_dirs_total = nd;
  s->n_slots = (int64_t)p.slots.size();
  return DH2_OK;
}

dh2_status dh2_plan_export(dh2_plan pl, int64_t* perm, int64_t* cl_first, int64_t* cl_size,
                           int32_t* cl_level, int64_t* cl_parent, double* cl_box,
                           int32_t* level_ndirs, double* dirs, int32_t* sd, int64_t* adm,
                           int64_t* near, int64_t* slots) {
  if (!pl) {
    g_err = "NULL plan";
    return DH2_ERR_ARG;
  }
  const Plan& p = pl->plan;
  if (perm) std::copy(p.perm.begin(), p.perm.end(), perm);
  for (size_t t = 0; t < p.cl.size(); ++t) {
    const Cluster& c = p.cl[t];
    if (cl_first) cl_first[t] = c.first;
    if (cl_size) cl_size[t] = c.size;
    if (cl_level) cl_level[t] = c.level;
    if (cl_parent) cl_parent[t] = c.parent;
    if (cl_box)
      for (int d = 0; d < 3; ++d) {
        cl_box[6 * t + d] = c.lo[d];
        cl_box[6 * t + 3 + d] = c.hi[d];
      }
  }
  int64_t off = 0;
  for (int l = 0; l <= p.depth; ++l) {
    const int64_t nd = (int64_t)p.dirs[l].size() / 3;
    if (level_ndirs) level_ndirs[l] = (int32_t)nd;
    for (int64_t c = 0; c < nd; ++c) {
      if (dirs)
        for (int d = 0; d < 3; ++d) dirs[3 * (off + c) + d] = p.dirs[l][3 * c + d];
      if (sd) sd[off + c] = l < p.depth ? p.sd[l][c] : -1;
    }
    off += nd;
  }
  for (size_t b = 0; b < p.adm.size(); ++b)
    if (adm) {
      adm[3 * b] = p.adm[b].t;
      adm[3 * b + 1] = p.adm[b].s;
      adm[3 * b + 2] = p.adm[b].c;
    }
  for (size_t b = 0; b < p.near.size(); ++b)
    if (near) {
      near[2 * b] = p.near[b].t;
      near[2 * b + 1] = p.near[b].s;
    }
  for (size_t q = 0; q < p.slots.size(); ++q)
    if (slots) {
      slots[3 * q] = p.slots[q].t;
      slots[3 * q + 1] = p.slots[q].c;
      slots[3 * q + 2] = (p.slot_row[q] ? 1 : 0) | (p.slot_col[q] ? 2 : 0);
    }
  return DH2_OK;
}

dh2_status dh2_plan_rank_features(dh2_plan pl, double tol, int kind, float* out) {
  if (!pl || !out || (kind != 0 && kind != 1) || !(tol >= 0.0)) {
    g_err = "NULL plan or output, kind not 0 / 1, or tol < 0";
    return DH2_ERR_ARG;
  }
  try {
    std::vector<float> f;
    rank_features(pl->plan, tol, kind == 0, f);
    std::copy(f.begin(), f.end(), out);
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return DH2_ERR_OOM;
  }
  return DH2_OK;
}

void dh2_plan_free(dh2_plan p) { delete p; }

}  // extern "C"
