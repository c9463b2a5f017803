// Host-side hierarchy of the DH^2 matrix: cluster tree, directions, block tree
// and the per-level work lists derived from them (Section 2 of Boerm & Boerst,
// "Hybrid matrix compression for high-frequency problems").
//
// Every decision (split axis, split side, admissibility, nearest direction)
// is taken in IEEE double arithmetic in a fixed operation order; this file is
// compiled with -ffp-contract=off so that the result is reproducible.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace dh2 {

struct Cluster {
  int64_t first = 0;      // position of the first index in the permutation
  int64_t size = 0;       // number of triangles
  int32_t level = 0;
  int64_t parent = -1;
  int64_t child[2] = {-1, -1};
  int32_t nchild = 0;
  double lo[3] = {0, 0, 0};
  double hi[3] = {0, 0, 0};
  double diam = 0;
  bool leaf() const { return nchild == 0; }
};

struct AdmBlock {
  int64_t t, s;
  int32_t c;    // direction index in D_{level(t)}
};

struct NearBlock {
  int64_t t, s;
};

// A (cluster, direction) pair that carries a basis.
struct Slot {
  int64_t t;
  int32_t c;
};

struct Plan {
  // inputs
  int64_t n = 0;
  double kappa = 0, eta = 1, eta1 = 10;
  int order = 0, leafsize = 0, k = 0;

  // cluster tree
  std::vector<int64_t> perm;             // cluster order -> triangle index
  std::vector<Cluster> cl;
  int32_t depth = 0;

  // directions: per level, 3 doubles per direction; dir_m[l] = 0 means D_l = {0}
  std::vector<std::vector<double>> dirs;
  std::vector<int32_t> dir_m;
  std::vector<std::vector<int32_t>> sd;  // sd[l][c] in D_{l+1}, l < depth

  // block tree leaves in recursion order
  std::vector<AdmBlock> adm;
  std::vector<NearBlock> near;

  // slots: every (t,c) with a row or column basis (downward closed)
  std::vector<Slot> slots;               // sorted by (level, t, c)
  std::vector<uint8_t> slot_row, slot_col;  // member of the row / column active set
  // lookup (t,c) -> slot: per cluster, sorted direction list with slot ids
  std::vector<std::vector<std::pair<int32_t, int64_t>>> cl_slots;

  // per slot: admissible blocks in which it is the row (t) resp. column (s) cluster,
  // blocks sorted by the other cluster index
  std::vector<int64_t> row_ptr, row_blk;   // CSR over slots
  std::vector<int64_t> col_ptr, col_blk;

  int64_t slot_of(int64_t t, int32_t c) const;
  int32_t son_dir(int64_t t, int32_t c) const {  // sd_{level(t)}(c)
    return sd[cl[t].level][c];
  }
  const double* dir(int64_t t, int32_t c) const { return &dirs[cl[t].level][3 * (size_t)c]; }
};

// Builds the hierarchy.  vertices: [nv][3]; triangles: [n][3] (validated by the caller).
// Returns an empty string on success, else an error message.
std::string build_plan(const double* vertices, int64_t nv, const int32_t* triangles, int64_t n,
                       double kappa, int order, double eta, int leafsize, double eta1, Plan& p);

}  // namespace dh2
