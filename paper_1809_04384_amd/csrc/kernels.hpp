// Descriptors and launch wrappers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev.hpp"

namespace dh2 {

// quadrature rules as barycentric coordinates + weights summing to one
struct QuadTab {
  double b7[7][3];
  double w7[7];
  double b16[16][3];
  double w16[16];
  double b9[9][3];    // the paper's rule of order 3 (Duffy-collapsed 3 x 3 Gauss)
  double w9[9];
};

// Sauter-Erichsen-Schwab rules of the paper's quadrature: the Gauss-Legendre
// rule on [0, 1] used in each of the four cube coordinates.
constexpr int kSesOrder = 5;
struct SesTab {
  double g[kSesOrder], gw[kSesOrder];
};

// One touching triangle pair (Section 5): the entry at element offset off of
// the near-field storage; vertex indices of the two triangles in the order
// that puts the shared part first (a shared vertex as A, a shared edge as
// A -> B of both); kind 1 common vertex, 2 common edge, 3 identical.
struct TouchDesc {
  int64_t off;
  int32_t va[3], vb[3];
  int32_t kind, pad;
};

struct NearDesc {     // inadmissible leaf t x s
  int64_t row0, col0; // first cluster-order position of t and s
  int32_t nr, nc;
  int64_t off;        // element offset of the column-major block
};

struct LeafDesc {     // leaf basis V_tc
  int64_t row0;
  int32_t nr;
  int32_t cl;
  int64_t dir;        // global direction index (row of the direction table)
  int64_t off;
};

struct TransDesc {    // transfer E_{t'c}
  int32_t child, parent;
  int64_t dir_parent, dir_child;
  int64_t off;
};

struct CoupDesc {     // coupling S_b of block (t, s, c)
  int32_t t, s;
  int64_t dir;
};

struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int32_t M, N, K, lda, ldb, ldc;
  int32_t opA, opB;   // 0 = N, 1 = T, 2 = C (conjugate transpose)
  int32_t accumulate;
  int32_t upper;      // FP64 kernel only: skip the 32 x 32 tiles of C below its diagonal
                      // (a Hermitian product whose upper triangle is all that is read)
  int32_t tri;        // zeros known in an operand (upper trapezoidal R factors of a QR):
                      // bit 0: op(A)[i][j] = 0 for j < i; bit 1: op(B)[j][n] = 0 for j < n.
                      // A tile then starts its K loop at its first row (bit 0) or column
                      // (bit 1); the products it skips are exact zeros, so C is unchanged.
  int32_t pad_;
  double alpha_re, alpha_im;
};

struct FoldTask {
  void* R;            // n x n FP64 complex, column-major
  int32_t n, ldr;
  int32_t piece_begin, piece_end;
  int32_t init_zero;  // start from R = 0
  int32_t compact;    // final fold: move the nonzero rows to the top, zero the rest
  int32_t* count;     // receives the number of nonzero rows when compacting (may be NULL)
};

struct FoldPiece {
  const void* P;      // rows x n complex of the piece precision, column-major
  int32_t rows, ld;
};

// Gram form of the total weights.  A slot's Gram matrix is the sum of the
// Gram matrices of its stacked-row segments; k_gram_sum adds the segments'
// upper triangles into the slot's (init: starting from zero), k_pchol turns it
// into a factor R with R^H R = G.
struct GramSumTask {
  void* G;            // nw x nw FP64 complex, leading dimension ldg (upper triangle written,
                      // or all of it when full)
  int32_t nw, ldg;
  int32_t src_begin, src_end;   // source matrices nw x nw, leading dimension ldg
  int32_t init, full;
};
void launch_gram_sum(const GramSumTask* t, int64_t ntasks, const void* const* srcs, hipStream_t st);

// Scaling of stacked rows: out[off + r] = 1 / w[index] for r < rows (zero when
// w[index] is not positive), the factor omega_b^-1 of the rows of block b in
// the total weights; then every row r of a segment (rows x cols, leading
// dimension rows) is multiplied by its factor f[r].
struct RowWeightTask {
  int64_t off;
  int32_t rows, pad;
  int64_t index;
};
void launch_row_weights(const RowWeightTask* t, int64_t ntasks, const double* w, double* out, hipStream_t st);
struct SegScaleTask {
  void* A;
  const double* f;
  int32_t rows, cols;
};
void launch_scale_segments(const SegScaleTask* t, int64_t ntasks, int maxcols, hipStream_t st);

struct PcholTask {
  void* G;            // in: Hermitian positive semi-definite nw x nw, leading dimension ldg
                      // (upper triangle read); out: R in rows 0 .. r-1 (nw columns, the
                      // original column order), rows r .. nw-1 zero
  void* scratch;      // nw (nw + 1) / 2 complex doubles, used when they do not fit in LDS
  int32_t nw, ldg;
  int32_t* count;     // receives r
};
// bytes of LDS k_pchol needs for order nw when the packed matrix is held there
size_t pchol_lds_bytes(int nw);
bool pchol_fits_lds(int nw);
void launch_pchol(const PcholTask* t, int64_t ntasks, int maxnw, hipStream_t st);

struct SvdTask {
  const void* B;      // rows x m FP64 complex, leading dimension ldb (exact truncation: the
                      // m x m R factor of A^H, rows = m)
  void* U;            // m x m output: the accumulated rotations V sorted by singular value
                      // (the left singular vectors of A = B^H); may be NULL
  double* sig;        // m singular values, descending
  int32_t* rank;      // chosen rank, -1 when the discarded norm alone exceeds the tolerance; may be NULL
  void* scratch;      // (rows + m) m complex doubles when not in LDS
  int32_t m, ldb, ldu, norm_mode;
  double eps;
  int32_t rows;       // rows of B (0 = m)
  int32_t ldw;
  void* W;            // rows x m output: the rotated columns of B divided by their norms,
                      // sorted (an orthonormal basis of range(B)); columns at or below
                      // 1e-13 of the largest are zero; may be NULL
  const double* resid; // Frobenius norm already discarded (its square is added to the rank
                       // rule's tail); may be NULL
};

// Gaussian sketch matrices: Omega (rows x cols, leading dimension ld), entry
// (i, j) = z0 + i z1 from Philox4x32-10 (counter (i, j, stream, 0), key (seed,
// 0)) and the Box-Muller transform.
struct SketchDesc {
  void* Om;
  int32_t rows, cols, ld, pad;
  int64_t stream;
};
void launch_sketch_omega(const SketchDesc* d, int64_t nd, uint32_t seed, hipStream_t st);

struct FrobDesc {
  const void* A;
  int32_t M, N, ld;
  int32_t pad;
  int64_t index;
};

// Spectral norm of M (rt x rs, leading dimension ldm) from the normalised power
// Gs (p x p, leading dimension ldg) of its Gram matrix: side 0 Gs ~ (M^* M)^(2^j)
// with p = rs, side 1 Gs ~ (M M^*)^(2^j) with p = rt.  out[index] = |M|_2.
constexpr int kSpecMaxP = 512;
struct SpecDesc {
  const void* G;
  const void* M;
  int32_t p, ldg, rt, rs, ldm, side;
  int64_t index;
};

struct CopyDesc {
  const void* src;
  void* dst;
  int32_t M, N, lds, ldd;
};

void launch_tri_data(int64_t n, const double* V, const int32_t* T, const int64_t* perm,
                     const QuadTab& qt, double* x7, double* w7, double* x16, double* w16,
                     double* x9, double* w9, double* self_lap, hipStream_t st);
// nq = 16: Q16 x Q16 and the closed-form self term; nq = 9: the paper's 9 x 9
// rule for every pair of distinct triangles (touching pairs are overwritten by
// launch_touch, the diagonal is left 0 for it)
template <typename R>
void launch_near(const NearDesc* d, int64_t nb, double kappa, const double* xq, const double* wq,
                 const double* self_lap, void* out, int nq, hipStream_t st);
// Sauter-Erichsen-Schwab entries of touching pairs, written over the near field
template <typename R>
void launch_touch(const TouchDesc* d, int64_t nt, const double* V, const SesTab& tab, double kappa,
                  void* out, hipStream_t st);
// far rule of nq points per triangle (7, or the paper's 9)
template <typename R>
void launch_leaf_basis(const LeafDesc* d, int64_t nb, const ChebTab& ct, double kappa,
                       const double* xf, const double* wf, int nq, const double* box, const double* dirs,
                       void* out, hipStream_t st);
template <typename R>
void launch_transfer(const TransDesc* d, int64_t nb, const ChebTab& ct, double kappa,
                     const double* box, const double* dirs, void* out, hipStream_t st);
template <typename R>
void launch_coupling(const CoupDesc* d, int64_t nb, const ChebTab& ct, double kappa,
                     const double* box, const double* dirs, void* out, hipStream_t st);

// C = alpha A S_b (conj 0) or alpha A S_b^H (conj 1) with S_b of block
// (t, s, dir) evaluated inside the product (k_gemm_coupling); A is M x k,
// column-major; C is M x k, FP64 data; form: the products on the FP64 (0) or
// FP32 (1) matrix cores or in the split-BF16x3 form (2), as the handle's other
// products.  mt: rows per chunk / 32 (1, 2 or 4); the
// caller groups the products by M (M <= 32 mt, or any M for mt = 4).
struct CoupGemmDesc {
  const void* A;
  void* C;
  int32_t M, lda, ldc;
  int32_t t, s;
  int32_t conj;
  int32_t tri;        // bit 0: A[i][j] = 0 for j < i (as GemmDesc.tri)
  int32_t pad_;
  int64_t dir;
  double alpha;
};
void launch_gemm_coupling(const CoupGemmDesc* d, int64_t nitems, int mt, const ChebTab& ct, double kappa,
                          const double* box, const double* dirs, int form, hipStream_t st);
template <typename R>
void launch_gemm(const GemmDesc* d, int64_t nitems, int maxM, int maxN, hipStream_t st);
// The same products on FP64 data with split-BF16x3 MFMA products and FP32 accumulation
void launch_gemm_bf16x3(const GemmDesc* d, int64_t nitems, int maxM, int maxN, hipStream_t st);
// The same products on FP64 data on the FP32 matrix cores (operands rounded to FP32, FP32 accumulation)
void launch_gemm_f32(const GemmDesc* d, int64_t nitems, int maxM, int maxN, hipStream_t st);
void set_lds_limit(size_t bytes);
int fold_rows_per_chunk(int n);
template <typename PT>
void launch_fold(const FoldTask* t, int64_t ntasks, const FoldPiece* p, int n, hipStream_t st);
// maxm, maxr: the largest m and rows of the tasks (LDS sizing)
void launch_jacobi(const SvdTask* t, int64_t ntasks, int maxm, int maxr, hipStream_t st);
template <typename R>
void launch_frob(const FrobDesc* d, int64_t nb, double* out, hipStream_t st);
// A <- A 2^-e per matrix (FP64 complex, FrobDesc.A is written), 2^(e-1) <= max |a| < 2^e
void launch_scale_pow2(const FrobDesc* d, int64_t nb, hipStream_t st);
void launch_spec_final(const SpecDesc* d, int64_t nb, double* out, hipStream_t st);
template <typename R>
void launch_copy(const CopyDesc* d, int64_t nb, hipStream_t st);
// dst (N x M, leading dimension ldd) = transpose of src (M x N, leading dimension lds), per descriptor
template <typename R>
void launch_transpose_blocks(const CopyDesc* d, int64_t nb, hipStream_t st);
void launch_narrow(const void* a, void* b, int64_t n, hipStream_t st);
// complex128 -> complex64 of many small arrays: dst[i] = src[i], i < n
struct NarrowDesc {
  const void* src;
  void* dst;
  int64_t n;
};
void launch_narrow_list(const NarrowDesc* d, int64_t nd, hipStream_t st);

}  // namespace dh2
