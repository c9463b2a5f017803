// Matvec of the compressed matrix: descriptors and launch wrappers (matvec.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dh2 {

// One term of an output: y[i, r] += sum_j op(A)[i, j] x[j + r ldx], j < K.
struct MvTerm {
  const void* A;
  const void* x;
  int32_t K, lda, ldx, op;   // op: 0 = A, 2 = A^H
};

// One output matrix y (M x nrhs, leading dimension ldy) and its term range.
struct MvOut {
  void* y;
  int32_t M, ldy;
  int32_t term_begin, term_end;
  int32_t accumulate;        // keep the current contents of y
  int32_t pad;
};

// Near field, one entry per leaf row cluster: rows [row0, row0 + nr) of Y get
// sum over segments of A (nr x ncols, leading dimension lda) times X rows
// [x0, x0 + ncols).  A segment is an inadmissible block restricted to the rows
// of this leaf.
struct NearRow {
  int64_t row0;
  int32_t nr;
  int32_t seg_begin, seg_end;
  int32_t pad;
};
struct NearSeg {
  const void* A;
  int64_t x0;
  int32_t lda, ncols;
};

// Block row of the matrix-core product: y (nr x nrhs, leading dimension ldy) =
// sum over the segments [seg_begin, seg_end) of A (nr x ncols, leading
// dimension lda) times rows [x0, x0 + ncols) of a row-major right-hand side
// XT[row * nrhs + r].  Used for the near field (Y rows of a leaf) and the
// coupling phase (y_tc of a row slot).
struct MfRow {
  void* y;
  int32_t ldy, nr;
  int32_t seg_begin, seg_end;
};
// Rows of a block-row launch per XCD: workgroup b runs on XCD b % 8, and XCD
// x takes the list entries [off[x], off[x + 1]) in order.  The grid has
// 8 * width workgroups, width = the largest share.
struct XcdSplit {
  int32_t off[9];
  int32_t width;
};
// zero16: 16 zero elements (device), read in place of right-hand-side entries
// outside a segment.  role: 0 near field, 1 coupling (names the kernel only).
// variant: pipeline shape, 0 .. mv_rows_variants() - 1 (0 = default).
template <typename R>
void launch_mv_rows_mfma(const MfRow* rows, const XcdSplit& split, const NearSeg* segs, const void* XT,
                         const void* zero16, int nrhs, int role, int variant, hipStream_t st);
int mv_rows_variants();

// Row-major copy of one slot vector: dst[(row0 + j) * nrhs + r] = src[j + r k].
struct SlotT {
  const void* src;
  int64_t row0;
  int32_t k, pad;
};
template <typename R>
void launch_mv_slot_transpose(const SlotT* d, int64_t cnt, void* dst, int nrhs, hipStream_t st);

// The generic transpose of the gathered X into row-major XT (XT[p nrhs + r]).
template <typename R>
void launch_mv_transpose(const void* X, void* XT, int64_t n, int nrhs, hipStream_t st);

template <typename R>
void launch_mv_terms(const MvOut* outs, int64_t nout, const MvTerm* terms, int nrhs, hipStream_t st);
template <typename R>
void launch_mv_permute(const void* src, void* dst, const int64_t* perm, int64_t n, int nrhs,
                       int gather, hipStream_t st);

}  // namespace dh2
