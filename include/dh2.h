/*
 * dh2.h -- C ABI of the MI355X (gfx950) library for the hybrid directional
 * H^2-matrix (DH^2) compression of the Helmholtz single-layer Galerkin matrix
 * (S. Boerm, C. Boerst, "Hybrid matrix compression for high-frequency
 * problems", arXiv 1809.04384).
 *
 * The matrix (Section 1, eq. (matrix)) is G_ij = int_{T_i} int_{T_j} g(x,y)
 * dy dx for the indicator functions of the triangles T_i of a surface mesh,
 * with g(x,y) = exp(i kappa |x-y|) / (4 pi |x-y|) (eq. (helmholtz)).
 * dh2_build constructs a DH^2 approximation by directional Chebyshev
 * interpolation (Section 2) and recompresses it algebraically (Section 3.2);
 * dh2_matvec applies the result.
 *
 * Conventions
 *   - complex numbers are interleaved (re, im) pairs of the handle's precision;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP device
 *     memory of the device that was current when the handle was built;
 *   - every function returns a dh2_status; on failure dh2_last_error() gives a
 *     message (thread-local, valid until the next call on the same thread);
 *     invalid arguments are detected before any side effect;
 *   - distinct handles may be used from different threads concurrently; one
 *     handle must not be used from two threads at the same time.
 */
#ifndef DH2_H
#define DH2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DH2_OK = 0,
  DH2_ERR_ARG = 1,       /* invalid argument (nothing was changed)            */
  DH2_ERR_GEOMETRY = 2,  /* index out of range or degenerate (zero-area) triangle */
  DH2_ERR_OOM = 3,       /* device or host allocation failed                  */
  DH2_ERR_DEVICE = 4,    /* HIP runtime error (no device, launch failure ...)  */
  DH2_ERR_NUMERIC = 5    /* non-finite value produced                         */
} dh2_status;

/* Surface mesh.  Host memory, read during the call only (the library copies
 * what it needs).  vertices: [n_vertices][3] row-major doubles; triangles:
 * [n_triangles][3] 0-based vertex indices.  The unknowns are the triangles
 * (piecewise-constant basis, Section 5), so n = n_triangles. */
typedef struct {
  int64_t n_vertices;
  const double* vertices;
  int64_t n_triangles;
  const int32_t* triangles;
} dh2_geometry;

/* Precision of a handle.
 *   DH2_FP64  everything in FP64; X / Y are complex128.
 *   DH2_FP32  the near field is evaluated and stored in FP32; the matrix
 *             products of the recompression (weighted couplings, block weights,
 *             total-weight pieces, basis changes, projections) run on the FP32
 *             matrix cores with FP32 accumulation on FP64 data; the recompressed
 *             couplings and bases are then rounded to complex64 and the matvec
 *             runs in FP32 on complex64 X / Y.
 *   DH2_BF16X3  the FP32 form with the matrix products of the recompression
 *             on the BF16 matrix cores instead: each FP64 operand
 *             is split into two bf16 parts and a product takes three of the four
 *             part products, accumulated in FP32 (about 2^-16 relative per
 *             product); ranks may differ from the FP64 form at near-ties.
 * Householder QR and SVD of the recompression are FP64 in all forms. */
typedef enum { DH2_FP64 = 0, DH2_FP32 = 1, DH2_BF16X3 = 2 } dh2_precision;

/* Error control of the recompression (Section 5).  Block weights
 * omega_b = |R_tc S_b R_sc^*|, the norm of the interpolated block, and the
 * rank rule per cluster and direction on the block-normalised total-weight
 * matrix with singular values sigma_1 >= sigma_2 >= ...:
 *   DH2_NORM_FROBENIUS  Frobenius norm; rank = smallest k with
 *                       sum_{i>k} sigma_i^2 <= eps^2 (the default, used for the
 *                       sphere and cube experiments of Section 5)
 *   DH2_NORM_SPECTRAL   spectral norm; rank = smallest k with sigma_{k+1} <= eps
 *                       (the variant of the sphere experiment at doubled wave
 *                       numbers, Section 5) */
typedef enum { DH2_NORM_FROBENIUS = 0, DH2_NORM_SPECTRAL = 1 } dh2_norm;

/* Truncation of the recompression (Section 3.2):
 *   DH2_RANKS_EXACT    the SVD of every truncation matrix (default);
 *   DH2_RANKS_LEARNED  the learned-rank form: a small multilayer perceptron
 *                      (12 features of geometry, direction, kappa and tol per
 *                      cluster and direction; three hidden layers of 128; BF16
 *                      weights, FP32 accumulation) predicts the rank, which sizes
 *                      a randomized range finder (Gaussian sketch with 8 extra
 *                      columns); the rank is then chosen by the same rule with the
 *                      norm the sketch discards added, and a slot whose discarded
 *                      norm alone exceeds the tolerance is truncated exactly
 *                      (FP64) instead.  Ranks are never below the exact ones and
 *                      each truncation meets the same block-relative bound. */
typedef enum { DH2_RANKS_EXACT = 0, DH2_RANKS_LEARNED = 1 } dh2_rank_mode;

/* How the total weight matrices Zhat_tc (Section 3.2) are factored.
 * HOUSEHOLDER: skinny QR of the stacked rows by Householder reflections, as the
 *   construction of the total weights states.
 * GRAM: the Gram matrix of the stacked rows (Zhat^H Zhat, a sum of FP64
 *   matrix-core products over row segments) factored by Cholesky with diagonal
 *   pivoting, Zhat = R with R^H R = the Gram matrix.  Zhat^H Zhat, which is all
 *   the truncation uses, is the same up to rounding; rounding now acts on the
 *   squares of the singular values, so this form is taken only for tol >= 1e-7
 *   (smaller tolerances use HOUSEHOLDER; dh2_stats.weights_gram says which ran).
 *   The blocks' share of the Gram matrices is formed together with the block
 *   weights, in two passes over the admissible blocks (column-slot order, then
 *   row-slot order; dh2_stats.ms_block_weights covers both), the inherited rows
 *   and the factorisation in a top-down pass (ms_total_weights).  The workspace
 *   must hold one block: 4 k^2 complex doubles and k doubles (DH2_ERR_OOM
 *   otherwise). */
typedef enum { DH2_WEIGHTS_HOUSEHOLDER = 0, DH2_WEIGHTS_GRAM = 1 } dh2_weights_mode;

/* Quadrature of the Galerkin entries (piecewise-constant basis on flat
 * triangles).
 * DH2_QUAD_DEFAULT: the near field by the 16-point Duffy-collapsed Gauss rule on
 *   both triangles, its diagonal by singularity subtraction (closed-form Laplace
 *   part plus the 16 x 16 rule on the bounded remainder); the leaf bases by the
 *   7-point rule.
 * DH2_QUAD_PAPER: the rules of Section 5: Sauter-Erichsen-Schwab quadrature of
 *   order 5 (5^4 tensor Gauss points per region of the regularising
 *   coordinates) for triangle pairs that share a vertex, an edge, or are
 *   identical; Gauss quadrature with the Duffy transformation of order 3 (3 x 3
 *   points per triangle) for every other near-field pair and for the leaf
 *   bases.  A touching pair is integrated with the triangle of lower index (in
 *   the caller's numbering) first, so the matrix stays exactly symmetric. */
typedef enum { DH2_QUAD_DEFAULT = 0, DH2_QUAD_PAPER = 1 } dh2_quadrature;

/* Optional settings.  Zero-initialise, set size = sizeof(dh2_options), then
 * override fields; zero fields take the defaults given here. */
typedef struct {
  uint32_t size;
  int32_t precision;  /* dh2_precision, default DH2_FP64                               */
  double eta1;        /* direction parameter eta_1 of eq. (admissibility) and of the
                         Remark on the construction of directions; default 10 (Section 5) */
  int32_t max_nrhs;   /* largest nrhs dh2_matvec will be called with; the matvec
                         workspace is reserved at build time.  Default 16.          */
  int32_t norm;       /* dh2_norm, default DH2_NORM_FROBENIUS                        */
  void* stream;       /* hipStream_t for all work of this handle; NULL = default stream */
  double workspace_gb;/* device workspace for the recompression batches; default 8 */
  int32_t rank_mode;  /* dh2_rank_mode, default DH2_RANKS_EXACT */
  int32_t sketch_rank;/* learned-rank form only: when > 0, every slot's predicted rank is
                         this value and no columns are added (a test hook) */
  int32_t autotune;   /* pipeline shape of the matrix-core block-row products (near field
                         and coupling phase): 0 = the default shape; 1 = time every shape
                         on this handle's own data at the end of the build and keep the
                         fastest per phase and right-hand-side class (nrhs <= 16, > 16),
                         another shape replacing the default only when more than 3 %
                         faster; 2 + v = use shape v everywhere (0 <= v < 4, a test hook).
                         Every shape gives the same results bit for bit. */
  int32_t weights;    /* dh2_weights_mode, default DH2_WEIGHTS_HOUSEHOLDER */
  int32_t quadrature; /* dh2_quadrature, default DH2_QUAD_DEFAULT */
} dh2_options;

typedef struct dh2_problem* dh2_handle;

/* Build the compressed matrix (synchronous: returns when the representation is
 * on the device).
 *   geometry  surface mesh (see dh2_geometry)
 *   kappa     wave number, >= 0
 *   order     Chebyshev points per axis m >= 1; interpolation rank k = m^3 (Section 5)
 *   eta       admissibility parameter eta_2 > 0 of the standard and parabolic
 *             conditions, eq. (admissibility), second and third line
 *   leafsize  maximal number of triangles in a leaf cluster, >= 1
 *   tol       recompression accuracy eps >= 0: per cluster and direction the rank is
 *             the smallest with sum_{i>k} sigma_i^2 <= eps^2 for the block-normalised
 *             total-weight matrices (block-relative Frobenius control, Section 5;
 *             options.norm = DH2_NORM_SPECTRAL: the smallest with sigma_{k+1} <= eps);
 *             tol = 0 keeps every nonzero singular value
 *   out       receives the handle; *out is set to NULL on failure
 * Errors: DH2_ERR_ARG (bad scalar), DH2_ERR_GEOMETRY (index out of range,
 * zero-area triangle, n < 1), DH2_ERR_OOM, DH2_ERR_DEVICE.  Partial builds are
 * freed. */
dh2_status dh2_build(const dh2_geometry* geometry, double kappa, int order, double eta,
                     int leafsize, double tol, dh2_handle* out);

/* As dh2_build with options (NULL = defaults). */
dh2_status dh2_build_ex(const dh2_geometry* geometry, double kappa, int order, double eta,
                        int leafsize, double tol, const dh2_options* options, dh2_handle* out);

/* Y = Gtilde X, the product with the compressed matrix: forward transform,
 * coupling, backward transform and near field (the product implied by
 * eq. (vsw) with the nested bases of eq. (nested)).
 *   X, Y   device pointers, column-major n x nrhs (leading dimension n),
 *          interleaved complex of the handle's precision, in the caller's
 *          triangle order; Y is overwritten; X and Y must not overlap
 *   nrhs   1 <= nrhs <= max_nrhs of the handle
 * Enqueued on the handle's stream; returns without synchronising and without
 * allocating.  Errors: DH2_ERR_ARG (NULL handle or pointer, nrhs out of
 * range), DH2_ERR_DEVICE (launch failure). */
dh2_status dh2_matvec(dh2_handle h, const void* X, void* Y, int nrhs);

/* dh2_matvec enqueued on `stream` (a hipStream_t; NULL = the default stream)
 * instead of the handle's stream.  Calls on one handle must not overlap in
 * time (they share its work buffers).  Errors as dh2_matvec. */
dh2_status dh2_matvec_stream(dh2_handle h, const void* X, void* Y, int nrhs, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dh2_matvec
 * enqueued on `stream` (NULL = the default stream) with its staging (gathered
 * X, its row-major copy, Y in cluster order, the coefficient vectors) in a
 * static device array of the library instead of the handle's buffers.  The
 * array holds 64 MiB per GPU, is allocated when the library is loaded on a
 * device and is kept until the process ends; this call allocates and frees
 * nothing.  The handle's staging for max_nrhs right-hand sides must fit
 * (about 6 n max_nrhs elements of the handle's complex type plus the
 * coefficient vectors); larger handles get DH2_ERR_ARG (build them with a
 * smaller max_nrhs).  All calls on one GPU share the array, whatever the
 * handle: calls that overlap in time on one GPU race and give wrong results.
 * Nothing in the array needs clearing between calls (every call writes each
 * staging entry before reading it).  The result equals dh2_matvec's bit for
 * bit.  Errors: as dh2_matvec; DH2_ERR_ARG also when the staging does not fit
 * or the current device is not the handle's. */
dh2_status dh2_matvec_noalloc(dh2_handle h, const void* X, void* Y, int nrhs, void* stream);

/* dh2_matvec with per-phase timing, for benchmarks: runs the same kernels,
 * records HIP events on the handle's stream between the phases and waits for
 * them (this call synchronises).  phase_ms[7] receives milliseconds of:
 * 0 gather of X into cluster order, 1 forward transform, 2 coupling,
 * 3 backward transform, 4 near field, 5 leaf output, 6 scatter of Y.
 * near_bytes (may be NULL) receives the near-field matrix bytes streamed by
 * phase 4.  Errors as dh2_matvec. */
dh2_status dh2_matvec_profile(dh2_handle h, const void* X, void* Y, int nrhs, double* phase_ms,
                              double* near_bytes);

/* Releases all device and host memory of the handle.  It first waits for all
 * work on the device (products enqueued on other streams by
 * dh2_matvec_stream or a batch may still read the handle's buffers), so it
 * must not be called while a stream of this device is being captured into a
 * graph.  NULL is a no-op. */
void dh2_free(dh2_handle h);

/* Builds of many problems side by side: problem i is what dh2_build_ex returns
 * for (geometries[i], kappa[i], order[i], eta[i], leafsize[i], tol[i], options),
 * built by one of up to `threads` host threads (0 = 8) on a stream of its own, so
 * the GPU runs the phases of several builds at once (small problems fill a
 * fraction of it each).  options->stream is ignored: every handle owns its
 * stream, which dh2_free destroys.  out receives count handles; on failure all
 * entries are NULL, every partial build is freed and the message names the
 * first failing problem.  Errors: as dh2_build_ex; DH2_ERR_ARG for NULL arrays
 * or count < 1. */
dh2_status dh2_build_many(int count, const dh2_geometry* geometries, const double* kappa, const int* order,
                          const double* eta, const int* leafsize, const double* tol,
                          const dh2_options* options, int threads, dh2_handle* out);

/* ---------------------------------------------------------------------------
 * Many products as one launch: a batch holds Y_i = Gtilde_i X_i for count
 * distinct handles (problems of any sizes, one precision), recorded once into
 * a HIP graph whose branches run the problems side by side (up to 8
 * concurrent branches, problems dealt round-robin), and replayed by one graph
 * launch.  Small problems, which fill a fraction of the GPU each, then share
 * it.  Each product is exactly the one dh2_matvec computes.
 *   handles  count distinct handles (a handle twice would race on its buffers)
 *   X, Y     count device pointers each, laid out as for dh2_matvec; the
 *            pointers are recorded: later runs read and write the same memory
 *   nrhs     1 <= nrhs <= max_nrhs of every handle
 *   stream   hipStream_t the graph is launched on; NULL = a stream owned by
 *            the batch, and then dh2_batch_run waits for the products
 *   out      receives the batch; *out is NULL on failure
 * The handles must outlive the batch.  Errors: DH2_ERR_ARG (NULL or repeated
 * handle, mixed precisions, nrhs out of range, count < 1), DH2_ERR_DEVICE
 * (capture or instantiation failed). */
typedef struct dh2_batch_s* dh2_batch;
dh2_status dh2_batch_create(const dh2_handle* handles, const void* const* X, void* const* Y, int nrhs,
                            int count, void* stream, dh2_batch* out);
/* One graph launch of all products (returns without synchronising unless the
 * batch owns its stream).  Errors: DH2_ERR_ARG (NULL), DH2_ERR_DEVICE. */
dh2_status dh2_batch_run(dh2_batch b);
/* Releases the graph and the batch's streams and events after waiting for the
 * batch's stream (a launch may still run).  The handles stay valid.  NULL is a
 * no-op. */
void dh2_batch_free(dh2_batch b);

/* Message of the last failure on this thread ("" if none). */
const char* dh2_last_error(void);

/* Counts, ranks, storage and timings of a built handle. */
typedef struct {
  uint32_t size;            /* set to sizeof(dh2_stats) by the caller */
  int32_t k;                /* interpolation rank m^3 */
  int64_t n, n_clusters, n_leaves, depth;
  int64_t n_adm, n_near;    /* admissible / inadmissible leaves of the block tree */
  int64_t n_slots, n_row_slots, n_col_slots;  /* (cluster, direction) pairs with bases */
  int64_t near_entries;     /* sum over inadmissible leaves of #t * #s */
  int64_t coupling_entries; /* sum over admissible leaves of k_tc * k_W,sc after recompression */
  int64_t basis_entries;    /* leaf bases + transfer matrices, rows and columns, after recompression */
  int32_t rank_max_row, rank_max_col;
  double rank_mean_row, rank_mean_col;
  double matvec_bytes;      /* algorithmic bytes of one matvec with nrhs = 1 (matrix data read once) */
  double matvec_bytes_per_rhs; /* additional algorithmic bytes per right-hand side */
  double ms_structure, ms_near, ms_interp, ms_basis_weights, ms_block_weights,
      ms_total_weights, ms_truncation, ms_projection, ms_total;
  double gemm_flops;        /* real flops of the build's complex matrix products, 8 M N K each
                               (4 N (N + 1) K for a Hermitian N x N product of which only the
                               upper triangle is formed; with a basis weight R_tc as a factor,
                               whose row i is zero left of column i, only the products outside
                               those zeros) */
  int64_t gemm_launches;    /* kernel launches of those products */
  double qr_flops;          /* real flops of the Householder QR steps of the recompression:
                               folding M rows into an n x n triangular factor counts 8 M n^2,
                               a factor started from zero subtracts (8/3) min(M, n)^3 */
  /* Workspace batches of the recompression phases (the interpolated couplings
   * S_b are generated per batch and never stored) and the (cluster, direction)
   * pairs of the two total-weight passes whose stacked rows were folded over
   * more than one batch. */
  int64_t batches_basis_weights, batches_block_weights, batches_total_weights_row,
      batches_total_weights_col, batches_truncation, batches_projection;
  int64_t slots_straddled;
  /* Regeneration factor: interpolated couplings S_b generated during the build,
   * divided by the number of admissible blocks (each phase that needs S_b
   * generates it again). */
  double coupling_regeneration;
  /* Learned-rank form: slots truncated through a sketch, sketches that missed the
   * tolerance and were truncated exactly, and the time of the rank prediction. */
  int64_t sketch_slots, sketch_fallbacks;
  double ms_rank_predict;
  /* Pipeline shapes of the block-row products in use: [0] near field and [1]
   * coupling for nrhs <= 16, [2] and [3] for nrhs > 16; the time the autotuner
   * took (0 without it). */
  int32_t mv_variant[4];
  double ms_autotune;
  int32_t weights_gram;     /* 1 when the total weights were factored in the Gram form */
  /* The part of coupling_regeneration evaluated inside the products that use
   * S_b (FP64 handles: the rows R S_b and R S_b^H of the Gram form with the
   * Frobenius norm, and the projection's C_tc S_b), so never stored. */
  double coupling_in_products;
  /* DH2_QUAD_PAPER: touching triangle pairs integrated by the Sauter-Erichsen-
   * Schwab rules (pairs of mirrored near-field blocks are copied, not counted). */
  int64_t touching_pairs;
} dh2_stats;

dh2_status dh2_get_stats(dh2_handle h, dh2_stats* s);

/* ---------------------------------------------------------------------------
 * Host-only hierarchy (no GPU needed): cluster tree, directions and block tree
 * exactly as dh2_build constructs them (Section 2: Definitions 'cluster tree',
 * 'directions', 'block tree', Remark 'construction of directions').  Used to
 * inspect and test the structure. */
typedef struct dh2_plan_s* dh2_plan;

typedef struct {
  int64_t n, n_clusters, depth, n_adm, n_near, n_dirs_total, n_slots;
} dh2_plan_sizes;

dh2_status dh2_plan_create(const dh2_geometry* geometry, double kappa, int order, double eta,
                           int leafsize, double eta1, dh2_plan* out);
dh2_status dh2_plan_get_sizes(dh2_plan p, dh2_plan_sizes* s);
/* Copies the hierarchy into caller-owned host arrays (any may be NULL):
 *   perm[n]                 cluster order -> triangle index
 *   cl_first[nc], cl_size[nc], cl_level[nc], cl_parent[nc] (-1 for the root)
 *   cl_box[nc][6]           lo_x, lo_y, lo_z, hi_x, hi_y, hi_z of the vertex box
 *   level_ndirs[depth+1]    #D_l (1 for D_l = {0})
 *   dirs[n_dirs_total][3]   directions of all levels, level after level
 *   sd[n_dirs_total]        son direction index in D_{l+1} (-1 on the last level)
 *   adm[n_adm][3]           (t, s, direction index) in block-recursion order
 *   near[n_near][2]         (t, s) in block-recursion order
 *   slots[n_slots][3]       (t, direction index, flags: 1 = row basis, 2 = column basis) */
dh2_status dh2_plan_export(dh2_plan p, int64_t* perm, int64_t* cl_first, int64_t* cl_size,
                           int32_t* cl_level, int64_t* cl_parent, double* cl_box,
                           int32_t* level_ndirs, double* dirs, int32_t* sd, int64_t* adm,
                           int64_t* near, int64_t* slots);
/* Features of the learned rank predictor (see DH2_RANKS_LEARNED) of every slot,
 * n_slots x 12 floats row-major into caller-owned host memory: kind 0 for the
 * row bases (blocks in which the cluster is the row cluster), 1 for the column
 * bases.  Features: log2 #t, level / depth, kappa diam(B_t), log10 tol (at
 * least -16), m, directional (|c| > 0), log2(1 + blocks of the slot's list),
 * log2(1 + blocks of its ancestors' lists), leaf, shortest / longest side of
 * B_t, log2(1 + triangles of the other clusters of its list), eta.
 * Errors: DH2_ERR_ARG (NULL, kind, tol < 0). */
dh2_status dh2_plan_rank_features(dh2_plan p, double tol, int kind, float* out);
void dh2_plan_free(dh2_plan p);

/* ---------------------------------------------------------------------------
 * Inspection of a built handle (tests): copies one intermediate matrix to a
 * caller-owned host buffer of complex doubles, column-major.  Call with
 * out = NULL to query rows / cols.  FP32 handles are widened to FP64.
 *   what = DH2_INSPECT_NEAR        index = inadmissible leaf (recursion order): #t x #s block
 *          DH2_INSPECT_LEAF_BASIS  index = slot of a leaf cluster: V_tc, #t x k (Section 2)
 *          DH2_INSPECT_TRANSFER    index = 2*slot + child: E_{t'c}, k x k (eq. (nested_apx))
 *          DH2_INSPECT_RANK_ROW    index ignored: k_tc of every slot (-1 if no row basis), n_slots x 1
 *          DH2_INSPECT_RANK_COL    same for the column basis
 *          DH2_INSPECT_SIGMA_ROW   index = slot: singular values of the truncation step
 *          DH2_INSPECT_SIGMA_COL   same for the column pass
 *          DH2_INSPECT_OMEGA       index ignored: block weights |G_int restricted to b|_F, n_adm x 1
 *          DH2_INSPECT_BASIS_WEIGHT      index = slot: R_tc with V_tc = P_tc R_tc (eq. (basis_weights_def))
 *          DH2_INSPECT_TOTAL_WEIGHT_ROW  index = slot: Zhat_tc of the row pass (eq. (recomp_weight_full));
 *                                  for a leaf with #t < k the projected weight, the R factor of
 *                                  Z_tc^* V_tc^H (rows x #t), whose Gram matrix is V Zhat^H Zhat V^H
 *          DH2_INSPECT_TOTAL_WEIGHT_COL  index = slot: Zhat of the column pass (adjoint matrix)
 *          DH2_INSPECT_COUPLING    index = admissible leaf: S_b = (g_c(xi_t,nu, xi_s,mu)), k x k
 *          DH2_INSPECT_RANK_PRED_ROW  index ignored: learned-rank form, predicted rank of every
 *                                  slot's row basis, n_slots x 1 (DH2_ERR_ARG otherwise)
 *          DH2_INSPECT_RANK_PRED_COL  same for the column bases
 * Real-valued results are returned in the real parts. */
enum {
  DH2_INSPECT_NEAR = 1,
  DH2_INSPECT_LEAF_BASIS = 2,
  DH2_INSPECT_TRANSFER = 3,
  DH2_INSPECT_RANK_ROW = 4,
  DH2_INSPECT_RANK_COL = 5,
  DH2_INSPECT_SIGMA_ROW = 6,
  DH2_INSPECT_SIGMA_COL = 7,
  DH2_INSPECT_OMEGA = 8,
  DH2_INSPECT_BASIS_WEIGHT = 9,
  DH2_INSPECT_TOTAL_WEIGHT_ROW = 10,
  DH2_INSPECT_TOTAL_WEIGHT_COL = 11,
  DH2_INSPECT_COUPLING = 12,
  DH2_INSPECT_RANK_PRED_ROW = 13,
  DH2_INSPECT_RANK_PRED_COL = 14
};
dh2_status dh2_inspect(dh2_handle h, int what, int64_t index, double* out, int64_t* rows,
                       int64_t* cols);

#ifdef __cplusplus
}
#endif
#endif /* DH2_H */
