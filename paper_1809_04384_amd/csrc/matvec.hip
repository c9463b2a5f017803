// Matvec Y = Gtilde X of the compressed DH^2 matrix (the product implied by
// eq. (vsw) with the nested bases of eq. (nested), Boerm & Boerst, arXiv
// 1809.04384): forward transform x_sc = Q_sc^* X_s (leaves) and
// x_sc = sum F_{s'c}^* x_{s'c'} (inner clusters), coupling y_tc = sum_b Stilde_b x_sc,
// backward transform y_{t'c'} += F_{t'c} y_tc, leaf output Q_tc y_tc, and the
// near field N_b X_s.  Every phase is a list of small dense products
// described on the host (MvOut / MvTerm); outputs are disjoint within a launch,
// so no atomics are needed and the result is deterministic.
#include "matvec.hpp"
#include "dev.hpp"

namespace dh2 {

template <typename R>
__global__ void __launch_bounds__(256) k_mv_terms(const MvOut* __restrict__ outs,
                                                  const MvTerm* __restrict__ terms, int nrhs) {
  const MvOut o = outs[blockIdx.x];
  cpx<R>* y = (cpx<R>*)o.y;
  const int total = o.M * nrhs;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = e % o.M, r = e / o.M;
    cpx<R> acc{0, 0};
    if (o.accumulate) acc = y[i + (int64_t)r * o.ldy];
    for (int tt = o.term_begin; tt < o.term_end; ++tt) {
      const MvTerm t = terms[tt];
      const cpx<R>* A = (const cpx<R>*)t.A;
      const cpx<R>* x = (const cpx<R>*)t.x + (int64_t)r * t.ldx;
      if (t.op == 0) {
        for (int j = 0; j < t.K; ++j) cfma(acc, A[i + (int64_t)j * t.lda], x[j]);
      } else {
        const cpx<R>* a = A + (int64_t)i * t.lda;
        for (int j = 0; j < t.K; ++j) cfmac(acc, a[j], x[j]);
      }
    }
    y[i + (int64_t)r * o.ldy] = acc;
  }
}

// Matrix-core block-row product (any number of right-hand sides), used by the
// near field (a row = a leaf cluster, its segments = the inadmissible blocks
// restricted to its rows) and by the coupling phase (a row = a row slot (t, c),
// its segments = the recompressed couplings Stilde_b of its admissible blocks).
// A 16x16x4 MFMA multiplies a 16-row, 4-column slice of a segment by the
// matching 4 x 16 slice of the row-major right-hand side; lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  The complex product uses three real
// products,
//   T1 = (Re A + Im A) Re X,  T2 = Re A (Im X - Re X),  T3 = Im A (Re X + Im X),
//   Re Y = T1 - T3,  Im Y = T1 + T2,
// so every matrix entry is loaded once (one 16-byte load per lane, coalesced
// along the column) and feeds three MFMAs.  A workgroup owns one row (64 rows =
// four row tiles per pass); its waves take interleaved segments, the loads of
// the next column slice are issued before the products of the current one, and
// the wave partial sums are added in LDS.  Workgroups are mapped so that each
// XCD walks a contiguous range of rows (neighbouring rows share right-hand-side
// rows in that XCD's L2).
typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));
template <typename R>
struct Mfma;
template <>
struct Mfma<double> {
  typedef mf64x4 acc_t;
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of accumulator element e in lane l (its column is l % 16)
  static __device__ __forceinline__ int row(int l, int e) { return 4 * e + (l >> 4); }
};
template <>
struct Mfma<float> {
  typedef mf32x4 acc_t;
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
};

// Loads through a global (address space 1) pointer: the pointers of the
// descriptors are generic, and generic (flat) loads make the compiler wait for
// every outstanding load before the first use.
template <typename R>
__device__ __forceinline__ cpx<R> gload(const cpx<R>* p) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)p;
  return cpx<R>{v.x, v.y};
}

// The matrix entries are read once per product: in FP64, non-temporal loads
// keep them from displacing the right-hand-side rows, which the neighbouring
// rows of the same XCD read again, from L2 (near field 9.3 -> 8.8 ms at
// n = 131k).  The 8-byte complex64 loads of FP32 stream faster as ordinary
// loads (5.0 ms against 5.4 ms non-temporal).
template <typename R>
__device__ __forceinline__ cpx<R> gload_nt(const cpx<R>* p) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  if constexpr (sizeof(R) == 8) {
    const v2 v = __builtin_nontemporal_load((const __attribute__((address_space(1))) v2*)p);
    return cpx<R>{v.x, v.y};
  } else {
    const v2 v = *(const __attribute__((address_space(1))) v2*)p;
    return cpx<R>{v.x, v.y};
  }
}

// One pass of a block row: rows [r0, r0 + nr) (NT = ceil(nr / 16) row tiles)
// and right-hand sides [c0, c0 + 16), over the T steps of this wave; the wave
// partial sums are added into red[rhs][row] (one wave after the other).
template <typename R, int KU, int S, int NT, int NC>
__device__ __forceinline__ void mf_pass(const MfRow& rw, const NearSeg* __restrict__ segs,
                                        const cpx<R>* __restrict__ XT, const cpx<R>* __restrict__ zero16,
                                        int nrhs, int wave, int T, int r0, int nr, int c0,
                                        cpx<R> (&red)[NC][16][65]) {
  typedef typename Mfma<R>::acc_t acc_t;
  constexpr int SW = 4 * KU;
  const int lane = threadIdx.x & 63;
  const int kc = lane >> 4, rr = lane & 15;
  bool bact[NC];
#pragma unroll
  for (int ch = 0; ch < NC; ++ch) bact[ch] = c0 + 16 * ch + rr < nrhs;
  acc_t t1[NC][NT], t2[NC][NT], t3[NC][NT];
#pragma unroll
  for (int ch = 0; ch < NC; ++ch)
#pragma unroll
    for (int rt = 0; rt < NT; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) t1[ch][rt][e] = t2[ch][rt][e] = t3[ch][rt][e] = R(0);
  if (T > 0) {
    cpx<R> a[S][KU][NT], x[S][KU][NC];
    // fetch position: segment fsg (descriptor fs), first column fj0.  Past the
    // last segment fs keeps a valid address with no columns, so every load
    // stays in bounds and the stage is zero.
    int fsg = rw.seg_begin + wave, fj0 = 0;
    NearSeg fs = segs[fsg];
    // Loads are never masked (a select would wait for the data): rows past nr
    // read row nr - 1 (those outputs are dropped), columns past the segment
    // read its last column, and their right-hand side comes from zero16, so
    // they add nothing.
    auto fetch = [&](cpx<R> (&fa)[KU][NT], cpx<R> (&fx)[KU][NC]) {
      const cpx<R>* A = (const cpx<R>*)fs.A + r0;
      const cpx<R>* xb = XT + fs.x0 * nrhs + c0 + rr;
      const int jl = max(fs.ncols - 1, 0);
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int j = fj0 + 4 * u + kc;
        const int jc = min(j, jl);
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
          const cpx<R>* xp = (j < fs.ncols && bact[ch]) ? xb + (int64_t)j * nrhs + 16 * ch : zero16 + rr;
          fx[u][ch] = gload(xp);
        }
#pragma unroll
        for (int rt = 0; rt < NT; ++rt) fa[u][rt] = gload_nt(A + min(rt * 16 + rr, nr - 1) + (int64_t)jc * fs.lda);
      }
    };
    auto advance = [&]() {
      fj0 += SW;
      if (fj0 >= fs.ncols) {
        fsg += 4;
        fj0 = 0;
        if (fsg < rw.seg_end) fs = segs[fsg];
        else fs.ncols = 0;
      }
    };
#pragma unroll
    for (int st = 0; st < S - 1; ++st) {
      fetch(a[st], x[st]);
      advance();
    }
    for (int done = 0; done < T; done += S) {
#pragma unroll
      for (int st = 0; st < S; ++st) {
        fetch(a[(st + S - 1) % S], x[(st + S - 1) % S]);
        advance();
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
          for (int ch = 0; ch < NC; ++ch) {
            const cpx<R> xv = x[st][u][ch];
            const R b1 = xv.x, b2 = xv.y - xv.x, b3 = xv.x + xv.y;
#pragma unroll
            for (int rt = 0; rt < NT; ++rt) {
              const cpx<R> av = a[st][u][rt];
              t1[ch][rt] = Mfma<R>::mac(av.x + av.y, b1, t1[ch][rt]);
              t2[ch][rt] = Mfma<R>::mac(av.x, b2, t2[ch][rt]);
              t3[ch][rt] = Mfma<R>::mac(av.y, b3, t3[ch][rt]);
            }
          }
      }
    }
  }
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int ch = 0; ch < NC; ++ch)
#pragma unroll
        for (int rt = 0; rt < NT; ++rt) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = rt * 16 + Mfma<R>::row(lane, e);
            const cpx<R> v{t1[ch][rt][e] - t3[ch][rt][e], t1[ch][rt][e] + t2[ch][rt][e]};
            if (w == 0) red[ch][rr][row] = v;
            else red[ch][rr][row] = red[ch][rr][row] + v;
          }
        }
    }
    __syncthreads();
  }
}

// ROLE only names the instantiation (0 near field, 1 coupling) so that the two
// uses are told apart in kernel traces.
template <typename R, int KU, int S, int ROLE, int NC, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) k_mv_rows_mfma(const MfRow* __restrict__ rows,
                                                      const NearSeg* __restrict__ segs,
                                                      const cpx<R>* __restrict__ XT,
                                                      const cpx<R>* __restrict__ zero16, int nrhs,
                                                      XcdSplit split) {
  // KU 4-column slices per step; S register stages (S - 1 steps in flight)
  constexpr int SW = 4 * KU;
  // XCD-aware order: workgroup b runs on XCD b % 8; XCD x takes its share of
  // the row list in order
  const int b = blockIdx.x;
  const int xcd = b & 7, i = b >> 3;
  if (i >= split.off[xcd + 1] - split.off[xcd]) return;
  const MfRow rw = rows[split.off[xcd] + i];
  cpx<R>* __restrict__ Y = (cpx<R>*)rw.y;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  __shared__ cpx<R> red[NC][16][65];
  // steps of this wave: its segments are seg_begin + wave + 4 i
  int T = 0;
  for (int sg = rw.seg_begin + wave; sg < rw.seg_end; sg += 4) T += (segs[sg].ncols + SW - 1) / SW;
  for (int r0 = 0; r0 < rw.nr; r0 += 64) {
    const int nr = min(64, rw.nr - r0);
    const int ntile = (nr + 15) >> 4;
    for (int c0 = 0; c0 < nrhs; c0 += 16 * NC) {
      if (ntile == 1) mf_pass<R, KU, S, 1, NC>(rw, segs, XT, zero16, nrhs, wave, T, r0, nr, c0, red);
      else if (ntile == 2) mf_pass<R, KU, S, 2, NC>(rw, segs, XT, zero16, nrhs, wave, T, r0, nr, c0, red);
      else if (ntile == 3) mf_pass<R, KU, S, 3, NC>(rw, segs, XT, zero16, nrhs, wave, T, r0, nr, c0, red);
      else mf_pass<R, KU, S, 4, NC>(rw, segs, XT, zero16, nrhs, wave, T, r0, nr, c0, red);
      for (int e = tid; e < NC * 16 * 64; e += 256) {
        const int row = e & 63, r = (e >> 6) & 15, ch = e >> 10;
        const int c = c0 + 16 * ch + r;
        if (row < nr && c < nrhs) Y[r0 + row + (int64_t)c * rw.ldy] = red[ch][r][row];
      }
      __syncthreads();
    }
  }
}

// Pipeline shapes of the block-row kernel, picked per handle and role by the
// build's autotuner (dh2_options.autotune): KU 4-column slices per step, S
// register stages, WPE waves per SIMD the register allocation is sized for.
// Variant 0 is the default.
template <typename R, int ROLE, int NC>
static void launch_variant(int variant, dim3 g, const MfRow* rows, const NearSeg* segs, const cpx<R>* xt,
                           const cpx<R>* z, int nrhs, const XcdSplit& split, hipStream_t st) {
  const dim3 b(256);
  switch (variant) {
    case 1:
      hipLaunchKernelGGL((k_mv_rows_mfma<R, 1, 3, ROLE, NC, 2>), g, b, 0, st, rows, segs, xt, z, nrhs, split);
      break;
    case 2:
      hipLaunchKernelGGL((k_mv_rows_mfma<R, 1, 6, ROLE, NC, 1>), g, b, 0, st, rows, segs, xt, z, nrhs, split);
      break;
    case 3:
      hipLaunchKernelGGL((k_mv_rows_mfma<R, 2, 3, ROLE, NC, 1>), g, b, 0, st, rows, segs, xt, z, nrhs, split);
      break;
    default:
      hipLaunchKernelGGL((k_mv_rows_mfma<R, 1, 4, ROLE, NC, 2>), g, b, 0, st, rows, segs, xt, z, nrhs, split);
      break;
  }
}

int mv_rows_variants() { return 4; }

template <typename R>
void launch_mv_rows_mfma(const MfRow* rows, const XcdSplit& split, const NearSeg* segs, const void* XT,
                         const void* zero16, int nrhs, int role, int variant, hipStream_t st) {
  if (split.width <= 0) return;
  // FP32 with more than 16 right-hand sides: two 16-wide chunks per pass, so
  // the matrix is streamed once per 32 right-hand sides (FP64 accumulators
  // for two chunks would not fit the registers of two waves per SIMD)
  const dim3 g((unsigned)(8 * split.width));
  const cpx<R>* xt = (const cpx<R>*)XT;
  const cpx<R>* z = (const cpx<R>*)zero16;
  if constexpr (sizeof(R) == 4) {
    if (nrhs > 16) {
      if (role == 0) launch_variant<R, 0, 2>(variant, g, rows, segs, xt, z, nrhs, split, st);
      else launch_variant<R, 1, 2>(variant, g, rows, segs, xt, z, nrhs, split, st);
      return;
    }
  }
  if (role == 0) launch_variant<R, 0, 1>(variant, g, rows, segs, xt, z, nrhs, split, st);
  else launch_variant<R, 1, 1>(variant, g, rows, segs, xt, z, nrhs, split, st);
}
template void launch_mv_rows_mfma<double>(const MfRow*, const XcdSplit&, const NearSeg*, const void*, const void*,
                                          int, int, int, hipStream_t);
template void launch_mv_rows_mfma<float>(const MfRow*, const XcdSplit&, const NearSeg*, const void*, const void*,
                                         int, int, int, hipStream_t);

// row-major copies of the slot vectors x_sc (k x nrhs, leading dimension k):
// dst[(row0 + j) * nrhs + r] = src[j + r k]; a workgroup per slot
template <typename R>
__global__ void __launch_bounds__(256) k_mv_slot_transpose(const SlotT* __restrict__ d,
                                                           cpx<R>* __restrict__ dst, int nrhs) {
  const SlotT t = d[blockIdx.x];
  const cpx<R>* src = (const cpx<R>*)t.src;
  for (int e = threadIdx.x; e < t.k * nrhs; e += blockDim.x) {
    const int j = e / nrhs, r = e % nrhs;
    dst[(t.row0 + j) * nrhs + r] = src[j + (int64_t)r * t.k];
  }
}

template <typename R>
void launch_mv_slot_transpose(const SlotT* d, int64_t cnt, void* dst, int nrhs, hipStream_t st) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_mv_slot_transpose<R>, dim3((unsigned)cnt), dim3(256), 0, st, d, (cpx<R>*)dst, nrhs);
}
template void launch_mv_slot_transpose<double>(const SlotT*, int64_t, void*, int, hipStream_t);
template void launch_mv_slot_transpose<float>(const SlotT*, int64_t, void*, int, hipStream_t);

// row-major copy of the gathered X: XT[p * nrhs + r] = Xp[p + r n]
template <typename R>
__global__ void k_mv_transpose(const cpx<R>* __restrict__ Xp, cpx<R>* __restrict__ XT, int64_t n,
                               int nrhs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t p = e / nrhs, r = e % nrhs;
  XT[e] = Xp[p + r * n];
}

template <typename R>
void launch_mv_transpose(const void* X, void* XT, int64_t n, int nrhs, hipStream_t st) {
  const int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_mv_transpose<R>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     (const cpx<R>*)X, (cpx<R>*)XT, n, nrhs);
}
template void launch_mv_transpose<double>(const void*, void*, int64_t, int, hipStream_t);
template void launch_mv_transpose<float>(const void*, void*, int64_t, int, hipStream_t);

// gather: dst[p + r n] = src[perm[p] + r n];  scatter: dst[perm[p] + r n] = src[p + r n]
template <typename R>
__global__ void k_mv_permute(const cpx<R>* __restrict__ src, cpx<R>* __restrict__ dst,
                             const int64_t* __restrict__ perm, int64_t n, int nrhs, int gather) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t p = e % n, r = e / n;
  if (gather) dst[p + r * n] = src[perm[p] + r * n];
  else dst[perm[p] + r * n] = src[p + r * n];
}

template <typename R>
void launch_mv_terms(const MvOut* outs, int64_t nout, const MvTerm* terms, int nrhs, hipStream_t st) {
  for (int64_t o0 = 0; o0 < nout; o0 += (1 << 30)) {
    const int64_t cnt = nout - o0 < (1 << 30) ? nout - o0 : (1 << 30);
    hipLaunchKernelGGL(k_mv_terms<R>, dim3((unsigned)cnt), dim3(256), 0, st, outs + o0, terms, nrhs);
  }
}
template void launch_mv_terms<double>(const MvOut*, int64_t, const MvTerm*, int, hipStream_t);
template void launch_mv_terms<float>(const MvOut*, int64_t, const MvTerm*, int, hipStream_t);

template <typename R>
void launch_mv_permute(const void* src, void* dst, const int64_t* perm, int64_t n, int nrhs,
                       int gather, hipStream_t st) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL(k_mv_permute<R>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     (const cpx<R>*)src, (cpx<R>*)dst, perm, n, nrhs, gather);
}
template void launch_mv_permute<double>(const void*, void*, const int64_t*, int64_t, int, int,
                                        hipStream_t);
template void launch_mv_permute<float>(const void*, void*, const int64_t*, int64_t, int, int,
                                       hipStream_t);

}  // namespace dh2
