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
