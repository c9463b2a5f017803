// HIP kernels of the DH^2 build (gfx950, wave64).  Each kernel cites the part
// of Boerm & Boerst (arXiv 1809.04384) it computes.  Complex data is
// interleaved (re, im); matrices are column-major unless stated.
#include "kernels.hpp"

#include <atomic>

#include <type_traits>

#include <hip/hip_runtime.h>

#include <algorithm>

namespace dh2 {

// ---------------------------------------------------------------------------
// Per-triangle data (Section 5: piecewise-constant basis on flat triangles).
// Triangle at cluster position p is user triangle perm[p].  Outputs in
// cluster order: 7-, 16- and 9-point quadrature points / weights and the
// closed-form Laplace self integral int_T int_T 1/|x-y| divided by 4 pi:
//   (4 A^2 / 3) sum_e (1/l_e) log(L / (L - 2 l_e)),  L = perimeter.
__global__ void k_tri_data(int64_t n, const double* __restrict__ V, const int32_t* __restrict__ T,
                           const int64_t* __restrict__ perm, QuadTab qt, double* __restrict__ x7,
                           double* __restrict__ w7, double* __restrict__ x16,
                           double* __restrict__ w16, double* __restrict__ x9, double* __restrict__ w9,
                           double* __restrict__ self_lap) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t u = perm[p];
  double P[3][3];
  for (int v = 0; v < 3; ++v)
    for (int d = 0; d < 3; ++d) P[v][d] = V[3 * (int64_t)T[3 * u + v] + d];
  double e1[3], e2[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = P[1][d] - P[0][d];
    e2[d] = P[2][d] - P[0][d];
  }
  const double cx = e1[1] * e2[2] - e1[2] * e2[1];
  const double cy = e1[2] * e2[0] - e1[0] * e2[2];
  const double cz = e1[0] * e2[1] - e1[1] * e2[0];
  const double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
  for (int q = 0; q < 7; ++q) {
    for (int d = 0; d < 3; ++d)
      x7[(p * 7 + q) * 3 + d] = qt.b7[q][0] * P[0][d] + qt.b7[q][1] * P[1][d] + qt.b7[q][2] * P[2][d];
    w7[p * 7 + q] = area * qt.w7[q];
  }
  for (int q = 0; q < 16; ++q) {
    for (int d = 0; d < 3; ++d)
      x16[(p * 16 + q) * 3 + d] =
          qt.b16[q][0] * P[0][d] + qt.b16[q][1] * P[1][d] + qt.b16[q][2] * P[2][d];
    w16[p * 16 + q] = area * qt.w16[q];
  }
  for (int q = 0; q < 9; ++q) {
    for (int d = 0; d < 3; ++d)
      x9[(p * 9 + q) * 3 + d] = qt.b9[q][0] * P[0][d] + qt.b9[q][1] * P[1][d] + qt.b9[q][2] * P[2][d];
    w9[p * 9 + q] = area * qt.w9[q];
  }
  double l[3];
  for (int e = 0; e < 3; ++e) {
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    const double dx = P[a][0] - P[b][0], dy = P[a][1] - P[b][1], dz = P[a][2] - P[b][2];
    l[e] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  const double L = l[0] + l[1] + l[2];
  double s = 0.0;
  for (int e = 0; e < 3; ++e) s += log(L / (L - 2.0 * l[e])) / l[e];
  self_lap[p] = (4.0 * area * area / 3.0) * s * (0.25 / M_PI);
}

// ---------------------------------------------------------------------------
// Near field (Definition of the DH^2 representation: inadmissible leaves are
// stored as dense arrays).  Entry (i,j) of block t x s:
//   i != j: sum_{p,q<16} w_i,p w_j,q g(x_i,p, y_j,q),  g = exp(i kappa r) / (4 pi r)
//   i == j: Laplace closed form + sum w w rho(r), rho(r) = (exp(i kappa r) - 1) / r,
//           rho(0) = i kappa (singularity subtraction).
// One workgroup per block, one thread per entry; the quadrature data of the row
// triangles is read through the caches, that of the column triangles from LDS.
// Output column-major, leading dimension #t.  NQ = 16: the rules above; NQ =
// 9: the paper's rule of order 3 on both triangles for every pair of distinct
// triangles, the diagonal left 0 (touching pairs take k_touch afterwards).
template <typename R, int NQ>
__global__ void __launch_bounds__(256) k_near(const NearDesc* __restrict__ blocks, double kappa,
                                              const double* __restrict__ xq,
                                              const double* __restrict__ wq,
                                              const double* __restrict__ self_lap,
                                              cpx<R>* __restrict__ out) {
  const NearDesc d = blocks[blockIdx.x];
  const R kap = (R)kappa;
  const R inv4pi = (R)(0.25 / M_PI);
  // the NQ points and weights of up to 64 column triangles, staged in LDS per
  // chunk of columns: every evaluation reads them from there (the lanes of a
  // wave mostly share one column, so the reads are broadcasts)
  __shared__ double cp[64 * NQ][4];
  for (int c0 = 0; c0 < d.nc; c0 += 64) {
    const int cn = min(64, d.nc - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < cn * NQ; e += blockDim.x) {
      const int64_t gj = d.col0 + c0 + e / NQ;
      const int q = e % NQ;
      cp[e][0] = xq[gj * 3 * NQ + 3 * q];
      cp[e][1] = xq[gj * 3 * NQ + 3 * q + 1];
      cp[e][2] = xq[gj * 3 * NQ + 3 * q + 2];
      cp[e][3] = wq[gj * NQ + q];
    }
    __syncthreads();
    const int64_t total = (int64_t)d.nr * cn;
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
      const int i = (int)(e % d.nr);
      const int jj = (int)(e / d.nr);
      const int64_t gi = d.row0 + i, gj = d.col0 + c0 + jj;
      const double* xi = xq + gi * 3 * NQ;
      const double* wi = wq + gi * NQ;
      const double(*pj)[4] = cp + jj * NQ;
      R sre = 0, sim = 0;
      if (gi != gj) {
        for (int p = 0; p < NQ; ++p) {
          const double ax = xi[3 * p], ay = xi[3 * p + 1], az = xi[3 * p + 2];
          R accr = 0, acci = 0;
          for (int q = 0; q < NQ; ++q) {
            const R dx = (R)(ax - pj[q][0]), dy = (R)(ay - pj[q][1]), dz = (R)(az - pj[q][2]);
            const R r2 = dx * dx + dy * dy + dz * dz;
            const R ir = rsqrt_r(r2);
            const R r = r2 * ir;
            R sn, cs;
            sincos_r(kap * r, &sn, &cs);
            const R f = (R)pj[q][3] * ir;
            accr += f * cs;
            acci += f * sn;
          }
          sre += (R)wi[p] * accr;
          sim += (R)wi[p] * acci;
        }
        sre *= inv4pi;
        sim *= inv4pi;
      } else if (NQ == 16) {
        for (int p = 0; p < NQ; ++p) {
          const double ax = xi[3 * p], ay = xi[3 * p + 1], az = xi[3 * p + 2];
          for (int q = 0; q < NQ; ++q) {
            const R w = (R)(wi[p] * pj[q][3]);
            const R dx = (R)(ax - pj[q][0]), dy = (R)(ay - pj[q][1]), dz = (R)(az - pj[q][2]);
            const R r = sqrt_r(dx * dx + dy * dy + dz * dz);
            if (r == (R)0) {
              sim += w * kap;
            } else {
              R sh, ch, sn, cs;
              sincos_r((R)0.5 * kap * r, &sh, &ch);
              sincos_r(kap * r, &sn, &cs);
              sre += w * ((R)-2 * sh * sh) / r;
              sim += w * sn / r;
            }
          }
        }
        sre = (R)self_lap[gi] + sre * inv4pi;
        sim = sim * inv4pi;
      }
      out[d.off + i + (int64_t)(c0 + jj) * d.nr] = cpx<R>{sre, sim};
    }
  }
}

// ---------------------------------------------------------------------------
// Touching pairs with the paper's quadrature (Section 5): Sauter-Erichsen-
// Schwab rules of order 5 for triangles that share a vertex (kind 1), an edge
// (2) or are identical (3).  With the reference triangle {0 <= s2 <= s1 <= 1}
// and chi(s) = A + s1 (B - A) + s2 (C - B) for the ordered vertices of each
// triangle (the shared part first), the entry is
//   (4 |Ta| |Tb| / (4 pi)) sum over the regions and the 5^4 tensor Gauss
//   points (xi, e1, e2, e3) of w * J * exp(i kappa r) / r,  r = |chi_a(s) - chi_b(t)|,
// where each region maps the cube onto part of the pair of reference
// triangles with Jacobian J, which vanishes where x = y (identical: six
// regions, J = xi^3 e1^2 e2; common edge: five, J = xi^3 e1^2 for the first
// and xi^3 e1^2 e2 for the others; common vertex: two, J = xi^3 e2).  One
// workgroup per pair; the entry overwrites the near-field value of the pair.
template <typename R>
__global__ void __launch_bounds__(256) k_touch(const TouchDesc* __restrict__ dd, const double* __restrict__ V,
                                               SesTab tab, double kappa, cpx<R>* __restrict__ out) {
  const TouchDesc d = dd[blockIdx.x];
  double A[3], U[3], W[3], A2[3], U2[3], W2[3];
  for (int k = 0; k < 3; ++k) {
    const double a = V[3 * (int64_t)d.va[0] + k], b = V[3 * (int64_t)d.va[1] + k], c = V[3 * (int64_t)d.va[2] + k];
    A[k] = a;
    U[k] = b - a;
    W[k] = c - b;
    const double a2 = V[3 * (int64_t)d.vb[0] + k], b2 = V[3 * (int64_t)d.vb[1] + k],
                 c2 = V[3 * (int64_t)d.vb[2] + k];
    A2[k] = a2;
    U2[k] = b2 - a2;
    W2[k] = c2 - b2;
  }
  constexpr int NP = kSesOrder * kSesOrder * kSesOrder * kSesOrder;
  const int nreg = d.kind == 3 ? 6 : (d.kind == 2 ? 5 : 2);
  double sre = 0.0, sim = 0.0;
  for (int e = threadIdx.x; e < nreg * NP; e += blockDim.x) {
    const int reg = e / NP, q = e % NP;
    const int i0 = q % kSesOrder, i1 = (q / kSesOrder) % kSesOrder, i2 = (q / (kSesOrder * kSesOrder)) % kSesOrder,
              i3 = q / (kSesOrder * kSesOrder * kSesOrder);
    const double xi = tab.g[i0], e1 = tab.g[i1], e2 = tab.g[i2], e3 = tab.g[i3];
    double w = tab.gw[i0] * tab.gw[i1] * tab.gw[i2] * tab.gw[i3];
    double s1, s2, t1, t2;
    if (d.kind == 3) {
      w *= xi * xi * xi * e1 * e1 * e2;
      switch (reg) {
        case 0: s1 = xi; s2 = xi * (1 - e1 + e1 * e2); t1 = xi * (1 - e1 * e2 * e3); t2 = xi * (1 - e1); break;
        case 1: s1 = xi * (1 - e1 * e2 * e3); s2 = xi * (1 - e1); t1 = xi; t2 = xi * (1 - e1 + e1 * e2); break;
        case 2: s1 = xi; s2 = xi * e1 * (1 - e2 + e2 * e3); t1 = xi * (1 - e1 * e2); t2 = xi * e1 * (1 - e2); break;
        case 3: s1 = xi * (1 - e1 * e2); s2 = xi * e1 * (1 - e2); t1 = xi; t2 = xi * e1 * (1 - e2 + e2 * e3); break;
        case 4: s1 = xi * (1 - e1 * e2 * e3); s2 = xi * e1 * (1 - e2 * e3); t1 = xi; t2 = xi * e1 * (1 - e2); break;
        default: s1 = xi; s2 = xi * e1 * (1 - e2); t1 = xi * (1 - e1 * e2 * e3); t2 = xi * e1 * (1 - e2 * e3); break;
      }
    } else if (d.kind == 2) {
      w *= xi * xi * xi * e1 * e1 * (reg == 0 ? 1.0 : e2);
      switch (reg) {
        case 0: s1 = xi; s2 = xi * e1 * e3; t1 = xi * (1 - e1 * e2); t2 = xi * e1 * (1 - e2); break;
        case 1: s1 = xi; s2 = xi * e1; t1 = xi * (1 - e1 * e2 * e3); t2 = xi * e1 * e2 * (1 - e3); break;
        case 2: s1 = xi * (1 - e1 * e2); s2 = xi * e1 * (1 - e2); t1 = xi; t2 = xi * e1 * e2 * e3; break;
        case 3: s1 = xi * (1 - e1 * e2 * e3); s2 = xi * e1 * e2 * (1 - e3); t1 = xi; t2 = xi * e1; break;
        default: s1 = xi * (1 - e1 * e2 * e3); s2 = xi * e1 * (1 - e2 * e3); t1 = xi; t2 = xi * e1 * e2; break;
      }
    } else {
      w *= xi * xi * xi * e2;
      if (reg == 0) { s1 = xi; s2 = xi * e1; t1 = xi * e2; t2 = xi * e2 * e3; }
      else { s1 = xi * e2; s2 = xi * e2 * e3; t1 = xi; t2 = xi * e1; }
    }
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double dx = (A[k] + s1 * U[k] + s2 * W[k]) - (A2[k] + t1 * U2[k] + t2 * W2[k]);
      r2 += dx * dx;
    }
    const double ir = rsqrt_r(r2);
    double sn, cs;
    sincos_fast(kappa * (r2 * ir), &sn, &cs);
    sre += w * ir * cs;
    sim += w * ir * sn;
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = sre;
  red[1][threadIdx.x] = sim;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    auto cross2 = [](const double* u, const double* v) {
      const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
      return sqrt(cx * cx + cy * cy + cz * cz);
    };
    // 4 |Ta| |Tb| / (4 pi) = |2 Ta| |2 Tb| / (4 pi)
    const double scale = cross2(U, W) * cross2(U2, W2) * (0.25 / M_PI);
    out[d.off] = cpx<R>{(R)(red[0][0] * scale), (R)(red[1][0] * scale)};
  }
}

// ---------------------------------------------------------------------------
// Leaf bases (Section 2): V_tc[i,nu] = sum_{q<nq} w_q exp(i kappa <x_q,c>) L_{t,nu}(x_q)
// for the triangles i of leaf t, with the far rule (7 points, or the paper's 9).
// Output #t x k, column-major.
template <typename R>
__global__ void __launch_bounds__(256) k_leaf_basis(const LeafDesc* __restrict__ dd, ChebTab ct,
                                                    double kappa, const double* __restrict__ xf,
                                                    const double* __restrict__ wf, int nq,
                                                    const double* __restrict__ box,
                                                    const double* __restrict__ dirs,
                                                    cpx<R>* __restrict__ out) {
  const LeafDesc d = dd[blockIdx.x];
  const int m = ct.m;
  const int k = m * m * m;
  const double lo[3] = {box[6 * d.cl], box[6 * d.cl + 1], box[6 * d.cl + 2]};
  const double hi[3] = {box[6 * d.cl + 3], box[6 * d.cl + 4], box[6 * d.cl + 5]};
  const double c[3] = {dirs[3 * d.dir], dirs[3 * d.dir + 1], dirs[3 * d.dir + 2]};
  const int64_t total = (int64_t)d.nr * k;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = (int)(e % d.nr);
    const int nu = (int)(e / d.nr);
    const int jx = nu % m, jy = (nu / m) % m, jz = nu / (m * m);
    const int64_t g = d.row0 + i;
    double sre = 0, sim = 0;
    for (int q = 0; q < nq; ++q) {
      const double* x = xf + (g * nq + q) * 3;
      double Lx[kMaxOrder], Ly[kMaxOrder], Lz[kMaxOrder];
      lagrange<double>(ct, to_ref(x[0], lo[0], hi[0]), Lx);
      lagrange<double>(ct, to_ref(x[1], lo[1], hi[1]), Ly);
      lagrange<double>(ct, to_ref(x[2], lo[2], hi[2]), Lz);
      const double L = Lx[jx] * Ly[jy] * Lz[jz];
      double sn, cs;
      sincos_fast(kappa * (x[0] * c[0] + x[1] * c[1] + x[2] * c[2]), &sn, &cs);
      const double f = wf[g * nq + q] * L;
      sre += f * cs;
      sim += f * sn;
    }
    out[d.off + e] = cpx<R>{(R)sre, (R)sim};
  }
}

// ---------------------------------------------------------------------------
// Transfer matrices (eq. (nested_apx)): for child t' of t, direction c of t,
// c' = sd(c): E_{t'c}[nu',nu] = exp(i kappa <xi_{t'nu'}, c - c'>) L_{t,nu}(xi_{t'nu'}).
// Output k x k column-major.
template <typename R>
__global__ void __launch_bounds__(256) k_transfer(const TransDesc* __restrict__ dd, ChebTab ct,
                                                  double kappa, const double* __restrict__ box,
                                                  const double* __restrict__ dirs,
                                                  cpx<R>* __restrict__ out) {
  const TransDesc d = dd[blockIdx.x];
  const int m = ct.m;
  const int k = m * m * m;
  const double* bp = box + 6 * d.parent;
  const double* bc = box + 6 * d.child;
  double dc[3];
  for (int a = 0; a < 3; ++a) dc[a] = dirs[3 * d.dir_parent + a] - dirs[3 * d.dir_child + a];
  for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += blockDim.x) {
    const int nu1 = (int)(e % k);   // row: child point
    const int nu = (int)(e / k);    // column: parent polynomial
    const int ix = nu1 % m, iy = (nu1 / m) % m, iz = nu1 / (m * m);
    const double xi[3] = {axis_point(ct, bc[0], bc[3], ix), axis_point(ct, bc[1], bc[4], iy),
                          axis_point(ct, bc[2], bc[5], iz)};
    const int jx = nu % m, jy = (nu / m) % m, jz = nu / (m * m);
    double Lx[kMaxOrder], Ly[kMaxOrder], Lz[kMaxOrder];
    lagrange<double>(ct, to_ref(xi[0], bp[0], bp[3]), Lx);
    lagrange<double>(ct, to_ref(xi[1], bp[1], bp[4]), Ly);
    lagrange<double>(ct, to_ref(xi[2], bp[2], bp[5]), Lz);
    const double L = Lx[jx] * Ly[jy] * Lz[jz];
    double sn, cs;
    sincos_fast(kappa * (xi[0] * dc[0] + xi[1] * dc[1] + xi[2] * dc[2]), &sn, &cs);
    out[d.off + e] = cpx<R>{(R)(L * cs), (R)(L * sn)};
  }
}

// One entry of a coupling matrix S_b (defined below, before k_coupling) at the
// interpolation points x_t of the row cluster and x_s of the column cluster.
// Shared by k_coupling (S_b stored) and k_gemm_coupling (S_b formed inside a
// product), so the two give the same bits.
__device__ __forceinline__ z64 coupling_entry(double xt, double yt, double zt, double xs, double ys, double zs,
                                              const double (&c)[3], double kappa) {
  const double f0 = 0.25 / M_PI;
  const double dx = xt - xs;
  const double dy = yt - ys;
  const double dz = zt - zs;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsqrt_r(r2);
  const double r = r2 * ir;
  double sn, cs;
  sincos_fast(kappa * (r - (dx * c[0] + dy * c[1] + dz * c[2])), &sn, &cs);
  const double f = f0 * ir;
  return z64{f * cs, f * sn};
}

// ---------------------------------------------------------------------------
// Coupling matrices (Section 2): S_b[nu,mu] = g_c(xi_{t,nu}, xi_{s,mu}),
// g_c(x,y) = exp(i kappa (|x-y| - <x-y,c>)) / (4 pi |x-y|).  One workgroup per
// block of the batch; output k x k column-major at out + item * k * k.
template <typename R>
__global__ void __launch_bounds__(256) k_coupling(const CoupDesc* __restrict__ dd, ChebTab ct,
                                                  double kappa, const double* __restrict__ box,
                                                  const double* __restrict__ dirs,
                                                  cpx<R>* __restrict__ out) {
  const CoupDesc d = dd[blockIdx.x];
  const int m = ct.m;
  const int k = m * m * m;
  const double* bt = box + 6 * d.t;
  const double* bs = box + 6 * d.s;
  const double c[3] = {dirs[3 * d.dir], dirs[3 * d.dir + 1], dirs[3 * d.dir + 2]};
  // interpolation points of t (rows) and s (columns): xi_nu = (x_{jx}, y_{jy}, z_{jz}),
  // nu = jx + m (jy + m jz); the point tables are built once per block
  __shared__ double pt[3][kMaxOrder], ps[3][kMaxOrder];
  __shared__ double qs[3][kMaxOrder * kMaxOrder * kMaxOrder];
  if (threadIdx.x < 3 * m) {
    const int a = threadIdx.x / m, j = threadIdx.x % m;
    pt[a][j] = axis_point(ct, bt[a], bt[a + 3], j);
    ps[a][j] = axis_point(ct, bs[a], bs[a + 3], j);
  }
  __syncthreads();
  for (int mu = threadIdx.x; mu < k; mu += blockDim.x) {
    qs[0][mu] = ps[0][mu % m];
    qs[1][mu] = ps[1][(mu / m) % m];
    qs[2][mu] = ps[2][mu / (m * m)];
  }
  __syncthreads();
  cpx<R>* o = out + (int64_t)blockIdx.x * k * k;
  // thread = row nu (its point in registers), the column points are read from
  // LDS (the same for every lane of an iteration); writes are coalesced
  const int ng = blockDim.x / 128;
  for (int nu0 = 0; nu0 < k; nu0 += 128) {
    const int nu = nu0 + (threadIdx.x & 127);
    if (nu >= k) continue;
    const double xt = pt[0][nu % m], yt = pt[1][(nu / m) % m], zt = pt[2][nu / (m * m)];
    for (int mu = threadIdx.x >> 7; mu < k; mu += ng) {
      const z64 v = coupling_entry(xt, yt, zt, qs[0][mu], qs[1][mu], qs[2][mu], c, kappa);
      o[nu + (int64_t)mu * k] = cpx<R>{(R)v.x, (R)v.y};
    }
  }
}

// ---------------------------------------------------------------------------
// Batched complex GEMM, C = alpha op(A) op(B) (+ C if accumulate), op in
// {N, T, C (conjugate transpose)}.  32 x 32 output tile per workgroup of 256
// threads (2 x 2 outputs each), K staged through LDS in slices of 16.
// Matrix-core tile products: a 16x16x4 MFMA multiplies A (16 x 4) by
// B (4 x 16); lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
typedef double gm_f64x4 __attribute__((ext_vector_type(4)));
typedef float gm_f32x4 __attribute__((ext_vector_type(4)));
template <typename R>
struct GMfma;
template <>
struct GMfma<double> {
  typedef gm_f64x4 acc_t;
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * e + (l >> 4); }
};
template <>
struct GMfma<float> {
  typedef gm_f32x4 acc_t;
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
};

// Batched complex GEMM C = alpha op(A) op(B) (+ C), the products of the
// recompression (Section 3.2: weighted couplings R S^*, transfers, basis
// changes and projections).  A workgroup computes a 32 x 32 tile: 16-deep
// slices of op(A) and op(B) are staged in LDS (transposition and conjugation
// happen there), and each wave multiplies a 16 x 16 sub-tile on the matrix
// cores, four real products per complex product:
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B.
// S: storage type of A, B and C; R: the matrix-core type of the products
// (S = double, R = float: FP64 data multiplied on the FP32 matrix cores with
// FP32 accumulation).  Registers are sized for seven waves per SIMD (the
// FP64 products per build at n = 131072: five 1336 ms, six 1270, seven 1245).
// XCD-aware order of a 2-d grid: workgroup b of the linear order runs on XCD
// b % 8, so the logical index is remapped to give each XCD a contiguous range
// of the logical order (the tiles of one product run on one XCD and share its
// L2).  Returns (x, y) of the logical workgroup.
__device__ __forceinline__ void xcd_remap(int& x, int& y) {
  const unsigned gx = gridDim.x, total = gx * gridDim.y;
  const unsigned b = blockIdx.x + gx * blockIdx.y;
  const unsigned q = total / 8, r = total % 8, xcd = b % 8;
  const unsigned l = xcd * q + min(xcd, r) + b / 8;
  x = (int)(l % gx);
  y = (int)(l / gx);
}

template <typename S, typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) k_gemm(const GemmDesc* __restrict__ dd, int ntm) {
  typedef typename GMfma<R>::acc_t acc_t;
  int bx, by;
  xcd_remap(bx, by);
  const GemmDesc d = dd[by];
  const int tm = bx % ntm, tn = bx / ntm;
  const int m0 = tm * 32, n0 = tn * 32;
  if (m0 >= d.M || n0 >= d.N) return;
  if (d.upper && m0 >= n0 + 32) return;
  const cpx<S>* A = (const cpx<S>*)d.A;
  const cpx<S>* B = (const cpx<S>*)d.B;
  cpx<S>* C = (cpx<S>*)d.C;
  __shared__ cpx<R> As[16][33];
  __shared__ cpx<R> Bs[16][33];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sm = (wave & 1) * 16, sn = (wave >> 1) * 16;   // sub-tile of this wave
  const int li = lane & 15, lk = lane >> 4;
  acc_t cre, cim;
#pragma unroll
  for (int e = 0; e < 4; ++e) cre[e] = cim[e] = R(0);
  // Slice loads: consecutive threads read consecutive memory for every op
  // (for op = N the fast index is the row of the stored matrix, otherwise the
  // column); the next slice is loaded into registers while the current one
  // is multiplied.
  cpx<R> va[2], vb[2];
  auto load_slice = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      int i, kk;
      if (d.opA == 0) { i = e % 32; kk = e / 32; }
      else { kk = e % 16; i = e / 16; }
      const int gi = m0 + i, gk = k0 + kk;
      cpx<S> v{0, 0};
      if (gi < d.M && gk < d.K) {
        if (d.opA == 0) v = A[gi + (int64_t)gk * d.lda];
        else {
          v = A[gk + (int64_t)gi * d.lda];
          if (d.opA == 2) v = conj(v);
        }
      }
      va[h] = cpx<R>{(R)v.x, (R)v.y};
      int kb, j;
      if (d.opB == 0) { kb = e % 16; j = e / 16; }
      else { j = e % 32; kb = e / 32; }
      const int gkb = k0 + kb, gj = n0 + j;
      cpx<S> w{0, 0};
      if (gkb < d.K && gj < d.N) {
        if (d.opB == 0) w = B[gkb + (int64_t)gj * d.ldb];
        else {
          w = B[gj + (int64_t)gkb * d.ldb];
          if (d.opB == 2) w = conj(w);
        }
      }
      vb[h] = cpx<R>{(R)w.x, (R)w.y};
    }
  };
  auto store_slice = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      if (d.opA == 0) As[e / 32][e % 32] = va[h];
      else As[e % 16][e / 16] = va[h];
      if (d.opB == 0) Bs[e % 16][e / 16] = vb[h];
      else Bs[e / 32][e % 32] = vb[h];
    }
  };
  // first slice: 0, or past the known zeros of a trapezoidal operand (m0 and
  // n0 are multiples of the slice depth)
  const int kb = max((d.tri & 1) ? m0 : 0, (d.tri & 2) ? n0 : 0);
  load_slice(kb);
  for (int k0 = kb; k0 < d.K; k0 += 16) {
    store_slice();
    __syncthreads();
    if (k0 + 16 < d.K) load_slice(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const cpx<R> a = As[ks + lk][sm + li];
      const cpx<R> b = Bs[ks + lk][sn + li];
      cre = GMfma<R>::mac(a.x, b.x, cre);
      cre = GMfma<R>::mac(-a.y, b.y, cre);
      cim = GMfma<R>::mac(a.x, b.y, cim);
      cim = GMfma<R>::mac(a.y, b.x, cim);
    }
    __syncthreads();
  }
  const cpx<S> al{(S)d.alpha_re, (S)d.alpha_im};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int gi = m0 + sm + GMfma<R>::row(lane, e), gj = n0 + sn + li;
    if (gi < d.M && gj < d.N) {
      const cpx<S> v = al * cpx<S>{(S)cre[e], (S)cim[e]};
      cpx<S>& dst = C[gi + (int64_t)gj * d.ldc];
      dst = d.accumulate ? dst + v : v;
    }
  }
}

// ---------------------------------------------------------------------------
// Products with a coupling matrix that is never stored: C = alpha A S_b or
// C = alpha A S_b^H (A: M x k, column-major), the entries of S_b evaluated in
// the product's B slices (coupling_entry, the bits k_coupling stores).  The
// recompression takes S_b only through such products in its Frobenius-norm
// passes (R_tc S_b, R_sc S_b^H / omega_b) and in the projection (C_tc S_b),
// so the k^2 coupling of a block need not go through HBM.  A workgroup owns 32
// columns of C and all of its rows, in chunks of 32 MT rows: every entry of
// S_b is evaluated once per chunk, the 16 x 32 B slice of the next step while
// the matrix cores multiply the current one.  Each wave holds MT 16 x 16
// sub-tiles; per sub-tile the accumulation order is that of k_gemm (same
// slices, same MFMA sequence), so with coupling_entry's values the result
// equals k_gemm on a stored S_b bit for bit.  Slices that lie in the known
// zeros of a trapezoidal A (tri bit 0) are skipped per sub-tile.  MT = 1, 2, 4
// is chosen per product by its row count (fewer accumulators and loads, more
// waves in flight to hide the evaluation's latency when M is small); NW waves
// per workgroup hold 4 MT / NW sub-tiles each, registers sized for WPE waves
// per SIMD (128-row chunks: eight waves of two sub-tiles, four per SIMD).
// RM: the matrix-core type; RM = float is the FP32 form's product (operands
// rounded to FP32 as they are staged, f32 MFMA, FP32 accumulation, FP64
// result), the bits of k_gemm<double, float> on a stored S_b.
template <typename RM, int MT, int NW, int WPE>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
k_gemm_coupling(const CoupGemmDesc* __restrict__ dd, ChebTab ct, double kappa, const double* __restrict__ box,
                const double* __restrict__ dirs) {
  typedef typename GMfma<RM>::acc_t acc_t;
  constexpr int NT = 64 * NW;                 // threads
  constexpr int RC = 32 * MT;                 // rows per chunk
  constexpr int NL = RC * 16 / NT;            // A entries per thread and slice
  constexpr int NB = 512 / NT;                // B entries per thread and slice
  constexpr int SPW = 4 * MT / NW;            // 16 x 16 sub-tiles per wave
  static_assert(SPW >= 1 && NL >= 1 && NB >= 1, "shape");
  int bx, by;
  xcd_remap(bx, by);
  const CoupGemmDesc d = dd[by];
  const int m = ct.m;
  const int k = m * m * m;
  const int n0 = bx * 32;
  if (n0 >= k || d.M <= 0) return;
  const z64* A = (const z64*)d.A;
  z64* C = (z64*)d.C;
  __shared__ double pt[3][kMaxOrder], ps[3][kMaxOrder];
  __shared__ cpx<RM> As[16][RC + 1];
  __shared__ cpx<RM> Bs[16][33];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int sn = (wave & 1) * 16;             // sub-tile column
  const int sm0 = (wave >> 1) * 16;           // sub-tile rows sm0 + 8 NW u, u < SPW
  if (tid < 3 * m) {
    const int a = tid / m, j = tid % m;
    const double* bt = box + 6 * d.t;
    const double* bs = box + 6 * d.s;
    pt[a][j] = axis_point(ct, bt[a], bt[a + 3], j);
    ps[a][j] = axis_point(ct, bs[a], bs[a + 3], j);
  }
  __syncthreads();
  const double c[3] = {dirs[3 * d.dir], dirs[3 * d.dir + 1], dirs[3 * d.dir + 2]};
  // B slice entries of this thread: row kk of the slice, columns jb + NT / 16 h, h < NB.
  // op(S)[j][n] is S_b[j][n] (the K index a point of t, the column one of s)
  // or conj(S_b[n][j]) (the K index a point of s, the column one of t).
  const int kk = tid & 15, jb = tid >> 4;
  const bool cj = d.conj != 0;
  double nx[NB], ny[NB], nz[NB];
  bool nok[NB];
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    const int n = min(n0 + jb + (NT / 16) * h, k - 1);
    const int i0 = n % m, i1 = (n / m) % m, i2 = n / (m * m);
    nok[h] = n0 + jb + (NT / 16) * h < k;
    nx[h] = cj ? pt[0][i0] : ps[0][i0];
    ny[h] = cj ? pt[1][i1] : ps[1][i1];
    nz[h] = cj ? pt[2][i2] : ps[2][i2];
  }
  // A slice entries of this thread: row ia (the same in every slice), slice
  // rows ka0 + NT / RC u
  const int ia = tid & (RC - 1), ka0 = tid / RC;
  const z64 al{d.alpha, 0.0};
  for (int mc = 0; mc < d.M; mc += RC) {
    const int rows = min(RC, d.M - mc);
    // wave-uniform: a wave whose A rows all lie past M loads nothing
    const bool wload = ((wave * 64) & (RC - 1)) < rows;
    acc_t cre[SPW], cim[SPW];
#pragma unroll
    for (int u = 0; u < SPW; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) cre[u][e] = cim[u][e] = RM(0);
    z64 va[NL], vb[NB];
    auto load_slice = [&](int k0) __attribute__((always_inline)) {
      const int j = k0 + kk;
      const bool kok = j < k;
      const int jc = min(j, k - 1);
      const int i0 = jc % m, i1 = (jc / m) % m, i2 = jc / (m * m);
      const double kx = cj ? ps[0][i0] : pt[0][i0];
      const double ky = cj ? ps[1][i1] : pt[1][i1];
      const double kz = cj ? ps[2][i2] : pt[2][i2];
#pragma unroll
      for (int h = 0; h < NB; ++h) {
        // x_t is the K point (S_b) or the column point (S_b^H)
        const double xt = cj ? nx[h] : kx, yt = cj ? ny[h] : ky, zt = cj ? nz[h] : kz;
        const double xs = cj ? kx : nx[h], ys = cj ? ky : ny[h], zs = cj ? kz : nz[h];
        z64 v = coupling_entry(xt, yt, zt, xs, ys, zs, c, kappa);
        if (cj) v.y = -v.y;
        vb[h] = (kok && nok[h]) ? v : z64{0.0, 0.0};
      }
      // unmasked loads from a clamped (valid) address, then a select
      if (wload) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
          const int ka = k0 + ka0 + (NT / RC) * u;
          typedef double v2 __attribute__((ext_vector_type(2)));
          const v2 w = *(const __attribute__((address_space(1))) v2*)(A + mc + min(ia, rows - 1) +
                                                                      (int64_t)min(ka, k - 1) * d.lda);
          const bool ok = ia < rows && ka < k;
          va[u] = z64{ok ? w.x : 0.0, ok ? w.y : 0.0};
        }
      } else {
#pragma unroll
        for (int u = 0; u < NL; ++u) va[u] = z64{0.0, 0.0};
      }
    };
    load_slice(0);
    for (int k0 = 0; k0 < k; k0 += 16) {
#pragma unroll
      for (int u = 0; u < NL; ++u) As[ka0 + (NT / RC) * u][ia] = cpx<RM>{(RM)va[u].x, (RM)va[u].y};
#pragma unroll
      for (int h = 0; h < NB; ++h) Bs[kk][jb + (NT / 16) * h] = cpx<RM>{(RM)vb[h].x, (RM)vb[h].y};
      __syncthreads();
      if (k0 + 16 < k) load_slice(k0 + 16);
#pragma unroll
      for (int u = 0; u < SPW; ++u) {
        const int ms = sm0 + 8 * NW * u;
        // wave-uniform: rows past M, or a slice wholly left of a trapezoidal A's diagonal
        if (ms < rows && !((d.tri & 1) && k0 + 16 <= mc + ms)) {
#pragma unroll
          for (int ks = 0; ks < 16; ks += 4) {
            const cpx<RM> a = As[ks + lk][ms + li];
            const cpx<RM> b = Bs[ks + lk][sn + li];
            cre[u] = GMfma<RM>::mac(a.x, b.x, cre[u]);
            cre[u] = GMfma<RM>::mac(-a.y, b.y, cre[u]);
            cim[u] = GMfma<RM>::mac(a.x, b.y, cim[u]);
            cim[u] = GMfma<RM>::mac(a.y, b.x, cim[u]);
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
      const int ms = sm0 + 8 * NW * u;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = ms + GMfma<RM>::row(lane, e), gj = n0 + sn + li;
        if (gi < rows && gj < k) C[mc + gi + (int64_t)gj * d.ldc] = al * z64{(double)cre[u][e], (double)cim[u][e]};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split-BF16x3 form of k_gemm (same descriptors, FP64 complex data in and
// out) with the products on the BF16 matrix cores.  Each operand x is taken
// to FP32 and split as x = hi + lo, hi = x rounded to bf16, lo = (x - hi)
// rounded to bf16; a product is hi hi' + hi lo' + lo hi' (the dropped lo lo'
// and the rounding of lo leave about 2^-16 of the product), accumulated in
// FP32 and written in FP64.  Per 16-deep slice a wave issues 12 MFMAs
// (16x16x16 bf16): three per real product of Re C += Re A Re B - Im A Im B,
// Im C += Re A Im B + Im A Re B, kept in four accumulators.
typedef short gm_bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rn(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ void split_bf16(double x, unsigned short& hi, unsigned short& lo) {
  const float f = (float)x;
  hi = bf16_rn(f);
  lo = bf16_rn(f - __uint_as_float((unsigned)hi << 16));
}

__global__ void __launch_bounds__(256) k_gemm_bf16x3(const GemmDesc* __restrict__ dd, int ntm) {
  int bx, by;
  xcd_remap(bx, by);
  const GemmDesc d = dd[by];
  const int tm = bx % ntm, tn = bx / ntm;
  const int m0 = tm * 32, n0 = tn * 32;
  if (m0 >= d.M || n0 >= d.N) return;
  const z64* A = (const z64*)d.A;
  const z64* B = (const z64*)d.B;
  z64* C = (z64*)d.C;
  // [part][row of op(A) | column of op(B)][k]; parts: Re hi, Re lo, Im hi, Im lo.
  // Rows are padded to 20 entries (40 B) so the 8-byte operand reads of a wave
  // fall in distinct banks.
  __shared__ __align__(16) unsigned short As[4][32][20];
  __shared__ __align__(16) unsigned short Bs[4][32][20];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sm = (wave & 1) * 16, sn = (wave >> 1) * 16;
  const int li = lane & 15, lk = lane >> 4;
  gm_f32x4 rr, ii, ri, ir;
#pragma unroll
  for (int e = 0; e < 4; ++e) rr[e] = ii[e] = ri[e] = ir[e] = 0.f;
  z64 va[2], vb[2];
  auto load_slice = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      int i, kk;
      if (d.opA == 0) { i = e % 32; kk = e / 32; }
      else { kk = e % 16; i = e / 16; }
      const int gi = m0 + i, gk = k0 + kk;
      z64 v{0, 0};
      if (gi < d.M && gk < d.K) {
        if (d.opA == 0) v = A[gi + (int64_t)gk * d.lda];
        else {
          v = A[gk + (int64_t)gi * d.lda];
          if (d.opA == 2) v = conj(v);
        }
      }
      va[h] = v;
      int kb, j;
      if (d.opB == 0) { kb = e % 16; j = e / 16; }
      else { j = e % 32; kb = e / 32; }
      const int gkb = k0 + kb, gj = n0 + j;
      z64 w{0, 0};
      if (gkb < d.K && gj < d.N) {
        if (d.opB == 0) w = B[gkb + (int64_t)gj * d.ldb];
        else {
          w = B[gj + (int64_t)gkb * d.ldb];
          if (d.opB == 2) w = conj(w);
        }
      }
      vb[h] = w;
    }
  };
  auto store_slice = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      int i, kk, j, kb;
      if (d.opA == 0) { i = e % 32; kk = e / 32; }
      else { kk = e % 16; i = e / 16; }
      if (d.opB == 0) { kb = e % 16; j = e / 16; }
      else { j = e % 32; kb = e / 32; }
      split_bf16(va[h].x, As[0][i][kk], As[1][i][kk]);
      split_bf16(va[h].y, As[2][i][kk], As[3][i][kk]);
      split_bf16(vb[h].x, Bs[0][j][kb], Bs[1][j][kb]);
      split_bf16(vb[h].y, Bs[2][j][kb], Bs[3][j][kb]);
    }
  };
  const int kb = max((d.tri & 1) ? m0 : 0, (d.tri & 2) ? n0 : 0);
  load_slice(kb);
  for (int k0 = kb; k0 < d.K; k0 += 16) {
    store_slice();
    __syncthreads();
    if (k0 + 16 < d.K) load_slice(k0 + 16);
    gm_bf16x4 a[4], b[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      a[p] = *(const gm_bf16x4*)&As[p][sm + li][4 * lk];
      b[p] = *(const gm_bf16x4*)&Bs[p][sn + li][4 * lk];
    }
    rr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[1], rr, 0, 0, 0);
    rr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[0], rr, 0, 0, 0);
    rr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[0], rr, 0, 0, 0);
    ii = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[3], ii, 0, 0, 0);
    ii = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[3], b[2], ii, 0, 0, 0);
    ii = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[2], ii, 0, 0, 0);
    ri = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[3], ri, 0, 0, 0);
    ri = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[2], ri, 0, 0, 0);
    ri = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[2], ri, 0, 0, 0);
    ir = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[1], ir, 0, 0, 0);
    ir = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[3], b[0], ir, 0, 0, 0);
    ir = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[0], ir, 0, 0, 0);
    __syncthreads();
  }
  const z64 al{d.alpha_re, d.alpha_im};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    // f32 16x16 output: element e of lane l is row 4 (l >> 4) + e, column l & 15
    const int gi = m0 + sm + 4 * lk + e, gj = n0 + sn + li;
    if (gi < d.M && gj < d.N) {
      const z64 v = al * z64{(double)rr[e] - (double)ii[e], (double)ri[e] + (double)ir[e]};
      z64& dst = C[gi + (int64_t)gj * d.ldc];
      dst = d.accumulate ? dst + v : v;
    }
  }
}

// The split-BF16x3 form of k_gemm_coupling: the same chunks, slices and
// evaluation of S_b, the operands split into bf16 hi and lo parts as they are
// staged (the split of k_gemm_bf16x3, so the bits of k_gemm_bf16x3 on a stored
// S_b), twelve 16x16x16 bf16 MFMAs per sub-tile and slice.
template <int MT, int NW, int WPE>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
k_gemm_coupling_bf16x3(const CoupGemmDesc* __restrict__ dd, ChebTab ct, double kappa,
                       const double* __restrict__ box, const double* __restrict__ dirs) {
  constexpr int NT = 64 * NW;
  constexpr int RC = 32 * MT;
  constexpr int NL = RC * 16 / NT;
  constexpr int NB = 512 / NT;
  constexpr int SPW = 4 * MT / NW;
  static_assert(SPW >= 1 && NL >= 1 && NB >= 1, "shape");
  int bx, by;
  xcd_remap(bx, by);
  const CoupGemmDesc d = dd[by];
  const int m = ct.m;
  const int k = m * m * m;
  const int n0 = bx * 32;
  if (n0 >= k || d.M <= 0) return;
  const z64* A = (const z64*)d.A;
  z64* C = (z64*)d.C;
  __shared__ double pt[3][kMaxOrder], ps[3][kMaxOrder];
  // [part][row of A | column of op(S)][k]; parts Re hi, Re lo, Im hi, Im lo
  __shared__ __align__(16) unsigned short As[4][RC][20];
  __shared__ __align__(16) unsigned short Bs[4][32][20];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int sn = (wave & 1) * 16;
  const int sm0 = (wave >> 1) * 16;
  if (tid < 3 * m) {
    const int a = tid / m, j = tid % m;
    const double* bt = box + 6 * d.t;
    const double* bs = box + 6 * d.s;
    pt[a][j] = axis_point(ct, bt[a], bt[a + 3], j);
    ps[a][j] = axis_point(ct, bs[a], bs[a + 3], j);
  }
  __syncthreads();
  const double c[3] = {dirs[3 * d.dir], dirs[3 * d.dir + 1], dirs[3 * d.dir + 2]};
  const int kk = tid & 15, jb = tid >> 4;
  const bool cj = d.conj != 0;
  double nx[NB], ny[NB], nz[NB];
  bool nok[NB];
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    const int n = min(n0 + jb + (NT / 16) * h, k - 1);
    const int i0 = n % m, i1 = (n / m) % m, i2 = n / (m * m);
    nok[h] = n0 + jb + (NT / 16) * h < k;
    nx[h] = cj ? pt[0][i0] : ps[0][i0];
    ny[h] = cj ? pt[1][i1] : ps[1][i1];
    nz[h] = cj ? pt[2][i2] : ps[2][i2];
  }
  const int ia = tid & (RC - 1), ka0 = tid / RC;
  const z64 al{d.alpha, 0.0};
  for (int mc = 0; mc < d.M; mc += RC) {
    const int rows = min(RC, d.M - mc);
    const bool wload = ((wave * 64) & (RC - 1)) < rows;
    gm_f32x4 rr[SPW], ii[SPW], ri[SPW], ir[SPW];
#pragma unroll
    for (int u = 0; u < SPW; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) rr[u][e] = ii[u][e] = ri[u][e] = ir[u][e] = 0.f;
    z64 va[NL], vb[NB];
    auto load_slice = [&](int k0) __attribute__((always_inline)) {
      const int j = k0 + kk;
      const bool kok = j < k;
      const int jc = min(j, k - 1);
      const int i0 = jc % m, i1 = (jc / m) % m, i2 = jc / (m * m);
      const double kx = cj ? ps[0][i0] : pt[0][i0];
      const double ky = cj ? ps[1][i1] : pt[1][i1];
      const double kz = cj ? ps[2][i2] : pt[2][i2];
#pragma unroll
      for (int h = 0; h < NB; ++h) {
        const double xt = cj ? nx[h] : kx, yt = cj ? ny[h] : ky, zt = cj ? nz[h] : kz;
        const double xs = cj ? kx : nx[h], ys = cj ? ky : ny[h], zs = cj ? kz : nz[h];
        z64 v = coupling_entry(xt, yt, zt, xs, ys, zs, c, kappa);
        if (cj) v.y = -v.y;
        vb[h] = (kok && nok[h]) ? v : z64{0.0, 0.0};
      }
      if (wload) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
          const int ka = k0 + ka0 + (NT / RC) * u;
          typedef double v2 __attribute__((ext_vector_type(2)));
          const v2 w = *(const __attribute__((address_space(1))) v2*)(A + mc + min(ia, rows - 1) +
                                                                      (int64_t)min(ka, k - 1) * d.lda);
          const bool ok = ia < rows && ka < k;
          va[u] = z64{ok ? w.x : 0.0, ok ? w.y : 0.0};
        }
      } else {
#pragma unroll
        for (int u = 0; u < NL; ++u) va[u] = z64{0.0, 0.0};
      }
    };
    load_slice(0);
    for (int k0 = 0; k0 < k; k0 += 16) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int ka = ka0 + (NT / RC) * u;
        split_bf16(va[u].x, As[0][ia][ka], As[1][ia][ka]);
        split_bf16(va[u].y, As[2][ia][ka], As[3][ia][ka]);
      }
#pragma unroll
      for (int h = 0; h < NB; ++h) {
        const int jj = jb + (NT / 16) * h;
        split_bf16(vb[h].x, Bs[0][jj][kk], Bs[1][jj][kk]);
        split_bf16(vb[h].y, Bs[2][jj][kk], Bs[3][jj][kk]);
      }
      __syncthreads();
      if (k0 + 16 < k) load_slice(k0 + 16);
      gm_bf16x4 b[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) b[p] = *(const gm_bf16x4*)&Bs[p][sn + li][4 * lk];
#pragma unroll
      for (int u = 0; u < SPW; ++u) {
        const int ms = sm0 + 8 * NW * u;
        if (ms < rows && !((d.tri & 1) && k0 + 16 <= mc + ms)) {
          gm_bf16x4 a[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) a[p] = *(const gm_bf16x4*)&As[p][ms + li][4 * lk];
          rr[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[1], rr[u], 0, 0, 0);
          rr[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[0], rr[u], 0, 0, 0);
          rr[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[0], rr[u], 0, 0, 0);
          ii[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[3], ii[u], 0, 0, 0);
          ii[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[3], b[2], ii[u], 0, 0, 0);
          ii[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[2], ii[u], 0, 0, 0);
          ri[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[3], ri[u], 0, 0, 0);
          ri[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[2], ri[u], 0, 0, 0);
          ri[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[2], ri[u], 0, 0, 0);
          ir[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[1], ir[u], 0, 0, 0);
          ir[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[3], b[0], ir[u], 0, 0, 0);
          ir[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[0], ir[u], 0, 0, 0);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
      const int ms = sm0 + 8 * NW * u;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = ms + 4 * lk + e, gj = n0 + sn + li;
        if (gi < rows && gj < k)
          C[mc + gi + (int64_t)gj * d.ldc] =
              al * z64{(double)rr[u][e] - (double)ii[u][e], (double)ri[u][e] + (double)ir[u][e]};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Householder fold (FP64): R <- R factor of [R; P_1; P_2; ...] for an n x n
// upper triangular R (column-major, leading dimension ldr) and pieces P
// (rows x n, column-major).  This is the QR step of the basis weights
// (eq. (basis_weights_def)) and of the total weights (skinny QR of Z_tc^*,
// eq. (recomp_weight_full)); only R is kept, as in the paper.
// Column j: x = (R[j,j], P[:,j]); beta = -phase(R[j,j]) |x| with |x| taken
// through a max-abs scale; d = R[j,j] - beta, u = (1, P[:,j] / d),
// tau = (beta - R[j,j]) / beta; H = I - tau u u^H satisfies H^H x = beta e_0.
// |u_i| <= 1 and 1 <= |tau| <= 2, so no intermediate is squared: bases with
// columns many orders of magnitude below the others (flat boxes) stay exact.
// A column whose remaining entries are below 1e-14 of the staged rows'
// maximum is skipped (rounding residue of a rank-deficient piece).
// Blocked form: panels of NB columns are reduced column by column, the
// panel's reflectors are accumulated as I - V T V^H (V = [I; Y], Y the u
// vectors, T upper triangular) and the trailing columns get
// C <- C - V T^H (V^H C) with all threads.  Rows of the current piece are
// staged in LDS (row-major, CH rows), followed by the NB rows of R of the
// current panel, so the serial column steps never wait on global memory.
constexpr int kFoldNB = 4;
constexpr int kFoldThreads = 512;

// Cross-lane sums without the LDS crossbar: DPP row operations (quad swaps,
// half-row and row mirrors) give every lane the sum of its aligned group of
// 4, 8 or 16 lanes; the four row sums of a wave are then read with readlane.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// sum over aligned groups of G lanes (G = 4, 8, 16); every lane of a group gets it
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_mov<0xB1>(v);                 // lanes i ^ 1
  v += dpp_mov<0x4E>(v);                 // lanes i ^ 2
  if (G >= 8) v += dpp_mov<0x141>(v);    // half-row mirror
  if (G >= 16) v += dpp_mov<0x140>(v);   // row mirror
  return v;
}
// The four row values of a wave (every lane of row r holding the value of row
// r) combined across rows with the gfx950 lane swaps (upper and lower halves,
// then odd and even rows) instead of readlanes; every lane combines
// (r0 op r2) op (r1 op r3) in the same order, so all lanes get the same bits.
template <bool MAX>
__device__ __forceinline__ double rows_combine(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)(b & 0xffffffffLL), hi = (unsigned)(b >> 32);
  const auto sl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto sh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double a0 = __builtin_bit_cast(double, ((long long)sh[0] << 32) | sl[0]);
  const double a1 = __builtin_bit_cast(double, ((long long)sh[1] << 32) | sl[1]);
  const double h = MAX ? fmax(a0, a1) : a0 + a1;
  const long long c = __builtin_bit_cast(long long, h);
  const unsigned clo = (unsigned)(c & 0xffffffffLL), chi = (unsigned)(c >> 32);
  const auto tl = __builtin_amdgcn_permlane16_swap(clo, clo, false, false);
  const auto th = __builtin_amdgcn_permlane16_swap(chi, chi, false, false);
  const double b0 = __builtin_bit_cast(double, ((long long)th[0] << 32) | tl[0]);
  const double b1 = __builtin_bit_cast(double, ((long long)th[1] << 32) | tl[1]);
  return MAX ? fmax(b0, b1) : b0 + b1;
}
// sum over the whole wave (all lanes active), the same value in every lane
__device__ __forceinline__ double wave_sum(double v) { return rows_combine<false>(group_sum<16>(v)); }
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_mov<0xB1>(v));
  v = fmax(v, dpp_mov<0x4E>(v));
  v = fmax(v, dpp_mov<0x141>(v));
  v = fmax(v, dpp_mov<0x140>(v));
  return rows_combine<true>(v);
}

// Global-memory accesses through address space 1: the task pointers are
// generic, and generic (flat) accesses would make every LDS access wait for
// them.
template <typename T>
__device__ __forceinline__ cpx<T> gld(const cpx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)p;
  return cpx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gst(cpx<T>* p, cpx<T> x) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  *(__attribute__((address_space(1))) v2*)p = v2{x.x, x.y};
}

template <typename PT>
__global__ void __launch_bounds__(kFoldThreads) k_fold(const FoldTask* __restrict__ tasks,
                                                       const FoldPiece* __restrict__ pieces, int ch) {
  extern __shared__ double lds_raw[];
  const FoldTask tk = tasks[blockIdx.x];
  const int n = tk.n;
  z64* R = (z64*)tk.R;
  z64* P = (z64*)lds_raw;                       // [ch][n]
  z64* Rp = P + (size_t)ch * n;                 // [4][NB][n]: rows of R of four panels
  __shared__ z64 s_tauc[2][kFoldNB];            // conj(tau) per panel column (0 if skipped)
  __shared__ double s_wmax[kFoldThreads / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  constexpr int nwaves = kFoldThreads / 64;
  if (tk.init_zero)
    for (int e = tid; e < n * n; e += kFoldThreads) {
      const int i = e % n, j = e / n;
      gst(R + i + (int64_t)j * tk.ldr, z64{0, 0});
    }
  __syncthreads();
  // ---- panel factorization, by wave 0 alone: lane i holds row i of the
  // chunk (p <= 64) for the panel columns j0 .. j0 + nb - 1.  A reflector
  // changes only its own pivot row of R (Rb, the panel's rows), so every panel
  // entry of R is read once before its single update.  Reductions are DPP
  // wave sums; the dot products of a reflector with the later panel columns
  // run together.  Writes the reflectors into P and conj(tau) into tc_out.
  auto factor_panel = [&](z64* Rb, z64* tc_out, int j0, int nb, int p, double skip_below) {
    const bool rowok = lane < p;
    z64 y[kFoldNB], tcs[kFoldNB];
    // the panel block of R (rows and columns j0 .. j0 + nb - 1), upper part,
    // read once; reflector jl changes only row jl of it
    z64 rb[kFoldNB][kFoldNB];
#pragma unroll
    for (int a = 0; a < kFoldNB; ++a) {
      y[a] = (rowok && a < nb) ? P[lane * n + j0 + a] : z64{0, 0};
      tcs[a] = z64{0, 0};
#pragma unroll
      for (int c = 0; c < kFoldNB; ++c) rb[a][c] = (c >= a && c < nb) ? Rb[a * n + j0 + c] : z64{0, 0};
    }
#pragma unroll
    for (int jl = 0; jl < kFoldNB; ++jl) {
      if (jl < nb) {
        const int j = j0 + jl;
        const double mx = wave_max(fmax(fabs(y[jl].x), fabs(y[jl].y)));
        const double sq = wave_sum(y[jl].x * y[jl].x + y[jl].y * y[jl].y);
        if (mx <= skip_below) {
          y[jl] = z64{0, 0};
        } else {
          // Scaled by an exact power of two 2^e >= max|x| (no rounding, no
          // over- or underflow in the squares).  With q = |alpha|, S = |x|:
          // beta = -alpha S / q, tau = 1 + q / S (real), and the reflector
          // entries x_i / (alpha - beta) = x_i conj(alpha) / (q^2 + q S).
          const z64 a = rb[jl][jl];
          int ex;
          (void)frexp(fmax(mx, fmax(fabs(a.x), fabs(a.y))), &ex);
          const double inv = ldexp(1.0, -ex);
          double part;
          if (mx > 1e-140 && mx < 1e140) {
            part = sq * inv * inv;
          } else {
            part = wave_sum((y[jl].x * inv) * (y[jl].x * inv) + (y[jl].y * inv) * (y[jl].y * inv));
          }
          const z64 as{a.x * inv, a.y * inv};
          const double a2 = abs2(as);
          const double S = sqrt(a2 + part);
          const double qa = sqrt(a2);
          z64 beta_s, dinv;
          double tau;
          if (qa > 0.0) {
            const double f = 1.0 / (a2 + qa * S);
            dinv = z64{as.x * f, -as.y * f};
            const double rr = S / qa;
            beta_s = z64{-as.x * rr, -as.y * rr};
            tau = 1.0 + qa / S;
          } else {
            dinv = z64{1.0 / S, 0.0};
            beta_s = z64{-S, 0.0};
            tau = 1.0;
          }
          y[jl] = z64{y[jl].x * inv, y[jl].y * inv} * dinv;
          const z64 tc{tau, 0.0};
          tcs[jl] = tc;
          rb[jl][jl] = z64{ldexp(beta_s.x, ex), ldexp(beta_s.y, ex)};
          z64 w[kFoldNB];
#pragma unroll
          for (int jc = 0; jc < kFoldNB; ++jc) {
            w[jc] = z64{0, 0};
            if (jc > jl) cfmac(w[jc], y[jl], y[jc]);
          }
#pragma unroll
          for (int jc = 0; jc < kFoldNB; ++jc) {
            if (jc > jl) {
              w[jc].x = wave_sum(w[jc].x);
              w[jc].y = wave_sum(w[jc].y);
            }
          }
#pragma unroll
          for (int jc = 0; jc < kFoldNB; ++jc) {
            if (jc > jl && jc < nb) {
              const z64 sw = rb[jl][jc] + w[jc];
              const z64 tw{tc.x * sw.x, tc.x * sw.y};
              y[jc] = y[jc] - y[jl] * tw;
              rb[jl][jc] = rb[jl][jc] - tw;
            }
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < kFoldNB; ++a)
      if (rowok && a < nb) P[lane * n + j0 + a] = y[a];
#pragma unroll
    for (int a = 0; a < kFoldNB; ++a)
      if (lane == a) tc_out[a] = tcs[a];
    if (lane == 0)
#pragma unroll
      for (int a = 0; a < kFoldNB; ++a)
#pragma unroll
        for (int c = 0; c < kFoldNB; ++c)
          if (c >= a && c < nb) Rb[a * n + j0 + c] = rb[a][c];
  };
  // ---- apply the reflectors of panel j0 .. j0 + nb - 1 (in P, conj(tau) in
  // tc_in, R rows in Rb) one after another to columns [cb, ce):
  //   w = R[a, jj] + y_a^H P[:, jj],  R[a, jj] -= conj(tau_a) w,  P[:, jj] -= y_a conj(tau_a) w.
  // 16 lanes per column (slot), lane q holds rows q, q + 16, q + 32, q + 48
  // (p <= 64) of the column and of every reflector in registers; the sums over
  // the 16 lanes of a column are DPP row reductions.  Every lane of the wave
  // takes part (the reductions need the whole row).
  auto apply_panel = [&](z64* Rb, const z64* tc_in, int j0, int nb, int cb, int ce, int slot, int nslots,
                         int p) {
    const int qg = lane & 15;
    z64 yv[4][kFoldNB], tcv[kFoldNB];
#pragma unroll
    for (int a = 0; a < kFoldNB; ++a) {
      tcv[a] = a < nb ? tc_in[a] : z64{0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = qg + 16 * r;
        yv[r][a] = (i < p && a < nb) ? P[i * n + j0 + a] : z64{0, 0};
      }
    }
    for (int jb = cb; jb < ce; jb += nslots) {
      const int jj = jb + slot;
      const bool colok = jj < ce;
      z64 pv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = qg + 16 * r;
        pv[r] = (colok && i < p) ? P[i * n + jj] : z64{0, 0};
      }
      // the R entries of this column (one per reflector) are read up front:
      // reflector a changes only entry a
      z64 rj[kFoldNB];
#pragma unroll
      for (int a = 0; a < kFoldNB; ++a) rj[a] = (colok && a < nb) ? Rb[a * n + jj] : z64{0, 0};
#pragma unroll
      for (int a = 0; a < kFoldNB; ++a) {
        if (a < nb) {
          // conj(y) p over this lane's four rows as a tree (short dependency chain)
          z64 t[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            t[r] = z64{0, 0};
            cfmac(t[r], yv[r][a], pv[r]);
          }
          z64 w = (t[0] + t[1]) + (t[2] + t[3]);
          w.x = group_sum<16>(w.x);
          w.y = group_sum<16>(w.y);
          const z64 sw = rj[a] + w;
          const z64 tw{tcv[a].x * sw.x - tcv[a].y * sw.y, tcv[a].x * sw.y + tcv[a].y * sw.x};
#pragma unroll
          for (int r = 0; r < 4; ++r) pv[r] = pv[r] - yv[r][a] * tw;
          rj[a] = rj[a] - tw;
        }
      }
      if (colok && qg == 0)
#pragma unroll
        for (int a = 0; a < kFoldNB; ++a)
          if (a < nb) Rb[a * n + jj] = rj[a];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = qg + 16 * r;
        if (colok && i < p) P[i * n + jj] = pv[r];
      }
    }
  };
  // Rows stream through LDS in chunks of up to ch rows, filled from as many
  // consecutive pieces as fit (stacking order does not change the R factor).
  int pc = tk.piece_begin, pr0 = 0;                      // next piece and its next row
  while (pc < tk.piece_end && pieces[pc].rows <= 0) ++pc;
  while (pc < tk.piece_end) {
    {
      int p = 0;
      double lmax = 0.0;
      while (p < ch && pc < tk.piece_end) {
        const FoldPiece pp = pieces[pc];
        const cpx<PT>* src = (const cpx<PT>*)pp.P;
        const int take = min(ch - p, pp.rows - pr0);
        // four loads in flight per thread before their LDS stores
        for (int e0 = tid; e0 < take * n; e0 += 4 * kFoldThreads) {
          cpx<PT> v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kFoldThreads;
            const int i = e % take, j = e / take;
            if (e < take * n) v[u] = gld(src + (pr0 + i) + (int64_t)j * pp.ld);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kFoldThreads;
            const int i = e % take, j = e / take;
            if (e < take * n) {
              P[(p + i) * n + j] = z64{(double)v[u].x, (double)v[u].y};
              lmax = fmax(lmax, fmax(fabs((double)v[u].x), fabs((double)v[u].y)));
            }
          }
        }
        p += take;
        pr0 += take;
        if (pr0 >= pp.rows) {
          ++pc;
          pr0 = 0;
          while (pc < tk.piece_end && pieces[pc].rows <= 0) ++pc;
        }
      }
      lmax = wave_max(lmax);
      if (lane == 0) s_wmax[wave] = lmax;
      __syncthreads();
      double cmax = 0.0;
      for (int w = 0; w < nwaves; ++w) cmax = fmax(cmax, s_wmax[w]);
      const double skip_below = 1e-14 * cmax;
      // Panels of kFoldNB columns with one panel of look-ahead: while waves
      // 1..7 apply panel q to the columns after panel q + 1 (and fetch the R
      // rows of panel q + 2), wave 0 applies panel q to the columns of panel
      // q + 1 and factors that panel.  Panel q keeps its rows of R in Rp
      // buffer q % 4 and its conj(tau) in s_tauc buffer q % 2, so one barrier
      // per panel suffices.
      auto load_rows = [&](int q0, int t0, int nthr) {   // R rows of panel q0 -> buffer q0 % 4
        const int jb = q0 * kFoldNB;
        const int nbq = min(kFoldNB, n - jb);
        z64* Rb = Rp + (size_t)(q0 % 4) * kFoldNB * n;
        for (int e = t0; e < nbq * (n - jb); e += nthr) {
          const int a = e % nbq, jj = jb + e / nbq;
          Rb[a * n + jj] = gld(R + jb + a + (int64_t)jj * tk.ldr);
        }
      };
      load_rows(0, tid, kFoldThreads);
      if (kFoldNB < n) load_rows(1, tid, kFoldThreads);
      __syncthreads();
      if (wave == 0) factor_panel(Rp, s_tauc[0], 0, min(kFoldNB, n), p, skip_below);
      __syncthreads();
      for (int q = 0, j0 = 0; j0 < n; ++q, j0 += kFoldNB) {
        const int nb = min(kFoldNB, n - j0);
        const int pe = j0 + nb;                 // end of panel q
        const int nb2 = min(kFoldNB, n - pe);
        const int pe2 = pe + nb2;               // end of panel q + 1
        z64* Rq = Rp + (size_t)(q % 4) * kFoldNB * n;
        z64* Rn = Rp + (size_t)((q + 1) % 4) * kFoldNB * n;
        if (wave == 0) {
          if (nb2 > 0) {
            apply_panel(Rq, s_tauc[q % 2], j0, nb, pe, pe2, lane >> 4, 4, p);
            factor_panel(Rn, s_tauc[(q + 1) % 2], pe, nb2, p, skip_below);
          }
        } else {
          // R rows of panel q + 2: loads issued before the update, stored after it
          const int jb2 = pe2;
          const int nb3 = min(kFoldNB, n - jb2);
          constexpr int kPre = (kFoldNB * kMaxOrder * kMaxOrder * kMaxOrder + 64 * (nwaves - 1) - 1) /
                               (64 * (nwaves - 1));
          z64 pre[kPre];
          const int t1 = tid - 64;
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const int e = t1 + u * 64 * (nwaves - 1);
            if (nb3 > 0 && e < nb3 * (n - jb2)) {
              const int a = e % nb3, jj = jb2 + e / nb3;
              pre[u] = gld(R + jb2 + a + (int64_t)jj * tk.ldr);
            }
          }
          if (pe2 < n)
            apply_panel(Rq, s_tauc[q % 2], j0, nb, pe2, n, (wave - 1) * 4 + (lane >> 4), 4 * (nwaves - 1), p);
          z64* R3 = Rp + (size_t)((q + 2) % 4) * kFoldNB * n;
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const int e = t1 + u * 64 * (nwaves - 1);
            if (nb3 > 0 && e < nb3 * (n - jb2)) {
              const int a = e % nb3, jj = jb2 + e / nb3;
              R3[a * n + jj] = pre[u];
            }
          }
        }
        __syncthreads();
        // rows of panel q of R back to global memory
        for (int e = tid; e < nb * (n - j0); e += kFoldThreads) {
          const int a = e % nb, jj = j0 + e / nb;
          gst(R + j0 + a + (int64_t)jj * tk.ldr, Rq[a * n + jj]);
        }
      }
      __syncthreads();
    }
  }
  if (tk.compact) {
    // A row is filled iff its diagonal is nonzero: reflectors write beta != 0
    // there and never touch rows they skip.  Filled rows are independent (upper
    // triangular with nonzero pivots), so there are at most rank <= folded rows
    // of them; move them to the top in pivot order and clear the rest.
    __shared__ int s_rows[kMaxOrder * kMaxOrder * kMaxOrder];
    __shared__ int s_cnt;
    if (tid == 0) {
      int c = 0;
      for (int j = 0; j < n; ++j) {
        const z64 dg = gld(R + j + (int64_t)j * tk.ldr);
        if (dg.x != 0.0 || dg.y != 0.0) s_rows[c++] = j;
      }
      s_cnt = c;
      if (tk.count) *tk.count = c;
    }
    __syncthreads();
    const int c = s_cnt;
    for (int jj = tid; jj < n; jj += kFoldThreads) {
      for (int r = 0; r < c; ++r) {
        const int i = s_rows[r];
        if (i != r) gst(R + r + (int64_t)jj * tk.ldr, gld(R + i + (int64_t)jj * tk.ldr));
      }
      for (int r = c; r < n; ++r) gst(R + r + (int64_t)jj * tk.ldr, z64{0, 0});
    }
  }
}

// ---------------------------------------------------------------------------
// Truncation SVD (FP64): one-sided (Hestenes) Jacobi on the m columns of a
// rows x m matrix B with round-robin pairs.  With rows = m and B the R factor
// of A^H, the accumulated rotations V are the left singular vectors of A =
// B^H and the column norms its singular values (exact truncation).  With
// rows > m (the sketch path of the learned-rank form) the normalised rotated
// columns W give an orthonormal basis of range(B), and V the left singular
// vectors of B^H.  The rank rule (smallest k with res^2 + sum_{i>k}
// sigma_i^2 <= eps^2, or max(sigma_{k+1}, res) <= eps; Section 3.1: lowest
// rank meeting the bound) is applied in the epilogue; res is the Frobenius
// norm a sketch has already discarded (0 for the exact path), and rank -1
// reports that it alone exceeds the tolerance.
// The input is scaled by a power of two to unit magnitude, and rotations with
// a numerically zero column are skipped, so no product of tiny quantities
// reaches the subnormal range (where the rotation phase would lose its bits).
// Workspace: (rows + m) m complex (B and V), in LDS when lds != 0, else in
// global scratch given by the task.
// eight waves: a round's column pairs (up to m / 2) are spread over more waves
// of the one workgroup that the LDS footprint leaves on a CU
constexpr int kJacobiThreads = 512, kJacobiWaves = kJacobiThreads / 64;

__global__ void __launch_bounds__(kJacobiThreads) k_jacobi(const SvdTask* __restrict__ tasks, int use_lds) {
  extern __shared__ double lds_raw[];
  const SvdTask tk = tasks[blockIdx.x];
  const int m = tk.m;
  const int r = tk.rows > 0 ? tk.rows : m;
  const int mp = (m + 1) & ~1;   // padded to even
  z64* B = use_lds ? (z64*)lds_raw : (z64*)tk.scratch;
  z64* V = B + (int64_t)r * m;
  __shared__ int s_rot;
  __shared__ double s_sig[512];
  __shared__ int s_ord[512];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  __shared__ double s_wmax[kJacobiWaves];
  const z64* Bin = (const z64*)tk.B;
  double lmax = 0.0;
  for (int e = tid; e < r * m; e += kJacobiThreads) {
    const int i = e % r, j = e / r;
    const z64 v = Bin[i + (int64_t)j * tk.ldb];
    lmax = fmax(lmax, fmax(fabs(v.x), fabs(v.y)));
  }
  for (int off = 32; off > 0; off >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, off));
  if (lane == 0) s_wmax[wave] = lmax;
  __syncthreads();
  // exact power-of-two scaling to unit magnitude; sigma is scaled back at the end
  int sexp = 0;
  {
    double mx = 0.0;
    for (int w = 0; w < kJacobiWaves; ++w) mx = fmax(mx, s_wmax[w]);
    if (mx > 0.0) frexp(mx, &sexp);
  }
  for (int e = tid; e < r * m; e += kJacobiThreads) {
    const int i = e % r, j = e / r;
    const z64 v = Bin[i + (int64_t)j * tk.ldb];
    B[e] = z64{ldexp(v.x, -sexp), ldexp(v.y, -sexp)};
  }
  for (int e = tid; e < m * m; e += kJacobiThreads) {
    const int i = e % m, j = e / m;
    V[e] = z64{i == j ? 1.0 : 0.0, 0.0};
  }
  // squared Frobenius norm of the scaled B (rotations keep it): a column whose
  // squared norm is at or below 1e-30 of it (1e-15 of the norm, about 5 units
  // of rounding) carries no singular value that rounding does not already
  // blur, and rotating it against another column changes that column by at
  // most as much; such pairs are skipped, so columns of rounding noise do not
  // keep the sweeps going
  double fro = 0.0;
  for (int e = tid; e < r * m; e += kJacobiThreads) fro += abs2(B[e]);
  for (int off = 32; off > 0; off >>= 1) fro += __shfl_xor(fro, off);
  __syncthreads();
  if (lane == 0) s_wmax[wave] = fro;
  __syncthreads();
  double fro_all = 0.0;
  for (int w = 0; w < kJacobiWaves; ++w) fro_all += s_wmax[w];
  const double tiny = fmax(1e-200, 1e-30 * fro_all);
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < mp - 1; ++round) {
      // round-robin pairing: position 0 stays, the others turn by one place a
      // round; position i > 0 holds column 1 + (i - 1 - round) mod (mp - 1)
      for (int pr = wave; pr < mp / 2; pr += kJacobiWaves) {
        const int i1 = mp - 1 - pr;
        int p = pr == 0 ? 0 : 1 + ((pr - 1 - round) % (mp - 1) + (mp - 1)) % (mp - 1);
        int q = 1 + ((i1 - 1 - round) % (mp - 1) + (mp - 1)) % (mp - 1);
        if (p >= m || q >= m) continue;
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double a = 0, b = 0;
        z64 g{0, 0};
        for (int i = lane; i < r; i += 64) {
          const z64 bp = B[i + p * r], bq = B[i + q * r];
          a += abs2(bp);
          b += abs2(bq);
          cfmac(g, bp, bq);
        }
        for (int off = 32; off > 0; off >>= 1) {
          a += __shfl_xor(a, off);
          b += __shfl_xor(b, off);
          g.x += __shfl_xor(g.x, off);
          g.y += __shfl_xor(g.y, off);
        }
        // columns at or below 1e-100 of unit scale are numerically zero; the
        // test |g| <= 1e-15 |b_p| |b_q| uses the norms, whose product cannot
        // underflow here, so the phase g / |g| below stays exact
        if (fmin(a, b) <= tiny) continue;
        const double ag = sqrt(abs2(g));
        if (ag <= 1e-15 * sqrt(a) * sqrt(b)) continue;
        const double zeta = (b - a) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
        const z64 e{g.x / ag, -g.y / ag};   // exp(-i phi), phi = arg g
        for (int i = lane; i < r; i += 64) {
          const z64 bp = B[i + p * r], bq = B[i + q * r];
          const z64 ebq = e * bq;
          B[i + p * r] = z64{c * bp.x - s * ebq.x, c * bp.y - s * ebq.y};
          B[i + q * r] = z64{s * bp.x + c * ebq.x, s * bp.y + c * ebq.y};
        }
        for (int i = lane; i < m; i += 64) {
          const z64 vp = V[i + p * m], vq = V[i + q * m];
          const z64 evq = e * vq;
          V[i + p * m] = z64{c * vp.x - s * evq.x, c * vp.y - s * evq.y};
          V[i + q * m] = z64{s * vp.x + c * evq.x, s * vp.y + c * evq.y};
        }
        if (lane == 0) s_rot = 1;
      }
      __syncthreads();
    }
    if (!s_rot) break;
    __syncthreads();
  }
  // singular values = column norms of B (scaled), sorted descending (stable)
  for (int j = wave; j < m; j += kJacobiWaves) {
    double a = 0;
    for (int i = lane; i < r; i += 64) a += abs2(B[i + j * r]);
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if (lane == 0) s_sig[j] = sqrt(a);
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < m; ++j) s_ord[j] = j;
    for (int j = 0; j < m; ++j) {
      int best = j;
      for (int l = j + 1; l < m; ++l)
        if (s_sig[s_ord[l]] > s_sig[s_ord[best]]) best = l;
      const int t = s_ord[best];
      for (int l = best; l > j; --l) s_ord[l] = s_ord[l - 1];
      s_ord[j] = t;
    }
    const double res2 = tk.resid ? (*tk.resid) * (*tk.resid) : 0.0;
    int kk = m;
    if (tk.norm_mode == 0) {
      double tail = res2;
      for (int i = m - 1; i >= 0; --i) {
        const double sv = ldexp(s_sig[s_ord[i]], sexp);
        tail += sv * sv;
        if (tail <= tk.eps * tk.eps) kk = i;
        else break;
      }
      if (res2 > tk.eps * tk.eps) kk = -1;
    } else {
      while (kk > 0 && ldexp(s_sig[s_ord[kk - 1]], sexp) <= tk.eps) --kk;
      if (sqrt(res2) > tk.eps) kk = -1;
    }
    if (tk.rank) *tk.rank = kk;
    for (int j = 0; j < m; ++j) tk.sig[j] = ldexp(s_sig[s_ord[j]], sexp);
  }
  __syncthreads();
  if (tk.U) {
    z64* U = (z64*)tk.U;
    for (int e = tid; e < m * m; e += kJacobiThreads) {
      const int i = e % m, j = e / m;
      U[i + (int64_t)j * tk.ldu] = V[i + s_ord[j] * m];
    }
  }
  if (tk.W) {
    z64* W = (z64*)tk.W;
    const double top = s_sig[s_ord[0]];
    for (int e = tid; e < r * m; e += kJacobiThreads) {
      const int i = e % r, j = e / r;
      const double sj = s_sig[s_ord[j]];
      const z64 v = B[i + s_ord[j] * r];
      W[i + (int64_t)j * tk.ldw] = sj > 1e-13 * top ? z64{v.x / sj, v.y / sj} : z64{0, 0};
    }
  }
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds of two 32 x 32 -> 64 bit products
// with the published multipliers and Weyl key increments.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void __launch_bounds__(256) k_sketch_omega(const SketchDesc* __restrict__ dd, uint32_t seed) {
  const SketchDesc d = dd[blockIdx.x];
  z64* Om = (z64*)d.Om;
  for (int e = threadIdx.x; e < d.rows * d.cols; e += 256) {
    const int i = e % d.rows, j = e / d.rows;
    uint32_t c[4] = {(uint32_t)i, (uint32_t)j, (uint32_t)d.stream, (uint32_t)(d.stream >> 32)};
    philox4x32_10(c, seed, 0u);
    // Box-Muller: u1 in (0, 1], u2 in [0, 1)
    const double u1 = ((double)c[0] + 1.0) * 0x1p-32;
    const double u2 = (double)c[1] * 0x1p-32;
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(6.283185307179586 * u2, &sn, &cs);
    Om[i + (int64_t)j * d.ld] = z64{rad * cs, rad * sn};
  }
}

void launch_sketch_omega(const SketchDesc* d, int64_t nd, uint32_t seed, hipStream_t st) {
  if (nd > 0) hipLaunchKernelGGL(k_sketch_omega, dim3((unsigned)nd), dim3(256), 0, st, d, seed);
}

// Frobenius norms of a batch of matrices (block weights omega_b).
template <typename R>
__global__ void __launch_bounds__(256) k_frob(const FrobDesc* __restrict__ dd, double* __restrict__ out) {
  const FrobDesc d = dd[blockIdx.x];
  const cpx<R>* A = (const cpx<R>*)d.A;
  double acc = 0;
  for (int64_t e = threadIdx.x; e < (int64_t)d.M * d.N; e += 256) {
    const int i = (int)(e % d.M), j = (int)(e / d.M);
    const cpx<R> v = A[i + (int64_t)j * d.ld];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[d.index] = sqrt(red[0]);
}

// Exact power-of-two normalisation of a batch of matrices in place: A <- A 2^-e
// with 2^(e-1) <= max |a_ij| < 2^e (real and imaginary parts); a zero matrix
// stays zero.  Keeps the repeated squaring of the Gram matrices (spectral block
// weights) in range without rounding.
__global__ void __launch_bounds__(256) k_scale_pow2(const FrobDesc* __restrict__ dd) {
  const FrobDesc d = dd[blockIdx.x];
  z64* A = (z64*)const_cast<void*>(d.A);
  const int64_t cnt = (int64_t)d.M * d.N;
  double mx = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += 256) {
    const z64 v = A[(e % d.M) + (e / d.M) * (int64_t)d.ld];
    mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (!(red[0] > 0.0)) return;
  int ex = 0;
  frexp(red[0], &ex);
  for (int64_t e = threadIdx.x; e < cnt; e += 256) {
    z64& v = A[(e % d.M) + (e / d.M) * (int64_t)d.ld];
    v = z64{ldexp(v.x, -ex), ldexp(v.y, -ex)};
  }
}

// Largest singular value of M (rt x rs) from a high power of its Gram matrix:
// Gs ~ (M^* M)^(2^j) (side 0, p = rs) or (M M^*)^(2^j) (side 1, p = rt).  The
// column v of Gs with the largest norm lies, up to a component that the powers
// have driven below rounding, in the dominant eigenspace, so the Rayleigh
// quotient |M v| / |v| (side 0) or |M^* v| / |v| (side 1) is |M|_2.  A zero M
// gives 0.  One workgroup per matrix; p <= kSpecMaxP.
__global__ void __launch_bounds__(256) k_spec_final(const SpecDesc* __restrict__ dd, double* __restrict__ out) {
  const SpecDesc d = dd[blockIdx.x];
  const z64* G = (const z64*)d.G;
  const z64* M = (const z64*)d.M;
  const int tid = threadIdx.x;
  __shared__ double s_val[256];
  __shared__ int s_idx[256];
  __shared__ z64 s_v[kSpecMaxP];
  // column of largest norm (ties: the smallest index)
  double best = -1.0;
  int bi = 0;
  for (int j = tid; j < d.p; j += 256) {
    double a = 0.0;
    for (int i = 0; i < d.p; ++i) {
      const z64 g = G[i + (int64_t)j * d.ldg];
      a += g.x * g.x + g.y * g.y;
    }
    if (a > best) {
      best = a;
      bi = j;
    }
  }
  s_val[tid] = best;
  s_idx[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      const double o = s_val[tid + s];
      const int oi = s_idx[tid + s];
      if (o > s_val[tid] || (o == s_val[tid] && oi < s_idx[tid])) {
        s_val[tid] = o;
        s_idx[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (!(s_val[0] > 0.0)) {
    if (tid == 0) out[d.index] = 0.0;
    return;
  }
  const int jv = s_idx[0];
  for (int i = tid; i < d.p; i += 256) s_v[i] = G[i + (int64_t)jv * d.ldg];
  __syncthreads();
  double vv = 0.0, yy = 0.0;
  for (int i = tid; i < d.p; i += 256) vv += s_v[i].x * s_v[i].x + s_v[i].y * s_v[i].y;
  if (d.side == 0) {
    for (int i = tid; i < d.rt; i += 256) {
      double ar = 0.0, ai = 0.0;
      for (int j = 0; j < d.rs; ++j) {
        const z64 a = M[i + (int64_t)j * d.ldm], v = s_v[j];
        ar += a.x * v.x - a.y * v.y;
        ai += a.x * v.y + a.y * v.x;
      }
      yy += ar * ar + ai * ai;
    }
  } else {
    for (int j = tid; j < d.rs; j += 256) {
      double ar = 0.0, ai = 0.0;
      for (int i = 0; i < d.rt; ++i) {
        const z64 a = M[i + (int64_t)j * d.ldm], v = s_v[i];
        ar += a.x * v.x + a.y * v.y;
        ai += a.x * v.y - a.y * v.x;
      }
      yy += ar * ar + ai * ai;
    }
  }
  __syncthreads();
  s_val[tid] = vv;
  __shared__ double s_y[256];
  s_y[tid] = yy;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      s_val[tid] += s_val[tid + s];
      s_y[tid] += s_y[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) out[d.index] = sqrt(s_y[0] / s_val[0]);
}

// Copy of a sub-matrix (column selection / layout change).
template <typename R>
__global__ void k_copy(const CopyDesc* __restrict__ dd) {
  const CopyDesc d = dd[blockIdx.x];
  const cpx<R>* s = (const cpx<R>*)d.src;
  cpx<R>* t = (cpx<R>*)d.dst;
  for (int64_t e = threadIdx.x; e < (int64_t)d.M * d.N; e += blockDim.x) {
    const int i = (int)(e % d.M), j = (int)(e / d.M);
    t[i + (int64_t)j * d.ldd] = s[i + (int64_t)j * d.lds];
  }
}

// Mirror near-field blocks: dst (N x M, leading dimension ldd) = src^T for
// src (M x N, leading dimension lds).  The Galerkin matrix is symmetric, so
// the inadmissible block (s, t) is the transpose of (t, s); 32 x 32 tiles go
// through LDS so that reads and writes are both coalesced.
template <typename R>
__global__ void __launch_bounds__(256) k_transpose_blocks(const CopyDesc* __restrict__ dd) {
  const CopyDesc d = dd[blockIdx.x];
  const cpx<R>* src = (const cpx<R>*)d.src;
  cpx<R>* dst = (cpx<R>*)d.dst;
  __shared__ cpx<R> tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int i0 = 0; i0 < d.M; i0 += 32)
    for (int j0 = 0; j0 < d.N; j0 += 32) {
      for (int jj = ty; jj < 32; jj += 8) {
        const int i = i0 + tx, j = j0 + jj;
        if (i < d.M && j < d.N) tile[jj][tx] = src[i + (int64_t)j * d.lds];
      }
      __syncthreads();
      for (int ii = ty; ii < 32; ii += 8) {
        const int j = j0 + tx, i = i0 + ii;
        if (i < d.M && j < d.N) dst[j + (int64_t)i * d.ldd] = tile[tx][ii];
      }
      __syncthreads();
    }
}

// FP64 -> FP32 narrowing of a complex array (basis data of the FP32 form).
__global__ void k_narrow(const z64* __restrict__ a, z32* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = z32{(float)a[i].x, (float)a[i].y};
}

__global__ void __launch_bounds__(256) k_narrow_list(const NarrowDesc* __restrict__ d) {
  const NarrowDesc t = d[blockIdx.x];
  const z64* a = (const z64*)t.src;
  z32* b = (z32*)t.dst;
  for (int64_t i = threadIdx.x; i < t.n; i += blockDim.x) b[i] = z32{(float)a[i].x, (float)a[i].y};
}

// ---------------------------------------------------------------------------
// launch wrappers
void launch_tri_data(int64_t n, const double* V, const int32_t* T, const int64_t* perm,
                     const QuadTab& qt, double* x7, double* w7, double* x16, double* w16,
                     double* x9, double* w9, double* self_lap, hipStream_t st) {
  hipLaunchKernelGGL(k_tri_data, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, V, T,
                     perm, qt, x7, w7, x16, w16, x9, w9, self_lap);
}

template <typename R>
void launch_near(const NearDesc* d, int64_t nb, double kappa, const double* xq, const double* wq,
                 const double* self_lap, void* out, int nq, hipStream_t st) {
  for (int64_t b0 = 0; b0 < nb; b0 += 1 << 30) {
    const int64_t cnt = std::min<int64_t>(nb - b0, 1 << 30);
    if (nq == 9)
      hipLaunchKernelGGL((k_near<R, 9>), dim3((unsigned)cnt), dim3(256), 0, st, d + b0, kappa, xq, wq,
                         self_lap, (cpx<R>*)out);
    else
      hipLaunchKernelGGL((k_near<R, 16>), dim3((unsigned)cnt), dim3(256), 0, st, d + b0, kappa, xq, wq,
                         self_lap, (cpx<R>*)out);
  }
}
template void launch_near<double>(const NearDesc*, int64_t, double, const double*, const double*,
                                  const double*, void*, int, hipStream_t);
template void launch_near<float>(const NearDesc*, int64_t, double, const double*, const double*,
                                 const double*, void*, int, hipStream_t);

template <typename R>
void launch_leaf_basis(const LeafDesc* d, int64_t nb, const ChebTab& ct, double kappa,
                       const double* xf, const double* wf, int nq, const double* box, const double* dirs,
                       void* out, hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_leaf_basis<R>, dim3((unsigned)nb), dim3(256), 0, st, d, ct, kappa, xf, wf, nq,
                       box, dirs, (cpx<R>*)out);
}
template void launch_leaf_basis<double>(const LeafDesc*, int64_t, const ChebTab&, double,
                                        const double*, const double*, int, const double*,
                                        const double*, void*, hipStream_t);

template <typename R>
void launch_touch(const TouchDesc* d, int64_t nt, const double* V, const SesTab& tab, double kappa,
                  void* out, hipStream_t st) {
  for (int64_t b0 = 0; b0 < nt; b0 += 1 << 30) {
    const int64_t cnt = std::min<int64_t>(nt - b0, 1 << 30);
    hipLaunchKernelGGL(k_touch<R>, dim3((unsigned)cnt), dim3(256), 0, st, d + b0, V, tab, kappa,
                       (cpx<R>*)out);
  }
}
template void launch_touch<double>(const TouchDesc*, int64_t, const double*, const SesTab&, double, void*,
                                   hipStream_t);
template void launch_touch<float>(const TouchDesc*, int64_t, const double*, const SesTab&, double, void*,
                                  hipStream_t);

template <typename R>
void launch_transfer(const TransDesc* d, int64_t nb, const ChebTab& ct, double kappa,
                     const double* box, const double* dirs, void* out, hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_transfer<R>, dim3((unsigned)nb), dim3(256), 0, st, d, ct, kappa, box, dirs,
                       (cpx<R>*)out);
}
template void launch_transfer<double>(const TransDesc*, int64_t, const ChebTab&, double,
                                      const double*, const double*, void*, hipStream_t);

template <typename R>
void launch_coupling(const CoupDesc* d, int64_t nb, const ChebTab& ct, double kappa,
                     const double* box, const double* dirs, void* out, hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_coupling<R>, dim3((unsigned)nb), dim3(256), 0, st, d, ct, kappa, box, dirs,
                       (cpx<R>*)out);
}
template void launch_coupling<double>(const CoupDesc*, int64_t, const ChebTab&, double,
                                      const double*, const double*, void*, hipStream_t);

template <typename RM>
static void launch_gemm_coupling_t(const CoupGemmDesc* d, int64_t nitems, int mt, const ChebTab& ct,
                                   double kappa, const double* box, const double* dirs, hipStream_t st) {
  const int k = ct.m * ct.m * ct.m;
  const int ntn = (k + 31) / 32;
  for (int64_t i0 = 0; i0 < nitems; i0 += 65535) {
    const int64_t cnt = std::min<int64_t>(nitems - i0, 65535);
    const dim3 g((unsigned)ntn, (unsigned)cnt);
    if (mt == 1)
      hipLaunchKernelGGL((k_gemm_coupling<RM, 1, 4, 4>), g, dim3(256), 0, st, d + i0, ct, kappa, box, dirs);
    else if (mt == 2)
      hipLaunchKernelGGL((k_gemm_coupling<RM, 2, 4, 3>), g, dim3(256), 0, st, d + i0, ct, kappa, box, dirs);
    else
      hipLaunchKernelGGL((k_gemm_coupling<RM, 4, 8, 4>), g, dim3(512), 0, st, d + i0, ct, kappa, box, dirs);
  }
}
void launch_gemm_coupling(const CoupGemmDesc* d, int64_t nitems, int mt, const ChebTab& ct, double kappa,
                          const double* box, const double* dirs, int form, hipStream_t st) {
  if (form == 1) {
    launch_gemm_coupling_t<float>(d, nitems, mt, ct, kappa, box, dirs, st);
    return;
  }
  if (form == 0) {
    launch_gemm_coupling_t<double>(d, nitems, mt, ct, kappa, box, dirs, st);
    return;
  }
  const int k = ct.m * ct.m * ct.m;
  const int ntn = (k + 31) / 32;
  for (int64_t i0 = 0; i0 < nitems; i0 += 65535) {
    const int64_t cnt = std::min<int64_t>(nitems - i0, 65535);
    const dim3 g((unsigned)ntn, (unsigned)cnt);
    if (mt == 1)
      hipLaunchKernelGGL((k_gemm_coupling_bf16x3<1, 4, 3>), g, dim3(256), 0, st, d + i0, ct, kappa, box, dirs);
    else if (mt == 2)
      hipLaunchKernelGGL((k_gemm_coupling_bf16x3<2, 4, 3>), g, dim3(256), 0, st, d + i0, ct, kappa, box, dirs);
    else
      hipLaunchKernelGGL((k_gemm_coupling_bf16x3<4, 8, 4>), g, dim3(512), 0, st, d + i0, ct, kappa, box, dirs);
  }
}

template <typename R>
void launch_gemm(const GemmDesc* d, int64_t nitems, int maxM, int maxN, hipStream_t st) {
  if (nitems <= 0 || maxM <= 0 || maxN <= 0) return;
  const int ntm = (maxM + 31) / 32, ntn = (maxN + 31) / 32;
  for (int64_t i0 = 0; i0 < nitems; i0 += 65535) {
    const int64_t cnt = std::min<int64_t>(nitems - i0, 65535);
    hipLaunchKernelGGL((k_gemm<R, R>), dim3((unsigned)(ntm * ntn), (unsigned)cnt), dim3(256), 0, st,
                       d + i0, ntm);
  }
}
template void launch_gemm<double>(const GemmDesc*, int64_t, int, int, hipStream_t);

void launch_gemm_bf16x3(const GemmDesc* d, int64_t nitems, int maxM, int maxN, hipStream_t st) {
  if (nitems <= 0 || maxM <= 0 || maxN <= 0) return;
  const int ntm = (maxM + 31) / 32, ntn = (maxN + 31) / 32;
  for (int64_t i0 = 0; i0 < nitems; i0 += 65535) {
    const int64_t cnt = std::min<int64_t>(nitems - i0, 65535);
    hipLaunchKernelGGL(k_gemm_bf16x3, dim3((unsigned)(ntm * ntn), (unsigned)cnt), dim3(256), 0, st, d + i0, ntm);
  }
}

void launch_gemm_f32(const GemmDesc* d, int64_t nitems, int maxM, int maxN, hipStream_t st) {
  if (nitems <= 0 || maxM <= 0 || maxN <= 0) return;
  const int ntm = (maxM + 31) / 32, ntn = (maxN + 31) / 32;
  for (int64_t i0 = 0; i0 < nitems; i0 += 65535) {
    const int64_t cnt = std::min<int64_t>(nitems - i0, 65535);
    hipLaunchKernelGGL((k_gemm<double, float>), dim3((unsigned)(ntm * ntn), (unsigned)cnt), dim3(256), 0, st,
                       d + i0, ntm);
  }
}

// per-workgroup LDS bytes usable for dynamic buffers, and of the device; set by
// every build (the same values for one device), read by the launchers, so
// atomic: builds may run in several host threads
static std::atomic<size_t> g_lds_limit{65536};
static std::atomic<size_t> g_lds_total{65536};

void set_lds_limit(size_t bytes) {
  g_lds_total = bytes;
  // keep 12 KB for the kernels' static shared variables
  g_lds_limit = bytes > 24576 ? bytes - 12288 : 12288;
}

// The panel factorization keeps one chunk row per lane of a wave, so a chunk
// has at most 64 rows.
int fold_rows_per_chunk(int n) {
  // the fold's own static LDS is below 4 KB
  int ch = (int)((g_lds_total - 4096) / ((size_t)n * 16)) - 4 * kFoldNB;
  if (ch > 64) ch = 64;
  if (ch < 1) ch = 1;
  return ch;
}

template <typename PT>
void launch_fold(const FoldTask* t, int64_t ntasks, const FoldPiece* p, int n, hipStream_t st) {
  if (ntasks <= 0) return;
  const int ch = fold_rows_per_chunk(n);
  const size_t lds = (size_t)(ch + 4 * kFoldNB) * n * 16;
  hipLaunchKernelGGL(k_fold<PT>, dim3((unsigned)ntasks), dim3(kFoldThreads), lds, st, t, p, ch);
}
template void launch_fold<double>(const FoldTask*, int64_t, const FoldPiece*, int, hipStream_t);
template void launch_fold<float>(const FoldTask*, int64_t, const FoldPiece*, int, hipStream_t);

// ---------------------------------------------------------------------------
// Gram form of the total weights.

__global__ void __launch_bounds__(256) k_gram_sum(const GramSumTask* __restrict__ tasks,
                                                  const void* const* __restrict__ srcs) {
  const GramSumTask t = tasks[blockIdx.x];
  z64* G = (z64*)t.G;
  const int nn = t.nw * t.nw;
  for (int e = blockIdx.y * 256 + threadIdx.x; e < nn; e += 256 * gridDim.y) {
    const int i = e % t.nw, j = e / t.nw;
    if (i > j && !t.full) continue;
    const int64_t o = i + (int64_t)j * t.ldg;
    z64 v = t.init ? z64{0, 0} : G[o];
    for (int q = t.src_begin; q < t.src_end; ++q) v = v + ((const z64*)srcs[q])[o];
    G[o] = v;
  }
}

void launch_gram_sum(const GramSumTask* t, int64_t ntasks, const void* const* srcs, hipStream_t st) {
  if (ntasks > 0)
    hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)ntasks, 8), dim3(256), 0, st, t, srcs);
}

__global__ void k_row_weights(const RowWeightTask* __restrict__ tasks, int64_t ntasks,
                              const double* __restrict__ w, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntasks) return;
  const RowWeightTask t = tasks[i];
  const double wv = w[t.index];
  const double s = wv > 0.0 ? 1.0 / wv : 0.0;
  for (int r = 0; r < t.rows; ++r) out[t.off + r] = s;
}

// a workgroup per (segment, group of 16 columns); each thread keeps the
// factors of its rows while it walks the columns
__global__ void __launch_bounds__(256) k_scale_segments(const SegScaleTask* __restrict__ tasks) {
  const SegScaleTask t = tasks[blockIdx.x];
  z64* A = (z64*)t.A;
  const int j0 = blockIdx.y * 16, j1 = min(t.cols, j0 + 16);
  for (int r = threadIdx.x; r < t.rows; r += 256) {
    const double f = t.f[r];
    z64* a = A + r + (int64_t)j0 * t.rows;
    for (int j = j0; j < j1; ++j, a += t.rows) *a = f * *a;
  }
}

void launch_scale_segments(const SegScaleTask* t, int64_t ntasks, int maxcols, hipStream_t st) {
  if (ntasks > 0)
    hipLaunchKernelGGL(k_scale_segments, dim3((unsigned)ntasks, (unsigned)((maxcols + 15) / 16)), dim3(256), 0, st, t);
}

void launch_row_weights(const RowWeightTask* t, int64_t ntasks, const double* w, double* out, hipStream_t st) {
  if (ntasks > 0)
    hipLaunchKernelGGL(k_row_weights, dim3((unsigned)((ntasks + 255) / 256)), dim3(256), 0, st, t, ntasks, w, out);
}

// column of packed upper-triangle entry e (entries of column j are j (j + 1) / 2
// .. j (j + 1) / 2 + j)
__device__ __forceinline__ int packed_col(int e) {
  int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while ((j + 1) * (j + 2) / 2 <= e) ++j;
  while (j * (j + 1) / 2 > e) --j;
  return j;
}

// largest value (smallest index on ties) over the workgroup; red: 8 slots
__device__ __forceinline__ void argmax256(double& v, int& i, double* rv, int* ri) {
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(i, off);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rv[w] = v;
    ri[w] = i;
  }
  __syncthreads();
  v = rv[0];
  i = ri[0];
  for (int q = 1; q < 4; ++q)
    if (rv[q] > v || (rv[q] == v && ri[q] < i)) {
      v = rv[q];
      i = ri[q];
    }
  __syncthreads();
}

// Cholesky factorisation with diagonal pivoting of a Hermitian positive
// semi-definite matrix, outer-product form.  Each step takes the largest
// remaining diagonal entry of the Schur complement as pivot and stops once it
// is at or below nw 2^-52 times the largest diagonal entry of G: what remains
// is rounding noise (for semi-definite matrices this pivoting makes the
// factorisation backward stable).  Row j of R is the j-th pivot row of the
// Schur complement divided by the square root of its pivot, kept in the
// original column order, so that R^H R = G without a permutation.  The
// matrix is held packed (upper triangle, column by column) in LDS, or in the
// task's scratch when it does not fit.
__global__ void __launch_bounds__(256) k_pchol(const PcholTask* __restrict__ tasks, int use_lds) {
  const PcholTask t = tasks[blockIdx.x];
  const int nw = t.nw, tid = threadIdx.x;
  const int64_t ldg = t.ldg;
  z64* G = (z64*)t.G;
  const int npk = nw * (nw + 1) / 2;
  extern __shared__ z64 dyn[];
  z64* l = dyn;                                   // nw: the current pivot row / sqrt(pivot)
  double* d = (double*)(dyn + nw);                // nw: diagonal of the Schur complement
  z64* U = use_lds ? dyn + nw + (nw + 1) / 2 : (z64*)t.scratch;
  __shared__ double rv[4];
  __shared__ int ri[4];
  for (int e = tid; e < npk; e += 256) {
    const int j = packed_col(e), i = e - j * (j + 1) / 2;
    U[e] = G[i + j * ldg];
  }
  for (int i = tid; i < nw; i += 256) d[i] = G[i + i * ldg].x;
  __syncthreads();
  double v0 = -INFINITY;
  int i0 = 0x7fffffff;
  for (int i = tid; i < nw; i += 256)
    if (d[i] > v0 || (d[i] == v0 && i < i0)) {
      v0 = d[i];
      i0 = i;
    }
  argmax256(v0, i0, rv, ri);
  const double delta = (double)nw * 0x1p-52 * v0;
  int r = 0;
  for (int step = 0; step < nw; ++step) {
    double bv = -INFINITY;
    int p = 0x7fffffff;
    for (int i = tid; i < nw; i += 256)
      if (d[i] > bv || (d[i] == bv && i < p)) {
        bv = d[i];
        p = i;
      }
    argmax256(bv, p, rv, ri);
    if (!(bv > delta) || !(v0 > 0.0)) break;
    const double piv = sqrt(bv), ipiv = 1.0 / piv;
    for (int i = tid; i < nw; i += 256) {
      z64 li{0, 0};
      if (i != p && d[i] != -INFINITY) {
        const z64 g = p <= i ? U[i * (i + 1) / 2 + p] : conj(U[p * (p + 1) / 2 + i]);
        li = ipiv * g;
      }
      l[i] = li;
      G[step + i * ldg] = i == p ? z64{piv, 0.0} : li;
    }
    __syncthreads();
    if (tid == 0) d[p] = -INFINITY;
    for (int e = tid; e < npk; e += 256) {
      const int j = packed_col(e), i = e - j * (j + 1) / 2;
      const z64 li = l[i], lj = l[j];
      if ((li.x == 0.0 && li.y == 0.0) || (lj.x == 0.0 && lj.y == 0.0)) continue;
      z64 u = U[e];
      u.x -= li.x * lj.x + li.y * lj.y;
      u.y -= li.x * lj.y - li.y * lj.x;
      U[e] = u;
      if (i == j) d[i] = u.x;
    }
    __syncthreads();
    r = step + 1;
  }
  const int rest = nw - r;
  for (int e = tid; e < rest * nw; e += 256) {
    const int i = r + e % rest, j = e / rest;
    G[i + j * ldg] = z64{0, 0};
  }
  if (tid == 0 && t.count) *t.count = r;
}

size_t pchol_lds_bytes(int nw) {
  return ((size_t)nw * (nw + 1) / 2 + (size_t)nw + (size_t)(nw + 1) / 2) * 16;
}

bool pchol_fits_lds(int nw) { return pchol_lds_bytes(nw) <= g_lds_limit; }

void launch_pchol(const PcholTask* t, int64_t ntasks, int maxnw, hipStream_t st) {
  if (ntasks <= 0) return;
  const int use_lds = pchol_fits_lds(maxnw) ? 1 : 0;
  const size_t lds = use_lds ? pchol_lds_bytes(maxnw) : ((size_t)maxnw + (size_t)(maxnw + 1) / 2) * 16;
  hipLaunchKernelGGL(k_pchol, dim3((unsigned)ntasks), dim3(256), lds, st, t, use_lds);
}

void launch_jacobi(const SvdTask* t, int64_t ntasks, int maxm, int maxr, hipStream_t st) {
  if (ntasks <= 0) return;
  const size_t need = (size_t)(maxr + maxm) * maxm * 16;
  const int use_lds = need <= g_lds_limit ? 1 : 0;
  hipLaunchKernelGGL(k_jacobi, dim3((unsigned)ntasks), dim3(kJacobiThreads), use_lds ? need : 0, st, t, use_lds);
}

template <typename R>
void launch_frob(const FrobDesc* d, int64_t nb, double* out, hipStream_t st) {
  if (nb > 0) hipLaunchKernelGGL(k_frob<R>, dim3((unsigned)nb), dim3(256), 0, st, d, out);
}
template void launch_frob<double>(const FrobDesc*, int64_t, double*, hipStream_t);
template void launch_frob<float>(const FrobDesc*, int64_t, double*, hipStream_t);

void launch_scale_pow2(const FrobDesc* d, int64_t nb, hipStream_t st) {
  if (nb > 0) hipLaunchKernelGGL(k_scale_pow2, dim3((unsigned)nb), dim3(256), 0, st, d);
}

void launch_spec_final(const SpecDesc* d, int64_t nb, double* out, hipStream_t st) {
  if (nb > 0) hipLaunchKernelGGL(k_spec_final, dim3((unsigned)nb), dim3(256), 0, st, d, out);
}

template <typename R>
void launch_copy(const CopyDesc* d, int64_t nb, hipStream_t st) {
  if (nb > 0) hipLaunchKernelGGL(k_copy<R>, dim3((unsigned)nb), dim3(256), 0, st, d);
}
template void launch_copy<double>(const CopyDesc*, int64_t, hipStream_t);
template void launch_copy<float>(const CopyDesc*, int64_t, hipStream_t);

template <typename R>
void launch_transpose_blocks(const CopyDesc* d, int64_t nb, hipStream_t st) {
  for (int64_t o = 0; o < nb; o += (1 << 30)) {
    const int64_t cnt = nb - o < (1 << 30) ? nb - o : (1 << 30);
    hipLaunchKernelGGL(k_transpose_blocks<R>, dim3((unsigned)cnt), dim3(256), 0, st, d + o);
  }
}
template void launch_transpose_blocks<double>(const CopyDesc*, int64_t, hipStream_t);
template void launch_transpose_blocks<float>(const CopyDesc*, int64_t, hipStream_t);

void launch_narrow(const void* a, void* b, int64_t n, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const z64*)a, (z32*)b, n);
}

void launch_narrow_list(const NarrowDesc* d, int64_t nd, hipStream_t st) {
  for (int64_t o = 0; o < nd; o += (1 << 30)) {
    const int64_t cnt = nd - o < (1 << 30) ? nd - o : (1 << 30);
    hipLaunchKernelGGL(k_narrow_list, dim3((unsigned)cnt), dim3(256), 0, st, d + o);
  }
}

}  // namespace dh2
