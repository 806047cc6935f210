// Gauss-quadrature form of the operator (paper §2.3: Gauss quadrature, isoparametric geometry
// evaluated at every quadrature point). Each element integrates with the q = p + 1 point
// Gauss-Legendre rule per axis: the GLL basis is interpolated to the points by I~ (I~_qi =
// l_i(eta_q)) and differentiated by D~ = I~ D, so the reference gradient is
//   u_x = (D~ (x) I~ (x) I~) u,  u_y = (I~ (x) D~ (x) I~) u,  u_z = (I~ (x) I~ (x) D~) u
// (factors along x, y, z), w = G~ grad u at every point with G~ = w~ mu(x_q) detJ J^{-1} J^{-T},
// and y_e = sum_a B_a^T w_a. Every element matrix is dense, unlike the collocated form; the sum
// factorization keeps the product at O(n^4) per element: five passes along coordinate lines,
// one line per thread, each pass in place in LDS (a thread reads all of its line into
// registers before writing it back), so three n^3 tiles per element suffice (3D, n = 17, FP64:
// 118 KB). The element vectors go to the element-vector buffer and the gather of the collocated
// product sums them and runs the epilogue.
#include <cstdint>

#include "dev_apply.h"
#include "fields.h"
#include "internal.h"

namespace gllmg {

namespace {

constexpr int kThreads = 256;

inline unsigned nblocks(int64_t n, int t = kThreads) { return (unsigned)((n + t - 1) / t); }

template <int N>
struct EpbG3 {
  static constexpr int v = (N * N >= 128) ? 1 : (256 / (N * N));
};
template <int N>
struct EpbG2 {
  static constexpr int v = 256 / N;
};

// ------------------------------------------------------------------ 3D product
// Thread (a0, a1) of an element: pass 1 and 5 along z at (x, y) = (a0, a1); passes 2 and 4
// along y at (x, z) = (a0, a1); pass 3 along x at (y, z) = (a0, a1). Tiles T0, T1, T2 hold
// the lines between passes.
template <int N, typename T, int EPB>
__global__ void __launch_bounds__(EPB * N * N)
k_apply3d_gauss(const T* __restrict__ x, T* __restrict__ F, const T* __restrict__ G,
                const T* __restrict__ Iq, const T* __restrict__ Dq, Grid g, int neumann) {
  constexpr int NN = N * N, NNN = N * N * N, P = N - 1;
  __shared__ T lds[2 * NN + 3 * EPB * NNN];
  T* sI = lds;
  T* sDq = lds + NN;
  const int t = threadIdx.x;
  for (int q = t; q < NN; q += EPB * NN) {
    sI[q] = Iq[q];
    sDq[q] = Dq[q];
  }
  const int le = t / NN, ij = t - le * NN;
  const int a0 = ij % N, a1 = ij / N;
  const uint32_t e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool valid = e < (uint32_t)g.E;
  const uint32_t ee = valid ? e : 0u;
  const uint32_t nexy = (uint32_t)g.ne[0] * (uint32_t)g.ne[1];
  const int ez = (int)(ee / nexy);
  const uint32_t rxy = ee - (uint32_t)ez * nexy;
  const int ey = (int)(rxy / (uint32_t)g.ne[0]);
  const int ex = (int)(rxy - (uint32_t)ey * g.ne[0]);
  T* T0 = lds + 2 * NN + le * 3 * NNN;
  T* T1 = T0 + NNN;
  T* T2 = T1 + NNN;
  const T* Ge = G + (int64_t)ee * (6 * NNN);
  // pass 1: the z-column of x at (a0, a1), interpolated and differentiated along z
  {
    const int gx = ex * P + a0, gy = ey * P + a1;
    const bool bxy = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1;
    const int64_t sxy = (int64_t)g.nn[0] * g.nn[1];
    const int64_t gb = gx + (int64_t)g.nn[0] * gy + sxy * (int64_t)(ez * P);
    T col[N];
#pragma unroll
    for (int k = 0; k < N; ++k) col[k] = x[gb + sxy * k];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int gz = ez * P + k;
      const bool bnd = bxy || gz == 0 || gz == g.nn[2] - 1;
      if (bnd && !neumann) col[k] = T(0);
    }
    __syncthreads();  // sI, sDq
#pragma unroll
    for (int kq = 0; kq < N; ++kq) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        s0 += sI[kq * N + k] * col[k];
        s1 += sDq[kq * N + k] * col[k];
      }
      T0[a0 + N * a1 + NN * kq] = s0;
      T1[a0 + N * a1 + NN * kq] = s1;
    }
  }
  __syncthreads();
  // pass 2: along y at (x, z) = (a0, a1): T0 -> I~_y T0 (in place), D~_y T0 -> T2; T1 -> I~_y T1
  {
    const int c = a0 + NN * a1;
    T v[N], w[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      v[j] = T0[c + N * j];
      w[j] = T1[c + N * j];
    }
#pragma unroll
    for (int jq = 0; jq < N; ++jq) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        s0 += sI[jq * N + j] * v[j];
        s1 += sDq[jq * N + j] * v[j];
        s2 += sI[jq * N + j] * w[j];
      }
      T0[c + N * jq] = s0;
      T2[c + N * jq] = s1;
      T1[c + N * jq] = s2;
    }
  }
  __syncthreads();
  // pass 3: along x at (y, z) = (a0, a1): the gradient at the row's Gauss points, w = G~ grad u,
  // and the transposed x-factors, back in place
  {
    const int base = N * a0 + NN * a1;
    T ra[N], rb[N], rc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      ra[i] = T0[base + i];
      rb[i] = T2[base + i];
      rc[i] = T1[base + i];
    }
    T wx[N], wy[N], wz[N];
#pragma unroll
    for (int iq = 0; iq < N; ++iq) {
      T ux = T(0), uy = T(0), uz = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        ux += sDq[iq * N + i] * ra[i];
        uy += sI[iq * N + i] * rb[i];
        uz += sI[iq * N + i] * rc[i];
      }
      const int q = base + iq;
      const T g0 = Ge[q], g1 = Ge[NNN + q], g2 = Ge[2 * NNN + q], g3 = Ge[3 * NNN + q],
              g4 = Ge[4 * NNN + q], g5 = Ge[5 * NNN + q];
      wx[iq] = g0 * ux + g1 * uy + g2 * uz;
      wy[iq] = g1 * ux + g3 * uy + g4 * uz;
      wz[iq] = g2 * ux + g4 * uy + g5 * uz;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int iq = 0; iq < N; ++iq) {
        s0 += sDq[iq * N + i] * wx[iq];
        s1 += sI[iq * N + i] * wy[iq];
        s2 += sI[iq * N + i] * wz[iq];
      }
      T0[base + i] = s0;
      T2[base + i] = s1;
      T1[base + i] = s2;
    }
  }
  __syncthreads();
  // pass 4: along y transposed at (x, z) = (a0, a1): T0 <- I~^T T0 + D~^T T2, T1 <- I~^T T1
  {
    const int c = a0 + NN * a1;
    T v[N], w[N], u[N];
#pragma unroll
    for (int jq = 0; jq < N; ++jq) {
      v[jq] = T0[c + N * jq];
      w[jq] = T2[c + N * jq];
      u[jq] = T1[c + N * jq];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int jq = 0; jq < N; ++jq) {
        s0 += sI[jq * N + j] * v[jq];
        s0 += sDq[jq * N + j] * w[jq];
        s1 += sI[jq * N + j] * u[jq];
      }
      T0[c + N * j] = s0;
      T1[c + N * j] = s1;
    }
  }
  __syncthreads();
  // pass 5: along z transposed at (x, y) = (a0, a1): y_e = I~^T T0 + D~^T T1
  {
    const int c = a0 + N * a1;
    T v[N], w[N];
#pragma unroll
    for (int kq = 0; kq < N; ++kq) {
      v[kq] = T0[c + NN * kq];
      w[kq] = T1[c + NN * kq];
    }
    if (!valid) return;
    T* Fe = F + (int64_t)ee * NNN + c;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      T s = T(0);
#pragma unroll
      for (int kq = 0; kq < N; ++kq) {
        s += sI[kq * N + k] * v[kq];
        s += sDq[kq * N + k] * w[kq];
      }
      Fe[NN * k] = s;
    }
  }
}

// ------------------------------------------------------------------ 2D product
// Thread a of an element: passes 1 and 3 along y at x = a, pass 2 along x at y = a.
template <int N, typename T, int EPB>
__global__ void __launch_bounds__(EPB * N)
k_apply2d_gauss(const T* __restrict__ x, T* __restrict__ F, const T* __restrict__ G,
                const T* __restrict__ Iq, const T* __restrict__ Dq, Grid g, int neumann) {
  constexpr int NN = N * N, P = N - 1;
  __shared__ T lds[2 * NN + 2 * EPB * NN];
  T* sI = lds;
  T* sDq = lds + NN;
  const int t = threadIdx.x;
  for (int q = t; q < NN; q += EPB * N) {
    sI[q] = Iq[q];
    sDq[q] = Dq[q];
  }
  const int le = t / N, a = t - le * N;
  const uint32_t e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool valid = e < (uint32_t)g.E;
  const uint32_t ee = valid ? e : 0u;
  const int ey = (int)(ee / (uint32_t)g.ne[0]);
  const int ex = (int)(ee - (uint32_t)ey * g.ne[0]);
  T* T0 = lds + 2 * NN + le * 2 * NN;
  T* T1 = T0 + NN;
  const T* Ge = G + (int64_t)ee * (3 * NN);
  {
    const int gx = ex * P + a;
    const bool bx = gx == 0 || gx == g.nn[0] - 1;
    T col[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int gy = ey * P + j;
      col[j] = x[gx + (int64_t)g.nn[0] * gy];
      const bool bnd = bx || gy == 0 || gy == g.nn[1] - 1;
      if (bnd && !neumann) col[j] = T(0);
    }
    __syncthreads();
#pragma unroll
    for (int jq = 0; jq < N; ++jq) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        s0 += sI[jq * N + j] * col[j];
        s1 += sDq[jq * N + j] * col[j];
      }
      T0[a + N * jq] = s0;
      T1[a + N * jq] = s1;
    }
  }
  __syncthreads();
  {
    const int base = N * a;
    T ra[N], rc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      ra[i] = T0[base + i];
      rc[i] = T1[base + i];
    }
    T wx[N], wy[N];
#pragma unroll
    for (int iq = 0; iq < N; ++iq) {
      T ux = T(0), uy = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        ux += sDq[iq * N + i] * ra[i];
        uy += sI[iq * N + i] * rc[i];
      }
      const int q = base + iq;
      const T g0 = Ge[q], g1 = Ge[NN + q], g2 = Ge[2 * NN + q];
      wx[iq] = g0 * ux + g1 * uy;
      wy[iq] = g1 * ux + g2 * uy;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int iq = 0; iq < N; ++iq) {
        s0 += sDq[iq * N + i] * wx[iq];
        s1 += sI[iq * N + i] * wy[iq];
      }
      T0[base + i] = s0;
      T1[base + i] = s1;
    }
  }
  __syncthreads();
  {
    T v[N], w[N];
#pragma unroll
    for (int jq = 0; jq < N; ++jq) {
      v[jq] = T0[a + N * jq];
      w[jq] = T1[a + N * jq];
    }
    if (!valid) return;
    T* Fe = F + (int64_t)ee * NN + a;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T s = T(0);
#pragma unroll
      for (int jq = 0; jq < N; ++jq) {
        s += sI[jq * N + j] * v[jq];
        s += sDq[jq * N + j] * w[jq];
      }
      Fe[N * j] = s;
    }
  }
}

// ------------------------------------------------------------------ setup kernels (FP64)
// Physical coordinates of every Gauss point: the isoparametric interpolant of the element's
// mapped nodes, x_q = sum_i (I~ (x) I~ (x) I~)_qi x_i. One thread per (element, point).
__global__ void __launch_bounds__(kThreads)
k_gauss_points(Grid g, int n, const double* __restrict__ Iq, const double* __restrict__ xn,
               double* __restrict__ xq) {
  const int dim = g.dim;
  const int nloc = dim == 3 ? n * n * n : n * n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.E * nloc) return;
  const int64_t e = t / nloc;
  const int q = (int)(t - e * nloc);
  const int ec[3] = {(int)(e % g.ne[0]), (int)((e / g.ne[0]) % g.ne[1]),
                     dim == 3 ? (int)(e / ((int64_t)g.ne[0] * g.ne[1])) : 0};
  const int qc[3] = {q % n, (q / n) % n, dim == 3 ? q / (n * n) : 0};
  const int64_t st[3] = {1, g.nn[0], (int64_t)g.nn[0] * g.nn[1]};
  const int p = n - 1;
  double acc[3] = {0, 0, 0};
  for (int k = 0; k < (dim == 3 ? n : 1); ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double wgt = Iq[qc[0] * n + i] * Iq[qc[1] * n + j];
        if (dim == 3) wgt *= Iq[qc[2] * n + k];
        const int64_t node = (ec[0] * p + i) * st[0] + (int64_t)(ec[1] * p + j) * st[1] +
                             (dim == 3 ? (int64_t)(ec[2] * p + k) * st[2] : 0);
        for (int a = 0; a < dim; ++a) acc[a] += wgt * xn[node * dim + a];
      }
  for (int a = 0; a < dim; ++a) xq[t * dim + a] = acc[a];
}

__global__ void __launch_bounds__(kThreads)
k_field_pts(int64_t npts, int dim, const double* __restrict__ pts, FieldDev f,
            double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npts) return;
  double x[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) x[a] = pts[t * dim + a];
  out[t] = field_eval(f, dim, x);
}

// Geometry at every Gauss point: J_ab = sum_i (M^b_x (x) M^b_y (x) M^b_z)_qi x_a(i), with
// M^b = D~ along b and I~ along the other axes; G~ = w~_q mu_q detJ J^{-1} J^{-T} and
// w~_q detJ. Layout [e][component][q] as the collocated factors.
template <int DIM>
__global__ void __launch_bounds__(kThreads)
k_geometry_gauss(Grid g, int n, const double* __restrict__ wg, const double* __restrict__ Iq,
                 const double* __restrict__ Dq, const double* __restrict__ xn,
                 const double* __restrict__ muq, double* __restrict__ G64, float* __restrict__ G32,
                 double* __restrict__ wdetq, int* __restrict__ flag) {
  const int nloc = DIM == 3 ? n * n * n : n * n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.E * nloc) return;
  const int64_t e = t / nloc;
  const int q = (int)(t - e * nloc);
  const int ec[3] = {(int)(e % g.ne[0]), (int)((e / g.ne[0]) % g.ne[1]),
                     DIM == 3 ? (int)(e / ((int64_t)g.ne[0] * g.ne[1])) : 0};
  const int qc[3] = {q % n, (q / n) % n, DIM == 3 ? q / (n * n) : 0};
  const int64_t st[3] = {1, g.nn[0], (int64_t)g.nn[0] * g.nn[1]};
  const int p = n - 1;
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int k = 0; k < (DIM == 3 ? n : 1); ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const int li[3] = {i, j, k};
        double wb[3];
        for (int b = 0; b < DIM; ++b) {
          double v = 1.0;
          for (int c = 0; c < DIM; ++c) v *= (c == b ? Dq : Iq)[qc[c] * n + li[c]];
          wb[b] = v;
        }
        int64_t node = 0;
        for (int c = 0; c < DIM; ++c) node += (int64_t)(ec[c] * p + li[c]) * st[c];
        for (int a = 0; a < DIM; ++a) {
          const double xa = xn[node * DIM + a];
          for (int b = 0; b < DIM; ++b) J[a][b] += wb[b] * xa;
        }
      }
  double wq = wg[qc[0]] * wg[qc[1]];
  if (DIM == 3) wq *= wg[qc[2]];
  double det, I[3][3];
  if (DIM == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    I[0][0] = J[1][1] / det;
    I[0][1] = -J[0][1] / det;
    I[1][0] = -J[1][0] / det;
    I[1][1] = J[0][0] / det;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    I[0][0] = c00 / det;
    I[1][0] = c01 / det;
    I[2][0] = c02 / det;
    I[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    I[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    I[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    I[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    I[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    I[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  if (!(det > 0.0)) atomicOr(flag, 1);
  const double m = muq[t];
  if (!(m > 0.0) || !isfinite(m)) atomicOr(flag, 2);
  const double sc = wq * m * det;
  const int ncomp = DIM == 3 ? 6 : 3;
  int c = 0;
  const int64_t base = e * (int64_t)ncomp * nloc + q;
  for (int a = 0; a < DIM; ++a)
    for (int b = a; b < DIM; ++b) {
      double s = 0.0;
      for (int k = 0; k < DIM; ++k) s += I[a][k] * I[b][k];
      const double v = sc * s;
      if (G64) G64[base + (int64_t)c * nloc] = v;
      if (G32) G32[base + (int64_t)c * nloc] = (float)v;
      ++c;
    }
  if (wdetq) wdetq[t] = wq * det;
}

// diag_e(i) = sum_q sum_ab G~_ab(q) B_a(q, i) B_b(q, i), B_a(q, i) = prod_c M^a_c[q_c, i_c]: one
// thread per (element, node), into the element-vector buffer.
__global__ void __launch_bounds__(kThreads)
k_diag_gauss(const double* __restrict__ G, const double* __restrict__ Iq,
             const double* __restrict__ Dq, Grid g, double* __restrict__ F) {
  const int n = g.p + 1, dim = g.dim;
  const int nloc = dim == 3 ? n * n * n : n * n;
  const int ncomp = dim == 3 ? 6 : 3;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.E * nloc) return;
  const int64_t e = t / nloc;
  const int i = (int)(t - e * nloc);
  const int ic[3] = {i % n, (i / n) % n, dim == 3 ? i / (n * n) : 0};
  const double* Ge = G + e * (int64_t)ncomp * nloc;
  double acc = 0.0;
  for (int q = 0; q < nloc; ++q) {
    const int qc[3] = {q % n, (q / n) % n, dim == 3 ? q / (n * n) : 0};
    double B[3];
    for (int a = 0; a < dim; ++a) {
      double v = 1.0;
      for (int c = 0; c < dim; ++c) v *= (c == a ? Dq : Iq)[qc[c] * n + ic[c]];
      B[a] = v;
    }
    int c = 0;
    for (int a = 0; a < dim; ++a)
      for (int b = a; b < dim; ++b) {
        const double gv = Ge[(int64_t)c * nloc + q];
        acc += (a == b ? 1.0 : 2.0) * gv * B[a] * B[b];
        ++c;
      }
  }
  F[t] = acc;
}

// Consistent mass M f on the element level: y_e = I~^T diag(w~ detJ) I~ f_e, one element per
// thread group as in the product (FP64; f is read at every node, boundary included).
template <int N, int DIM>
__global__ void __launch_bounds__(DIM == 3 ? N * N : N)
k_mass_gauss(const double* __restrict__ f, double* __restrict__ F,
             const double* __restrict__ wdetq, const double* __restrict__ Iq, Grid g) {
  constexpr int NN = N * N, NL = DIM == 3 ? N * N * N : N * N, P = N - 1;
  __shared__ double sI[NN];
  __shared__ double T0[NL];
  const int t = threadIdx.x;
  for (int q = t; q < NN; q += blockDim.x) sI[q] = Iq[q];
  const int64_t e = blockIdx.x;
  const int ex = (int)(e % g.ne[0]), ey = (int)((e / g.ne[0]) % g.ne[1]),
            ez = DIM == 3 ? (int)(e / ((int64_t)g.ne[0] * g.ne[1])) : 0;
  const int64_t sy = g.nn[0], sz = (int64_t)g.nn[0] * g.nn[1];
  const double* We = wdetq + e * NL;
  if constexpr (DIM == 3) {
    const int a0 = t % N, a1 = t / N;
    double col[N];
    for (int k = 0; k < N; ++k)
      col[k] = f[(ex * P + a0) + sy * (ey * P + a1) + sz * (ez * P + k)];
    __syncthreads();
    for (int kq = 0; kq < N; ++kq) {  // along z at (x, y) = (a0, a1)
      double s = 0.0;
      for (int k = 0; k < N; ++k) s += sI[kq * N + k] * col[k];
      T0[a0 + N * a1 + NN * kq] = s;
    }
    __syncthreads();
    {  // along y at (x, z) = (a0, a1)
      const int c = a0 + NN * a1;
      double v[N];
      for (int j = 0; j < N; ++j) v[j] = T0[c + N * j];
      for (int jq = 0; jq < N; ++jq) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += sI[jq * N + j] * v[j];
        T0[c + N * jq] = s;
      }
    }
    __syncthreads();
    {  // along x at (y, z) = (a0, a1), weights, and back along x
      const int base = N * a0 + NN * a1;
      double r[N], wv[N];
      for (int i = 0; i < N; ++i) r[i] = T0[base + i];
      for (int iq = 0; iq < N; ++iq) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) s += sI[iq * N + i] * r[i];
        wv[iq] = s * We[base + iq];
      }
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int iq = 0; iq < N; ++iq) s += sI[iq * N + i] * wv[iq];
        T0[base + i] = s;
      }
    }
    __syncthreads();
    {  // back along y
      const int c = a0 + NN * a1;
      double v[N];
      for (int jq = 0; jq < N; ++jq) v[jq] = T0[c + N * jq];
      for (int j = 0; j < N; ++j) {
        double s = 0.0;
        for (int jq = 0; jq < N; ++jq) s += sI[jq * N + j] * v[jq];
        T0[c + N * j] = s;
      }
    }
    __syncthreads();
    {  // back along z
      const int c = a0 + N * a1;
      double v[N];
      for (int kq = 0; kq < N; ++kq) v[kq] = T0[c + NN * kq];
      for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (int kq = 0; kq < N; ++kq) s += sI[kq * N + k] * v[kq];
        F[e * NL + c + NN * k] = s;
      }
    }
  } else {
    const int a = t;
    double col[N];
    for (int j = 0; j < N; ++j) col[j] = f[(ex * P + a) + sy * (ey * P + j)];
    __syncthreads();
    for (int jq = 0; jq < N; ++jq) {  // along y at x = a
      double s = 0.0;
      for (int j = 0; j < N; ++j) s += sI[jq * N + j] * col[j];
      T0[a + N * jq] = s;
    }
    __syncthreads();
    {  // along x at y = a, weights, back along x
      const int base = N * a;
      double r[N], wv[N];
      for (int i = 0; i < N; ++i) r[i] = T0[base + i];
      for (int iq = 0; iq < N; ++iq) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) s += sI[iq * N + i] * r[i];
        wv[iq] = s * We[base + iq];
      }
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int iq = 0; iq < N; ++iq) s += sI[iq * N + i] * wv[iq];
        T0[base + i] = s;
      }
    }
    __syncthreads();
    {  // back along y
      double v[N];
      for (int jq = 0; jq < N; ++jq) v[jq] = T0[a + N * jq];
      for (int j = 0; j < N; ++j) {
        double s = 0.0;
        for (int jq = 0; jq < N; ++jq) s += sI[jq * N + j] * v[jq];
        F[e * NL + a + N * j] = s;
      }
    }
  }
}

template <int N, typename T>
void apply_gauss_n(const Level& L, int neumann, const void* x, void* F, hipStream_t s) {
  const T* G = std::is_same<T, double>::value ? (const T*)L.G64 : (const T*)L.G32;
  const T* Iq = std::is_same<T, double>::value ? (const T*)L.Iq64 : (const T*)L.Iq32;
  const T* Dq = std::is_same<T, double>::value ? (const T*)L.Dq64 : (const T*)L.Dq32;
  if (L.g.dim == 3) {
    constexpr int EPB = EpbG3<N>::v;
    const unsigned nb = (unsigned)((L.g.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_apply3d_gauss<N, T, EPB>), dim3(nb), dim3(EPB * N * N), 0, s,
                       (const T*)x, (T*)F, G, Iq, Dq, L.g, neumann);
  } else {
    constexpr int EPB = EpbG2<N>::v;
    const unsigned nb = (unsigned)((L.g.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_apply2d_gauss<N, T, EPB>), dim3(nb), dim3(EPB * N), 0, s,
                       (const T*)x, (T*)F, G, Iq, Dq, L.g, neumann);
  }
  GLLMG_HIP(hipGetLastError());
}

template <typename T>
void apply_gauss_t(const Level& L, int neumann, const void* x, void* F, hipStream_t s) {
  switch (L.n) {
#define GLLMG_CASE(NV) \
  case NV:             \
    return apply_gauss_n<NV, T>(L, neumann, x, F, s);
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
#undef GLLMG_CASE
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
}

template <int N>
void mass_gauss_n(const Level& L, const double* f, double* F, const double* wdetq, hipStream_t s) {
  if (L.g.dim == 3)
    hipLaunchKernelGGL((k_mass_gauss<N, 3>), dim3((unsigned)L.g.E), dim3(N * N), 0, s, f, F,
                       wdetq, L.Iq64, L.g);
  else
    hipLaunchKernelGGL((k_mass_gauss<N, 2>), dim3((unsigned)L.g.E), dim3(N), 0, s, f, F, wdetq,
                       L.Iq64, L.g);
  GLLMG_HIP(hipGetLastError());
}

}  // namespace

void launch_apply_gauss(const Level& L, int prec, int neumann, const void* x, const Epi& ep,
                        void* F, hipStream_t s) {
  if (prec == 0)
    apply_gauss_t<double>(L, neumann, x, F, s);
  else
    apply_gauss_t<float>(L, neumann, x, F, s);
  launch_gather_in(L, prec, F, x, neumann, ep, s);
}

void launch_gauss_points(const Level& L, const double* xn, double* xq, hipStream_t s) {
  hipLaunchKernelGGL(k_gauss_points, dim3(nblocks(L.npts)), dim3(kThreads), 0, s, L.g, L.n,
                     L.Iq64, xn, xq);
  GLLMG_HIP(hipGetLastError());
}

void launch_field_pts(int64_t npts, int dim, const double* pts, const FieldDev& f, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_field_pts, dim3(nblocks(npts)), dim3(kThreads), 0, s, npts, dim, pts, f, out);
  GLLMG_HIP(hipGetLastError());
}

void launch_geometry_gauss(const Level& L, const double* xn, const double* muq, double* G64,
                           float* G32, double* wdetq, int* flag, hipStream_t s) {
  if (L.g.dim == 3)
    hipLaunchKernelGGL(k_geometry_gauss<3>, dim3(nblocks(L.npts)), dim3(kThreads), 0, s, L.g,
                       L.n, L.wg64, L.Iq64, L.Dq64, xn, muq, G64, G32, wdetq, flag);
  else
    hipLaunchKernelGGL(k_geometry_gauss<2>, dim3(nblocks(L.npts)), dim3(kThreads), 0, s, L.g,
                       L.n, L.wg64, L.Iq64, L.Dq64, xn, muq, G64, G32, wdetq, flag);
  GLLMG_HIP(hipGetLastError());
}

void launch_diag_gauss(const Level& L, double* diag, double* F, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_gauss, dim3(nblocks(L.npts)), dim3(kThreads), 0, s, L.G64, L.Iq64,
                     L.Dq64, L.g, F);
  GLLMG_HIP(hipGetLastError());
  launch_gather_full(L, F, diag, s);
}

void launch_mass_gauss(const Level& L, const double* f, const double* wdetq, double* F,
                       hipStream_t s) {
  switch (L.n) {
#define GLLMG_CASE(NV) \
  case NV:             \
    return mass_gauss_n<NV>(L, f, F, wdetq, s);
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
#undef GLLMG_CASE
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
}

}  // namespace gllmg
