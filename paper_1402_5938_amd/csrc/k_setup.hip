// Setup kernels: isoparametric geometry at the GLL points, lumped mass, field evaluation at
// the nodes, load vector, inverse diagonal and the Lanczos start vector.
#include "fields.h"
#include "internal.h"

namespace gllmg {

namespace {

constexpr int kThreads = 256;

inline unsigned nblocks(int64_t n, int t = kThreads) { return (unsigned)((n + t - 1) / t); }

// Geometry at one GLL point q of element e (paper §2.3): J_ab = d x_a / d xi_b of the degree-p
// interpolant of Phi through the element's nodes, sum_l D[q_b, l] x_a(node q with b -> l), from
// the physical coordinates xn of the level's nodes (N x dim); G = w_q mu_q detJ J^{-1} J^{-T}
// with mu_q = mun at the node (collocated quadrature: the points are the nodes); also w_q detJ.
template <int DIM>
__global__ void __launch_bounds__(kThreads)
k_geometry(Grid g, int n, const double* __restrict__ w, const double* __restrict__ D,
           const double* __restrict__ xn, const double* __restrict__ mun,
           double* __restrict__ G64, float* __restrict__ G32, double* __restrict__ wdet,
           int* __restrict__ flag) {
  int nloc = n * n;
  if (DIM == 3) nloc *= n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.E * nloc) return;
  const int64_t e = t / nloc;
  const int q = (int)(t - e * nloc);
  int ec[3], qc[3];
  ec[0] = (int)(e % g.ne[0]);
  ec[1] = (int)((e / g.ne[0]) % g.ne[1]);
  ec[2] = (DIM == 3) ? (int)(e / ((int64_t)g.ne[0] * g.ne[1])) : 0;
  qc[0] = q % n;
  qc[1] = (q / n) % n;
  qc[2] = (DIM == 3) ? q / (n * n) : 0;
  const int64_t st[3] = {1, g.nn[0], (int64_t)g.nn[0] * g.nn[1]};
  int64_t node = 0;  // global index of the point's node
  for (int a = 0; a < DIM; ++a) node += (int64_t)(ec[a] * (n - 1) + qc[a]) * st[a];
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int b = 0; b < DIM; ++b) {
    for (int l = 0; l < n; ++l) {
      const int64_t nb = node + (int64_t)(l - qc[b]) * st[b];
      const double dq = D[qc[b] * n + l];
      for (int a = 0; a < DIM; ++a) J[a][b] += dq * xn[nb * DIM + a];
    }
  }
  double wq = w[qc[0]] * w[qc[1]];
  if (DIM == 3) wq *= w[qc[2]];
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
  const double m = mun[node];
  if (!(m > 0.0) || !isfinite(m)) atomicOr(flag, 2);
  const double sc = wq * m * det;
  const int ncomp = (DIM == 3) ? 6 : 3;
  double Gv[6];
  int c = 0;
  for (int a = 0; a < DIM; ++a)
    for (int b = a; b < DIM; ++b) {
      double s = 0.0;
      for (int k = 0; k < DIM; ++k) s += I[a][k] * I[b][k];
      Gv[c++] = sc * s;
    }
  const int64_t base = e * (int64_t)ncomp * nloc + q;
  for (int k = 0; k < ncomp; ++k) {
    if (G64) G64[base + (int64_t)k * nloc] = Gv[k];
    if (G32) G32[base + (int64_t)k * nloc] = (float)Gv[k];
  }
  if (wdet) wdet[t] = wq * det;
}

// out[g] = sum over the elements containing node g of elem_vals[e][local index of g].
__global__ void k_gather_full(Grid g, int n, const double* __restrict__ ev, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  const int p = g.p;
  int gc[3];
  gc[0] = (int)(t % g.nn[0]);
  gc[1] = (int)((t / g.nn[0]) % g.nn[1]);
  gc[2] = (int)(t / ((int64_t)g.nn[0] * g.nn[1]));
  int ce[3][2], cl[3][2], cnt[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= g.dim) {
      cnt[a] = 1;
      ce[a][0] = 0;
      cl[a][0] = 0;
      continue;
    }
    const int r = gc[a] % p, e = gc[a] / p;
    if (r != 0) {
      cnt[a] = 1;
      ce[a][0] = e;
      cl[a][0] = r;
    } else {
      cnt[a] = 0;
      if (e > 0) { ce[a][cnt[a]] = e - 1; cl[a][cnt[a]] = p; ++cnt[a]; }
      if (e < g.ne[a]) { ce[a][cnt[a]] = e; cl[a][cnt[a]] = 0; ++cnt[a]; }
    }
  }
  const int nloc = (g.dim == 3) ? n * n * n : n * n;
  double acc = 0.0;
  for (int kz = 0; kz < cnt[2]; ++kz)
    for (int ky = 0; ky < cnt[1]; ++ky)
      for (int kx = 0; kx < cnt[0]; ++kx) {
        const int64_t e = ce[0][kx] + (int64_t)g.ne[0] * (ce[1][ky] + (int64_t)g.ne[1] * ce[2][kz]);
        const int l = cl[0][kx] + n * (cl[1][ky] + n * cl[2][kz]);
        acc += ev[e * nloc + l];
      }
  out[t] = acc;
}

__device__ inline void node_ref(const Grid& g, const double* xi, int64_t t, double* X, bool* bnd) {
  int gc[3];
  gc[0] = (int)(t % g.nn[0]);
  gc[1] = (int)((t / g.nn[0]) % g.nn[1]);
  gc[2] = (int)(t / ((int64_t)g.nn[0] * g.nn[1]));
  bool b = false;
  for (int a = 0; a < g.dim; ++a) {
    X[a] = ref_coord_global(gc[a], g.p, g.ne[a], xi);
    b = b || gc[a] == 0 || gc[a] == g.nn[a] - 1;
  }
  *bnd = b;
}

__global__ void k_node_coords(Grid g, const double* __restrict__ xi, FieldDev map, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  double X[3], x[3];
  bool bnd;
  node_ref(g, xi, t, X, &bnd);
  map_eval(map, g.dim, X, x);
  for (int a = 0; a < g.dim; ++a) out[t * g.dim + a] = x[a];
}

__global__ void k_eval_field(Grid g, const double* __restrict__ xi, FieldDev map, FieldDev f,
                             double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  double X[3], x[3];
  bool bnd;
  node_ref(g, xi, t, X, &bnd);
  map_eval(map, g.dim, X, x);
  out[t] = field_eval(f, g.dim, x);
}

// Nodal coordinates and mu of a coarser grid whose node (i, j, k) is node (s i, s j, s k) of the
// grid g0.
__global__ void k_subsample_nodal(Grid g0, Grid g, int stride, const double* __restrict__ xn0,
                                  const double* __restrict__ mu0, double* __restrict__ xn,
                                  double* __restrict__ mu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  const int64_t gc[3] = {t % g.nn[0], (t / g.nn[0]) % g.nn[1], t / ((int64_t)g.nn[0] * g.nn[1])};
  const int64_t src = gc[0] * stride + (int64_t)g0.nn[0] * (gc[1] * stride +
                                                            (int64_t)g0.nn[1] * gc[2] * stride);
  for (int a = 0; a < g.dim; ++a) xn[t * g.dim + a] = xn0[src * g.dim + a];
  mu[t] = mu0[src];
}

// A field at given physical node coordinates xn (N x dim).
__global__ void k_field_at(Grid g, const double* __restrict__ xn, FieldDev f, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  double x[3] = {0, 0, 0};
  for (int a = 0; a < g.dim; ++a) x[a] = xn[t * g.dim + a];
  out[t] = field_eval(f, g.dim, x);
}

__device__ inline bool on_boundary(const Grid& g, int64_t t) {
  const int gx = (int)(t % g.nn[0]);
  const int gy = (int)((t / g.nn[0]) % g.nn[1]);
  bool b = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1;
  if (g.dim == 3) {
    const int gz = (int)(t / ((int64_t)g.nn[0] * g.nn[1]));
    b = b || gz == 0 || gz == g.nn[2] - 1;
  }
  return b;
}

__global__ void k_rhs(Grid g, const double* __restrict__ mass, const double* __restrict__ f,
                      double* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  b[t] = on_boundary(g, t) ? 0.0 : mass[t] * f[t];
}

__global__ void k_dinv(Grid g, const double* __restrict__ diag, double* __restrict__ d64,
                       float* __restrict__ d32, int* __restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  double v = 0.0;
  if (!on_boundary(g, t)) {
    const double dg = diag[t];
    if (!(dg > 0.0) || !isfinite(dg)) atomicOr(flag, 4);
    v = 1.0 / dg;
  }
  d64[t] = v;
  if (d32) d32[t] = (float)v;
}

// SplitMix64 (Steele, Lea and Flood 2014) of the key seed ^ g ^ (level << 32), mapped to
// [0, 1) as (h >> 11) 2^-53, minus 1/2; zero on the boundary.
__global__ void k_start_vector(Grid g, uint64_t seed, int level, double* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  if (on_boundary(g, t)) {
    v[t] = 0.0;
    return;
  }
  uint64_t z = (seed ^ (uint64_t)t ^ ((uint64_t)level << 32)) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  v[t] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

// e = the sum of the unit vectors of the interior nodes whose interior indices (g_a - 1) are
// o_a mod c along every axis (one color of the coarse operator's assembly)
__global__ void k_color_unit(Grid g, int c, int ox, int oy, int oz, double* e) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  const int64_t nx = g.nn[0], ny = g.nn[1];
  const int gx = (int)(t % nx);
  const int64_t r = t / nx;
  const int gy = (int)(r % ny);
  const int gz = g.dim == 3 ? (int)(r / ny) : 0;
  bool hit = gx >= 1 && gx <= nx - 2 && gy >= 1 && gy <= ny - 2 && (gx - 1) % c == ox &&
             (gy - 1) % c == oy;
  if (g.dim == 3) hit = hit && gz >= 1 && gz <= g.nn[2] - 2 && (gz - 1) % c == oz;
  e[t] = hit ? 1.0 : 0.0;
}

}  // namespace

void launch_geometry(const Level& L, const double* xn, const double* mun, double* G64,
                     float* G32, double* wdet, int* flag, hipStream_t s) {
  const int64_t tot = L.npts;
  if (L.g.dim == 2)
    hipLaunchKernelGGL(k_geometry<2>, dim3(nblocks(tot)), dim3(kThreads), 0, s, L.g, L.n, L.w64,
                       L.D64, xn, mun, G64, G32, wdet, flag);
  else
    hipLaunchKernelGGL(k_geometry<3>, dim3(nblocks(tot)), dim3(kThreads), 0, s, L.g, L.n, L.w64,
                       L.D64, xn, mun, G64, G32, wdet, flag);
  GLLMG_HIP(hipGetLastError());
}

void launch_subsample_nodal(const Grid& g0, const Grid& g, int stride, const double* xn0,
                            const double* mu0, double* xn, double* mu, hipStream_t s) {
  hipLaunchKernelGGL(k_subsample_nodal, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g0, g, stride, xn0,
                     mu0, xn, mu);
  GLLMG_HIP(hipGetLastError());
}

void launch_field_at(const Grid& g, const double* xn, const FieldDev& f, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_field_at, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g, xn, f, out);
  GLLMG_HIP(hipGetLastError());
}

void launch_gather_full(const Level& L, const double* ev, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_full, dim3(nblocks(L.g.N)), dim3(kThreads), 0, s, L.g, L.n, ev, out);
  GLLMG_HIP(hipGetLastError());
}

void launch_node_coords(const Grid& g, const double* xi, const FieldDev& map, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_node_coords, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g, xi, map, out);
  GLLMG_HIP(hipGetLastError());
}

void launch_eval_field(const Grid& g, const double* xi, const FieldDev& map, const FieldDev& f,
                       double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_eval_field, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g, xi, map, f, out);
  GLLMG_HIP(hipGetLastError());
}

void launch_rhs(const Grid& g, const double* mass, const double* f, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g, mass, f, b);
  GLLMG_HIP(hipGetLastError());
}

void launch_dinv(const Grid& g, const double* diag, double* d64, float* d32, int* flag,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_dinv, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g, diag, d64, d32, flag);
  GLLMG_HIP(hipGetLastError());
}

void start_vector(const Grid& g, uint64_t seed, int level, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_start_vector, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g, seed, level, v);
  GLLMG_HIP(hipGetLastError());
}

void color_unit_vector(const Grid& g, int c, int ox, int oy, int oz, double* e, hipStream_t s) {
  hipLaunchKernelGGL(k_color_unit, dim3(nblocks(g.N)), dim3(kThreads), 0, s, g, c, ox, oy, oz, e);
  GLLMG_HIP(hipGetLastError());
}

}  // namespace gllmg
