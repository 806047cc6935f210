// Matrix-free sum-factorized operator y = A x (paper §2.3: tensorized O(p^4) matvec) and the
// operator diagonal (§3.2.1), for GLL quads and hexes of order 1..16.
//
// Per element e and GLL point q (collocated quadrature):
//   u_b(q) = sum_l D[q_b, l] x_e(q with coordinate b -> l)          (d forward contractions)
//   w_a(q) = sum_b G_ab(q) u_b(q)                                    (pointwise, G symmetric)
//   y_e(i) = sum_a sum_m D[m, i_a] w_a(i with coordinate a -> m)     (d transposed contractions)
// and y = sum_e Q_e^T y_e. The sum over elements is deterministic and atomic-free: a node in
// the interior of an element has exactly one contribution, written directly; contributions
// to nodes on element faces/edges/vertices go to a face buffer (compact per-element slots)
// and a second kernel adds, for every such node, the 2, 4 or 8 slots in a fixed order.
// Dirichlet data: boundary entries of x are read as 0 and boundary entries of y are set to 0.
#include "internal.h"

namespace gllmg {

namespace {

// Compact slot of an element-boundary local node (i, j, k) of an n^3 element: the k = 0
// plane (n^2), then for each 0 < k < n-1 the ring of the (i, j) plane (4(n-1)), then the
// k = n-1 plane. 2D uses the ring alone.
__host__ __device__ inline int slot_ring(int n, int i, int j) {
  if (j == 0) return i;
  if (j == n - 1) return n + 2 * (n - 2) + i;
  return n + 2 * (j - 1) + (i == 0 ? 0 : 1);
}
__host__ __device__ inline int slot3(int n, int i, int j, int k) {
  const int R = 4 * (n - 1);
  if (k == 0) return j * n + i;
  if (k == n - 1) return n * n + (n - 2) * R + j * n + i;
  return n * n + (k - 1) * R + slot_ring(n, i, j);
}
__host__ __device__ inline int nbnd(int n, int dim) {
  return dim == 3 ? n * n * n - (n - 2) * (n - 2) * (n - 2) : n * n - (n - 2) * (n - 2);
}

// Elements per workgroup so that a workgroup has about 256 threads (n^2 threads per element).
template <int N>
struct Epb {
  static constexpr int v = (N * N >= 128) ? 1 : (256 / (N * N));
};

// ------------------------------------------------------------------ 3D element kernel
template <int N, typename T, int EPB>
__global__ void __launch_bounds__(EPB * N * N)
k_apply3d(const T* __restrict__ x, T* __restrict__ y, T* __restrict__ F,
          const T* __restrict__ G, const T* __restrict__ Dm, Grid g, int neumann) {
  constexpr int NN = N * N, NNN = N * N * N, P = N - 1;
  constexpr int NB = NNN - (N - 2) * (N - 2) * (N - 2);
  __shared__ T sA[EPB * NNN];
  __shared__ T sB[EPB * NNN];
  const int t = threadIdx.x;
  const int le = t / NN;
  const int ij = t - le * NN;
  const int i = ij % N, j = ij / N;
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  const bool valid = e < g.E;
  const int64_t ee = valid ? e : 0;
  const int ex = (int)(ee % g.ne[0]);
  const int ey = (int)((ee / g.ne[0]) % g.ne[1]);
  const int ez = (int)(ee / ((int64_t)g.ne[0] * g.ne[1]));
  const int gx = ex * P + i, gy = ey * P + j;
  const bool bxy = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1;
  const int64_t sxy = (int64_t)g.nn[0] * g.nn[1];
  const int64_t gb = gx + (int64_t)g.nn[0] * gy + sxy * (int64_t)(ez * P);
  T* A = sA + le * NNN;
  T* B = sB + le * NNN;

  T xr[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int gz = ez * P + k;
    const bool bnd = bxy || gz == 0 || gz == g.nn[2] - 1;
    T v = T(0);
    if (valid && (neumann || !bnd)) v = x[gb + sxy * k];
    xr[k] = v;
    A[k * NN + ij] = v;
  }
  T Di[N], Dj[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    Di[l] = Dm[i * N + l];
    Dj[l] = Dm[j * N + l];
  }
  __syncthreads();

  T wx[N], wy[N], wz[N];
  const T* Ge = G + ee * (6 * NNN) + ij;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T ux = T(0), uy = T(0), uz = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      ux += Di[l] * A[k * NN + j * N + l];
      uy += Dj[l] * A[k * NN + l * N + i];
      uz += Dm[k * N + l] * xr[l];
    }
    const T g0 = Ge[0 * NNN + k * NN], g1 = Ge[1 * NNN + k * NN], g2 = Ge[2 * NNN + k * NN];
    const T g3 = Ge[3 * NNN + k * NN], g4 = Ge[4 * NNN + k * NN], g5 = Ge[5 * NNN + k * NN];
    wx[k] = g0 * ux + g1 * uy + g2 * uz;
    wy[k] = g1 * ux + g3 * uy + g4 * uz;
    wz[k] = g2 * ux + g4 * uy + g5 * uz;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    A[k * NN + ij] = wx[k];
    B[k * NN + ij] = wy[k];
  }
  T DiT[N], DjT[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    DiT[l] = Dm[l * N + i];
    DjT[l] = Dm[l * N + j];
  }
  __syncthreads();
  if (!valid) return;
  const bool inner_ij = i > 0 && i < N - 1 && j > 0 && j < N - 1;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      acc += DiT[l] * A[k * NN + j * N + l];
      acc += DjT[l] * B[k * NN + l * N + i];
      acc += Dm[l * N + k] * wz[l];
    }
    if (inner_ij && k > 0 && k < N - 1)
      y[gb + sxy * k] = acc;
    else
      F[e * NB + slot3(N, i, j, k)] = acc;
  }
}

// ------------------------------------------------------------------ 2D element kernel
template <int N, typename T, int EPB>
__global__ void __launch_bounds__(EPB * N * N)
k_apply2d(const T* __restrict__ x, T* __restrict__ y, T* __restrict__ F,
          const T* __restrict__ G, const T* __restrict__ Dm, Grid g, int neumann) {
  constexpr int NN = N * N, P = N - 1;
  constexpr int NB = 4 * (N - 1);
  __shared__ T sA[EPB * NN];
  __shared__ T sB[EPB * NN];
  const int t = threadIdx.x;
  const int le = t / NN;
  const int ij = t - le * NN;
  const int i = ij % N, j = ij / N;
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  const bool valid = e < g.E;
  const int64_t ee = valid ? e : 0;
  const int ex = (int)(ee % g.ne[0]);
  const int ey = (int)(ee / g.ne[0]);
  const int gx = ex * P + i, gy = ey * P + j;
  const bool bnd = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1;
  const int64_t gi = gx + (int64_t)g.nn[0] * gy;
  T* A = sA + le * NN;
  T* B = sB + le * NN;
  T xv = T(0);
  if (valid && (neumann || !bnd)) xv = x[gi];
  A[ij] = xv;
  __syncthreads();
  T ux = T(0), uy = T(0);
#pragma unroll
  for (int l = 0; l < N; ++l) {
    ux += Dm[i * N + l] * A[j * N + l];
    uy += Dm[j * N + l] * A[l * N + i];
  }
  const T* Ge = G + ee * (3 * NN) + ij;
  const T g0 = Ge[0], g1 = Ge[NN], g2 = Ge[2 * NN];
  const T wx = g0 * ux + g1 * uy;
  const T wy = g1 * ux + g2 * uy;
  __syncthreads();
  A[ij] = wx;
  B[ij] = wy;
  __syncthreads();
  if (!valid) return;
  T acc = T(0);
#pragma unroll
  for (int l = 0; l < N; ++l) {
    acc += Dm[l * N + i] * A[j * N + l];
    acc += Dm[l * N + j] * B[l * N + i];
  }
  if (i > 0 && i < N - 1 && j > 0 && j < N - 1)
    y[gi] = acc;
  else
    F[e * NB + slot_ring(N, i, j)] = acc;
}

// ------------------------------------------------------------------ face sums
// For every node on an element boundary: y[g] = sum of the face-buffer slots of the
// elements containing it (lower element first along each axis, z outermost); 0 on the
// domain boundary unless neumann.
template <typename T>
__global__ void __launch_bounds__(256)
k_facesum(const T* __restrict__ F, T* __restrict__ y, Grid g, int neumann) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  const int p = g.p, n = p + 1, dim = g.dim;
  int gc[3];
  gc[0] = (int)(t % g.nn[0]);
  gc[1] = (int)((t / g.nn[0]) % g.nn[1]);
  gc[2] = (dim == 3) ? (int)(t / ((int64_t)g.nn[0] * g.nn[1])) : 0;
  const int rx = gc[0] % p, ry = gc[1] % p, rz = (dim == 3) ? gc[2] % p : 1;
  if (rx != 0 && ry != 0 && rz != 0) return;  // element-interior node: written by the element kernel
  bool bnd = gc[0] == 0 || gc[0] == g.nn[0] - 1 || gc[1] == 0 || gc[1] == g.nn[1] - 1;
  if (dim == 3) bnd = bnd || gc[2] == 0 || gc[2] == g.nn[2] - 1;
  if (bnd && !neumann) {
    y[t] = T(0);
    return;
  }
  int ce[3][2], cl[3][2], cnt[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= dim) {
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
  const int NB = nbnd(n, dim);
  T acc = T(0);
  for (int kz = 0; kz < cnt[2]; ++kz)
    for (int ky = 0; ky < cnt[1]; ++ky)
      for (int kx = 0; kx < cnt[0]; ++kx) {
        const int64_t e = ce[0][kx] + (int64_t)g.ne[0] * (ce[1][ky] + (int64_t)g.ne[1] * ce[2][kz]);
        const int s = (dim == 3) ? slot3(n, cl[0][kx], cl[1][ky], cl[2][kz])
                                 : slot_ring(n, cl[0][kx], cl[1][ky]);
        acc += F[e * NB + s];
      }
  y[t] = acc;
}

// ------------------------------------------------------------------ diagonal
// diag_e(i) = sum_a sum_m D[m, i_a]^2 G_aa(i with a -> m) + sum_{a != b} D[i_a, i_a] D[i_b, i_b] G_ab(i)
// (the cross terms survive only where both D diagonal entries are nonzero: the element's
// boundary nodes). One thread per element point; FP64.
__global__ void __launch_bounds__(256)
k_diag(const double* __restrict__ G, const double* __restrict__ Dm, Grid g, double* __restrict__ y,
       double* __restrict__ F) {
  const int n = g.p + 1, dim = g.dim;
  const int nloc = dim == 3 ? n * n * n : n * n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.E * nloc) return;
  const int64_t e = t / nloc;
  const int q = (int)(t - e * nloc);
  int qc[3] = {q % n, (q / n) % n, dim == 3 ? q / (n * n) : 0};
  const int ncomp = dim == 3 ? 6 : 3;
  const double* Ge = G + e * (int64_t)ncomp * nloc;
  // component index of G_ab (a <= b) in the packed order 00 01 (02) 11 (12) (22)
  auto comp = [&](int a, int b) {
    if (dim == 2) return a == 0 ? (b == 0 ? 0 : 1) : 2;
    if (a == 0) return b;               // 00 01 02
    if (a == 1) return b == 1 ? 3 : 4;  // 11 12
    return 5;                           // 22
  };
  const int stride[3] = {1, n, n * n};
  double d = 0.0;
  for (int a = 0; a < dim; ++a) {
    const int ca = comp(a, a);
    for (int m = 0; m < n; ++m) {
      const double dm = Dm[m * n + qc[a]];
      const int qq = q + (m - qc[a]) * stride[a];
      d += dm * dm * Ge[(int64_t)ca * nloc + qq];
    }
  }
  for (int a = 0; a < dim; ++a)
    for (int b = a + 1; b < dim; ++b)
      d += 2.0 * Dm[qc[a] * n + qc[a]] * Dm[qc[b] * n + qc[b]] * Ge[(int64_t)comp(a, b) * nloc + q];
  const int ex = (int)(e % g.ne[0]);
  const int ey = (int)((e / g.ne[0]) % g.ne[1]);
  const int ez = dim == 3 ? (int)(e / ((int64_t)g.ne[0] * g.ne[1])) : 0;
  bool inner = qc[0] > 0 && qc[0] < n - 1 && qc[1] > 0 && qc[1] < n - 1;
  if (dim == 3) inner = inner && qc[2] > 0 && qc[2] < n - 1;
  if (inner) {
    const int64_t gi = (ex * g.p + qc[0]) + (int64_t)g.nn[0] *
                       ((ey * g.p + qc[1]) + (int64_t)g.nn[1] * (ez * g.p + qc[2]));
    y[gi] = d;
  } else {
    const int s = dim == 3 ? slot3(n, qc[0], qc[1], qc[2]) : slot_ring(n, qc[0], qc[1]);
    F[e * nbnd(n, dim) + s] = d;
  }
}

template <int N, typename T>
void apply_n(const Level& L, int neumann, const void* x, void* y, void* F, hipStream_t s) {
  const T* G = std::is_same<T, double>::value ? (const T*)L.G64 : (const T*)L.G32;
  const T* D = std::is_same<T, double>::value ? (const T*)L.D64 : (const T*)L.D32;
  constexpr int EPB = Epb<N>::v;
  const unsigned nb = (unsigned)((L.g.E + EPB - 1) / EPB);
  if (L.g.dim == 3)
    hipLaunchKernelGGL((k_apply3d<N, T, EPB>), dim3(nb), dim3(EPB * N * N), 0, s, (const T*)x,
                       (T*)y, (T*)F, G, D, L.g, neumann);
  else
    hipLaunchKernelGGL((k_apply2d<N, T, EPB>), dim3(nb), dim3(EPB * N * N), 0, s, (const T*)x,
                       (T*)y, (T*)F, G, D, L.g, neumann);
  GLLMG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_facesum<T>, dim3((unsigned)((L.g.N + 255) / 256)), dim3(256), 0, s,
                     (const T*)F, (T*)y, L.g, neumann);
  GLLMG_HIP(hipGetLastError());
}

template <typename T>
void apply_t(const Level& L, int neumann, const void* x, void* y, void* F, hipStream_t s) {
  switch (L.n) {
#define GLLMG_CASE(NV) \
  case NV:             \
    return apply_n<NV, T>(L, neumann, x, y, F, s);
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
#undef GLLMG_CASE
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
}

}  // namespace

size_t face_buffer_elems(const Level& L) { return (size_t)L.g.E * nbnd(L.n, L.g.dim); }

void launch_apply(const Level& L, int prec, int neumann, const void* x, void* y, void* F,
                  hipStream_t s) {
  if (prec == 0)
    apply_t<double>(L, neumann, x, y, F, s);
  else
    apply_t<float>(L, neumann, x, y, F, s);
}

void launch_diag(const Level& L, double* diag, double* F, hipStream_t s) {
  const int64_t tot = L.npts;
  hipLaunchKernelGGL(k_diag, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L.G64, L.D64,
                     L.g, diag, F);
  GLLMG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_facesum<double>, dim3((unsigned)((L.g.N + 255) / 256)), dim3(256), 0, s,
                     (const double*)F, diag, L.g, 0);
  GLLMG_HIP(hipGetLastError());
}

}  // namespace gllmg
