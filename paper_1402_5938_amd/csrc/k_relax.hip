// Multicolor Gauss-Seidel passes of the SSOR smoother (paper §3.2.1, §4.3 "SSOR(2,1)").
//
// Coloring: n^2 colors, n = p + 1. A node with global grid indices (gx, gy[, gz]) has color
//   2D: (gx mod n) + n (gy mod n)            3D: ((gx + gz) mod n) + n ((gy + gz) mod n).
// Under collocated GLL quadrature the stiffness couples two nodes only if an element holds
// both and, in 3D, they share a grid coordinate (the B_a^T G_ab B_b terms reach along the
// coordinate lines and planes through a node); within one element distinct indices along an
// axis have distinct residues mod n, so nodes of one color never couple. One launch updates
// every interior node of one color,
//   x_i <- x_i + omega dinv_i (b_i - (A x)_i),
// each node's row (A x)_i formed matrix-free from the elements around it by a group of lanes.
// A row reads only nodes of other colors (and its own), so the threads of a launch never read
// what another writes: a whole color at once is the node-by-node Gauss-Seidel update. A forward
// sweep launches colors 0..C-1, a backward sweep C-1..0.
//
// The row of element e at its local node (i, j, k): with q running along the coordinate line
// of axis a through the node,
//   (A_e x)(i,j,k) = sum_a sum_m D[m, i_a] w_a(q_m),   w_a = sum_b G_ab u_b,
//   u_b(q) = sum_l D[q_b, l] x(q with coordinate b -> l),
// so a row needs x on the three coordinate planes through the node (3D; the whole element in
// 2D) and G on the three lines: 9 n^2 + O(n) multiply-adds per element in 3D. The elements
// around a node are summed lower element first per axis, z outermost. x must be 0 at boundary
// nodes (the smoother clears them first); boundary rows are not updated.
#include <cstdint>

#include "internal.h"

namespace gllmg {

namespace {

constexpr int kGsT = 256;

// Lanes per node: lane m of a node's group evaluates the terms at position m (and m + LPN, ...)
// along the coordinate lines through the node; the group then sums its lanes.
template <int N>
struct Lpn {
  static constexpr int v = N <= 4 ? 4 : (N <= 8 ? 8 : 16);
};

// The terms of position m of element e's row at its local node (i, j, k): for each axis a the
// point q on the a-line through the node with q_a = m,
//   D[m, i_a] (G_a0 u_0(q) + G_a1 u_1(q) + G_a2 u_2(q)),  u_b(q) = sum_l D[q_b, l] x(q, b -> l).
template <int N, typename T>
__device__ __forceinline__ T terms3d(const T* __restrict__ x, const T* __restrict__ Ge,
                                     const T* __restrict__ sD, int64_t base, int64_t sy,
                                     int64_t sz, int i, int j, int k, int m) {
  constexpr int NN = N * N, NNN = N * N * N;
  auto X = [&](int a, int b, int c) { return x[base + a + sy * b + sz * c]; };
  T acc = T(0);
  {  // a = 0: q = (m, j, k)
    T u0 = T(0), u1 = T(0), u2 = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      u0 += sD[m * N + l] * X(l, j, k);
      u1 += sD[j * N + l] * X(m, l, k);
      u2 += sD[k * N + l] * X(m, j, l);
    }
    const int q = m + N * j + NN * k;
    acc += sD[m * N + i] * (Ge[q] * u0 + Ge[NNN + q] * u1 + Ge[2 * NNN + q] * u2);
  }
  {  // a = 1: q = (i, m, k)
    T u0 = T(0), u1 = T(0), u2 = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      u0 += sD[i * N + l] * X(l, m, k);
      u1 += sD[m * N + l] * X(i, l, k);
      u2 += sD[k * N + l] * X(i, m, l);
    }
    const int q = i + N * m + NN * k;
    acc += sD[m * N + j] * (Ge[NNN + q] * u0 + Ge[3 * NNN + q] * u1 + Ge[4 * NNN + q] * u2);
  }
  {  // a = 2: q = (i, j, m)
    T u0 = T(0), u1 = T(0), u2 = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      u0 += sD[i * N + l] * X(l, j, m);
      u1 += sD[j * N + l] * X(i, l, m);
      u2 += sD[m * N + l] * X(i, j, l);
    }
    const int q = i + N * j + NN * m;
    acc += sD[m * N + k] * (Ge[2 * NNN + q] * u0 + Ge[4 * NNN + q] * u1 + Ge[5 * NNN + q] * u2);
  }
  return acc;
}

template <int N, typename T>
__device__ __forceinline__ T terms2d(const T* __restrict__ x, const T* __restrict__ Ge,
                                     const T* __restrict__ sD, int64_t base, int64_t sy, int i,
                                     int j, int m) {
  constexpr int NN = N * N;
  auto X = [&](int a, int b) { return x[base + a + sy * b]; };
  T acc = T(0);
  {  // a = 0: q = (m, j)
    T u0 = T(0), u1 = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      u0 += sD[m * N + l] * X(l, j);
      u1 += sD[j * N + l] * X(m, l);
    }
    const int q = m + N * j;
    acc += sD[m * N + i] * (Ge[q] * u0 + Ge[NN + q] * u1);
  }
  {  // a = 1: q = (i, m)
    T u0 = T(0), u1 = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      u0 += sD[i * N + l] * X(l, m);
      u1 += sD[m * N + l] * X(i, l);
    }
    const int q = i + N * m;
    acc += sD[m * N + j] * (Ge[NN + q] * u0 + Ge[2 * NN + q] * u1);
  }
  return acc;
}

// The elements around an interior grid index gi along an axis: the one below first.
// Returns the count (1 or 2); e[0], loc[0] and e[1], loc[1].
__device__ __forceinline__ int axis_elems(int gi, int p, int* e, int* loc) {
  if (gi % p == 0) {
    e[0] = gi / p - 1;
    loc[0] = p;
    e[1] = gi / p;
    loc[1] = 0;
    return 2;
  }
  e[0] = gi / p;
  loc[0] = gi - e[0] * p;
  return 1;
}

// One color of a Gauss-Seidel sweep. Lane group t / LPN -> node (kx, ky, gz) (2D: gz = 0): the
// node is (ox + n kx, oy + n ky, gz) with ox, oy the color's residues, shifted by gz in 3D.
// Each lane sums its positions over the elements around the node (lower element first per
// axis, z outermost); the group adds its lanes by an xor butterfly (the same sum in every lane)
// and its first lane writes the update.
template <int N, int DIM, typename T>
__global__ void __launch_bounds__(kGsT)
k_gs_color(T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ dinv,
           const T* __restrict__ G, const T* __restrict__ Dm, Grid g, int ca, int cb, int cx,
           int cy, T omega) {
  constexpr int LPN = Lpn<N>::v;
  __shared__ T sD[N * N];
  for (int q = threadIdx.x; q < N * N; q += blockDim.x) sD[q] = Dm[q];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kGsT + threadIdx.x;
  const int lane = (int)(t % LPN);
  const int64_t nid = t / LPN;
  const int64_t per = (int64_t)cx * cy;
  bool ok = nid < per * g.nn[2];
  const int gz = ok ? (int)(nid / per) : 0;
  const int rem = ok ? (int)(nid - (int64_t)gz * per) : 0;
  const int ky = rem / cx, kx = rem - ky * cx;
  const int ox = DIM == 3 ? ((ca - gz) % N + N) % N : ca;
  const int oy = DIM == 3 ? ((cb - gz) % N + N) % N : cb;
  const int gx = ox + kx * N, gy = oy + ky * N;
  ok = ok && gx > 0 && gx < g.nn[0] - 1 && gy > 0 && gy < g.nn[1] - 1;
  if (DIM == 3) ok = ok && gz > 0 && gz < g.nn[2] - 1;
  const int p = N - 1;
  const int64_t sy = g.nn[0], sz = (int64_t)g.nn[0] * g.nn[1];
  T acc = T(0);
  if (ok) {
    int exs[2], lxs[2], eys[2], lys[2], ezs[2] = {0, 0}, lzs[2] = {0, 0};
    const int nx = axis_elems(gx, p, exs, lxs);
    const int ny = axis_elems(gy, p, eys, lys);
    const int nz = DIM == 3 ? axis_elems(gz, p, ezs, lzs) : 1;
    constexpr int NLOC = DIM == 3 ? N * N * N : N * N;
    constexpr int NC = DIM == 3 ? 6 : 3;
    for (int c = 0; c < nz; ++c)
      for (int bb = 0; bb < ny; ++bb)
        for (int a = 0; a < nx; ++a) {
          const int ex = exs[a], ey = eys[bb], ez = ezs[c];
          const int64_t e = ex + (int64_t)g.ne[0] * (ey + (int64_t)g.ne[1] * ez);
          const int64_t base = (int64_t)ex * p + sy * ((int64_t)ey * p) + sz * ((int64_t)ez * p);
          const T* Ge = G + e * (NC * NLOC);
          for (int m = lane; m < N; m += LPN) {
            if constexpr (DIM == 3)
              acc += terms3d<N, T>(x, Ge, sD, base, sy, sz, lxs[a], lys[bb], lzs[c], m);
            else
              acc += terms2d<N, T>(x, Ge, sD, base, sy, lxs[a], lys[bb], m);
          }
        }
  }
#pragma unroll
  for (int off = LPN / 2; off >= 1; off /= 2) acc += __shfl_xor(acc, off, LPN);
  if (ok && lane == 0) {
    const int64_t node = gx + sy * gy + sz * gz;
    x[node] = x[node] + omega * dinv[node] * (b[node] - acc);
  }
}

// ------------------------------------------------------------------ assembled entries
// Packed index of G_ab (a <= b): 00 01 02 11 12 22 in 3D, 00 01 11 in 2D.
__device__ __forceinline__ int gcomp(int dim, int a, int b) {
  if (a > b) {
    const int t = a;
    a = b;
    b = t;
  }
  if (dim == 2) return a == 0 ? b : 2;
  if (a == 0) return b;
  return a == 1 ? 2 + b : 5;
}

// (K_e)_ij of the collocated element stiffness sum_q B_q^T G_q B_q between local nodes li and
// lj of element e: B_a(q, i) = D[q_a, i_a] when q agrees with i off axis a, so
//   a = b: i, j on one a-line: sum_m D[m, i_a] G_aa(i with a -> m) D[m, j_a];
//   a != b: i, j agree on the remaining axis (3D); the one point q = (q_a = j_a, q_b = i_b, rest
//           = i) gives D[j_a, i_a] G_ab(q) D[i_b, j_b].
__device__ double elem_entry(const double* __restrict__ Ge, const double* __restrict__ Dm, int n,
                             int dim, const int* li, const int* lj) {
  const int nloc = dim == 3 ? n * n * n : n * n;
  const int st[3] = {1, n, n * n};
  double k = 0.0;
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) {
      if (a == b) {
        bool line = true;
        for (int c = 0; c < dim; ++c)
          if (c != a && li[c] != lj[c]) line = false;
        if (!line) continue;
        int q0 = 0;
        for (int c = 0; c < dim; ++c)
          if (c != a) q0 += li[c] * st[c];
        const double* Gaa = Ge + (int64_t)gcomp(dim, a, a) * nloc;
        for (int m = 0; m < n; ++m)
          k += Dm[m * n + li[a]] * Gaa[q0 + m * st[a]] * Dm[m * n + lj[a]];
      } else {
        if (dim == 3) {
          const int c3 = 3 - a - b;
          if (li[c3] != lj[c3]) continue;
        }
        int q = lj[a] * st[a] + li[b] * st[b];
        if (dim == 3) q += li[3 - a - b] * st[3 - a - b];
        k += Dm[lj[a] * n + li[a]] * Ge[(int64_t)gcomp(dim, a, b) * nloc + q] * Dm[li[b] * n + lj[b]];
      }
    }
  return k;
}

// l1 row sums of the interior block: out_i = sum_j |A_ij| over interior nodes j, A_ij = the sum
// of (K_e)_ij over the elements holding both nodes (0 at boundary rows). One thread per node;
// the candidates j are the nodes of the elements around i that share a grid coordinate with i
// (3D) or any node of them (2D). FP64, setup only.
__global__ void __launch_bounds__(256)
k_l1_rowsum(const double* __restrict__ G, const double* __restrict__ Dm, Grid g,
            double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  const int dim = g.dim, p = g.p, n = p + 1;
  const int gi[3] = {(int)(t % g.nn[0]), (int)((t / g.nn[0]) % g.nn[1]),
                     dim == 3 ? (int)(t / ((int64_t)g.nn[0] * g.nn[1])) : 0};
  for (int a = 0; a < dim; ++a)
    if (gi[a] == 0 || gi[a] == g.nn[a] - 1) {
      out[t] = 0.0;
      return;
    }
  // per axis: the elements around gi (one below first) and the range of their nodes
  int ea[3][2], na[3], lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= dim) {
      na[a] = 1;
      ea[a][0] = ea[a][1] = 0;
      lo[a] = hi[a] = 0;
      continue;
    }
    if (gi[a] % p == 0) {
      na[a] = 2;
      ea[a][0] = gi[a] / p - 1;
      ea[a][1] = gi[a] / p;
    } else {
      na[a] = 1;
      ea[a][0] = ea[a][1] = gi[a] / p;
    }
    lo[a] = ea[a][0] * p;
    hi[a] = ea[a][na[a] - 1] * p + p;
  }
  const int nloc = dim == 3 ? n * n * n : n * n;
  const int ncomp = dim == 3 ? 6 : 3;
  double acc = 0.0;
  for (int jz = lo[2]; jz <= hi[2]; ++jz)
    for (int jy = lo[1]; jy <= hi[1]; ++jy)
      for (int jx = lo[0]; jx <= hi[0]; ++jx) {
        const int gj[3] = {jx, jy, jz};
        bool inter = true;
        for (int a = 0; a < dim; ++a) inter = inter && gj[a] > 0 && gj[a] < g.nn[a] - 1;
        if (!inter) continue;
        if (dim == 3 && gj[0] != gi[0] && gj[1] != gi[1] && gj[2] != gi[2]) continue;
        // per axis the elements holding both: both around gi if gj == gi, else the one on gj's side
        int ce[3][2], nc[3];
        for (int a = 0; a < 3; ++a) {
          if (a >= dim) {
            nc[a] = 1;
            ce[a][0] = 0;
          } else if (gj[a] == gi[a]) {
            nc[a] = na[a];
            ce[a][0] = ea[a][0];
            ce[a][1] = ea[a][1];
          } else {
            nc[a] = 1;
            ce[a][0] = (na[a] == 2 && gj[a] > gi[a]) ? ea[a][1] : ea[a][0];
          }
        }
        double aij = 0.0;
        for (int cz = 0; cz < nc[2]; ++cz)
          for (int cy = 0; cy < nc[1]; ++cy)
            for (int cx = 0; cx < nc[0]; ++cx) {
              const int e3[3] = {ce[0][cx], ce[1][cy], ce[2][cz]};
              int li[3], lj[3];
              for (int a = 0; a < 3; ++a) {
                li[a] = a < dim ? gi[a] - e3[a] * p : 0;
                lj[a] = a < dim ? gj[a] - e3[a] * p : 0;
              }
              const int64_t e = e3[0] + (int64_t)g.ne[0] * (e3[1] + (int64_t)g.ne[1] * e3[2]);
              aij += elem_entry(G + e * (int64_t)ncomp * nloc, Dm, n, dim, li, lj);
            }
        acc += fabs(aij);
      }
  out[t] = acc;
}

// ------------------------------------------------------------------ element block Jacobi
// Blocks (§3.2.3, §4.4.3): element e owns, along each axis, its local nodes 0..p-1 (the last
// element also p, always a boundary node), so every interior node lies in exactly one block.
// Block e is stored as a padded P x P matrix, P = p^d, over the slots s = i + p (j + p k) of the
// local nodes [0, p)^d: slots of owned interior nodes hold A restricted to them, slots of
// boundary nodes (local 0 on an element at the low domain face) an identity row and column, so
// the inverse of the padded matrix is the block inverse beside an identity.

// The elements holding global grid index gi along an axis (one below first; 1 or 2).
__device__ __forceinline__ int holders(int gi, int p, int ne, int* e) {
  if (gi % p == 0 && gi > 0 && gi < ne * p) {
    e[0] = gi / p - 1;
    e[1] = gi / p;
    return 2;
  }
  e[0] = e[1] = min(gi / p, ne - 1);
  return 1;
}

// A_ij of the assembled stiffness between global nodes gi and gj: (K_e)_ij summed over the
// elements holding both.
__device__ double assembled_entry(const double* __restrict__ G, const double* __restrict__ Dm,
                                  const Grid& g, const int* gi, const int* gj) {
  const int dim = g.dim, p = g.p, n = p + 1;
  int ce[3][2], nc[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= dim) {
      nc[a] = 1;
      ce[a][0] = 0;
      continue;
    }
    int ei[2], ej[2];
    const int ni = holders(gi[a], p, g.ne[a], ei), nj = holders(gj[a], p, g.ne[a], ej);
    nc[a] = 0;
    for (int u = 0; u < ni; ++u)
      for (int v = 0; v < nj; ++v)
        if (ei[u] == ej[v]) ce[a][nc[a]++] = ei[u];
    if (nc[a] == 0) return 0.0;
  }
  const int nloc = dim == 3 ? n * n * n : n * n;
  const int ncomp = dim == 3 ? 6 : 3;
  double aij = 0.0;
  for (int cz = 0; cz < nc[2]; ++cz)
    for (int cy = 0; cy < nc[1]; ++cy)
      for (int cx = 0; cx < nc[0]; ++cx) {
        const int e3[3] = {ce[0][cx], ce[1][cy], ce[2][cz]};
        int li[3], lj[3];
        for (int a = 0; a < 3; ++a) {
          li[a] = a < dim ? gi[a] - e3[a] * p : 0;
          lj[a] = a < dim ? gj[a] - e3[a] * p : 0;
        }
        const int64_t e = e3[0] + (int64_t)g.ne[0] * (e3[1] + (int64_t)g.ne[1] * e3[2]);
        aij += elem_entry(G + e * (int64_t)ncomp * nloc, Dm, n, dim, li, lj);
      }
  return aij;
}

// Fill the padded blocks: one thread per (element, row slot, column slot).
__global__ void __launch_bounds__(256)
k_block_fill(const double* __restrict__ G, const double* __restrict__ Dm, Grid g, int P,
             double* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t PP = (int64_t)P * P;
  if (t >= g.E * PP) return;
  const int64_t e = t / PP;
  const int rs = (int)((t - e * PP) / P), cs = (int)(t - e * PP - (int64_t)rs * P);
  const int dim = g.dim, p = g.p;
  const int ex = (int)(e % g.ne[0]), ey = (int)((e / g.ne[0]) % g.ne[1]),
            ez = (int)(e / ((int64_t)g.ne[0] * g.ne[1]));
  const int eo[3] = {ex * p, ey * p, ez * p};
  const int ls[2][3] = {{rs % p, (rs / p) % p, dim == 3 ? rs / (p * p) : 0},
                        {cs % p, (cs / p) % p, dim == 3 ? cs / (p * p) : 0}};
  int gi[3] = {0, 0, 0}, gj[3] = {0, 0, 0};
  bool bi = false, bj = false;
  for (int a = 0; a < dim; ++a) {
    gi[a] = eo[a] + ls[0][a];
    gj[a] = eo[a] + ls[1][a];
    bi = bi || gi[a] == 0;
    bj = bj || gj[a] == 0;
  }
  double v;
  if (bi || bj)
    v = rs == cs ? 1.0 : 0.0;
  else
    v = assembled_entry(G, Dm, g, gi, gj);
  B[t] = v;
}

// In-place inverse of each P x P block by Gauss-Jordan elimination without pivoting (the blocks
// are SPD, so every pivot is positive): at step k, with the old row k and column k kept,
//   a_kk <- 1/a_kk,  a_kj <- a_kj / a_kk,  a_ik <- -a_ik / a_kk,  a_ij <- a_ij - a_ik a_kj / a_kk.
// One workgroup per block; the block lives in global memory (P <= kBlockMaxP).
constexpr int kBlockMaxP = 1024;
__global__ void __launch_bounds__(1024) k_block_invert(double* __restrict__ B, int P, int* flag) {
  double* A = B + (int64_t)blockIdx.x * P * P;
  __shared__ double rowk[kBlockMaxP], colk[kBlockMaxP];
  const int64_t PP = (int64_t)P * P;
  for (int k = 0; k < P; ++k) {
    for (int q = threadIdx.x; q < P; q += blockDim.x) {
      rowk[q] = A[(int64_t)k * P + q];
      colk[q] = A[(int64_t)q * P + k];
    }
    __syncthreads();
    const double akk = rowk[k];
    if (!(akk > 0.0)) {
      if (threadIdx.x == 0) atomicOr(flag, 8);
      return;  // the whole workgroup sees the same pivot and leaves together
    }
    const double piv = 1.0 / akk;
    for (int64_t q = threadIdx.x; q < PP; q += blockDim.x) {
      const int i = (int)(q / P), j = (int)(q - (int64_t)i * P);
      double v;
      if (i == k)
        v = j == k ? piv : rowk[j] * piv;
      else if (j == k)
        v = -colk[i] * piv;
      else
        v = A[q] - colk[i] * rowk[j] * piv;
      A[q] = v;
    }
    __syncthreads();
  }
}

// One block-Jacobi update x <- x + omega B^{-1} r per element: the workgroup gathers r at the
// element's slots into LDS, each thread forms z_s = sum_t Binv[t][s] r_t for its slots (the
// stored inverse read by columns: consecutive threads, consecutive words) and updates the owned
// interior nodes. r at boundary slots is 0.
template <typename T, int DIM>
__global__ void __launch_bounds__(256)
k_block_apply(const T* __restrict__ Binv, const T* __restrict__ r, T* __restrict__ x, Grid g,
              int P, T omega) {
  extern __shared__ unsigned char smem[];
  T* sr = (T*)smem;
  const int64_t e = blockIdx.x;
  const int p = g.p;
  const int ex = (int)(e % g.ne[0]), ey = (int)((e / g.ne[0]) % g.ne[1]),
            ez = DIM == 3 ? (int)(e / ((int64_t)g.ne[0] * g.ne[1])) : 0;
  const int64_t sy = g.nn[0], sz = (int64_t)g.nn[0] * g.nn[1];
  auto node = [&](int s, bool* bnd) {
    const int i = s % p, j = (s / p) % p, k = DIM == 3 ? s / (p * p) : 0;
    const int gx = ex * p + i, gy = ey * p + j, gz = ez * p + k;
    *bnd = gx == 0 || gy == 0 || (DIM == 3 && gz == 0);
    return gx + sy * gy + sz * gz;
  };
  for (int s = threadIdx.x; s < P; s += blockDim.x) {
    bool bnd;
    const int64_t gidx = node(s, &bnd);
    sr[s] = bnd ? T(0) : r[gidx];
  }
  __syncthreads();
  const T* Be = Binv + e * (int64_t)P * P;
  for (int s = threadIdx.x; s < P; s += blockDim.x) {
    T z = T(0);
    for (int t = 0; t < P; ++t) z += Be[(int64_t)t * P + s] * sr[t];
    bool bnd;
    const int64_t gidx = node(s, &bnd);
    if (!bnd) x[gidx] = x[gidx] + omega * z;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero_boundary(T* __restrict__ v, Grid g) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.N) return;
  const int gx = (int)(t % g.nn[0]);
  const int gy = (int)((t / g.nn[0]) % g.nn[1]);
  const int gz = (int)(t / ((int64_t)g.nn[0] * g.nn[1]));
  bool bnd = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1;
  if (g.dim == 3) bnd = bnd || gz == 0 || gz == g.nn[2] - 1;
  if (bnd) v[t] = T(0);
}

template <int N, typename T>
void gs_color_n(const Level& L, const T* G, const T* D, const void* b, void* x, const void* dinv,
                int color, double omega, hipStream_t s) {
  const Grid& g = L.g;
  const int ca = color % N, cb = color / N;
  const int cx = (g.nn[0] + N - 1) / N, cy = (g.nn[1] + N - 1) / N;
  const int64_t threads = (int64_t)cx * cy * g.nn[2] * Lpn<N>::v;
  const unsigned nb = (unsigned)((threads + kGsT - 1) / kGsT);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_gs_color<N, 3, T>), dim3(nb), dim3(kGsT), 0, s, (T*)x, (const T*)b,
                       (const T*)dinv, G, D, g, ca, cb, cx, cy, (T)omega);
  else
    hipLaunchKernelGGL((k_gs_color<N, 2, T>), dim3(nb), dim3(kGsT), 0, s, (T*)x, (const T*)b,
                       (const T*)dinv, G, D, g, ca, cb, cx, cy, (T)omega);
  GLLMG_HIP(hipGetLastError());
}

template <typename T>
void gs_color_t(const Level& L, const void* b, void* x, const void* dinv, int color, double omega,
                hipStream_t s) {
  const T* G = std::is_same<T, double>::value ? (const T*)L.G64 : (const T*)L.G32;
  const T* D = std::is_same<T, double>::value ? (const T*)L.D64 : (const T*)L.D32;
  switch (L.n) {
#define GLLMG_CASE(NV) \
  case NV:             \
    return gs_color_n<NV, T>(L, G, D, b, x, dinv, color, omega, s);
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
#undef GLLMG_CASE
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
}

}  // namespace

void launch_gs_color(const Level& L, int prec, const void* b, void* x, const void* dinv, int color,
                     double omega, hipStream_t s) {
  GLLMG_CHECK(color >= 0 && color < L.n * L.n, GLLMG_EINVAL, "color out of range");
  if (prec == 0)
    gs_color_t<double>(L, b, x, dinv, color, omega, s);
  else
    gs_color_t<float>(L, b, x, dinv, color, omega, s);
}

void launch_l1_rowsum(const Level& L, double* out, hipStream_t s) {
  const unsigned nb = (unsigned)((L.g.N + 255) / 256);
  hipLaunchKernelGGL(k_l1_rowsum, dim3(nb), dim3(256), 0, s, L.G64, L.D64, L.g, out);
  GLLMG_HIP(hipGetLastError());
}

int block_slots(const Level& L) {
  int P = 1;
  for (int a = 0; a < L.g.dim; ++a) P *= L.g.p;
  return P;
}

void launch_block_setup(const Level& L, double* B, int* flag, hipStream_t s) {
  const int P = block_slots(L);
  GLLMG_CHECK(P <= kBlockMaxP, GLLMG_EUNSUPPORTED,
              "block Jacobi: element blocks of p^d > 1024 unknowns are not supported");
  const int64_t tot = L.g.E * (int64_t)P * P;
  hipLaunchKernelGGL(k_block_fill, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L.G64,
                     L.D64, L.g, P, B);
  GLLMG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_block_invert, dim3((unsigned)L.g.E), dim3(1024), 0, s, B, P, flag);
  GLLMG_HIP(hipGetLastError());
}

void launch_block_apply(const Level& L, int prec, const void* Binv, const void* r, void* x,
                        double omega, hipStream_t s) {
  const int P = block_slots(L);
  const size_t lds = (size_t)P * (prec == 0 ? sizeof(double) : sizeof(float));
  const dim3 grid((unsigned)L.g.E), block(256);
  if (prec == 0) {
    if (L.g.dim == 3)
      hipLaunchKernelGGL((k_block_apply<double, 3>), grid, block, lds, s, (const double*)Binv,
                         (const double*)r, (double*)x, L.g, P, omega);
    else
      hipLaunchKernelGGL((k_block_apply<double, 2>), grid, block, lds, s, (const double*)Binv,
                         (const double*)r, (double*)x, L.g, P, omega);
  } else {
    if (L.g.dim == 3)
      hipLaunchKernelGGL((k_block_apply<float, 3>), grid, block, lds, s, (const float*)Binv,
                         (const float*)r, (float*)x, L.g, P, (float)omega);
    else
      hipLaunchKernelGGL((k_block_apply<float, 2>), grid, block, lds, s, (const float*)Binv,
                         (const float*)r, (float*)x, L.g, P, (float)omega);
  }
  GLLMG_HIP(hipGetLastError());
}

void zero_boundary(const Level& L, int prec, void* v, hipStream_t s) {
  const unsigned nb = (unsigned)((L.g.N + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_zero_boundary<double>, dim3(nb), dim3(256), 0, s, (double*)v, L.g);
  else
    hipLaunchKernelGGL(k_zero_boundary<float>, dim3(nb), dim3(256), 0, s, (float*)v, L.g);
  GLLMG_HIP(hipGetLastError());
}

}  // namespace gllmg
