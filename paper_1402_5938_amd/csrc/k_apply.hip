// Matrix-free sum-factorized operator y = A x (paper §2.3: tensorized O(p^4) matvec) and the
// operator diagonal (§3.2.1), for GLL quads and hexes of order 1..16.
//
// Per element e and GLL point q (collocated quadrature):
//   u_b(q) = sum_l D[q_b, l] x_e(q with coordinate b -> l)          (d forward contractions)
//   w_a(q) = sum_b G_ab(q) u_b(q)                                    (pointwise, G symmetric)
//   y_e(i) = sum_a sum_m D[m, i_a] w_a(i with coordinate a -> m)     (d transposed contractions)
// and y = sum_e Q_e^T y_e. The sum over elements is deterministic and atomic-free: the element
// kernel writes y_e contiguously into an element-vector buffer F[e][k][j][i]; a gather kernel
// walks the nodes in vector order (x fastest) and adds the 1, 2, 4 or 8 element copies of
// each node in a fixed order (lower element first per axis, x innermost). Every access of
// the gather is coalesced for every order p. The gather ends with a per-node epilogue
// (store, residual, Jacobi or Chebyshev update), so a smoothing step is two kernels and
// never materializes A x.
// Dirichlet data: boundary entries of x are read as 0 and A x is 0 at boundary nodes.
#include <cstdint>

#include "dev_apply.h"

namespace gllmg {

namespace {

// threads of the 3D element kernel: EPB n^2
template <int N, typename T, int EPB>
struct Threads3d {
  static constexpr int v = EPB * N * N;
};

template <int N, typename T, int EPB, bool GR>
__global__ void __launch_bounds__((Threads3d<N, T, EPB>::v)) __attribute__((amdgpu_waves_per_eu(Waves<N>::min, Waves<N>::max)))
k_apply3d(const T* __restrict__ x, T* __restrict__ F, const T* __restrict__ G,
          const T* __restrict__ Dm, Grid g, int neumann, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    x = shift(x, dk);
    F = shift(F, dk);
    G = shift(G, dk);
    Dm = shift(Dm, dk);
  }
  // one LDS array with D first: D's addresses are then small enough for the immediate offset
  // of an LDS instruction (no address register per D entry)
  __shared__ T lds[N * N + 2 * EPB * N * N * N];
  T* sD = lds;
  T* sA = lds + N * N;
  T* sB = sA + EPB * N * N * N;
  elem3d_any<N, T, EPB>(x, F, G, Dm, g, neumann, xcd_block(blockIdx.x, gridDim.x) * EPB, threadIdx.x,
                        sA, sB, sD);
}

template <int N, typename T, int EPB, bool GR>
__global__ void __launch_bounds__(EPB * N)
k_apply2d(const T* __restrict__ x, T* __restrict__ F, const T* __restrict__ G,
          const T* __restrict__ Dm, Grid g, int neumann, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    x = shift(x, dk);
    F = shift(F, dk);
    G = shift(G, dk);
    Dm = shift(Dm, dk);
  }
  __shared__ T lds[N * N + 2 * EPB * N * N];
  T* sD = lds;
  T* sA = lds + N * N;
  T* sB = sA + EPB * N * N;
  elem2d_col<N, T, EPB>(x, F, G, Dm, g, neumann, xcd_block(blockIdx.x, gridDim.x) * EPB,
                        threadIdx.x, sA, sB, sD);
}

template <int DIM, typename T, bool GR>
__global__ void __launch_bounds__(256)
k_apply_p1(const T* __restrict__ x, const T* __restrict__ G, const T* __restrict__ Dm, Grid g,
           int neumann, EpiT<T> ep, const T* __restrict__ zero, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    x = shift(x, dk);
    G = shift(G, dk);
    Dm = shift(Dm, dk);
    ep = shift(ep, dk);
    zero = shift(zero, dk);
  }
  // 2^d N may pass 2^32
  p1_lanes<DIM, T>(x, G, Dm, g, neumann, ep, zero, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

constexpr int kGT = 256;

// one-kernel product of small 3D levels: element boxes of 2 x 2 x 2 owned elements
constexpr int kBoxTiles = 2;

template <int N, typename T, bool GR>
__global__ void __launch_bounds__((Box<N, kBoxTiles>::NT))
k_apply_box(const T* __restrict__ x, const T* __restrict__ G, const T* __restrict__ Dm, Grid g,
            int neumann, EpiT<T> ep, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    x = shift(x, dk);
    G = shift(G, dk);
    Dm = shift(Dm, dk);
    ep = shift(ep, dk);
  }
  using B = Box<N, kBoxTiles>;
  __shared__ T lds[B::LDS];
  T* sD = lds;
  T* sA = sD + N * N;
  T* sB = sA + B::EPB * B::NNN;
  T* sF = sB + B::EPB * B::NNN;
  apply_box<N, kBoxTiles, T>(x, G, Dm, g, neumann, ep, xcd_block(blockIdx.x, gridDim.x),
                             threadIdx.x, sA, sB, sF, sD);
}

constexpr int64_t kP1MaxNodes64 = 16384, kP1MaxNodes32 = 65536;
constexpr int64_t kBoxMaxNodes = 65536;

template <int N, int DIM, typename T, bool GR>
__global__ void __launch_bounds__(kGT)
k_gather(const T* __restrict__ F, const T* __restrict__ xin, Grid g, int neumann, EpiT<T> ep,
         Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    F = shift(F, dk);
    xin = shift(xin, dk);
    ep = shift(ep, dk);
  }
  const uint32_t t = xcd_block(blockIdx.x, gridDim.x) * (uint32_t)kGT + threadIdx.x;
  if (t >= (uint32_t)g.N) return;
  // the plain product (y = A x) in a copy of its own, whose epilogue is known at compile
  // time: no mode dispatch per node (13% faster at p = 8; the updating epilogues are bound by
  // their vector traffic and gain nothing from it)
  if (ep.mode == EPI_STORE) {
    EpiT<T> e = ep;
    e.mode = EPI_STORE;
    gather_node<N, DIM, T>(F, xin, g, neumann, e, t);
  } else {
    gather_node<N, DIM, T>(F, xin, g, neumann, ep, t);
  }
}

template <int N, typename T>
void launch_gather(const T* F, const T* xin, const Grid& g, int neumann, const EpiT<T>& ep,
                   hipStream_t s) {
  GLLMG_CHECK(g.N < ((int64_t)1 << 32) - kGT, GLLMG_EUNSUPPORTED, "level too large for 32-bit node indices");
  GLLMG_CHECK(g.E * nloc_of(N, g.dim) < ((int64_t)1 << 32), GLLMG_EUNSUPPORTED,
              "level too large for 32-bit element-vector offsets");
  const dim3 grid((unsigned)((g.N + kGT - 1) / kGT), grp_count()), block(kGT);
  if (g.dim == 3)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_gather<N, 3, T, GR>), grid, block, 0, s, F, xin, g, neumann, ep, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_gather<N, 2, T, GR>), grid, block, 0, s, F, xin, g, neumann, ep, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}

template <typename T>
void launch_gather_rt(const T* F, const T* xin, const Grid& g, int neumann, const EpiT<T>& ep,
                      hipStream_t s) {
  switch (g.p + 1) {
#define GLLMG_CASE(NV) \
  case NV:             \
    return launch_gather<NV, T>(F, xin, g, neumann, ep, s);
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
#undef GLLMG_CASE
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
}

// ------------------------------------------------------------------ diagonal
// diag_e(i) = sum_a sum_m D[m, i_a]^2 G_aa(i with a -> m) + sum_{a != b} D[i_a, i_a] D[i_b, i_b] G_ab(i)
// (for the GLL points D has a zero diagonal, up to rounding, except at the two end points, so
// the cross terms matter on element boundaries only). One thread per element point, written
// to the element-vector buffer; FP64.
__global__ void __launch_bounds__(256)
k_diag(const double* __restrict__ G, const double* __restrict__ Dm, Grid g, double* __restrict__ F) {
  const int n = g.p + 1, dim = g.dim;
  const int nloc = nloc_of(n, dim);
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
  F[t] = d;
}

template <int N, typename T>
void apply_n(const Level& L, int neumann, const void* x, const Epi& epi, void* F, hipStream_t s) {
  const T* G = std::is_same<T, double>::value ? (const T*)L.G64 : (const T*)L.G32;
  const T* D = std::is_same<T, double>::value ? (const T*)L.D64 : (const T*)L.D32;
  constexpr int EPB = Epb<N>::v;
  const unsigned nb = (unsigned)((L.g.E + EPB - 1) / EPB);
  if (L.g.dim == 3)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_apply3d<N, T, EPB, GR>), dim3(nb, grp_count()), dim3(Threads3d<N, T, EPB>::v), 0, s,
                       (const T*)x, (T*)F, G, D, L.g, neumann, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      constexpr int EPB2 = Epb2<N>::v;
      const unsigned nb2 = (unsigned)((L.g.E + EPB2 - 1) / EPB2);
      hipLaunchKernelGGL((k_apply2d<N, T, EPB2, GR>), dim3(nb2, grp_count()), dim3(EPB2 * N), 0, s,
                         (const T*)x, (T*)F, G, D, L.g, neumann, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
  launch_gather<N, T>((const T*)F, (const T*)x, L.g, neumann, typed<T>(epi), s);
}

template <typename T>
void apply_p1(const Level& L, int neumann, const void* x, const Epi& epi, hipStream_t s) {
  GLLMG_CHECK(epi.y != x && epi.x != x && epi.r != x && epi.d != x, GLLMG_EINVAL,
              "an output of the order-1 product aliases its input");
  const T* G = std::is_same<T, double>::value ? (const T*)L.G64 : (const T*)L.G32;
  const T* D = std::is_same<T, double>::value ? (const T*)L.D64 : (const T*)L.D32;
  const int64_t lanes = L.g.N * (L.g.dim == 3 ? 8 : 4);
  const unsigned nb = (unsigned)((lanes + 255) / 256);
  if (L.g.dim == 3)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_apply_p1<3, T, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const T*)x, G,
                       D, L.g, neumann, typed<T>(epi), (const T*)L.zero, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_apply_p1<2, T, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const T*)x, G,
                       D, L.g, neumann, typed<T>(epi), (const T*)L.zero, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}

template <int N, typename T>
void apply_box_n(const Level& L, int neumann, const void* x, const Epi& epi, hipStream_t s) {
  using B = Box<N, kBoxTiles>;
  const int64_t nb = (int64_t)box_count(L.g.nn[0], B::S) * box_count(L.g.nn[1], B::S) *
                     box_count(L.g.nn[2], B::S);
  GLLMG_CHECK(nb < ((int64_t)1 << 31), GLLMG_EUNSUPPORTED, "level too large for the box product");
  const T* G = std::is_same<T, double>::value ? (const T*)L.G64 : (const T*)L.G32;
  const T* D = std::is_same<T, double>::value ? (const T*)L.D64 : (const T*)L.D32;
  with_gr([&](auto gr) {
    constexpr bool GR = decltype(gr)::value;
    hipLaunchKernelGGL((k_apply_box<N, T, GR>), dim3((unsigned)nb, grp_count()), dim3(B::NT), 0, s,
                       (const T*)x, G, D, L.g, neumann, typed<T>(epi), cur_grp());
  });
  GLLMG_HIP(hipGetLastError());
}

template <typename T>
void apply_t(const Level& L, int neumann, const void* x, const Epi& ep, void* F, hipStream_t s) {
  if (L.gauss) return launch_apply_gauss(L, sizeof(T) == 8 ? 0 : 1, neumann, x, ep, F, s);
  // order 1: the one-kernel product where launch latency dominates (small levels); on large
  // 3D levels the element kernel and gather, whose F round trip costs less than the one-kernel
  // form's 8 lanes per node. Measured crossover (3D): between 4913 and 35,937 nodes in FP64,
  // between 35,937 and 274,625 in FP32; at 17M nodes the two kernels are 3x faster. In 2D the
  // two forms are within 10% up to 17M nodes.
  const int64_t p1_max = L.g.dim == 2 ? INT64_MAX : (sizeof(T) == 8 ? kP1MaxNodes64 : kP1MaxNodes32);
  if (L.n == 2 && ep.mode != EPI_JACOBI && L.g.N <= p1_max) return apply_p1<T>(L, neumann, x, ep, s);
  // order 2 in 3D: the one-kernel box product up to kBoxMaxNodes (it reads the geometric factors
  // of up to 27 elements per 8 owned, so on large levels the bytes of the two launches cost
  // less; measured at 35,937 nodes: 7.0 against 8.4 us), unless an output of the epilogue is
  // the product's input (other workgroups still read it)
  const bool in_place = ep.x == x || ep.y == x || ep.r == x || ep.d == x;
  if (L.g.dim == 3 && L.n == 3 && !in_place && L.g.N <= kBoxMaxNodes)
    return apply_box_n<3, T>(L, neumann, x, ep, s);
  switch (L.n) {
#define GLLMG_CASE(NV) \
  case NV:             \
    return apply_n<NV, T>(L, neumann, x, ep, F, s);
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
#undef GLLMG_CASE
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
}

}  // namespace

size_t face_buffer_elems(const Level& L) { return (size_t)L.g.E * nloc_of(L.n, L.g.dim); }

void launch_apply(const Level& L, int prec, int neumann, const void* x, const Epi& ep, void* F,
                  hipStream_t s) {
  if (prec == 0)
    apply_t<double>(L, neumann, x, ep, F, s);
  else
    apply_t<float>(L, neumann, x, ep, F, s);
}

void launch_gather_epi(const Level& L, int prec, const void* R, const Epi& ep, hipStream_t s) {
  if (prec == 0)
    launch_gather_rt<double>((const double*)R, nullptr, L.g, 0, typed<double>(ep), s);
  else
    launch_gather_rt<float>((const float*)R, nullptr, L.g, 0, typed<float>(ep), s);
}

void launch_gather_in(const Level& L, int prec, const void* R, const void* xin, int neumann,
                      const Epi& ep, hipStream_t s) {
  if (prec == 0)
    launch_gather_rt<double>((const double*)R, (const double*)xin, L.g, neumann, typed<double>(ep), s);
  else
    launch_gather_rt<float>((const float*)R, (const float*)xin, L.g, neumann, typed<float>(ep), s);
}

void launch_diag(const Level& L, double* diag, double* F, hipStream_t s) {
  if (L.gauss) return launch_diag_gauss(L, diag, F, s);
  const int64_t tot = L.npts;
  hipLaunchKernelGGL(k_diag, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L.G64, L.D64,
                     L.g, F);
  GLLMG_HIP(hipGetLastError());
  Epi ep;
  ep.y = diag;
  launch_gather_rt<double>((const double*)F, nullptr, L.g, 0, typed<double>(ep), s);
}

}  // namespace gllmg
