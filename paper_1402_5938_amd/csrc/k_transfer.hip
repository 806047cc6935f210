// Level transfers (paper §2.2): the prolongation P evaluates the coarse basis at the fine nodes
// and the restriction is its transpose, between the interior unknowns of the Dirichlet problem.
//
// The meshes are uniform, so between a coarse element and each fine element inside it (one
// under p-coarsening, 2 per axis under h-coarsening) P is the same tensor product of a small
// 1D matrix Pl[child][i][c] = l_c(position of fine node i in the coarse element's reference
// interval) for every element. Both directions therefore run element by element, as three 1D
// contractions (two in 2D) in LDS, one kernel launch each instead of one pass per axis over the
// global grid:
// * prolongation: one fine element per work unit reads its parent's coarse nodes, contracts and
//   writes the fine nodes it owns (local indices 0..p-1 per axis, and p in the last element
//   along an axis), so every fine node is written once and x += P e needs no atomics;
// * restriction: a fine node shared by m fine elements enters each of them with weight 1/m
//   (m = 1, 2, 4, 8: exact in binary floating point), so the element contributions add up to
//   P^T r. One coarse element per work unit sums its children's contracted contributions in a
//   fixed order into a coarse element vector; the gather kernel of the operator product then
//   adds the copies of shared coarse nodes in a fixed order and runs the coarse level's first
//   smoothing step as its epilogue.
// Boundary values of the input are read as 0 and boundary outputs are 0 (left unchanged when
// adding).
#include <type_traits>

#include "dev_transfer.h"

namespace gllmg {

namespace {

template <int MF, int NCH, int DIM, typename T, bool GR>
__global__ void __launch_bounds__(XEpb<MF>::v * MF * MF)
k_prolong(const T* __restrict__ xc, T* __restrict__ xf, const T* __restrict__ Pl, Grid gf,
          Grid gc, int add, const T* __restrict__ zero, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    xc = shift(xc, dk);
    xf = shift(xf, dk);
    Pl = shift(Pl, dk);
    zero = shift(zero, dk);
  }
  using L = ProlongLds<MF, NCH, DIM, T>;
  __shared__ T s1[L::EPB * L::S1];
  __shared__ T s2[L::EPB * L::S2];
  __shared__ T sP[L::NP];
  prolong_elem<MF, NCH, DIM, T>(xc, xf, Pl, gf, gc, add, zero, blockIdx.x * (uint32_t)L::EPB,
                                threadIdx.x, s1, s2, sP);
}

template <int MF, int NCH, int DIM, typename T, bool GR>
__global__ void __launch_bounds__(XEpb<MF>::v * MF * MF)
k_restrict(const T* __restrict__ rf, T* __restrict__ R, const T* __restrict__ Pl, Grid gf,
           Grid gc, const T* __restrict__ zero, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    rf = shift(rf, dk);
    R = shift(R, dk);
    Pl = shift(Pl, dk);
    zero = shift(zero, dk);
  }
  using L = RestrictLds<MF, NCH, DIM, T>;
  __shared__ T su[L::EPB * L::SU];
  __shared__ T s1[L::EPB * L::S1];
  __shared__ T sP[L::NP];
  restrict_elem<MF, NCH, DIM, T>(rf, R, Pl, gf, gc, zero, blockIdx.x * (uint32_t)L::EPB,
                                 threadIdx.x, su, s1, sP);
}

template <int DIM, typename T, bool GR>
__global__ void __launch_bounds__(256)
k_restrict_p1h(const T* __restrict__ rf, Grid gf, Grid gc, EpiT<T> ep, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    rf = shift(rf, dk);
    ep = shift(ep, dk);
  }
  restrict_p1h_node<DIM, T>(rf, gf, gc, ep, blockIdx.x * blockDim.x + threadIdx.x);
}

template <int DIM, typename T, bool GR>
__global__ void __launch_bounds__(256)
k_prolong_p1h(const T* __restrict__ xc, T* __restrict__ xf, Grid gf, Grid gc, int add, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    xc = shift(xc, dk);
    xf = shift(xf, dk);
  }
  prolong_p1h_node<DIM, T>(xc, xf, gf, gc, add, blockIdx.x * blockDim.x + threadIdx.x);
}

template <int MF, int NCH, typename T>
void prolong_n(const Level& F, const Level& C, const T* Pl, const T* xc, T* xf, int add,
               hipStream_t s) {
  GLLMG_CHECK(F.n == MF && C.n == (Mc<MF, NCH>::v) && F.g.dim == C.g.dim, GLLMG_EINVAL,
              "levels do not match the transfer");
  constexpr int EPB = XEpb<MF>::v;
  const unsigned nb = (unsigned)((F.g.E + EPB - 1) / EPB);
  if (F.g.dim == 3)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_prolong<MF, NCH, 3, T, GR>), dim3(nb, grp_count()), dim3(EPB * MF * MF), 0, s,
                       xc, xf, Pl, F.g, C.g, add, (const T*)F.zero, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_prolong<MF, NCH, 2, T, GR>), dim3(nb, grp_count()), dim3(EPB * MF * MF), 0, s,
                       xc, xf, Pl, F.g, C.g, add, (const T*)F.zero, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}

template <int MF, int NCH, typename T>
void restrict_n(const Level& F, const Level& C, const T* Pl, const T* rf, T* R, hipStream_t s) {
  GLLMG_CHECK(F.n == MF && C.n == (Mc<MF, NCH>::v) && F.g.dim == C.g.dim, GLLMG_EINVAL,
              "levels do not match the transfer");
  constexpr int EPB = XEpb<MF>::v;
  const unsigned nb = (unsigned)((C.g.E + EPB - 1) / EPB);
  if (F.g.dim == 3)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_restrict<MF, NCH, 3, T, GR>), dim3(nb, grp_count()), dim3(EPB * MF * MF), 0, s,
                       rf, R, Pl, F.g, C.g, (const T*)F.zero, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_restrict<MF, NCH, 2, T, GR>), dim3(nb, grp_count()), dim3(EPB * MF * MF), 0, s,
                       rf, R, Pl, F.g, C.g, (const T*)F.zero, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}

// runtime order and coarsening kind -> template instance
template <typename T, typename Fn>
void dispatch(const Level& F, Fn&& fn) {
  const bool h = F.tp.nch == 2;
#define GLLMG_CASE(MF)                                        \
  case MF:                                                    \
    if (h)                                                    \
      fn(std::integral_constant<int, MF>{}, std::integral_constant<int, 2>{}); \
    else                                                      \
      fn(std::integral_constant<int, MF>{}, std::integral_constant<int, 1>{}); \
    return;
  switch (F.n) {
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
#undef GLLMG_CASE
}

}  // namespace

void launch_prolong(const Level& F, const Level& C, int prec, const void* xc, void* xf, bool add,
                    hipStream_t s) {
  const int a = add ? 1 : 0;
  if (F.n == 2 && F.tp.nch == 2) {
    GLLMG_CHECK(C.n == 2 && F.g.dim == C.g.dim, GLLMG_EINVAL, "levels do not match the transfer");
    const unsigned nb = (unsigned)((F.g.N + 255) / 256);
    if (prec == 0 && F.g.dim == 3)
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_prolong_p1h<3, double, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const double*)xc, (double*)xf, F.g, C.g, a, cur_grp());
      });
    else if (prec == 0)
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_prolong_p1h<2, double, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const double*)xc, (double*)xf, F.g, C.g, a, cur_grp());
      });
    else if (F.g.dim == 3)
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_prolong_p1h<3, float, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const float*)xc, (float*)xf, F.g, C.g, a, cur_grp());
      });
    else
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_prolong_p1h<2, float, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const float*)xc, (float*)xf, F.g, C.g, a, cur_grp());
      });
    GLLMG_HIP(hipGetLastError());
    return;
  }
  if (prec == 0)
    dispatch<double>(F, [&](auto mf, auto nch) {
      prolong_n<decltype(mf)::value, decltype(nch)::value, double>(F, C, F.tp.P64, (const double*)xc,
                                                                  (double*)xf, a, s);
    });
  else
    dispatch<float>(F, [&](auto mf, auto nch) {
      prolong_n<decltype(mf)::value, decltype(nch)::value, float>(F, C, F.tp.P32, (const float*)xc,
                                                                 (float*)xf, a, s);
    });
}

void launch_restrict(const Level& F, const Level& C, int prec, const void* rf, const Epi& ep,
                     void* R, hipStream_t s) {
  if (F.n == 2 && F.tp.nch == 2) {
    GLLMG_CHECK(C.n == 2 && F.g.dim == C.g.dim, GLLMG_EINVAL, "levels do not match the transfer");
    const unsigned nb = (unsigned)((C.g.N + 255) / 256);
    if (prec == 0 && F.g.dim == 3)
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_restrict_p1h<3, double, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const double*)rf, F.g, C.g, typed<double>(ep), cur_grp());
      });
    else if (prec == 0)
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_restrict_p1h<2, double, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const double*)rf, F.g, C.g, typed<double>(ep), cur_grp());
      });
    else if (F.g.dim == 3)
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_restrict_p1h<3, float, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const float*)rf, F.g, C.g, typed<float>(ep), cur_grp());
      });
    else
      with_gr([&](auto gr) {
        constexpr bool GR = decltype(gr)::value;
        hipLaunchKernelGGL((k_restrict_p1h<2, float, GR>), dim3(nb, grp_count()), dim3(256), 0, s, (const float*)rf, F.g, C.g, typed<float>(ep), cur_grp());
      });
    GLLMG_HIP(hipGetLastError());
    return;
  }
  if (prec == 0)
    dispatch<double>(F, [&](auto mf, auto nch) {
      restrict_n<decltype(mf)::value, decltype(nch)::value, double>(F, C, F.tp.P64, (const double*)rf,
                                                                   (double*)R, s);
    });
  else
    dispatch<float>(F, [&](auto mf, auto nch) {
      restrict_n<decltype(mf)::value, decltype(nch)::value, float>(F, C, F.tp.P32, (const float*)rf,
                                                                  (float*)R, s);
    });
  launch_gather_epi(C, prec, R, ep, s);
}

size_t restrict_buffer_elems(const Level& F, const Level& C) {
  (void)F;
  return (size_t)C.g.E * (C.g.dim == 3 ? (size_t)C.n * C.n * C.n : (size_t)C.n * C.n);
}

}  // namespace gllmg
