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

#include "internal.h"

namespace gllmg {

namespace {

constexpr int kXT = 256;

template <int M, int DIM>
struct Pow {
  static constexpr int v = DIM == 3 ? M * M * M : M * M;
};

// work units per workgroup: about kXT outputs per workgroup for small bricks
template <int CNT>
struct Epw {
  static constexpr int v = CNT >= kXT / 2 ? 1 : kXT / CNT;
};

// number of coarse nodes per axis of a coarse element: p-coarsening halves the order (rounding
// up), h-coarsening keeps it
template <int MF, int NCH>
struct Mc {
  static constexpr int v = NCH == 2 ? MF : (MF - 1 + 1) / 2 + 1;
};

__device__ inline bool on_bnd(int gidx, int nn) { return gidx == 0 || gidx == nn - 1; }

// ------------------------------------------------------------------ prolongation
// Work unit = fine element ef; parent coarse element ef / NCH per axis, child ef % NCH.
template <int MF, int NCH, int DIM, typename T>
__global__ void __launch_bounds__(kXT)
k_prolong(const T* __restrict__ xc, T* __restrict__ xf, const T* __restrict__ Pl, Grid gf,
          Grid gc, int add) {
  constexpr int MC = Mc<MF, NCH>::v;
  constexpr int CC = Pow<MC, DIM>::v, CF = Pow<MF, DIM>::v;
  constexpr int EPW = Epw<CF>::v;
  constexpr int S1 = DIM == 3 ? MF * MC * MC : MF * MC;  // after the z (3D) or y (2D) contraction
  constexpr int S2 = DIM == 3 ? MF * MF * MC : 1;        // after the y contraction (3D)
  constexpr int PF = MF - 1, PC = MC - 1;
  __shared__ T sx[EPW * CC];
  __shared__ T s1[EPW * S1];
  __shared__ T s2[EPW * S2];
  __shared__ T sP[NCH * MF * MC];
  const int tid = threadIdx.x;
  for (int q = tid; q < NCH * MF * MC; q += kXT) sP[q] = Pl[q];
  const int64_t e0 = (int64_t)blockIdx.x * EPW;
  // element coordinates of work unit le
  auto coords = [&](int le, int* ef) -> bool {
    const int64_t e = e0 + le;
    if (e >= gf.E) return false;
    ef[0] = (int)(e % gf.ne[0]);
    ef[1] = (int)((e / gf.ne[0]) % gf.ne[1]);
    ef[2] = DIM == 3 ? (int)(e / ((int64_t)gf.ne[0] * gf.ne[1])) : 0;
    return true;
  };
  // coarse brick of the parent element, boundary values read as 0
  for (int q = tid; q < EPW * CC; q += kXT) {
    const int le = q / CC, c = q - le * CC;
    int ef[3];
    T v = T(0);
    if (coords(le, ef)) {
      const int cx = c % MC, cy = (c / MC) % MC, cz = DIM == 3 ? c / (MC * MC) : 0;
      const int gx = (ef[0] / NCH) * PC + cx, gy = (ef[1] / NCH) * PC + cy;
      const int gz = DIM == 3 ? (ef[2] / NCH) * PC + cz : 0;
      bool b = on_bnd(gx, gc.nn[0]) || on_bnd(gy, gc.nn[1]);
      if (DIM == 3) b = b || on_bnd(gz, gc.nn[2]);
      if (!b) v = xc[gx + (int64_t)gc.nn[0] * (gy + (int64_t)gc.nn[1] * gz)];
    }
    sx[q] = v;
  }
  __syncthreads();
  if (DIM == 3) {
    // s1[le][kz][cy][cx] = sum_cz Pz[kz][cz] sx[le][cz][cy][cx]
    for (int q = tid; q < EPW * S1; q += kXT) {
      const int le = q / S1, r = q - le * S1;
      const int cx = r % MC, cy = (r / MC) % MC, kz = r / (MC * MC);
      int ef[3] = {0, 0, 0};
      coords(le, ef);
      const T* Pz = sP + (ef[2] % NCH) * MF * MC + kz * MC;
      const T* in = sx + le * CC + cy * MC + cx;
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < MC; ++c) acc += Pz[c] * in[c * MC * MC];
      s1[q] = acc;
    }
    __syncthreads();
    // s2[le][kz][jy][cx] = sum_cy Py[jy][cy] s1[le][kz][cy][cx]
    for (int q = tid; q < EPW * S2; q += kXT) {
      const int le = q / S2, r = q - le * S2;
      const int cx = r % MC, jy = (r / MC) % MF, kz = r / (MC * MF);
      int ef[3] = {0, 0, 0};
      coords(le, ef);
      const T* Py = sP + (ef[1] % NCH) * MF * MC + jy * MC;
      const T* in = s1 + le * S1 + kz * MC * MC + cx;
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < MC; ++c) acc += Py[c] * in[c * MC];
      s2[q] = acc;
    }
  } else {
    // s1[le][jy][cx] = sum_cy Py[jy][cy] sx[le][cy][cx]
    for (int q = tid; q < EPW * S1; q += kXT) {
      const int le = q / S1, r = q - le * S1;
      const int cx = r % MC, jy = r / MC;
      int ef[3] = {0, 0, 0};
      coords(le, ef);
      const T* Py = sP + (ef[1] % NCH) * MF * MC + jy * MC;
      const T* in = sx + le * CC + cx;
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < MC; ++c) acc += Py[c] * in[c * MC];
      s1[q] = acc;
    }
  }
  __syncthreads();
  // fine value at (ix, jy, kz) = sum_cx Px[ix][cx] s[.., cx]; written where owned
  const T* S = DIM == 3 ? s2 : s1;
  constexpr int SS = DIM == 3 ? S2 : S1;
  for (int q = tid; q < EPW * CF; q += kXT) {
    const int le = q / CF, r = q - le * CF;
    int ef[3];
    if (!coords(le, ef)) continue;
    const int ix = r % MF, jy = (r / MF) % MF, kz = DIM == 3 ? r / (MF * MF) : 0;
    const bool own = (ix < PF || ef[0] == gf.ne[0] - 1) && (jy < PF || ef[1] == gf.ne[1] - 1) &&
                     (DIM == 2 || kz < PF || ef[2] == gf.ne[2] - 1);
    if (!own) continue;
    const int gx = ef[0] * PF + ix, gy = ef[1] * PF + jy, gz = DIM == 3 ? ef[2] * PF + kz : 0;
    const int64_t g = gx + (int64_t)gf.nn[0] * (gy + (int64_t)gf.nn[1] * gz);
    bool b = on_bnd(gx, gf.nn[0]) || on_bnd(gy, gf.nn[1]);
    if (DIM == 3) b = b || on_bnd(gz, gf.nn[2]);
    if (b) {
      if (!add) xf[g] = T(0);
      continue;
    }
    const T* Px = sP + (ef[0] % NCH) * MF * MC + ix * MC;
    const T* in = S + le * SS + (DIM == 3 ? (kz * MF + jy) * MC : jy * MC);
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < MC; ++c) acc += Px[c] * in[c];
    xf[g] = add ? xf[g] + acc : acc;
  }
}

// ------------------------------------------------------------------ restriction
// Work unit = coarse element ec; its NCH^DIM children are summed in the fixed order z, y, x
// (child 0 first). Output: the coarse element vector R[ec][cz][cy][cx].
template <int MF, int NCH, int DIM, typename T>
__global__ void __launch_bounds__(kXT)
k_restrict(const T* __restrict__ rf, T* __restrict__ R, const T* __restrict__ Pl, Grid gf,
           Grid gc) {
  constexpr int MC = Mc<MF, NCH>::v;
  constexpr int CC = Pow<MC, DIM>::v, CF = Pow<MF, DIM>::v;
  constexpr int EPW = Epw<CF>::v;
  constexpr int S1 = DIM == 3 ? MF * MF * MC : MF * MC;  // after the x contraction
  constexpr int S2 = DIM == 3 ? MF * MC * MC : 1;        // after the y contraction (3D), in su
  constexpr int SU = CF > S2 ? CF : S2;
  constexpr int NC = DIM == 3 ? NCH * NCH * NCH : NCH * NCH;
  constexpr int PF = MF - 1;
  __shared__ T su[EPW * SU];
  __shared__ T s1[EPW * S1];
  __shared__ T sacc[EPW * CC];
  __shared__ T sP[NCH * MF * MC];
  const int tid = threadIdx.x;
  for (int q = tid; q < NCH * MF * MC; q += kXT) sP[q] = Pl[q];
  const int64_t e0 = (int64_t)blockIdx.x * EPW;
  auto coords = [&](int le, int* ec) -> bool {
    const int64_t e = e0 + le;
    if (e >= gc.E) return false;
    ec[0] = (int)(e % gc.ne[0]);
    ec[1] = (int)((e / gc.ne[0]) % gc.ne[1]);
    ec[2] = DIM == 3 ? (int)(e / ((int64_t)gc.ne[0] * gc.ne[1])) : 0;
    return true;
  };
  for (int ch = 0; ch < NC; ++ch) {
    const int chx = ch % NCH, chy = (ch / NCH) % NCH, chz = DIM == 3 ? ch / (NCH * NCH) : 0;
    // the child's fine values, weighted by 1 / (number of fine elements sharing the node)
    for (int q = tid; q < EPW * CF; q += kXT) {
      const int le = q / CF, r = q - le * CF;
      int ec[3];
      T v = T(0);
      if (coords(le, ec)) {
        const int ix = r % MF, jy = (r / MF) % MF, kz = DIM == 3 ? r / (MF * MF) : 0;
        const int fx = ec[0] * NCH + chx, fy = ec[1] * NCH + chy, fz = DIM == 3 ? ec[2] * NCH + chz : 0;
        const int gx = fx * PF + ix, gy = fy * PF + jy, gz = DIM == 3 ? fz * PF + kz : 0;
        bool b = on_bnd(gx, gf.nn[0]) || on_bnd(gy, gf.nn[1]);
        if (DIM == 3) b = b || on_bnd(gz, gf.nn[2]);
        if (!b) {
          T w = T(1);
          if (ix == 0 || ix == PF) w *= T(0.5);  // interior of the domain: shared along x
          if (jy == 0 || jy == PF) w *= T(0.5);
          if (DIM == 3 && (kz == 0 || kz == PF)) w *= T(0.5);
          v = w * rf[gx + (int64_t)gf.nn[0] * (gy + (int64_t)gf.nn[1] * gz)];
        }
      }
      su[le * SU + r] = v;
    }
    __syncthreads();
    // s1[le][k][j][cx] = sum_i Px[i][cx] su[le][k][j][i]
    for (int q = tid; q < EPW * S1; q += kXT) {
      const int le = q / S1, r = q - le * S1;
      const int cx = r % MC, row = r / MC;  // row = (k, j) or j
      const T* Px = sP + chx * MF * MC + cx;
      const T* in = su + le * SU + row * MF;
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < MF; ++i) acc += Px[i * MC] * in[i];
      s1[q] = acc;
    }
    __syncthreads();
    if (DIM == 3) {
      // su[le][k][cy][cx] = sum_j Py[j][cy] s1[le][k][j][cx]
      for (int q = tid; q < EPW * S2; q += kXT) {
        const int le = q / S2, r = q - le * S2;
        const int cx = r % MC, cy = (r / MC) % MC, k = r / (MC * MC);
        const T* Py = sP + chy * MF * MC + cy;
        const T* in = s1 + le * S1 + k * MF * MC + cx;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < MF; ++j) acc += Py[j * MC] * in[j * MC];
        su[le * SU + r] = acc;
      }
      __syncthreads();
      // sacc[le][cz][cy][cx] (+)= sum_k Pz[k][cz] su[le][k][cy][cx]
      for (int q = tid; q < EPW * CC; q += kXT) {
        const int le = q / CC, r = q - le * CC;
        const int cxy = r % (MC * MC), cz = r / (MC * MC);
        const T* Pz = sP + chz * MF * MC + cz;
        const T* in = su + le * SU + cxy;
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < MF; ++k) acc += Pz[k * MC] * in[k * MC * MC];
        sacc[q] = ch == 0 ? acc : sacc[q] + acc;
      }
    } else {
      // sacc[le][cy][cx] (+)= sum_j Py[j][cy] s1[le][j][cx]
      for (int q = tid; q < EPW * CC; q += kXT) {
        const int le = q / CC, r = q - le * CC;
        const int cx = r % MC, cy = r / MC;
        const T* Py = sP + chy * MF * MC + cy;
        const T* in = s1 + le * S1 + cx;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < MF; ++j) acc += Py[j * MC] * in[j * MC];
        sacc[q] = ch == 0 ? acc : sacc[q] + acc;
      }
    }
    __syncthreads();
  }
  for (int q = tid; q < EPW * CC; q += kXT) {
    const int le = q / CC;
    if (e0 + le < gc.E) R[(e0 + le) * CC + (q - le * CC)] = sacc[q];
  }
}

template <int MF, int NCH, typename T>
void prolong_n(const Level& F, const Level& C, const T* Pl, const T* xc, T* xf, int add,
               hipStream_t s) {
  GLLMG_CHECK(F.n == MF && C.n == (Mc<MF, NCH>::v) && F.g.dim == C.g.dim, GLLMG_EINVAL,
              "levels do not match the transfer");
  if (F.g.dim == 3) {
    constexpr int EPW = Epw<Pow<MF, 3>::v>::v;
    const unsigned nb = (unsigned)((F.g.E + EPW - 1) / EPW);
    hipLaunchKernelGGL((k_prolong<MF, NCH, 3, T>), dim3(nb), dim3(kXT), 0, s, xc, xf, Pl, F.g,
                       C.g, add);
  } else {
    constexpr int EPW = Epw<Pow<MF, 2>::v>::v;
    const unsigned nb = (unsigned)((F.g.E + EPW - 1) / EPW);
    hipLaunchKernelGGL((k_prolong<MF, NCH, 2, T>), dim3(nb), dim3(kXT), 0, s, xc, xf, Pl, F.g,
                       C.g, add);
  }
  GLLMG_HIP(hipGetLastError());
}

template <int MF, int NCH, typename T>
void restrict_n(const Level& F, const Level& C, const T* Pl, const T* rf, T* R, hipStream_t s) {
  GLLMG_CHECK(F.n == MF && C.n == (Mc<MF, NCH>::v) && F.g.dim == C.g.dim, GLLMG_EINVAL,
              "levels do not match the transfer");
  if (F.g.dim == 3) {
    constexpr int EPW = Epw<Pow<MF, 3>::v>::v;
    const unsigned nb = (unsigned)((C.g.E + EPW - 1) / EPW);
    hipLaunchKernelGGL((k_restrict<MF, NCH, 3, T>), dim3(nb), dim3(kXT), 0, s, rf, R, Pl, F.g,
                       C.g);
  } else {
    constexpr int EPW = Epw<Pow<MF, 2>::v>::v;
    const unsigned nb = (unsigned)((C.g.E + EPW - 1) / EPW);
    hipLaunchKernelGGL((k_restrict<MF, NCH, 2, T>), dim3(nb), dim3(kXT), 0, s, rf, R, Pl, F.g,
                       C.g);
  }
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
