// Device building blocks of the operator product: the element passes (3D, 2D), the node-order
// gather of element vectors and the order-1 lane product. Each is a __device__ function over an
// explicit element / row / lane index, shared by the product kernels (one launch per pass) and
// the batched solver (one workgroup per problem, looping over the passes).
#pragma once

#include "epilogue.h"
#include "internal.h"

namespace gllmg {

namespace {

__host__ __device__ inline int nloc_of(int n, int dim) { return dim == 3 ? n * n * n : n * n; }

// Elements per workgroup so that a workgroup has about 256 threads (n^2 threads per element).
template <int N>
struct Epb {
  static constexpr int v = (N * N >= 128) ? 1 : (256 / (N * N));
};

// An opaque use that makes the compiler compute v at this point (and not later, where it is
// consumed, which can keep all of its operands alive meanwhile).
template <typename T>
__device__ __forceinline__ void pin(T& v) {
  asm volatile("" : "+v"(v));
}

// Row r of the n x n matrix M (D or its transpose, stored one after the other), the same for
// every lane, read by scalar loads into scalar registers: the FMAs of a contraction then take
// their D operand from a scalar register instead of an LDS broadcast per term. M (the same
// for every lane, also where the compiler cannot tell, as in a device function's argument) is
// constant while a kernel runs. The empty asm hides the row's address from the optimizer, so
// each row is loaded where it is requested and not every row at the kernel's start, which
// would need more scalar registers than a wave has.
template <int N, typename T>
__device__ __forceinline__ void uniform_row(const T* M, int r, T (&out)[N]) {
  const uint64_t a = (uint64_t)(M + r * N);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const T* p = (const T*)(((uint64_t)hi << 32) | lo);
#if defined(__OPTIMIZE__)  // (unoptimized builds keep p in a vector register: no such hint)
  asm volatile("" : "+s"(p));
#endif
  using CT = const __attribute__((address_space(4))) T;
  CT* q = (CT*)p;
#pragma unroll
  for (int l = 0; l < N; ++l) out[l] = q[l];
}

// ------------------------------------------------------------------ 3D element kernel
// Thread (i, j) of an element keeps the column k = 0..p in registers; the x- and
// y-contractions read the element tile from LDS, the z-contraction works in registers.
// Occupancy range given to the compiler (waves per SIMD): no minimum above 1, which would
// force spills (measured slower), and at most 4 for the high-order pass, whose LDS tile
// allows few workgroups per CU anyway.
template <int N>
struct Waves {
  static constexpr int min = 1;
  static constexpr int max = N >= 12 ? 4 : 8;
};

// Which elements a pass of the element kernel works on, and where each one's element vector
// goes. ERange: elements ebase + le, the vector at F + e n^d (the level's element vectors).
struct ERange {
  __device__ bool elem(uint32_t ebase, int le, const Grid& g, uint32_t* e) const {
    *e = ebase + (uint32_t)le;
    return *e < (uint32_t)g.E;
  }
  __device__ int64_t out(uint32_t e, int, int nloc) const { return (int64_t)e * nloc; }
};

// EBox: the elements (e0 + l) of an EB^3 box, le = lx + EB (ly + EB lz), those outside the mesh
// left out; the vector of box element le at F + le n^d (a tile in LDS).
template <int EB>
struct EBox {
  int e0[3];
  __device__ bool elem(uint32_t, int le, const Grid& g, uint32_t* e) const {
    const int lx = le % EB, ly = (le / EB) % EB, lz = le / (EB * EB);
    const int ex = e0[0] + lx, ey = e0[1] + ly, ez = e0[2] + lz;
    const bool ok = ex >= 0 && ex < g.ne[0] && ey >= 0 && ey < g.ne[1] && ez >= 0 && ez < g.ne[2];
    *e = ok ? (uint32_t)ex + (uint32_t)g.ne[0] * ((uint32_t)ey + (uint32_t)g.ne[1] * (uint32_t)ez) : 0u;
    return ok;
  }
  __device__ int64_t out(uint32_t, int le, int nloc) const { return (int64_t)le * nloc; }
};

// One pass of the 3D element kernel over EPB elements (those of `map`, by default ebase..) by
// the threads t of a workgroup: t < EPB n^2 own a column, others only join the barriers. sA and
// sB hold EPB n^3 values, sD n^2. Consecutive calls that share the LDS must be separated by a
// barrier. With SR the z-contractions take D's rows and columns (the same for every lane) from
// scalar registers (uniform_row) instead of LDS broadcasts: measured 7-13% faster at n = 7 in
// FP64, 2-3% at n = 9, within +-2% below (kept on LDS there).
template <int N, typename T, int EPB, class Map = ERange, bool SR = (N >= 7)>
__device__ __forceinline__ void elem3d(const T* __restrict__ x, T* __restrict__ F,
                                       const T* __restrict__ G, const T* __restrict__ Dm,
                                       const Grid& g, int neumann, uint32_t ebase, int t,
                                       T* __restrict__ sA, T* __restrict__ sB,
                                       T* __restrict__ sD, const Map& map = Map{}) {
  constexpr int NN = N * N, NNN = N * N * N, P = N - 1;
  const bool act = t < EPB * NN;
  const int tt = act ? t : 0;
  const int le = tt / NN;
  const int ij = tt - le * NN;
  const int i = ij % N, j = ij / N;
  uint32_t e = 0u;
  const bool valid = act && map.elem(ebase, le, g, &e);
  const uint32_t ee = valid ? e : 0u;
  const uint32_t nexy = (uint32_t)g.ne[0] * (uint32_t)g.ne[1];
  const int ez = (int)(ee / nexy);
  const uint32_t rxy = ee - (uint32_t)ez * nexy;
  const int ey = (int)(rxy / (uint32_t)g.ne[0]);
  const int ex = (int)(rxy - (uint32_t)ey * g.ne[0]);
  const int gx = ex * P + i, gy = ey * P + j;
  const bool bxy = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1;
  const int64_t sxy = (int64_t)g.nn[0] * g.nn[1];
  const int64_t gb = gx + (int64_t)g.nn[0] * gy + sxy * (int64_t)(ez * P);
  T* A = sA + le * NNN;
  T* B = sB + le * NNN;

  // Every global load of the first phase is issued before any is consumed (all addresses are
  // in bounds: an out-of-range element reads element 0, thread t reads D[t mod n^2]): the x
  // column, the first PF planes of geometric factors (PF bounded by a register budget) and D.
  // measured on the 2.1M-node products: all planes for n <= 6; beyond, 4 planes in FP64 and
  // 2 in FP32 (more registers for prefetch cost occupancy, or spill, for less latency saved;
  // in FP32, 1 to 9 planes measured within noise at n = 5..11)
  constexpr int PF = N <= 6 ? N : (sizeof(T) == 8 ? 4 : 2);
  T xr[N];
#pragma unroll
  for (int k = 0; k < N; ++k) xr[k] = x[gb + sxy * k];
  const T* Ge = G + (int64_t)ee * (6 * NNN) + ij;
  T gp[PF][6];
#pragma unroll
  for (int k = 0; k < PF; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) gp[k][c] = Ge[c * NNN + k * NN];
  const T dval = Dm[ij];
  if (le == 0 && act) sD[ij] = dval;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int gz = ez * P + k;
    const bool bnd = bxy || gz == 0 || gz == g.nn[2] - 1;
    if (!valid || (bnd && !neumann)) xr[k] = T(0);
    if (act) A[k * NN + ij] = xr[k];
  }
  __syncthreads();
  T Di[N], Dj[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    Di[l] = sD[i * N + l];
    Dj[l] = sD[j * N + l];
  }

  T wx[N], wy[N], wz[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T ux = T(0), uy = T(0), uz = T(0);
    T dk[N];
    if constexpr (SR) uniform_row<N>(Dm, k, dk);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      ux += Di[l] * A[k * NN + j * N + l];
      uy += Dj[l] * A[k * NN + l * N + i];
      uz += (SR ? dk[l] : sD[k * N + l]) * xr[l];
    }
    T g0, g1, g2, g3, g4, g5;
    if (k < PF) {
      g0 = gp[k < PF ? k : 0][0];
      g1 = gp[k < PF ? k : 0][1];
      g2 = gp[k < PF ? k : 0][2];
      g3 = gp[k < PF ? k : 0][3];
      g4 = gp[k < PF ? k : 0][4];
      g5 = gp[k < PF ? k : 0][5];
    } else {
      g0 = Ge[0 * NNN + k * NN];
      g1 = Ge[1 * NNN + k * NN];
      g2 = Ge[2 * NNN + k * NN];
      g3 = Ge[3 * NNN + k * NN];
      g4 = Ge[4 * NNN + k * NN];
      g5 = Ge[5 * NNN + k * NN];
    }
    wx[k] = g0 * ux + g1 * uy + g2 * uz;
    wy[k] = g1 * ux + g3 * uy + g4 * uz;
    wz[k] = g2 * ux + g4 * uy + g5 * uz;
    // in FP64 from n = 9 on, forming the fluxes here (not at their uses after the barrier)
    // lowers the register count from two to three waves per SIMD (measured: 3% faster at
    // n = 9; at lower orders and in FP32 the compiler's placement is as fast or faster)
    if constexpr (sizeof(T) == 8 && N >= 9) {
      pin(wx[k]);
      pin(wy[k]);
      pin(wz[k]);
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      A[k * NN + ij] = wx[k];
      B[k * NN + ij] = wy[k];
    }
  }
  __syncthreads();
  if (!valid) return;
  T DiT[N], DjT[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    DiT[l] = sD[l * N + i];
    DjT[l] = sD[l * N + j];
  }
  T* Fe = F + map.out(e, le, NNN) + ij;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T acc = T(0);
    T dk[N];
    if constexpr (SR) uniform_row<N>(Dm + NN, k, dk);  // column k of D
#pragma unroll
    for (int l = 0; l < N; ++l) {
      acc += DiT[l] * A[k * NN + j * N + l];
      acc += DjT[l] * B[k * NN + l * N + i];
      acc += (SR ? dk[l] : sD[l * N + k]) * wz[l];
    }
    Fe[k * NN] = acc;
  }
}

// One row of the pointwise product w = G u, g0 u0 + g1 u1 + g2 u2, with its rounding fixed
// (two fused multiply-adds in this order) rather than left to the compiler's choice of which
// product to fuse, which can differ between two kernels that inline the same pass.
__device__ __forceinline__ double flux(double g0, double g1, double g2, double u0, double u1,
                                       double u2) {
  return __builtin_fma(g2, u2, __builtin_fma(g1, u1, g0 * u0));
}
__device__ __forceinline__ float flux(float g0, float g1, float g2, float u0, float u1, float u2) {
  return __builtin_fmaf(g2, u2, __builtin_fmaf(g1, u1, g0 * u0));
}

// High orders: the same element pass arranged for a register budget of two waves per SIMD
// (at most 256 registers per thread), where the low-order form needs more and runs one
// workgroup per CU, with no overlap of one element's loads and another's arithmetic:
// * the z-contraction reads the thread's own column back from LDS where registers are short
//   (FP64 n = 12, 13), else from a register copy of x;
// * the x-flux goes to the second LDS tile, still unused, as soon as it is formed, the
//   y-flux once every thread has finished reading the input tile;
// * the contractions run in chunks of C terms, software-pipelined: the LDS reads of
//   chunk s+1 are issued before the products of chunk s, with a scheduling barrier between
//   chunks so that the compiler does not hoist all reads of a plane (which is what fills the
//   registers otherwise);
// * D's rows and columns for the z-contractions (the same for every lane) come from scalar
//   loads one plane ahead into scalar registers (uniform_row), not from LDS: a third fewer
//   LDS reads than one LDS broadcast per term, and fewer instructions than one LDS read per
//   plane passed to the lanes by cross-lane reads; measured 5-13% faster at n = 13 and 17 on
//   8^3 to 20^3 hexes, FP32 and FP64, except FP64 n = 17 on 8^3 hexes (2% slower).
// The sums are formed in the same order as in elem3d.
// chunk length: measured best 1 in FP64 and 2 in FP32 (n = 13, 15, 17; FP64 with 1 against 3:
// 12-19% faster)
template <int N, typename T, int EPB>
__device__ __forceinline__ void elem3d_hp(const T* __restrict__ x, T* __restrict__ F,
                                          const T* __restrict__ G, const T* __restrict__ Dm,
                                          const Grid& g, int neumann, uint32_t ebase, int t,
                                          T* __restrict__ sA, T* __restrict__ sB,
                                          T* __restrict__ sD) {
  constexpr int NN = N * N, NNN = N * N * N, P = N - 1;
  constexpr int C = sizeof(T) == 8 ? 1 : 2, NC = (N + C - 1) / C, S = N * NC;
  const bool act = t < EPB * NN;
  const int tt = act ? t : 0;
  const int le = tt / NN;
  const int ij = tt - le * NN;
  const int i = ij % N, j = ij / N;
  const uint32_t e = ebase + le;
  const bool valid = act && e < (uint32_t)g.E;
  const uint32_t ee = valid ? e : 0u;
  const uint32_t nexy = (uint32_t)g.ne[0] * (uint32_t)g.ne[1];
  const int ez = (int)(ee / nexy);
  const uint32_t rxy = ee - (uint32_t)ez * nexy;
  const int ey = (int)(rxy / (uint32_t)g.ne[0]);
  const int ex = (int)(rxy - (uint32_t)ey * g.ne[0]);
  const int gx = ex * P + i, gy = ey * P + j;
  const bool bxy = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1;
  const int64_t sxy = (int64_t)g.nn[0] * g.nn[1];
  const int64_t gb = gx + (int64_t)g.nn[0] * gy + sxy * (int64_t)(ez * P);
  T* A = sA + le * NNN;
  T* B = sB + le * NNN;

  // loads issued before use (all in bounds, as in elem3d): the x column, the geometric factors
  // of the first PF planes (a ring refilled PF planes ahead) and D
  constexpr int PF = 2;
  const T* Ge = G + (int64_t)ee * (6 * NNN) + ij;
  T gp[PF][6];
#pragma unroll
  for (int k = 0; k < PF; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) gp[k][c] = Ge[c * NNN + k * NN];
  // The x column stays in registers for the z-contraction in FP32 (a quarter of the first
  // phase's LDS reads; measured 4-10% faster at n = 13, 15 and 17) and in FP64 from n = 14 on
  // (3-4% at n = 17); in FP64 at n = 12, 13 the registers would take the third wave per SIMD
  // (13-19% slower on 12^3 to 20^3 hexes).
  constexpr bool XREG = sizeof(T) == 4 || N >= 14;
  T xr[N];
  {
#pragma unroll
    for (int k = 0; k < N; ++k) xr[k] = x[gb + sxy * k];
    const T dval = Dm[ij];
    if (le == 0 && act) sD[ij] = dval;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int gz = ez * P + k;
      const bool bnd = bxy || gz == 0 || gz == g.nn[2] - 1;
      if (!valid || (bnd && !neumann)) xr[k] = T(0);
      if (act) A[k * NN + ij] = xr[k];
    }
  }
  __syncthreads();
  T Di[N], Dj[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    Di[l] = sD[i * N + l];
    Dj[l] = sD[j * N + l];
  }

  // phase 1: u = D-contractions of the tile along x, y, z; flux w = G u per node
  T bx[2][C], by[2][C], bz[2][C];
  T srow[2][N];  // row k of D (phase 1) or column k (phase 2), one plane ahead
  uniform_row<N>(Dm, 0, srow[0]);
  auto load1 = [&](int s, int buf) {
    const int k = s / NC, c = s - (s / NC) * NC;
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int l = c * C + q;
      if (l < N) {
        bx[buf][q] = A[k * NN + j * N + l];
        by[buf][q] = A[k * NN + l * N + i];
        if constexpr (!XREG) bz[buf][q] = A[l * NN + ij];
      }
    }
  };
  T wy[N], wz[N];
  T ux = T(0), uy = T(0), uz = T(0);
  load1(0, 0);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = s / NC, c = s - (s / NC) * NC;
    if (s + 1 < S) load1(s + 1 < S ? s + 1 : 0, (s + 1) & 1);
    __builtin_amdgcn_sched_barrier(0);
    if (c == 0 && k + 1 < N) uniform_row<N>(Dm, k + 1 < N ? k + 1 : 0, srow[(k + 1) & 1]);
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int l = c * C + q;
      if (l < N) {
        ux += Di[l] * bx[s & 1][q];
        uy += Dj[l] * by[s & 1][q];
        uz += srow[k & 1][l] * (XREG ? xr[l] : bz[s & 1][q]);
      }
    }
    if (c == NC - 1) {
      T gk[6];
#pragma unroll
      for (int cc = 0; cc < 6; ++cc) gk[cc] = gp[k % PF][cc];
      if (k + PF < N) {
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) gp[k % PF][cc] = Ge[cc * NNN + (k + PF < N ? k + PF : 0) * NN];
      }
      const T wx = flux(gk[0], gk[1], gk[2], ux, uy, uz);
      wy[k] = flux(gk[1], gk[3], gk[4], ux, uy, uz);
      wz[k] = flux(gk[2], gk[4], gk[5], ux, uy, uz);
      // form the fluxes here: otherwise the compiler sinks them to their uses after the
      // barrier and keeps u and the six factors of every plane alive instead
      pin(wy[k]);
      pin(wz[k]);
      if (act) B[k * NN + ij] = wx;
      ux = uy = uz = T(0);
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int k = 0; k < N; ++k) A[k * NN + ij] = wy[k];
  }
  __syncthreads();
  if (!valid) return;
  T DiT[N], DjT[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    DiT[l] = sD[l * N + i];
    DjT[l] = sD[l * N + j];
  }

  // phase 2: transposed contractions of the fluxes (x-flux in B, y-flux in A, z in registers)
  T cx[2][C], cy[2][C];
  uniform_row<N>(Dm + NN, 0, srow[0]);
  auto load2 = [&](int s, int buf) {
    const int k = s / NC, c = s - (s / NC) * NC;
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int l = c * C + q;
      if (l < N) {
        cx[buf][q] = B[k * NN + j * N + l];
        cy[buf][q] = A[k * NN + l * N + i];
      }
    }
  };
  T* Fe = F + (int64_t)e * NNN + ij;
  T acc = T(0);
  load2(0, 0);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = s / NC, c = s - (s / NC) * NC;
    if (s + 1 < S) load2(s + 1 < S ? s + 1 : 0, (s + 1) & 1);
    __builtin_amdgcn_sched_barrier(0);
    if (c == 0 && k + 1 < N) uniform_row<N>(Dm + NN, k + 1 < N ? k + 1 : 0, srow[(k + 1) & 1]);
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int l = c * C + q;
      if (l < N) {
        acc += DiT[l] * cx[s & 1][q];
        acc += DjT[l] * cy[s & 1][q];
        acc += srow[k & 1][l] * wz[l];
      }
    }
    if (c == NC - 1) {
      if (valid) Fe[k * NN] = acc;
      acc = T(0);
    }
  }
}

// elem3d or, from n = kHighpN on, elem3d_hp
constexpr int kHighpN = 12;
template <int N, typename T, int EPB>
__device__ __forceinline__ void elem3d_any(const T* __restrict__ x, T* __restrict__ F,
                                           const T* __restrict__ G, const T* __restrict__ Dm,
                                           const Grid& g, int neumann, uint32_t ebase, int t,
                                           T* __restrict__ sA, T* __restrict__ sB,
                                           T* __restrict__ sD) {
  if constexpr (N >= kHighpN)
    elem3d_hp<N, T, EPB>(x, F, G, Dm, g, neumann, ebase, t, sA, sB, sD);
  else
    elem3d<N, T, EPB>(x, F, G, Dm, g, neumann, ebase, t, sA, sB, sD);
}

// ------------------------------------------------------------------ 2D element kernel
// The 2D element pass with one thread per element column (i fixed, j = 0..p): the thread
// keeps its column of x and of the y-flux in registers, so the y-contractions take D rows that
// are the same for the whole wave (LDS broadcasts) and only the x-contractions read other
// threads' values from LDS. (One thread per node instead reads D per lane for every term:
// measured 1.7x slower at p = 8 and 2.5x at p = 16.) sA and sB hold EPB n^2 values, sD n^2.
// With SR the y-contractions take D's rows and columns from scalar registers (uniform_row):
// 3-21% faster at n = 17; at n = 5 and 9 between 7% faster and 7% slower (kept on LDS).
template <int N>
struct Epb2 {
  static constexpr int v = 256 / N;
};

template <int N, typename T, int EPB, bool SR = (N >= 13)>
__device__ __forceinline__ void elem2d_col(const T* __restrict__ x, T* __restrict__ F,
                                           const T* __restrict__ G, const T* __restrict__ Dm,
                                           const Grid& g, int neumann, uint32_t ebase, int t,
                                           T* __restrict__ sA, T* __restrict__ sB,
                                           T* __restrict__ sD) {
  constexpr int NN = N * N, P = N - 1;
  const bool act = t < EPB * N;
  const int tt = act ? t : 0;
  const int le = tt / N;
  const int i = tt - le * N;
  const uint32_t e = ebase + le;
  const bool valid = act && e < (uint32_t)g.E;
  const uint32_t ee = valid ? e : 0u;
  const int ey = (int)(ee / (uint32_t)g.ne[0]);
  const int ex = (int)(ee - (uint32_t)ey * g.ne[0]);
  const int gx = ex * P + i;
  const bool bx = gx == 0 || gx == g.nn[0] - 1;
  const int64_t nx = g.nn[0];
  const int64_t gb = gx + nx * (int64_t)(ey * P);
  T* A = sA + le * NN;
  T* B = sB + le * NN;
  // loads first: the x column, the factors of the first PF rows, D
  constexpr int PF = N < 4 ? N : 4;
  T xr[N];
#pragma unroll
  for (int j = 0; j < N; ++j) xr[j] = x[gb + nx * j];
  const T* Ge = G + (int64_t)ee * (3 * NN) + i;
  T gp[PF][3];
#pragma unroll
  for (int j = 0; j < PF; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) gp[j][c] = Ge[c * NN + j * N];
  for (int q = t; q < NN; q += EPB * N) sD[q] = Dm[q];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int gy = ey * P + j;
    const bool bnd = bx || gy == 0 || gy == g.nn[1] - 1;
    if (!valid || (bnd && !neumann)) xr[j] = T(0);
    if (act) A[j * N + i] = xr[j];
  }
  __syncthreads();
  T Di[N];
#pragma unroll
  for (int l = 0; l < N; ++l) Di[l] = sD[i * N + l];
  T wy[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T ux = T(0), uy = T(0);
    T dj[N];
    if constexpr (SR) uniform_row<N>(Dm, j, dj);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      ux += Di[l] * A[j * N + l];
      uy += (SR ? dj[l] : sD[j * N + l]) * xr[l];
    }
    T g0, g1, g2;
    if (j < PF) {
      g0 = gp[j < PF ? j : 0][0];
      g1 = gp[j < PF ? j : 0][1];
      g2 = gp[j < PF ? j : 0][2];
    } else {
      g0 = Ge[0 * NN + j * N];
      g1 = Ge[1 * NN + j * N];
      g2 = Ge[2 * NN + j * N];
    }
    const T wx = g0 * ux + g1 * uy;
    wy[j] = g1 * ux + g2 * uy;
    if (act) B[j * N + i] = wx;
  }
  __syncthreads();
  if (!valid) return;
  T DiT[N];
#pragma unroll
  for (int l = 0; l < N; ++l) DiT[l] = sD[l * N + i];
  T* Fe = F + (int64_t)e * NN + i;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T acc = T(0);
    T dj[N];
    if constexpr (SR) uniform_row<N>(Dm + NN, j, dj);  // column j of D
#pragma unroll
    for (int l = 0; l < N; ++l) {
      acc += DiT[l] * B[j * N + l];
      acc += (SR ? dj[l] : sD[l * N + j]) * wy[l];
    }
    Fe[j * N] = acc;
  }
}

// ------------------------------------------------------------------ order 1, one kernel
// At p = 1 an element has 2^d nodes, and the levels where it occurs (the bottom of the
// p-hierarchy and every coarser h-level) are small enough that two kernels per product are
// bound by launch latency. Here 2^d adjacent lanes serve one node, one lane per element around
// it (lane bits x, y, z = lower or upper element along the axis), each evaluating that
// element's contribution from the same factored form
//   y_e(l) = sum_a sum_m D[m, l_a] w_a(l with a -> m),  w_a(q) = sum_b G_ab(q) u_b(q),
//   u_b(q) = sum_m D[q_b, m] x_e(q with b -> m);
// the lanes then add their values by an xor butterfly (pairs, then pairs of pairs: the same
// fixed order in every lane, since floating-point addition commutes), and the first lane runs
// the epilogue. Lanes read their neighbours' inputs while others write outputs, so no output
// may be the product's input (the in-place Jacobi update takes the two-kernel path).
template <typename T>
__device__ inline T pick(int b, T v0, T v1) {
  return b ? v1 : v0;
}

// Lane gid of the order-1 product (2^d lanes per node; every lane of a wave must take part,
// for the butterfly).
template <int DIM, typename T>
__device__ __forceinline__ void p1_lanes(const T* __restrict__ x, const T* __restrict__ G,
                                         const T* __restrict__ Dm, const Grid& g, int neumann,
                                         const EpiT<T>& ep, const T* __restrict__ zero,
                                         uint64_t gid) {
  constexpr int NE = DIM == 3 ? 8 : 4;  // lanes per node = elements around it = points per element
  constexpr int NZ = DIM == 3 ? 2 : 1;
  const bool live = gid / NE < (uint64_t)g.N;
  const uint32_t t = live ? (uint32_t)(gid / NE) : 0u;  // N < 2^31
  const int k = (int)(gid % NE);
  const int nx = g.nn[0], ny = g.nn[1], nz = g.nn[2];
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const int gz = DIM == 3 ? (int)(t / nxy) : 0;
  const uint32_t rxy = t - (uint32_t)gz * nxy;
  const int gy = (int)(rxy / (uint32_t)nx);
  const int gx = (int)(rxy - (uint32_t)gy * nx);
  auto bnd = [&](int cx, int cy, int cz) {
    return cx == 0 || cx == nx - 1 || cy == 0 || cy == ny - 1 || (DIM == 3 && (cz == 0 || cz == nz - 1));
  };
  const bool bnode = !neumann && bnd(gx, gy, gz);
  const int kx = k & 1, ky = (k >> 1) & 1, kz = DIM == 3 ? k >> 2 : 0;
  const int ex = gx - 1 + kx, ey = gy - 1 + ky, ez = DIM == 3 ? gz - 1 + kz : 0;
  const bool ev = live && !bnode && ex >= 0 && ex < g.ne[0] && ey >= 0 && ey < g.ne[1] &&
                  ez >= 0 && ez < g.ne[2];
  const int64_t e = ev ? ex + (int64_t)g.ne[0] * (ey + (int64_t)g.ne[1] * ez) : 0;
  // the element's nodal values (boundary values read as 0 unless neumann: such lanes read the
  // zero instead) and the geometric factors, all loaded before use
  T xe[NZ][2][2];
#pragma unroll
  for (int c = 0; c < NZ; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int cx = ex + a, cy = ey + b, cz = DIM == 3 ? ez + c : 0;
        const bool m = ev && (neumann || !bnd(cx, cy, cz));
        xe[c][b][a] = *(m ? x + (cx + (int64_t)nx * (cy + (int64_t)ny * cz)) : zero);
      }
  // the epilogue's operands, by the lane that applies it
  EpiIn<T> in{};
  if (live && k == 0 && !bnode) in = epilogue_load(ep, t, x);
  // the node's local coordinates in the element (runtime bits: every access below that depends
  // on them is a select, so that all values stay in registers)
  const int lx = 1 - kx, ly = 1 - ky, lz = DIM == 3 ? 1 - kz : 0;
  constexpr int NC = DIM == 3 ? 6 : 3;
  const T* Ge = G + e * (NC * NE);
  T gq[DIM][2][NC];  // G at the points l with a -> m
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int qx = a == 0 ? m : lx, qy = a == 1 ? m : ly, qz = a == 2 ? m : lz;
      const int qi = qx + 2 * qy + (DIM == 3 ? 4 * qz : 0);
#pragma unroll
      for (int c = 0; c < NC; ++c) gq[a][m][c] = Ge[c * NE + qi];
    }
  const T D00 = Dm[0], D01 = Dm[1], D10 = Dm[2], D11 = Dm[3];
  auto X = [&](int i, int j, int l) {
    const T v0 = pick(j, pick(i, xe[0][0][0], xe[0][0][1]), pick(i, xe[0][1][0], xe[0][1][1]));
    if (DIM == 2) return v0;
    const T v1 = pick(j, pick(i, xe[NZ - 1][0][0], xe[NZ - 1][0][1]),
                      pick(i, xe[NZ - 1][1][0], xe[NZ - 1][1][1]));
    return pick(l, v0, v1);
  };
  auto Drow0 = [&](int q) { return pick(q, D00, D10); };  // D[q][0]
  auto Drow1 = [&](int q) { return pick(q, D01, D11); };  // D[q][1]
  T contrib = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int qx = a == 0 ? m : lx, qy = a == 1 ? m : ly, qz = a == 2 ? m : lz;
      const T ux = Drow0(qx) * X(0, qy, qz) + Drow1(qx) * X(1, qy, qz);
      const T uy = Drow0(qy) * X(qx, 0, qz) + Drow1(qy) * X(qx, 1, qz);
      const T* gc = gq[a][m];
      T wa;
      if (DIM == 3) {
        const T uz = Drow0(qz) * X(qx, qy, 0) + Drow1(qz) * X(qx, qy, 1);
        if (a == 0)
          wa = gc[0] * ux + gc[1] * uy + gc[2] * uz;
        else if (a == 1)
          wa = gc[1] * ux + gc[3] * uy + gc[4] * uz;
        else
          wa = gc[2] * ux + gc[4] * uy + gc[5] * uz;
      } else {
        wa = a == 0 ? gc[0] * ux + gc[1] * uy : gc[1] * ux + gc[2] * uy;
      }
      const int la = a == 0 ? lx : (a == 1 ? ly : lz);
      const T dm = m == 0 ? pick(la, D00, D01) : pick(la, D10, D11);  // D[m][l_a]
      contrib += dm * wa;
    }
  if (!ev) contrib = T(0);
#pragma unroll
  for (int off = 1; off < NE; off <<= 1) contrib += __shfl_xor(contrib, off, NE);
  if (!live || k != 0) return;
  if (bnode)
    epilogue_zero(ep, t);
  else
    epilogue(ep, t, contrib, in);
}

// ------------------------------------------------------------------ gather
// containing elements of grid coordinate c along one axis: (element, local index), lower first
__device__ inline int axis_cands(int c, int p, int ne, int* ce, int* cl) {
  const int e = c / p, r = c - e * p;
  if (r != 0) {
    ce[0] = e;
    cl[0] = r;
    return 1;
  }
  int k = 0;
  if (e > 0) {
    ce[k] = e - 1;
    cl[k] = p;
    ++k;
  }
  if (e < ne) {
    ce[k] = e;
    cl[k] = 0;
    ++k;
  }
  return k;
}

// Sum over the elements containing node (gx, gy, gz) of F[e][local index of the node], in the
// order z, y, x with the lower element first. Along y and z the candidates are the same for a
// whole grid row, so those branches are uniform where a wave covers one row; along x a missing
// second candidate re-reads the first (all loads are issued before the sum). Offsets into F
// are 32-bit (the launchers require E n^d < 2^32): 64-bit index arithmetic made the kernel
// bound by its integer instructions.
template <int N, int DIM, typename T>
__device__ __forceinline__ T gather_sum(const T* __restrict__ F, const Grid& g, int gx, int gy,
                                        int gz) {
  constexpr int P = N - 1, NL = DIM == 3 ? N * N * N : N * N;
  int cex[2], clx[2], cey[2], cly[2], cez[2] = {0, 0}, clz[2] = {0, 0};
  const int cx = axis_cands(gx, P, g.ne[0], cex, clx);
  const int cy = axis_cands(gy, P, g.ne[1], cey, cly);
  const int cz = DIM == 3 ? axis_cands(gz, P, g.ne[2], cez, clz) : 1;
  T v[2][2][2];
#pragma unroll
  for (int kz = 0; kz < 2; ++kz)
#pragma unroll
    for (int ky = 0; ky < 2; ++ky)
      if (kz < cz && ky < cy) {
        const uint32_t eyz =
            (uint32_t)g.ne[0] * ((uint32_t)cey[ky] + (uint32_t)g.ne[1] * (uint32_t)cez[kz]);
        const uint32_t lyz = (uint32_t)(N * (cly[ky] + N * clz[kz]));
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) {
          const int ax = kx < cx ? kx : 0;
          v[kz][ky][kx] = F[((uint32_t)cex[ax] + eyz) * (uint32_t)NL + ((uint32_t)clx[ax] + lyz)];
        }
      }
  T acc = T(0);
#pragma unroll
  for (int kz = 0; kz < 2; ++kz)
#pragma unroll
    for (int ky = 0; ky < 2; ++ky)
#pragma unroll
      for (int kx = 0; kx < 2; ++kx)
        if (kz < cz && ky < cy && kx < cx) acc += v[kz][ky][kx];
  return acc;
}

// acc = gather_sum at node t, then the epilogue; on the domain boundary A x = 0 (all epilogue
// outputs 0) unless neumann.
template <int N, int DIM, typename T>
__device__ __forceinline__ void gather_at(const T* __restrict__ F, const T* __restrict__ xin,
                                          const Grid& g, int neumann, const EpiT<T>& ep,
                                          int64_t t, int gx, int gy, int gz) {
  const bool bnd = gx == 0 || gx == g.nn[0] - 1 || gy == 0 || gy == g.nn[1] - 1 ||
                   (DIM == 3 && (gz == 0 || gz == g.nn[2] - 1));
  if (bnd && !neumann) {
    epilogue_zero(ep, t);
    return;
  }
  const EpiIn<T> in = epilogue_load(ep, t, xin);
  const T acc = gather_sum<N, DIM, T>(F, g, gx, gy, gz);
  epilogue(ep, t, acc, in);
}

// One node per thread in node order (t < N): consecutive threads walk a grid row, so a wave
// covers one row or the end of one and the start of the next.
template <int N, int DIM, typename T>
__device__ __forceinline__ void gather_node(const T* __restrict__ F, const T* __restrict__ xin,
                                            const Grid& g, int neumann, const EpiT<T>& ep,
                                            uint32_t t) {
  const uint32_t row = div_by_recip(t, (uint32_t)g.nn[0], g.rnn[0]);
  const int gx = (int)(t - row * (uint32_t)g.nn[0]);
  const int gz = DIM == 3 ? (int)div_by_recip(row, (uint32_t)g.nn[1], g.rnn[1]) : 0;
  const int gy = DIM == 3 ? (int)(row - (uint32_t)gz * (uint32_t)g.nn[1]) : (int)row;
  gather_at<N, DIM, T>(F, xin, g, neumann, ep, (int64_t)t, gx, gy, gz);
}

// Node row `row` (fixed y, z) of the gather, nodes lane, lane + nlanes, ... (a wave per row:
// the y and z candidates are uniform across it).
template <int N, int DIM, typename T>
__device__ __forceinline__ void gather_row(const T* __restrict__ F, const T* __restrict__ xin,
                                           const Grid& g, int neumann, const EpiT<T>& ep, int row,
                                           int lane, int nlanes) {
  const int gy = DIM == 3 ? row % g.nn[1] : row;
  const int gz = DIM == 3 ? row / g.nn[1] : 0;
  const int64_t rbase = (int64_t)g.nn[0] * row;
  for (int gx = lane; gx < g.nn[0]; gx += nlanes)
    gather_at<N, DIM, T>(F, xin, g, neumann, ep, rbase + gx, gx, gy, gz);
}

// ------------------------------------------------------------------ one-kernel product of small levels
// Workgroup b owns the nodes of a box of TB p nodes per axis (the last box along an axis also
// the mesh's last node) and computes, into LDS, the element vectors of every element that
// contains one of them: the (TB + 1)^3 elements from b TB - 1 on along each axis (those shared
// with neighbouring boxes are computed by each). Each owned node then sums its elements'
// values and applies the epilogue. The element pass is the element kernel's and the sum runs in
// the gather's order, so the result is that of the two launches to the bit, in one launch and
// one memory round trip: for levels where latency, not bytes, sets the time.
template <int N, int TB>
struct Box {
  static constexpr int P = N - 1, S = TB * P, EB = TB + 1, EPB = EB * EB * EB;
  static constexpr int NNN = N * N * N;
  static constexpr int OWN = S + 1;  // owned nodes per axis, at most
  static constexpr int NT = (EPB * N * N + 63) / 64 * 64;
  static constexpr int NPT = (OWN * OWN * OWN + NT - 1) / NT;
  static constexpr int LDS = N * N + 3 * EPB * NNN;  // sD, sA, sB, sF
};

// boxes along an axis of nn nodes: the last one also takes the final node
__host__ __device__ inline int box_count(int nn, int S) { return nn - 1 > S ? (nn - 2) / S + 1 : 1; }

// Sum over the elements of the box tile sF containing node (gx, gy, gz): gather_sum's order.
template <int N, int EB, typename T>
__device__ __forceinline__ T box_sum(const T* __restrict__ sF, const Grid& g, int gx, int gy,
                                     int gz, const int* e0) {
  constexpr int P = N - 1, NNN = N * N * N;
  int cex[2], clx[2], cey[2], cly[2], cez[2], clz[2];
  const int cx = axis_cands(gx, P, g.ne[0], cex, clx);
  const int cy = axis_cands(gy, P, g.ne[1], cey, cly);
  const int cz = axis_cands(gz, P, g.ne[2], cez, clz);
  T acc = T(0);
#pragma unroll
  for (int kz = 0; kz < 2; ++kz)
#pragma unroll
    for (int ky = 0; ky < 2; ++ky)
#pragma unroll
      for (int kx = 0; kx < 2; ++kx)
        if (kz < cz && ky < cy && kx < cx) {
          const int le = (cex[kx] - e0[0]) + EB * ((cey[ky] - e0[1]) + EB * (cez[kz] - e0[2]));
          acc += sF[le * NNN + clx[kx] + N * (cly[ky] + N * clz[kz])];
        }
  return acc;
}

// Box b of the level (b < product of box_count over the axes), threads t < Box::NT; sA, sB and
// sF hold Box::EPB n^3 values, sD n^2.
template <int N, int TB, typename T>
__device__ __forceinline__ void apply_box(const T* __restrict__ x, const T* __restrict__ G,
                                          const T* __restrict__ Dm, const Grid& g, int neumann,
                                          const EpiT<T>& ep, uint32_t b, int t,
                                          T* __restrict__ sA, T* __restrict__ sB,
                                          T* __restrict__ sF, T* __restrict__ sD) {
  using B = Box<N, TB>;
  const int nbx = box_count(g.nn[0], B::S), nby = box_count(g.nn[1], B::S);
  const int bz = (int)(b / (uint32_t)(nbx * nby));
  const int rb = (int)(b - (uint32_t)bz * (uint32_t)(nbx * nby));
  const int by = rb / nbx, bx = rb - by * nbx;
  const int nbz = box_count(g.nn[2], B::S);
  const int o[3] = {bx * B::S, by * B::S, bz * B::S};
  const int c[3] = {bx == nbx - 1 ? g.nn[0] - o[0] : B::S, by == nby - 1 ? g.nn[1] - o[1] : B::S,
                    bz == nbz - 1 ? g.nn[2] - o[2] : B::S};
  const int e0[3] = {bx * TB - 1, by * TB - 1, bz * TB - 1};
  // this thread's owned nodes and their epilogue operands, loaded with the element pass's
  int64_t tn[B::NPT];
  int gn[B::NPT][3];
  bool own[B::NPT], zero[B::NPT];
  EpiIn<T> in[B::NPT];
#pragma unroll
  for (int q = 0; q < B::NPT; ++q) {
    const int sl = t + q * B::NT;
    const int u = sl % B::OWN, v = (sl / B::OWN) % B::OWN, w = sl / (B::OWN * B::OWN);
    own[q] = sl < B::OWN * B::OWN * B::OWN && u < c[0] && v < c[1] && w < c[2];
    gn[q][0] = o[0] + u;
    gn[q][1] = o[1] + v;
    gn[q][2] = o[2] + w;
    const bool bnd = gn[q][0] == 0 || gn[q][0] == g.nn[0] - 1 || gn[q][1] == 0 ||
                     gn[q][1] == g.nn[1] - 1 || gn[q][2] == 0 || gn[q][2] == g.nn[2] - 1;
    zero[q] = bnd && !neumann;
    tn[q] = own[q] ? gn[q][0] + (int64_t)g.nn[0] * (gn[q][1] + (int64_t)g.nn[1] * gn[q][2]) : 0;
    in[q] = EpiIn<T>{};
    if (own[q] && !zero[q]) in[q] = epilogue_load(ep, tn[q], x);
  }
  elem3d<N, T, B::EPB, EBox<B::EB>>(x, sF, G, Dm, g, neumann, 0u, t, sA, sB, sD,
                                    EBox<B::EB>{{e0[0], e0[1], e0[2]}});
  __syncthreads();
#pragma unroll
  for (int q = 0; q < B::NPT; ++q) {
    if (!own[q]) continue;
    if (zero[q]) {
      epilogue_zero(ep, tn[q]);
      continue;
    }
    const T acc = box_sum<N, B::EB, T>(sF, g, gn[q][0], gn[q][1], gn[q][2], e0);
    epilogue(ep, tn[q], acc, in[q]);
  }
}

}  // namespace

}  // namespace gllmg
