// Device building blocks of the level transfers: element passes of the prolongation and the
// restriction, and the order-1 h-stencils, as __device__ functions over an explicit element or
// node index; shared by the transfer kernels and the batched solver.
#pragma once

#include "epilogue.h"
#include "internal.h"

namespace gllmg {

namespace {

template <int M, int DIM>
struct Pow {
  static constexpr int v = DIM == 3 ? M * M * M : M * M;
};

// number of coarse nodes per axis of a coarse element: p-coarsening halves the order (rounding
// up), h-coarsening keeps it
template <int MF, int NCH>
struct Mc {
  static constexpr int v = NCH == 2 ? MF : (MF - 1 + 1) / 2 + 1;
};

// Thread layout: MF x MF threads per element, thread (i, j) owning the line k = 0..MF-1 (3D)
// or the single node (i, j) (2D), as in the operator kernels; elements per workgroup so that a
// workgroup has about 256 threads. Index arithmetic is then done once per thread.
template <int MF>
struct XEpb {
  static constexpr int v = MF * MF >= 128 ? 1 : 256 / (MF * MF);
};

__device__ inline bool on_bnd(int gidx, int nn) { return gidx == 0 || gidx == nn - 1; }

// Coordinates of element e on a grid with ne elements per axis (32-bit: E < 2^31).
template <int DIM>
__device__ inline void elem_xyz(uint32_t e, const int* ne, int* c) {
  const uint32_t nxy = (uint32_t)ne[0] * (uint32_t)ne[1];
  c[2] = DIM == 3 ? (int)(e / nxy) : 0;
  const uint32_t r = DIM == 3 ? e - (uint32_t)c[2] * nxy : e;
  c[1] = (int)(r / (uint32_t)ne[0]);
  c[0] = (int)(r - (uint32_t)c[1] * ne[0]);
}

// ------------------------------------------------------------------ prolongation
// Work unit = fine element ef; parent coarse element ef / NCH per axis, child ef % NCH. Every
// global load (the 1D matrix, the parent's coarse nodes and, when adding, the old fine values)
// is issued before the first barrier; the contractions z, y, x then run through LDS (3D: the z
// contraction in the registers of the thread that loaded the coarse line).
template <int MF, int NCH, int DIM, typename T>
struct ProlongLds {
  static constexpr int MC = Mc<MF, NCH>::v, EPB = XEpb<MF>::v;
  static constexpr int S1 = DIM == 3 ? MF * MC * MC : MC * MC;
  static constexpr int S2 = DIM == 3 ? MF * MF * MC : MF * MC;
  static constexpr int NP = NCH * MF * MC;
};

// One pass over the EPB fine elements ebase.. by the threads t of a workgroup (t < EPB MF^2
// own a line; others only join the barriers). s1, s2 and sP hold EPB S1, EPB S2 and NP values
// (ProlongLds). Consecutive calls sharing the LDS must be separated by a barrier.
template <int MF, int NCH, int DIM, typename T>
__device__ __forceinline__ void prolong_elem(const T* __restrict__ xc, T* __restrict__ xf,
                                             const T* __restrict__ Pl, const Grid& gf,
                                             const Grid& gc, int add, const T* __restrict__ zero,
                                             uint32_t ebase, int t, T* __restrict__ s1,
                                             T* __restrict__ s2, T* __restrict__ sP) {
  constexpr int MC = Mc<MF, NCH>::v, EPB = XEpb<MF>::v, NN = MF * MF;
  constexpr int PF = MF - 1, PC = MC - 1, NP = NCH * MF * MC;
  constexpr int NT = EPB * NN, PP = (NP + NT - 1) / NT;
  constexpr int KZ = DIM == 3 ? MF : 1;  // fine nodes per thread
  constexpr int CZ = DIM == 3 ? MC : 1;  // coarse nodes per loading thread
  // 3D: s1[le][kz][cy][cx] (after z), s2[le][kz][jy][cx] (after y); 2D: s1[le][cy][cx] (loaded),
  // s2[le][jy][cx] (after y)
  constexpr int S1 = DIM == 3 ? MF * MC * MC : MC * MC;
  constexpr int S2 = DIM == 3 ? MF * MF * MC : MF * MC;
  const bool act = t < NT;
  const int tt = act ? t : 0;
  const int le = tt / NN, ij = tt - le * NN;
  const int i = ij % MF, j = ij / MF;
  const uint32_t e = ebase + le;
  const bool valid = act && e < (uint32_t)gf.E;
  int ef[3];
  elem_xyz<DIM>(valid ? e : 0u, gf.ne, ef);
  const int chx = ef[0] % NCH, chy = ef[1] % NCH, chz = ef[2] % NCH;
  // loads: the 1D matrix, the coarse line (threads i, j < MC), the old fine line (add)
  T pv[PP];
#pragma unroll
  for (int u = 0; u < PP; ++u) pv[u] = *(t + u * NT < NP ? Pl + t + u * NT : zero);
  const bool loader = valid && i < MC && j < MC;
  const int cgx = (ef[0] / NCH) * PC + i, cgy = (ef[1] / NCH) * PC + j;
  const bool cbxy = on_bnd(cgx, gc.nn[0]) || on_bnd(cgy, gc.nn[1]);
  const int64_t cbase = cgx + (int64_t)gc.nn[0] * cgy;
  const int64_t csz = (int64_t)gc.nn[0] * gc.nn[1];
  T cl[CZ];
#pragma unroll
  for (int c = 0; c < CZ; ++c) {
    const int cgz = DIM == 3 ? (ef[2] / NCH) * PC + c : 0;
    const bool ok = loader && !cbxy && !(DIM == 3 && on_bnd(cgz, gc.nn[2]));
    cl[c] = *(ok ? xc + (cbase + csz * cgz) : zero);
  }
  const int fgx = ef[0] * PF + i, fgy = ef[1] * PF + j;
  const bool ownxy = valid && (i < PF || ef[0] == gf.ne[0] - 1) && (j < PF || ef[1] == gf.ne[1] - 1);
  const bool fbxy = on_bnd(fgx, gf.nn[0]) || on_bnd(fgy, gf.nn[1]);
  const int64_t fbase = fgx + (int64_t)gf.nn[0] * fgy;
  const int64_t fsz = (int64_t)gf.nn[0] * gf.nn[1];
  auto fine_state = [&](int k) -> int {  // 0 not written here, 1 value, 2 boundary zero
    const int fgz = DIM == 3 ? ef[2] * PF + k : 0;
    const bool own = ownxy && (DIM == 2 || k < PF || ef[2] == gf.ne[2] - 1);
    if (!own) return 0;
    const bool b = fbxy || (DIM == 3 && on_bnd(fgz, gf.nn[2]));
    return b ? (add ? 0 : 2) : 1;
  };
  T old[KZ];
#pragma unroll
  for (int k = 0; k < KZ; ++k) {
    const int fgz = DIM == 3 ? ef[2] * PF + k : 0;
    old[k] = *(add && fine_state(k) == 1 ? xf + (fbase + fsz * fgz) : zero);
  }
#pragma unroll
  for (int u = 0; u < PP; ++u)
    if (act && t + u * NT < NP) sP[t + u * NT] = pv[u];
  if (DIM == 2 && loader) s1[le * S1 + j * MC + i] = cl[0];
  __syncthreads();
  if (DIM == 3 && loader) {
    // z: s1[kz][cy = j][cx = i] = sum_cz Pz[kz][cz] cl[cz]
    const T* Pz = sP + chz * MF * MC;
#pragma unroll
    for (int kz = 0; kz < MF; ++kz) {
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < CZ; ++c) acc += Pz[kz * MC + c] * cl[c];
      s1[le * S1 + (kz * MC + j) * MC + i] = acc;
    }
  }
  if (DIM == 3) __syncthreads();
  // y: s2[(kz)][jy = j][cx = i] = sum_cy Py[jy][cy] s1[(kz)][cy][cx], threads i < MC
  if (valid && i < MC) {
    const T* Py = sP + chy * MF * MC + j * MC;
#pragma unroll
    for (int kz = 0; kz < KZ; ++kz) {
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < MC; ++c) acc += Py[c] * s1[le * S1 + (kz * MC + c) * MC + i];
      s2[le * S2 + (kz * MF + j) * MC + i] = acc;
    }
  }
  __syncthreads();
  // x: fine (ix = i, jy = j, kz) = sum_cx Px[ix][cx] s2[(kz)][jy][cx]; written where owned
  const T* Px = sP + chx * MF * MC + i * MC;
#pragma unroll
  for (int kz = 0; kz < KZ; ++kz) {
    const int st = fine_state(kz);
    if (st == 0) continue;
    const int64_t g = fbase + fsz * (DIM == 3 ? ef[2] * PF + kz : 0);
    if (st == 2) {
      xf[g] = T(0);
      continue;
    }
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < MC; ++c) acc += Px[c] * s2[le * S2 + (kz * MF + j) * MC + c];
    xf[g] = add ? old[kz] + acc : acc;
  }
}

// ------------------------------------------------------------------ restriction
// Work unit = coarse element ec; its NCH^DIM children are summed in the fixed order z, y, x
// (child 0 first) into registers of the threads (i, j) < MC, which write the coarse element
// vector R[ec][cz][cy][cx]. A child's fine line is loaded while the previous child is being
// contracted: x through LDS, then y and z in registers (3D).
template <int MF, int NCH, int DIM, typename T>
struct RestrictLds {
  static constexpr int MC = Mc<MF, NCH>::v, EPB = XEpb<MF>::v;
  static constexpr int SU = DIM == 3 ? MF * MF * MF : MF * MF;
  static constexpr int S1 = DIM == 3 ? MF * MF * MC : MF * MC;
  static constexpr int NP = NCH * MF * MC;
};

// One pass over the EPB coarse elements ebase.. (conventions as prolong_elem; su, s1 and sP
// hold EPB SU, EPB S1 and NP values, RestrictLds).
template <int MF, int NCH, int DIM, typename T>
__device__ __forceinline__ void restrict_elem(const T* __restrict__ rf, T* __restrict__ R,
                                              const T* __restrict__ Pl, const Grid& gf,
                                              const Grid& gc, const T* __restrict__ zero,
                                              uint32_t ebase, int t, T* __restrict__ su,
                                              T* __restrict__ s1, T* __restrict__ sP) {
  constexpr int MC = Mc<MF, NCH>::v, EPB = XEpb<MF>::v, NN = MF * MF;
  constexpr int PF = MF - 1, NP = NCH * MF * MC;
  constexpr int NT = EPB * NN, PP = (NP + NT - 1) / NT;
  constexpr int KZ = DIM == 3 ? MF : 1;
  constexpr int NC = DIM == 3 ? NCH * NCH * NCH : NCH * NCH;
  constexpr int SU = DIM == 3 ? MF * MF * MF : MF * MF;  // su[le][k][j][i]
  constexpr int S1 = DIM == 3 ? MF * MF * MC : MF * MC;  // s1[le][k][j][cx]
  constexpr int CC = Pow<MC, DIM>::v;
  const bool act = t < NT;
  const int tt = act ? t : 0;
  const int le = tt / NN, ij = tt - le * NN;
  const int i = ij % MF, j = ij / MF;
  const uint32_t e = ebase + le;
  const bool valid = act && e < (uint32_t)gc.E;
  int ec[3];
  elem_xyz<DIM>(valid ? e : 0u, gc.ne, ec);
  const int64_t fsz = (int64_t)gf.nn[0] * gf.nn[1];
  // weight of the shared-node split along x and y for this thread's line
  const T wxy = ((i == 0 || i == PF) ? T(0.5) : T(1)) * ((j == 0 || j == PF) ? T(0.5) : T(1));
  // child ch's fine line of this thread: node index of each k (valid where w[k] != 0)
  auto line = [&](int ch, int64_t* base, bool* live) {
    const int chx = ch % NCH, chy = (ch / NCH) % NCH;
    const int gx = (ec[0] * NCH + chx) * PF + i, gy = (ec[1] * NCH + chy) * PF + j;
    *live = valid && !(on_bnd(gx, gf.nn[0]) || on_bnd(gy, gf.nn[1]));
    *base = gx + (int64_t)gf.nn[0] * gy;
  };
  auto zof = [&](int ch, int k) {
    const int chz = DIM == 3 ? ch / (NCH * NCH) : 0;
    return DIM == 3 ? (ec[2] * NCH + chz) * PF + k : 0;
  };
  T pv[PP];
#pragma unroll
  for (int u = 0; u < PP; ++u) pv[u] = *(t + u * NT < NP ? Pl + t + u * NT : zero);
  T col[KZ];
  {
    int64_t b;
    bool lv;
    line(0, &b, &lv);
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
      const int gz = zof(0, k);
      const bool ok = lv && !(DIM == 3 && on_bnd(gz, gf.nn[2]));
      col[k] = *(ok ? rf + (b + fsz * gz) : zero);
    }
  }
#pragma unroll
  for (int u = 0; u < PP; ++u)
    if (act && t + u * NT < NP) sP[t + u * NT] = pv[u];
  T acc[DIM == 3 ? MC : 1];
#pragma unroll
  for (int c = 0; c < (DIM == 3 ? MC : 1); ++c) acc[c] = T(0);
  for (int ch = 0; ch < NC; ++ch) {
    const int chx = ch % NCH, chy = (ch / NCH) % NCH, chz = DIM == 3 ? ch / (NCH * NCH) : 0;
    // weighted line into LDS (boundary nodes were read as 0)
    if (act) {
#pragma unroll
      for (int k = 0; k < KZ; ++k) {
        const T wz = (DIM == 3 && (k == 0 || k == PF)) ? T(0.5) : T(1);
        su[le * SU + (k * MF + j) * MF + i] = (wxy * wz) * col[k];
      }
    }
    __syncthreads();
    if (ch + 1 < NC) {
      int64_t b;
      bool lv;
      line(ch + 1, &b, &lv);
#pragma unroll
      for (int k = 0; k < KZ; ++k) {
        const int gz = zof(ch + 1, k);
        const bool ok = lv && !(DIM == 3 && on_bnd(gz, gf.nn[2]));
        col[k] = *(ok ? rf + (b + fsz * gz) : zero);
      }
    }
    // x: s1[k][j][cx = i] = sum_i' Px[i'][cx] su[k][j][i'], threads i < MC
    if (act && i < MC) {
      const T* Px = sP + chx * MF * MC + i;
#pragma unroll
      for (int k = 0; k < KZ; ++k) {
        T a = T(0);
#pragma unroll
        for (int m = 0; m < MF; ++m) a += Px[m * MC] * su[le * SU + (k * MF + j) * MF + m];
        s1[le * S1 + (k * MF + j) * MC + i] = a;
      }
    }
    __syncthreads();
    // y (and z in 3D): threads (cx = i, cy = j) < MC
    if (act && i < MC && j < MC) {
      const T* Py = sP + chy * MF * MC + j;
      if (DIM == 3) {
        const T* Pz = sP + chz * MF * MC;
#pragma unroll
        for (int k = 0; k < MF; ++k) {
          T a = T(0);
#pragma unroll
          for (int m = 0; m < MF; ++m) a += Py[m * MC] * s1[le * S1 + (k * MF + m) * MC + i];
#pragma unroll
          for (int c = 0; c < MC; ++c) acc[c] += Pz[k * MC + c] * a;
        }
      } else {
        T a = T(0);
#pragma unroll
        for (int m = 0; m < MF; ++m) a += Py[m * MC] * s1[le * S1 + m * MC + i];
        acc[0] += a;
      }
    }
    __syncthreads();
  }
  if (valid && i < MC && j < MC) {
    T* Re = R + (int64_t)e * CC;
    if (DIM == 3) {
#pragma unroll
      for (int c = 0; c < MC; ++c) Re[(c * MC + j) * MC + i] = acc[c];
    } else {
      Re[j * MC + i] = acc[0];
    }
  }
}

// ------------------------------------------------------------------ order 1, h-coarsening
// The coarse hat function of node I is 1 at fine node 2I and 1/2 at 2I - 1 and 2I + 1 along
// each axis, so at p = 1 both directions are short node stencils, one thread per output node
// and one launch each (these levels are small and launch-bound):
//   (P^T r)(I) = sum over s in {-1, 0, 1}^d of prod_a w(s_a) r(2I + s),  w(0) = 1, w(+-1) = 1/2
//   (P e)(i)   = per axis, the coarse value at i/2 (i even) or the mean of those at (i -+ 1)/2
// (the weights are powers of 2, so every product is exact). Sums run z, y, x, lower first.
template <int DIM, typename T>
__device__ __forceinline__ void restrict_p1h_node(const T* __restrict__ rf, const Grid& gf,
                                                  const Grid& gc, const EpiT<T>& ep, uint32_t t) {
  if (t >= (uint32_t)gc.N) return;
  const uint32_t nxy = (uint32_t)gc.nn[0] * (uint32_t)gc.nn[1];
  const int Iz = DIM == 3 ? (int)(t / nxy) : 0;
  const uint32_t r = t - (uint32_t)Iz * nxy;
  const int Iy = (int)(r / (uint32_t)gc.nn[0]);
  const int Ix = (int)(r - (uint32_t)Iy * gc.nn[0]);
  if (on_bnd(Ix, gc.nn[0]) || on_bnd(Iy, gc.nn[1]) || (DIM == 3 && on_bnd(Iz, gc.nn[2]))) {
    epilogue_zero(ep, t);
    return;
  }
  const EpiIn<T> in = epilogue_load(ep, t, (const T*)nullptr);
  // an interior coarse node's stencil lies inside the fine grid, off its boundary
  T acc = T(0);
#pragma unroll
  for (int sz = (DIM == 3 ? -1 : 0); sz <= (DIM == 3 ? 1 : 0); ++sz)
#pragma unroll
    for (int sy = -1; sy <= 1; ++sy)
#pragma unroll
      for (int sx = -1; sx <= 1; ++sx) {
        const T w = (sx ? T(0.5) : T(1)) * (sy ? T(0.5) : T(1)) * (sz ? T(0.5) : T(1));
        const int fx = 2 * Ix + sx, fy = 2 * Iy + sy, fz = DIM == 3 ? 2 * Iz + sz : 0;
        acc += w * rf[fx + (int64_t)gf.nn[0] * (fy + (int64_t)gf.nn[1] * fz)];
      }
  epilogue(ep, t, acc, in);
}

template <int DIM, typename T>
__device__ __forceinline__ void prolong_p1h_node(const T* __restrict__ xc, T* __restrict__ xf,
                                                 const Grid& gf, const Grid& gc, int add,
                                                 uint32_t t) {
  if (t >= (uint32_t)gf.N) return;
  const uint32_t nxy = (uint32_t)gf.nn[0] * (uint32_t)gf.nn[1];
  const int iz = DIM == 3 ? (int)(t / nxy) : 0;
  const uint32_t r = t - (uint32_t)iz * nxy;
  const int iy = (int)(r / (uint32_t)gf.nn[0]);
  const int ix = (int)(r - (uint32_t)iy * gf.nn[0]);
  if (on_bnd(ix, gf.nn[0]) || on_bnd(iy, gf.nn[1]) || (DIM == 3 && on_bnd(iz, gf.nn[2]))) {
    if (!add) xf[t] = T(0);
    return;
  }
  // per axis: coarse indices I0 (and I0 + 1 at odd fine indices) with weights 1 or 1/2
  const int cx = (ix & 1) ? 2 : 1, cy = (iy & 1) ? 2 : 1, cz = DIM == 3 ? ((iz & 1) ? 2 : 1) : 1;
  const int x0 = ix >> 1, y0 = iy >> 1, z0 = iz >> 1;
  const T wx = cx == 2 ? T(0.5) : T(1), wy = cy == 2 ? T(0.5) : T(1), wz = cz == 2 ? T(0.5) : T(1);
  T acc = T(0);
  for (int kz = 0; kz < cz; ++kz)
    for (int ky = 0; ky < cy; ++ky)
      for (int kx = 0; kx < cx; ++kx) {
        const int X = x0 + kx, Y = y0 + ky, Z = DIM == 3 ? z0 + kz : 0;
        const bool b = on_bnd(X, gc.nn[0]) || on_bnd(Y, gc.nn[1]) || (DIM == 3 && on_bnd(Z, gc.nn[2]));
        if (!b) acc += (wz * wy * wx) * xc[X + (int64_t)gc.nn[0] * (Y + (int64_t)gc.nn[1] * Z)];
      }
  xf[t] = add ? xf[t] + acc : acc;
}

}  // namespace

}  // namespace gllmg
