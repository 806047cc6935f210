// Batched persistent solver: one workgroup solves one problem (PCG with the V-cycle as
// preconditioner, Algorithm 1, or the V-cycle as solver), all problems of a batch in one
// launch. The workgroup runs every step of the solve itself, in the order and arithmetic of the
// stream path (the product passes, transfers, smoothers and coarse solve are the same device
// functions), with a barrier between passes and its dot products reduced in a fixed order
// inside the workgroup; a problem stops when it converges, breaks down or reaches maxit,
// independently of the others. Small problems, whose levels are too small to fill the GPU,
// are what this is for: the stream path pays a kernel launch per pass and level.
//
// The device code is instantiated per finest order n0 = p + 1 (the p-hierarchy's orders n0,
// n0/2 + 1, ..., 2) in the k_batch_*.hip files; the descriptor is in batch_desc.h.
#pragma once

#include "batch_desc.h"
#include "dev_apply.h"
#include "dev_transfer.h"

namespace gllmg {

namespace {

constexpr int kBT = kBatchThreads;

template <typename T>
struct LvlT;
template <>
struct LvlT<double> {
  static __device__ const double* G(const BatchLevel& L) { return L.G64; }
  static __device__ const double* D(const BatchLevel& L) { return L.D64; }
  static __device__ const double* dinv(const BatchLevel& L) { return L.dinv64; }
  static __device__ const double* P(const BatchLevel& L) { return L.P64; }
  static __device__ const double* Ainv(const BatchLevel& L) { return L.Ainv64; }
  static constexpr int pr = 0;
};
template <>
struct LvlT<float> {
  static __device__ const float* G(const BatchLevel& L) { return L.G32; }
  static __device__ const float* D(const BatchLevel& L) { return L.D32; }
  static __device__ const float* dinv(const BatchLevel& L) { return L.dinv32; }
  static __device__ const float* P(const BatchLevel& L) { return L.P32; }
  static __device__ const float* Ainv(const BatchLevel& L) { return L.Ainv32; }
  static constexpr int pr = 1;
};

// elements per pass of the element kernel inside the workgroup: threads and LDS permitting
template <int N, typename T>
struct BEpb {
  static constexpr int by_threads = kBT / (N * N) >= 1 ? kBT / (N * N) : 1;
  static constexpr int by_lds = (kBatchLdsBytes / (int)sizeof(T) - N * N) / (2 * N * N * N);
  static constexpr int v = by_threads < by_lds ? by_threads : (by_lds >= 1 ? by_lds : 1);
};

// Fixed-order workgroup sum (xor butterfly within each wave, then the waves in index order);
// every thread returns the same value.
__device__ inline double b_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kBT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// The stream path's order of the solve's FP64 reductions (k_dot_partial and k_pcg_xr, then
// k_sum_final): dot_grid(n) blocks of kDotThreads threads, thread t of block v adding the
// terms of entries v kDotThreads + t + m g kDotThreads in increasing m, each block's values
// added by the LDS tree of block_sum, then the block sums added the same way by one block. The
// workgroup runs two such blocks at a time (its halves), so that every scalar of the solve, and
// so every iterate, equals the stream path's bit for bit. term(i) gives entry i's term (and may
// update vectors at i: each entry is visited once). sh: kBT doubles; part: dot_grid(n) doubles.
constexpr int kHalves = kBT / kDotThreads;
static_assert(kBT % kDotThreads == 0, "the workgroup emulates whole reduction blocks");
static_assert((kBatchMaxNodes + kDotThreads - 1) / kDotThreads <= 64, "partials fit the LDS array");

__device__ inline void s_tree(double* sh) {  // each half: sh[h..h+255] -> sh[h]
  const int h = threadIdx.x / kDotThreads * kDotThreads, t = threadIdx.x % kDotThreads;
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[h + t] += sh[h + t + w];
    __syncthreads();
  }
}

template <class Term>
__device__ double s_reduce(int64_t n, double* sh, double* part, Term term) {
  const int g = dot_grid(n);
  const int t = threadIdx.x % kDotThreads;
  for (int v0 = 0; v0 < g; v0 += kHalves) {
    const int v = v0 + (int)threadIdx.x / kDotThreads;
    double acc = 0.0;
    if (v < g)
      for (int64_t i = (int64_t)v * kDotThreads + t; i < n; i += (int64_t)g * kDotThreads)
        acc += term(i);
    sh[threadIdx.x] = acc;
    __syncthreads();
    s_tree(sh);
    if (t == 0 && v < g) part[v] = sh[threadIdx.x];
    __syncthreads();
  }
  double acc = 0.0;
  if ((int)threadIdx.x < kDotThreads)
    for (int i = t; i < g; i += kDotThreads) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  s_tree(sh);
  const double s = sh[0];
  __syncthreads();
  return s;
}

template <typename T>
__device__ double s_dot(const T* a, const T* b, int64_t n, double* sh, double* part) {
  return s_reduce(n, sh, part, [&](int64_t i) { return (double)a[i] * (double)b[i]; });
}

template <typename T>
__device__ double b_dot(const T* a, const T* b, int64_t n, double* red) {
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBT) acc += (double)a[i] * (double)b[i];
  return b_sum(acc, red);
}

struct BatchCtx {
  const BatchProblem* P;
  const BatchLevel* L;  // in LDS
  char* lds;
  double* red;
  long long* applies;   // in LDS, updated by thread 0
};

// ------------------------------------------------------------------ product y = A x (+ epilogue)
// The passes below are separate functions (not inlined into the solve loop): each gets its
// own register allocation, as the corresponding kernel would.
template <int N, typename T>
__device__ __attribute__((noinline)) void b_apply_n(const BatchCtx& c, int l, const T* x,
                                                    const EpiT<T>& ep) {
  const BatchLevel& L = c.L[l];
  const Grid& g = L.g;
  const T* G = LvlT<T>::G(L);
  const T* D = LvlT<T>::D(L);
  T* F = (T*)c.P->F;
  if (N == 2 && ep.mode != EPI_JACOBI) {
    const uint64_t lanes = (uint64_t)g.N * 8;
    for (uint64_t base = 0; base < lanes; base += kBT)
      p1_lanes<3, T>(x, G, D, g, 0, ep, (const T*)c.P->zero, base + threadIdx.x);
    __syncthreads();
    return;
  }
  constexpr int EPB = BEpb<N, T>::v;
  T* sD = (T*)c.lds;
  T* sA = sD + N * N;
  T* sB = sA + EPB * N * N * N;
  for (uint32_t eb = 0; eb < (uint32_t)g.E; eb += EPB) {
    elem3d_any<N, T, EPB>(x, F, G, D, g, 0, eb, threadIdx.x, sA, sB, sD);
    __syncthreads();
  }
  const int nrows = (int)(g.N / g.nn[0]);
  for (int rb = 0; rb < nrows; rb += kBT / 64) {
    const int row = rb + (int)threadIdx.x / 64;
    if (row < nrows) gather_row<N, 3, T>(F, x, g, 0, ep, row, threadIdx.x & 63, 64);
  }
  __syncthreads();
}

// dispatch over the orders of the chain n0, n0/2 + 1, ..., 2
template <int N, typename T>
__device__ void b_apply_any(const BatchCtx& c, int l, int n, const T* x, const EpiT<T>& ep) {
  if (n == N) {
    b_apply_n<N, T>(c, l, x, ep);
    return;
  }
  if constexpr (N > 2) b_apply_any<N / 2 + 1, T>(c, l, n, x, ep);
}

template <int N0, typename T>
__device__ void b_apply(const BatchCtx& c, int l, const T* x, const Epi& e) {
  if (threadIdx.x == 0) c.applies[l] += 1;
  b_apply_any<N0, T>(c, l, c.L[l].n, x, typed<T>(e));
}

// the FP64 product on the finest level (order n0) of the outer iteration
template <int N0>
__device__ void b_apply0(const BatchCtx& c, const double* x, const Epi& e) {
  if (threadIdx.x == 0) c.applies[0] += 1;
  b_apply_n<N0, double>(c, 0, x, typed<double>(e));
}

// ------------------------------------------------------------------ transfers
template <int MF, int NCH, typename T>
__device__ __attribute__((noinline)) void b_prolong_n(const BatchCtx& c, int lf, const T* xc,
                                                      T* xf) {
  const BatchLevel& F = c.L[lf];
  const BatchLevel& C = c.L[lf + 1];
  if (MF == 2 && NCH == 2) {
    for (int64_t t = threadIdx.x; t < F.g.N; t += kBT)
      prolong_p1h_node<3, T>(xc, xf, F.g, C.g, 1, (uint32_t)t);
    __syncthreads();
    return;
  }
  using Ls = ProlongLds<MF, NCH, 3, T>;
  T* s1 = (T*)c.lds;
  T* s2 = s1 + Ls::EPB * Ls::S1;
  T* sP = s2 + Ls::EPB * Ls::S2;
  for (uint32_t eb = 0; eb < (uint32_t)F.g.E; eb += Ls::EPB) {
    prolong_elem<MF, NCH, 3, T>(xc, xf, LvlT<T>::P(F), F.g, C.g, 1, (const T*)c.P->zero, eb,
                                threadIdx.x, s1, s2, sP);
    __syncthreads();
  }
}

template <int MF, int NCH, typename T>
__device__ __attribute__((noinline)) void b_restrict_n(const BatchCtx& c, int lf, const T* rf,
                                                       const EpiT<T>& ep) {
  const BatchLevel& F = c.L[lf];
  const BatchLevel& C = c.L[lf + 1];
  if (MF == 2 && NCH == 2) {
    for (int64_t t = threadIdx.x; t < C.g.N; t += kBT)
      restrict_p1h_node<3, T>(rf, F.g, C.g, ep, (uint32_t)t);
    __syncthreads();
    return;
  }
  using Ls = RestrictLds<MF, NCH, 3, T>;
  constexpr int MC = Ls::MC;
  T* R = (T*)c.P->F;
  T* su = (T*)c.lds;
  T* s1 = su + Ls::EPB * Ls::SU;
  T* sP = s1 + Ls::EPB * Ls::S1;
  for (uint32_t eb = 0; eb < (uint32_t)C.g.E; eb += Ls::EPB) {
    restrict_elem<MF, NCH, 3, T>(rf, R, LvlT<T>::P(F), F.g, C.g, (const T*)c.P->zero, eb,
                                 threadIdx.x, su, s1, sP);
    __syncthreads();
  }
  const int nrows = (int)(C.g.N / C.g.nn[0]);
  for (int rb = 0; rb < nrows; rb += kBT / 64) {
    const int row = rb + (int)threadIdx.x / 64;
    if (row < nrows) gather_row<MC, 3, T>(R, nullptr, C.g, 0, ep, row, threadIdx.x & 63, 64);
  }
  __syncthreads();
}

// p-type transfers between chain orders (fine order MF), h-type at n0 (h-hierarchy) or at 2
template <int N0, int MF, typename T>
__device__ void b_transfer_any(const BatchCtx& c, int lf, int mf, int nch, bool restr,
                               const T* in, T* out, const EpiT<T>& ep) {
  if (mf == MF) {
    if (nch == 2) {
      if constexpr (MF == N0 || MF == 2) {
        if (restr)
          b_restrict_n<MF, 2, T>(c, lf, in, ep);
        else
          b_prolong_n<MF, 2, T>(c, lf, in, out);
      }
    } else if constexpr (MF > 2) {
      if (restr)
        b_restrict_n<MF, 1, T>(c, lf, in, ep);
      else
        b_prolong_n<MF, 1, T>(c, lf, in, out);
    }
    return;
  }
  if constexpr (MF > 2) b_transfer_any<N0, MF / 2 + 1, T>(c, lf, mf, nch, restr, in, out, ep);
}

template <int N0, typename T>
__device__ void b_restrict(const BatchCtx& c, int lf, const T* rf, const Epi& e) {
  b_transfer_any<N0, N0, T>(c, lf, c.L[lf].n, c.L[lf].nch, true, rf, nullptr, typed<T>(e));
}

template <int N0, typename T>
__device__ void b_prolong_add(const BatchCtx& c, int lf, const T* xc, T* xf) {
  b_transfer_any<N0, N0, T>(c, lf, c.L[lf].n, c.L[lf].nch, false, xc, xf, typed<T>(Epi{}));
}

// ------------------------------------------------------------------ coarse solve, vectors
template <typename T>
__device__ __attribute__((noinline)) void b_coarse(const BatchLevel& L, const T* b, T* x) {
  // the stream path's k_coarse, row by row: each wave forms rows w, w + waves, ..., lane l
  // summing the terms j = l, l + 64, ... and an xor butterfly adding the lanes (the same
  // order, so the same values)
  const Grid& g = L.g;
  const T* Ainv = LvlT<T>::Ainv(L);
  const int nx = g.nn[0], ny = g.nn[1], nz = g.nn[2];
  const int mx = nx - 2, my = ny - 2;
  for (int64_t t = threadIdx.x; t < g.N; t += kBT) {
    const int gx = (int)(t % nx), gy = (int)((t / nx) % ny), gz = (int)(t / ((int64_t)nx * ny));
    if (gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1 || gz == 0 || gz == nz - 1) x[t] = T(0);
  }
  auto node_of = [&](int64_t j) {
    const int64_t q = j / mx;
    const int jx = (int)(j - q * mx), jy = (int)(q % my), jz = (int)(q / my);
    return (jx + 1) + (int64_t)nx * ((jy + 1) + (int64_t)ny * (jz + 1));
  };
  const int lane = threadIdx.x & 63;
  for (int64_t row = threadIdx.x >> 6; row < L.nint; row += kBT / 64) {
    const T* a = Ainv + row * L.nint;
    T acc = T(0);
    for (int64_t j = lane; j < L.nint; j += 64) acc += a[j] * b[node_of(j)];
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) x[node_of(row)] = acc;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ smoothing and the V-cycle
template <int N0, typename T>
__device__ void b_smooth(const BatchCtx& c, int l, const T* b, T* x, int k, bool zero,
                         bool started) {
  const BatchLevel& L = c.L[l];
  const int64_t N = L.g.N;
  constexpr int pr = LvlT<T>::pr;
  if (k <= 0) {
    if (zero) {
      for (int64_t i = threadIdx.x; i < N; i += kBT) x[i] = T(0);
      __syncthreads();
    }
    return;
  }
  T* r = (T*)L.vr[pr];
  T* d = (T*)L.vd[pr];
  T* d2 = (T*)L.vd2[pr];
  const T* dinv = LvlT<T>::dinv(L);
  if (c.P->smoother == GLLMG_SMOOTH_JACOBI) {
    const T om = (T)c.P->omega;
    for (int it = 0; it < k; ++it) {
      if (it == 0 && zero) {
        if (!started) {
          for (int64_t i = threadIdx.x; i < N; i += kBT) x[i] = (om * dinv[i]) * b[i];
          __syncthreads();
        }
      } else {
        Epi ep;
        ep.mode = EPI_JACOBI;
        ep.x = x;
        ep.b = b;
        ep.dinv = dinv;
        ep.om = c.P->omega;
        b_apply<N0, T>(c, l, x, ep);
      }
    }
    return;
  }
  const double theta = L.theta, delta = L.delta;
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  const T* rin;
  if (zero) {
    if (!started) {
      const T th = (T)theta;
      for (int64_t i = threadIdx.x; i < N; i += kBT) d[i] = dinv[i] * b[i] / th;
      __syncthreads();
    }
    rin = b;
  } else {
    Epi ep;
    ep.mode = EPI_CHEB_START;
    ep.b = b;
    ep.r = r;
    ep.d = d;
    ep.dinv = dinv;
    ep.c1 = theta;
    b_apply<N0, T>(c, l, x, ep);
    rin = r;
  }
  for (int i = 1; i <= k; ++i) {
    const bool first_zero = zero && i == 1;
    if (i < k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      Epi ep;
      ep.mode = EPI_CHEB;
      ep.from_zero = first_zero ? 1 : 0;
      ep.last = i == k - 1 ? 1 : 0;
      ep.x = x;
      ep.rin = rin;
      ep.r = r;
      ep.d = d2;
      ep.dinv = dinv;
      ep.c1 = rn * rho;
      ep.c2 = 2.0 * rn / delta;
      b_apply<N0, T>(c, l, d, ep);
      T* t = d;
      d = d2;
      d2 = t;
      rin = r;
      rho = rn;
    } else if (k == 1) {
      for (int64_t j = threadIdx.x; j < N; j += kBT) x[j] = first_zero ? d[j] : x[j] + d[j];
      __syncthreads();
    }
  }
}

// e = V b on level 0 (b and e are vectors of precision T on level 0)
template <int N0, typename T>
__device__ void b_vcycle(const BatchCtx& c, const T* b0, T* x0) {
  constexpr int pr = LvlT<T>::pr;
  const int nl = c.P->nlev;
  const BatchProblem& P = *c.P;
  bool started = false;
  for (int l = 0; l + 1 < nl; ++l) {
    const BatchLevel& L = c.L[l];
    const BatchLevel& C = c.L[l + 1];
    const T* b = l == 0 ? b0 : (const T*)L.vb[pr];
    T* x = l == 0 ? x0 : (T*)L.vx[pr];
    b_smooth<N0, T>(c, l, b, x, P.nu_pre, true, started);
    Epi rs;  // r = b - A x
    rs.mode = EPI_RESIDUAL;
    rs.b = b;
    rs.r = L.vr[pr];
    b_apply<N0, T>(c, l, x, rs);
    Epi ep;  // b_c = P^T r and the coarse level's first smoothing step from 0
    ep.y = C.vb[pr];
    const bool fuse = C.has_coarse && P.nu_pre > 0;
    if (fuse && P.smoother == GLLMG_SMOOTH_JACOBI) {
      ep.mode = EPI_STORE_JACOBI0;
      ep.x = C.vx[pr];
      ep.dinv = LvlT<T>::dinv(C);
      ep.om = P.omega;
    } else if (fuse) {
      ep.mode = EPI_STORE_CHEB0;
      ep.d = C.vd[pr];
      ep.dinv = LvlT<T>::dinv(C);
      ep.c1 = C.theta;
    }
    b_restrict<N0, T>(c, l, (const T*)L.vr[pr], ep);
    started = fuse;
  }
  {
    const BatchLevel& L = c.L[nl - 1];
    const T* b = nl == 1 ? b0 : (const T*)L.vb[pr];
    T* x = nl == 1 ? x0 : (T*)L.vx[pr];
    b_coarse<T>(L, b, x);
  }
  for (int l = nl - 2; l >= 0; --l) {
    const BatchLevel& L = c.L[l];
    const BatchLevel& C = c.L[l + 1];
    const T* b = l == 0 ? b0 : (const T*)L.vb[pr];
    T* x = l == 0 ? x0 : (T*)L.vx[pr];
    b_prolong_add<N0, T>(c, l, (const T*)C.vx[pr], x);
    b_smooth<N0, T>(c, l, b, x, P.nu_post, false, false);
  }
}

// z = V r for the FP64 level-0 vectors, in the problem's V-cycle precision T; nr = ||r||_2
template <int N0, typename T>
__device__ void b_precond(const BatchCtx& c, const double* r, double* z, double nr) {
  if constexpr (sizeof(T) == 8) {
    b_vcycle<N0, double>(c, r, z);
  } else {  // FP32 V-cycle between casts, on r scaled by a power of two to norm about 1
    const BatchLevel& L = c.L[0];
    float* rb = (float*)L.vb[1];
    float* xb = (float*)L.vx[1];
    const double sc = pow2_inv_norm(nr * nr), isc = 1.0 / sc;
    for (int64_t i = threadIdx.x; i < L.g.N; i += kBT) rb[i] = (float)(r[i] * sc);
    __syncthreads();
    b_vcycle<N0, float>(c, rb, xb);
    for (int64_t i = threadIdx.x; i < L.g.N; i += kBT) z[i] = (double)xb[i] * isc;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ the solve
template <int N0, typename T>
__device__ void b_solve(BatchProblem* Pg, char* lds, double* red, double* sh, double* spart,
                        BatchLevel* sL, long long* sApp) {
  const int nl = Pg->nlev;
  for (int i = threadIdx.x; i < nl * (int)sizeof(BatchLevel) / 4; i += kBT)
    ((int*)sL)[i] = ((const int*)Pg->L)[i];
  if (threadIdx.x < kBatchMaxLevels) sApp[threadIdx.x] = 0;
  __syncthreads();
  BatchCtx c{Pg, sL, lds, red, sApp};
  const int64_t N = sL[0].g.N;
  const double* b = Pg->b;
  double* x = Pg->x;
  double *r = Pg->pr, *z = Pg->pz, *p = Pg->pp, *h = Pg->ph, *t = Pg->pt;
  const int mode = Pg->mode, maxit = Pg->maxit;
  const double rtol = Pg->rtol;
  {
    Epi rs;
    rs.mode = EPI_RESIDUAL;
    rs.b = b;
    rs.r = r;
    b_apply0<N0>(c, x, rs);
  }
  const double n0 = sqrt(s_dot<double>(r, r, N, sh, spart));
  if (threadIdx.x == 0) Pg->hist[0] = n0;
  int iters = 0, status = 1;
  double nr = n0;
  if (n0 == 0.0) status = 0;
  if (!isfinite(n0)) status = 2;
  if (status == 1) {
    double g = 0.0;
    if (mode == GLLMG_MODE_PCG) {
      b_precond<N0, T>(c, r, z, n0);
      g = s_dot<double>(z, r, N, sh, spart);
      for (int64_t i = threadIdx.x; i < N; i += kBT) p[i] = z[i];
      __syncthreads();
    }
    for (;;) {
      double ph = 1.0;
      if (mode == GLLMG_MODE_PCG) {
        Epi st;
        st.y = h;
        b_apply0<N0>(c, p, st);
        ph = s_dot<double>(p, h, N, sh, spart);
        const double al = g / ph;
        nr = sqrt(s_reduce(N, sh, spart, [&](int64_t i) {
          x[i] = x[i] + al * p[i];
          const double ri = r[i] - al * h[i];
          r[i] = ri;
          return ri * ri;
        }));
      } else {
        b_precond<N0, T>(c, r, z, nr);
        for (int64_t i = threadIdx.x; i < N; i += kBT) x[i] = x[i] + z[i];
        __syncthreads();
        Epi rs;
        rs.mode = EPI_RESIDUAL;
        rs.b = b;
        rs.r = r;
        b_apply0<N0>(c, x, rs);
        nr = sqrt(s_dot<double>(r, r, N, sh, spart));
      }
      ++iters;
      if (threadIdx.x == 0 && iters < kBatchHist) Pg->hist[iters] = nr;
      if ((mode == GLLMG_MODE_PCG && !(ph > 0.0)) || !isfinite(nr)) {
        status = 2;
        break;
      }
      if (nr <= rtol * n0) {
        status = 0;
        break;
      }
      if (iters >= maxit) break;
      if (mode == GLLMG_MODE_PCG) {
        b_precond<N0, T>(c, r, z, nr);
        const double gn = s_dot<double>(z, r, N, sh, spart);
        const double be = gn / g;
        for (int64_t i = threadIdx.x; i < N; i += kBT) p[i] = z[i] + be * p[i];
        __syncthreads();
        g = gn;
      }
    }
  }
  double rt = 0.0;
  if (n0 > 0.0 && isfinite(n0)) {
    Epi rs;
    rs.mode = EPI_RESIDUAL;
    rs.b = b;
    rs.r = t;
    b_apply0<N0>(c, x, rs);
    rt = sqrt(s_dot<double>(t, t, N, sh, spart)) / n0;
  }
  if (threadIdx.x == 0) {
    Pg->iters = iters;
    Pg->status = status;
    Pg->n0 = n0;
    Pg->nr = nr;
    Pg->relres_true = rt;
    for (int l = 0; l < kBatchMaxLevels; ++l) Pg->applies[l] = l < nl ? sApp[l] : 0;
  }
}

}  // namespace

// the persistent solver of finest order N0 (FP32 V-cycle, FP64 outer iteration): workgroup i
// solves problem a.p[i]
template <int N0>
__global__ void __launch_bounds__(kBatchThreads) k_batch(BatchArgs a) {
  __shared__ double lds[kBatchLdsBytes / 8];
  __shared__ double red[kBatchThreads / 64];
  __shared__ double sh[kBatchThreads];
  __shared__ double spart[64];
  __shared__ BatchLevel sL[kBatchMaxLevels];
  __shared__ long long sApp[kBatchMaxLevels];
  b_solve<N0, float>(a.p[blockIdx.x], (char*)lds, red, sh, spart, sL, sApp);
}

}  // namespace gllmg
