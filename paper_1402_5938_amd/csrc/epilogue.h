// Per-node epilogues of the node-order sums (operator product, restriction): what is done with
// each summed value. Shared by the kernels that end in such a sum.
#pragma once

#include "internal.h"

namespace gllmg {


// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on XCD i mod 8), and
// each XCD has its own L2. This bijection of [0, n) gives XCD x a contiguous range of logical
// workgroup indices, so that neighbouring elements (which share nodes) and neighbouring node
// rows meet in the same L2.
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_block(uint32_t i, uint32_t n) {
  const uint32_t q = n / kXcds, r = n % kXcds, x = i % kXcds;
  return x * q + (x < r ? x : r) + i / kXcds;
}

// Typed view of the epilogue.
template <typename T>
struct EpiT {
  int mode, from_zero, last;
  T* y;
  const T* b;
  T* x;
  const T* rin;
  T* r;
  T* d;
  const T* dinv;
  const T* e0;
  const T* e1;
  T c1, c2, om;
  const double* cc;
};

template <typename T>
__host__ __device__ EpiT<T> typed(const Epi& e) {
  return EpiT<T>{e.mode, e.from_zero, e.last, (T*)e.y, (const T*)e.b, (T*)e.x, (const T*)e.rin, (T*)e.r,
                 (T*)e.d, (const T*)e.dinv, (const T*)e.e0, (const T*)e.e1, (T)e.c1, (T)e.c2,
                 (T)e.om, e.cc};
}

// ------------------------------------------------------------------ launch groups
// pointer p of problem 0 moved to problem k (d = its byte offset); null stays null
template <typename P>
__device__ inline P* shift(P* p, int64_t d) {
  return p ? (P*)((char*)p + d) : p;
}

// Problem blockIdx.y of the launch: false if it is inactive; *d = its byte offset.
__device__ inline bool grp_begin(const Grp& g, int64_t* d) {
  const int k = blockIdx.y;
  if (g.act && g.act[k] == 0) return false;
  *d = g.dlt ? g.dlt[k] : 0;
  return true;
}

// the epilogue of problem k (offset d): its pointers and, from its table, its coefficients
template <typename T>
__device__ inline EpiT<T> shift(EpiT<T> e, int64_t d) {
  e.y = shift(e.y, d);
  e.b = shift(e.b, d);
  e.x = shift(e.x, d);
  e.rin = shift(e.rin, d);
  e.r = shift(e.r, d);
  e.d = shift(e.d, d);
  e.dinv = shift(e.dinv, d);
  e.e0 = shift(e.e0, d);
  e.e1 = shift(e.e1, d);
  if (e.cc) {
    const double* c = shift(e.cc, d);
    e.c1 = (T)c[0];
    e.c2 = (T)c[1];
  }
  return e;
}

// The operands that the epilogue of ep.mode reads at node g, besides the sum: loaded before the
// sum's own loads, so that both come in one memory round trip. xin is the product's input
// vector (read by the Jacobi and Chebyshev steps).
template <typename T>
struct EpiIn {
  T b, x, rin, dinv, xin, e0, e1;
};

template <typename T>
__device__ inline EpiIn<T> epilogue_load(const EpiT<T>& ep, int64_t g, const T* xin) {
  EpiIn<T> in{};
  switch (ep.mode) {
    case EPI_STORE:
      break;
    case EPI_RESIDUAL:
      in.b = ep.b[g];
      break;
    case EPI_JACOBI:
      in.xin = xin[g];
      in.b = ep.b[g];
      in.dinv = ep.dinv[g];
      break;
    case EPI_CHEB_START:
      in.b = ep.b[g];
      in.dinv = ep.dinv[g];
      break;
    case EPI_STORE_CHEB0:
    case EPI_STORE_JACOBI0:
      in.dinv = ep.dinv[g];
      break;
    case EPI_CHEB_D:
      in.xin = xin[g];
      in.rin = ep.rin[g];
      in.dinv = ep.dinv[g];
      break;
    case EPI_CHEB_SUM:
      in.xin = xin[g];
      if (!ep.from_zero) in.x = ep.x[g];
      in.e0 = ep.e0[g];
      if (ep.e1) in.e1 = ep.e1[g];
      in.rin = ep.rin[g];
      in.dinv = ep.dinv[g];
      break;
    default:  // EPI_CHEB
      in.xin = xin[g];
      if (!ep.from_zero) in.x = ep.x[g];
      in.rin = ep.rin[g];
      in.dinv = ep.dinv[g];
  }
  return in;
}

// acc = (A xin)_g; in = epilogue_load at g
template <typename T>
__device__ inline void epilogue(const EpiT<T>& ep, int64_t g, T acc, const EpiIn<T>& in) {
  switch (ep.mode) {
    case EPI_STORE:
      ep.y[g] = acc;
      break;
    case EPI_RESIDUAL:
      ep.r[g] = in.b - acc;
      break;
    case EPI_JACOBI:
      ep.x[g] = in.xin + (ep.om * in.dinv) * (in.b - acc);
      break;
    case EPI_CHEB_START: {  // r = b - A x, d = dinv r / theta (theta in c1)
      const T ri = in.b - acc;
      ep.r[g] = ri;
      ep.d[g] = in.dinv * ri / ep.c1;
      break;
    }
    case EPI_STORE_CHEB0:
      ep.y[g] = acc;
      ep.d[g] = in.dinv * acc / ep.c1;
      break;
    case EPI_STORE_JACOBI0:
      ep.y[g] = acc;
      ep.x[g] = (ep.om * in.dinv) * acc;
      break;
    case EPI_CHEB_D: {
      const T ri = in.rin - acc;
      ep.r[g] = ri;
      ep.d[g] = ep.c1 * in.xin + (ep.c2 * in.dinv) * ri;
      break;
    }
    case EPI_CHEB_SUM: {
      T xs = ep.from_zero ? in.e0 : in.x + in.e0;
      if (ep.e1) xs = xs + in.e1;
      const T ri = in.rin - acc;
      const T dn = ep.c1 * in.xin + (ep.c2 * in.dinv) * ri;
      ep.x[g] = (xs + in.xin) + dn;
      break;
    }
    default: {  // EPI_CHEB, input vector is d
      const T xo = ep.from_zero ? in.xin : in.x + in.xin;
      const T ri = in.rin - acc;
      const T dn = ep.c1 * in.xin + (ep.c2 * in.dinv) * ri;
      if (ep.last) {  // the polynomial's final step: x = (x + d) + d_next, r and d not needed
        ep.x[g] = xo + dn;
      } else {
        ep.x[g] = xo;
        ep.r[g] = ri;
        ep.d[g] = dn;
      }
    }
  }
}

// Dirichlet boundary node: every output of the epilogue is 0 there.
template <typename T>
__device__ inline void epilogue_zero(const EpiT<T>& ep, int64_t g) {
  switch (ep.mode) {
    case EPI_STORE:
      ep.y[g] = T(0);
      break;
    case EPI_RESIDUAL:
      ep.r[g] = T(0);
      break;
    case EPI_JACOBI:
      ep.x[g] = T(0);
      break;
    case EPI_CHEB_START:
      ep.r[g] = T(0);
      ep.d[g] = T(0);
      break;
    case EPI_STORE_CHEB0:
      ep.y[g] = T(0);
      ep.d[g] = T(0);
      break;
    case EPI_STORE_JACOBI0:
      ep.y[g] = T(0);
      ep.x[g] = T(0);
      break;
    case EPI_CHEB_D:
      ep.r[g] = T(0);
      ep.d[g] = T(0);
      break;
    case EPI_CHEB_SUM:
      ep.x[g] = T(0);
      break;
    default:
      ep.x[g] = T(0);
      if (!ep.last) {
        ep.r[g] = T(0);
        ep.d[g] = T(0);
      }
  }
}

}  // namespace gllmg
