// Device evaluation of the domain maps and scalar field families (see gllmg.h for the list).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace gllmg {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.1415926535897932384626433832795;

// x = Phi(X)
__device__ inline void map_eval(const FieldDev& m, int dim, const double* X, double* x) {
  if (m.kind == GLLMG_MAP_WARP_SINE) {
    const double a = m.param[0];
    if (dim == 2) {
      const double s0 = sin(kTwoPi * X[0]), s1 = sin(kTwoPi * X[1]);
      x[0] = X[0] + a * s1;
      x[1] = X[1] + a * s0;
    } else {
      const double s0 = sin(kTwoPi * X[0]), s1 = sin(kTwoPi * X[1]), s2 = sin(kTwoPi * X[2]);
      x[0] = X[0] + a * (s1 * s2);
      x[1] = X[1] + a * (s2 * s0);
      x[2] = X[2] + a * (s0 * s1);
    }
  } else if (m.kind == GLLMG_MAP_AFFINE) {
    for (int r = 0; r < dim; ++r) {
      double v = 0.0;
      for (int c = 0; c < dim; ++c) v += m.param[r * dim + c] * X[c];
      x[r] = v + m.param[dim * dim + r];
    }
  } else {
    for (int r = 0; r < dim; ++r) x[r] = X[r];
  }
}

__device__ inline double field_eval(const FieldDev& f, int dim, const double* x) {
  switch (f.kind) {
    case GLLMG_FIELD_CONST:
      return f.param[0];
    case GLLMG_FIELD_EXP_SINE_PRODUCT: {
      double prod = 1.0;
      for (int i = 0; i < dim; ++i) prod *= sin(kTwoPi * (x[i] + f.param[1 + i]));
      return exp(f.param[0] * prod);
    }
    case GLLMG_FIELD_EXP_FOURIER: {
      double gsum = 0.0;
      for (int j = 0; j < f.nmodes; ++j) {
        const double* md = f.modes + 5 * j;
        double kx = 0.0;
        for (int i = 0; i < dim; ++i) kx += md[i] * x[i];
        gsum += md[3] * cos(kTwoPi * kx + md[4]);
      }
      return exp(sqrt(2.0 / f.nmodes) * gsum);
    }
    case GLLMG_FIELD_SIN_PRODUCT: {
      double prod = 1.0;
      for (int i = 0; i < dim; ++i) prod *= sin(f.param[1] * kPi * x[i]);
      return f.param[0] * prod;
    }
    case GLLMG_FIELD_COS2_SUM: {
      double s = 0.0;
      for (int i = 0; i < dim; ++i) {
        const double c = cos(f.param[2] * kPi * x[i]);
        s += c * c;
      }
      return f.param[0] + f.param[1] * s;
    }
    default:
      return __builtin_nan("");
  }
}

// Reference coordinate of local node l of element e along an axis with ne elements.
__device__ inline double ref_coord(int e, int l, int ne, const double* xi) {
  return ((double)e + (xi[l] + 1.0) * 0.5) / (double)ne;
}

// Reference coordinate of global 1D grid index gi (order p, ne elements).
__device__ inline double ref_coord_global(int gi, int p, int ne, const double* xi) {
  int e = gi / p;
  if (e > ne - 1) e = ne - 1;
  return ref_coord(e, gi - e * p, ne, xi);
}

}  // namespace gllmg
