// Streaming kernels: the coarsest-level dense solve, the fused smoother updates, deterministic
// dot products and the PCG vector updates.
#include <algorithm>

#include "epilogue.h"

namespace gllmg {

namespace {

constexpr int kT = kDotThreads;  // 256
inline unsigned nb(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

// ------------------------------------------------------------------ coarsest level
// x = A_II^{-1} b on the interior nodes (dense inverse, rows in lexicographic interior order),
// 0 on the boundary. Blocks [0, nbn) zero the boundary nodes, one node per thread. Each block
// after them first copies b's interior entries, in row order, into LDS (at most 4096 values);
// then each of its waves forms one interior row: lane l sums the row's terms j = l, l + 64, ...
// in increasing j (the lanes read consecutive entries of the row), and an xor butterfly adds
// the 64 partial sums in a fixed order. The whole chip streams the inverse, however few nodes
// the level has.
constexpr int kCT = 512;
constexpr int kRowsPerBlock = kCT / 64;

template <typename T, bool GR>
__global__ void __launch_bounds__(kCT)
k_coarse(const T* __restrict__ Ainv, int nint, const T* __restrict__ b, T* __restrict__ x,
         Grid g, unsigned nbn, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    Ainv = shift(Ainv, dk);
    b = shift(b, dk);
    x = shift(x, dk);
  }
  extern __shared__ char coarse_lds[];
  T* sb = (T*)coarse_lds;
  const int nx = g.nn[0], ny = g.nn[1], nz = g.nn[2];
  const bool d3 = g.dim == 3;
  if (blockIdx.x < nbn) {
    const int64_t t = (int64_t)blockIdx.x * kCT + threadIdx.x;
    if (t >= g.N) return;
    const int gx = (int)(t % nx), gy = (int)((t / nx) % ny), gz = (int)(t / ((int64_t)nx * ny));
    const bool bnd = gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1 || (d3 && (gz == 0 || gz == nz - 1));
    if (bnd) x[t] = T(0);
    return;
  }
  const int mx = nx - 2, my = ny - 2;
  auto node_of = [&](int j) {
    const int q = j / mx;
    const int jx = j - q * mx, jy = q % my, jz = q / my;
    return (jx + 1) + (int64_t)nx * ((jy + 1) + (int64_t)ny * (d3 ? jz + 1 : 0));
  };
  for (int j = threadIdx.x; j < nint; j += kCT) sb[j] = b[node_of(j)];
  __syncthreads();
  const int row = (int)(blockIdx.x - nbn) * kRowsPerBlock + (int)(threadIdx.x >> 6);
  if (row >= nint) return;  // the whole wave
  const int lane = threadIdx.x & 63;
  const T* a = Ainv + (int64_t)row * nint;
  T acc = T(0);
#pragma unroll 8
  for (int j = lane; j < nint; j += 64) acc += a[j] * sb[j];
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) x[node_of(row)] = acc;
}

// ------------------------------------------------------------------ elementwise
template <typename T, bool GR> __global__ void k_copy(int64_t n, const T* a, T* o, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    a = shift(a, dk);
    o = shift(o, dk);
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i];
}
template <typename T, bool GR> __global__ void k_zero(int64_t n, T* o, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    o = shift(o, dk);
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = T(0);
}
template <typename T> __global__ void k_sub(int64_t n, const T* a, const T* b, T* o) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] - b[i];
}
template <typename T, bool GR> __global__ void k_axpy(int64_t n, T al, const T* x, T* y, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    x = shift(x, dk);
    y = shift(y, dk);
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = y[i] + al * x[i];
}
template <typename T> __global__ void k_scale_mul(int64_t n, T al, const T* a, const T* b, T* o) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = al * a[i] * b[i];
}
template <bool GR>
__global__ void k_c6432(int64_t n, const double* a, const double* rr, float* o, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    a = shift(a, dk);
    o = shift(o, dk);
    if (rr) rr = shift(rr, dk);
  }
  const double sc = rr ? pow2_inv_norm(*rr) : 1.0;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = (float)(a[i] * sc);
}
template <bool GR>
__global__ void k_c3264(int64_t n, const float* a, const double* rr, double* o, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    a = shift(a, dk);
    o = shift(o, dk);
    if (rr) rr = shift(rr, dk);
  }
  const double sc = rr ? 1.0 / pow2_inv_norm(*rr) : 1.0;  // exact: a power of two
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = (double)a[i] * sc;
}

__global__ void k_div(int64_t n, const double* a, double den, double* o) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] / den;
}
__global__ void k_sqrt(int64_t n, const double* a, double* o) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = sqrt(a[i]);
}
template <typename T> __global__ void k_recip_masked(int64_t n, T* v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = v[i] != T(0) ? T(1) / v[i] : T(0);
}

// Chebyshev start: r = b - t (t = A x; t == nullptr means x = 0 and r = b), d = dinv r / theta.
template <typename T, bool GR>
__global__ void k_cheb_start(int64_t n, const T* b, const T* t, const T* dinv, T theta, T* r, T* d,
                             const double* th, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    b = shift(b, dk);
    t = shift(t, dk);
    dinv = shift(dinv, dk);
    r = shift(r, dk);
    d = shift(d, dk);
    if (th) theta = (T)shift(th, dk)[0];
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T ri = b[i];
  if (t) {
    ri = ri - t[i];
    r[i] = ri;
  }
  d[i] = dinv[i] * ri / theta;
}

// One Chebyshev step after t = A d: x += d; r = rin - t; d = c1 d + (c2 dinv) r.
template <typename T>
__global__ void k_cheb_step(int64_t n, int from_zero, T* x, const T* rin, T* r, const T* t, T* d,
                            const T* dinv, T c1, T c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T di = d[i];
  x[i] = from_zero ? di : x[i] + di;
  const T ri = rin[i] - t[i];
  r[i] = ri;
  d[i] = c1 * di + (c2 * dinv[i]) * ri;
}

// Damped Jacobi: x += (omega dinv) (b - t), or x = (omega dinv) b from a zero guess.
template <typename T, bool GR>
__global__ void k_jacobi(int64_t n, int from_zero, T* x, const T* b, const T* t, const T* dinv, T om,
                         Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    x = shift(x, dk);
    b = shift(b, dk);
    t = shift(t, dk);
    dinv = shift(dinv, dk);
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (from_zero)
    x[i] = (om * dinv[i]) * b[i];
  else
    x[i] = x[i] + (om * dinv[i]) * (b[i] - t[i]);
}

// ------------------------------------------------------------------ deterministic reductions
// Each block accumulates a fixed strided subset in FP64 and reduces it by a fixed tree; a
// single block then sums the partials in a fixed tree. Same inputs and sizes give bitwise
// identical results.
__device__ inline double block_sum(double v) {
  __shared__ double sh[kT];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

template <typename T, bool GR>
__global__ void __launch_bounds__(kT) k_dot_partial(int64_t n, const T* a, const T* b, double* part,
                                                     Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    a = shift(a, dk);
    b = shift(b, dk);
    part = shift(part, dk);
  }
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    acc += (double)a[i] * (double)b[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// *out = the sum of the np partials; also to the pinned host scalar *hout if given (single
// problems only: it saves a separate copy before the host reads the value)
template <bool GR>
__global__ void __launch_bounds__(kT) k_sum_final(const double* part, int np, double* out,
                                                  double* hout, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    part = shift(part, dk);
    out = shift(out, dk);
    hout = nullptr;
  }
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kT) acc += part[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) {
    *out = s;
    if (hout) *hout = s;
  }
}


// ------------------------------------------------------------------ Lanczos building blocks
// Block-Gram-Schmidt against the basis V_0..V_{c-1} (columns of V with leading dimension ld):
// all c coefficients in one pass over w, then one update of w; every sum in a fixed order.
constexpr int kMdChunk = 8;

// part[v kMdBlocks + b] = the strided partial of V_v . w of block b, v = kMdChunk blockIdx.y + q
__global__ void __launch_bounds__(kT)
k_multidot(int64_t n, const double* V, int64_t ld, int c, const double* w, double* part) {
  __shared__ double sh[kMdChunk][kT];
  const int v0 = blockIdx.y * kMdChunk;
  double acc[kMdChunk];
#pragma unroll
  for (int q = 0; q < kMdChunk; ++q) acc[q] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double wi = w[i];
#pragma unroll
    for (int q = 0; q < kMdChunk; ++q)
      if (v0 + q < c) acc[q] += V[(int64_t)(v0 + q) * ld + i] * wi;
  }
  // the kMdChunk trees side by side (each the same tree as one at a time: bitwise the same
  // sums, with one barrier per level of the tree instead of one per level and coefficient)
#pragma unroll
  for (int q = 0; q < kMdChunk; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int q = 0; q < kMdChunk; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < kMdChunk && v0 + (int)threadIdx.x < c)
    part[(int64_t)(v0 + threadIdx.x) * kMdBlocks + blockIdx.x] = sh[threadIdx.x][0];
}

// coef[v] = sum over the np blocks of part[v kMdBlocks + b] (block v)
__global__ void __launch_bounds__(kT) k_md_final(const double* part, int np, double* coef) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < np; b += kT) acc += part[(int64_t)blockIdx.x * kMdBlocks + b];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) coef[blockIdx.x] = s;
}


// ------------------------------------------------------------------ Lanczos step, fused
// The vector passes of one Lanczos step, each doing what two of the kernels above do in turn,
// per entry with the same operations in the same order; those that end in a dot product run on
// the dot-product grid with its strided sums, so that every partial (and every result) is
// bitwise the one the separate kernels give.
// w = (1 sqd) w; partials of v . w
__global__ void __launch_bounds__(kT) k_lz_scale_dot(int64_t n, const double* sqd, double* w,
                                                     const double* v, double* part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double wi = 1.0 * sqd[i] * w[i];
    w[i] = wi;
    acc += v[i] * wi;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The sum of np partials, formed by every workgroup in k_sum_final's order (bitwise its
// result); the first workgroup also stores it to *out.
__device__ inline double sum_in_block(const double* part, int np, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kT) acc += part[i];
  const double s = block_sum(acc);
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = s;
  return s;
}

// alpha = the sum of the np partials; w = w - alpha vj, then (vjm1 != nullptr)
// w = w - sqrt(*n2) vjm1
__global__ void __launch_bounds__(kT) k_lz_axpy2(int64_t n, const double* part, int np,
                                                 double* alpha, const double* vj, const double* n2,
                                                 const double* vjm1, double* w) {
  const double a = sum_in_block(part, np, alpha);
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    double wi = w[i] + (-1.0 * a) * vj[i];
    if (vjm1) wi = wi + (-sqrt(n2[0])) * vjm1[i];
    w[i] = wi;
  }
}

// w -= sum_v coef[v] V_v (v ascending); partials of w . w
__global__ void __launch_bounds__(kT) k_md_sub_dot(int64_t n, const double* V, int64_t ld, int c,
                                                   const double* coef, double* w, double* part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    double wi = w[i];
    for (int v = 0; v < c; ++v) wi = wi - coef[v] * V[(int64_t)v * ld + i];
    w[i] = wi;
    acc += wi * wi;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// nn = the sum of the np partials (np = 0: nn = *n2); vn = w / sqrt(nn); t = (1 sqd) vn (w and
// vn may be the same vector)
__global__ void __launch_bounds__(kT) k_lz_next(int64_t n, const double* w, const double* part, int np,
                                                double* n2, const double* sqd, double* vn, double* t) {
  const double nn = np > 0 ? sum_in_block(part, np, n2) : n2[0];
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double v = w[i] / sqrt(nn);
    vn[i] = v;
    t[i] = 1.0 * sqd[i] * v;
  }
}

// dst[k cnt + i] = src[i] of problem k (blockIdx.y): a launch group's scalars side by side
__global__ void k_collect(const double* src, int cnt, double* dst, Grp gp) {
  int64_t dk;
  if (!grp_begin(gp, &dk)) return;
  if ((int)threadIdx.x < cnt) dst[(int64_t)blockIdx.y * cnt + threadIdx.x] = shift(src, dk)[threadIdx.x];
}

// alpha = scal[num] / scal[den]; x += alpha p; r -= alpha h; partial sums of r.r
template <bool GR>
__global__ void __launch_bounds__(kT)
k_pcg_xr(int64_t n, const double* scal, int inum, int iden, double* x, double* r, const double* p,
         const double* h, double* part, Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    scal = shift(scal, dk);
    x = shift(x, dk);
    r = shift(r, dk);
    p = shift(p, dk);
    h = shift(h, dk);
    part = shift(part, dk);
  }
  const double al = scal[inum] / scal[iden];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    x[i] = x[i] + al * p[i];
    const double ri = r[i] - al * h[i];
    r[i] = ri;
    acc += ri * ri;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta = scal[num] / scal[den]; p = z + beta p
template <bool GR>
__global__ void k_pcg_p(int64_t n, const double* scal, int inum, int iden, double* p, const double* z,
                        Grp gp) {
  if constexpr (GR) {
    int64_t dk;
    if (!grp_begin(gp, &dk)) return;
    scal = shift(scal, dk);
    p = shift(p, dk);
    z = shift(z, dk);
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double be = scal[inum] / scal[iden];
  p[i] = z[i] + be * p[i];
}

// Inner FP32 CG of the iterative refinement. alpha = scal[num] / scal[den] (FP64 dots of the
// FP32 vectors), applied in FP32: e += alpha p; r -= alpha h.
__global__ void __launch_bounds__(kT) k_ir_er(int64_t n, const double* scal, int inum, int iden,
                                              float* e, float* r, const float* p, const float* h) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float al = (float)(scal[inum] / scal[iden]);
  e[i] = e[i] + al * p[i];
  r[i] = r[i] - al * h[i];
}
// beta = scal[num] / scal[den]; p = z + beta p (FP32 vectors)
__global__ void __launch_bounds__(kT) k_ir_p(int64_t n, const double* scal, int inum, int iden,
                                             float* p, const float* z) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float be = (float)(scal[inum] / scal[iden]);
  p[i] = z[i] + be * p[i];
}
// x += e 2^k: the correction of the scaled residual back at the residual's scale (the power of
// two pow2_inv_norm(*rr) that scaled it), added in FP64
__global__ void __launch_bounds__(kT) k_ir_add(int64_t n, const float* e, const double* rr, double* x) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double sc = 1.0 / pow2_inv_norm(*rr);
  x[i] = x[i] + (double)e[i] * sc;
}

}  // namespace

void ir_update_er(int64_t n, const double* scal, int inum, int iden, float* e, float* r,
                  const float* p, const float* h, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  hipLaunchKernelGGL(k_ir_er, dim3(nb(n)), dim3(kT), 0, s, n, scal, inum, iden, e, r, p, h);
  GLLMG_HIP(hipGetLastError());
}
void ir_update_p(int64_t n, const double* scal, int inum, int iden, float* p, const float* z,
                 hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  hipLaunchKernelGGL(k_ir_p, dim3(nb(n)), dim3(kT), 0, s, n, scal, inum, iden, p, z);
  GLLMG_HIP(hipGetLastError());
}
void ir_add(int64_t n, const float* e, const double* rr, double* x, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  hipLaunchKernelGGL(k_ir_add, dim3(nb(n)), dim3(kT), 0, s, n, e, rr, x);
  GLLMG_HIP(hipGetLastError());
}

void launch_coarse_solve(const Level& L, int prec, const void* b, void* x, hipStream_t s) {
  GLLMG_CHECK(L.nint <= 4096, GLLMG_EUNSUPPORTED, "coarsest level above 4096 unknowns");
  const int nint = (int)L.nint;
  const unsigned nbn = (unsigned)((L.g.N + kCT - 1) / kCT);
  const dim3 grid(nbn + (unsigned)((nint + kRowsPerBlock - 1) / kRowsPerBlock), grp_count());
  if (prec == 0)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_coarse<double, GR>), grid, dim3(kCT), sizeof(double) * nint, s, L.Ainv64,
                         nint, (const double*)b, (double*)x, L.g, nbn, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_coarse<float, GR>), grid, dim3(kCT), sizeof(float) * nint, s, L.Ainv32,
                         nint, (const float*)b, (float*)x, L.g, nbn, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}

// A plain streaming copy, 16 bytes per lane (the achievable-bandwidth reference of the
// roofline figures): one read and one write of every byte.
__global__ void __launch_bounds__(256) k_stream_copy(int64_t n16, const uint4* __restrict__ a,
                                                     uint4* __restrict__ o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) o[i] = a[i];
}

void stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s, n16,
                     (const uint4*)src, (uint4*)dst);
  GLLMG_HIP(hipGetLastError());
}

void vec_copy(int prec, int64_t n, const void* a, void* o, hipStream_t s) {
  if (prec == 0)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_copy<double, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, (const double*)a, (double*)o, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_copy<float, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, (const float*)a, (float*)o, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}
void vec_zero(int prec, int64_t n, void* o, hipStream_t s) {
  if (prec == 0)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_zero<double, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, (double*)o, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_zero<float, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, (float*)o, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}
void vec_sub(int prec, int64_t n, const void* a, const void* b, void* o, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  if (prec == 0)
    hipLaunchKernelGGL(k_sub<double>, dim3(nb(n)), dim3(kT), 0, s, n, (const double*)a,
                       (const double*)b, (double*)o);
  else
    hipLaunchKernelGGL(k_sub<float>, dim3(nb(n)), dim3(kT), 0, s, n, (const float*)a,
                       (const float*)b, (float*)o);
  GLLMG_HIP(hipGetLastError());
}
void vec_axpy(int prec, int64_t n, double al, const void* x, void* y, hipStream_t s) {
  if (prec == 0)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_axpy<double, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, al, (const double*)x, (double*)y, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_axpy<float, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, (float)al, (const float*)x,
                       (float*)y, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}
void vec_scale_mul(int prec, int64_t n, double al, const void* a, const void* b, void* o,
                   hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  if (prec == 0)
    hipLaunchKernelGGL(k_scale_mul<double>, dim3(nb(n)), dim3(kT), 0, s, n, al, (const double*)a,
                       (const double*)b, (double*)o);
  else
    hipLaunchKernelGGL(k_scale_mul<float>, dim3(nb(n)), dim3(kT), 0, s, n, (float)al,
                       (const float*)a, (const float*)b, (float*)o);
  GLLMG_HIP(hipGetLastError());
}
void vec_div(int64_t n, const double* a, double den, double* o, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  hipLaunchKernelGGL(k_div, dim3(nb(n)), dim3(kT), 0, s, n, a, den, o);
  GLLMG_HIP(hipGetLastError());
}
void vec_sqrt(int64_t n, const double* a, double* o, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  hipLaunchKernelGGL(k_sqrt, dim3(nb(n)), dim3(kT), 0, s, n, a, o);
  GLLMG_HIP(hipGetLastError());
}
void vec_recip_masked(int prec, int64_t n, void* v, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  if (prec == 0)
    hipLaunchKernelGGL(k_recip_masked<double>, dim3(nb(n)), dim3(kT), 0, s, n, (double*)v);
  else
    hipLaunchKernelGGL(k_recip_masked<float>, dim3(nb(n)), dim3(kT), 0, s, n, (float*)v);
  GLLMG_HIP(hipGetLastError());
}
void cast_64_32(int64_t n, const double* a, float* o, hipStream_t s, const double* rr) {
  with_gr([&](auto gr) {
    constexpr bool GR = decltype(gr)::value;
    hipLaunchKernelGGL((k_c6432<GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, a, rr, o, cur_grp());
  });
  GLLMG_HIP(hipGetLastError());
}
void cast_32_64(int64_t n, const float* a, double* o, hipStream_t s, const double* rr) {
  with_gr([&](auto gr) {
    constexpr bool GR = decltype(gr)::value;
    hipLaunchKernelGGL((k_c3264<GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, a, rr, o, cur_grp());
  });
  GLLMG_HIP(hipGetLastError());
}
void cheb_start(int prec, int64_t n, const void* b, const void* t, const void* dinv, double theta,
                void* r, void* d, hipStream_t s, const double* th) {
  if (prec == 0)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_cheb_start<double, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, (const double*)b,
                       (const double*)t, (const double*)dinv, theta, (double*)r, (double*)d, th,
                       cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_cheb_start<float, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, (const float*)b,
                       (const float*)t, (const float*)dinv, (float)theta, (float*)r, (float*)d, th,
                       cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}
void cheb_step(int prec, int64_t n, int from_zero, void* x, const void* rin, void* r, const void* t,
               void* d, const void* dinv, double c1, double c2, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  if (prec == 0)
    hipLaunchKernelGGL(k_cheb_step<double>, dim3(nb(n)), dim3(kT), 0, s, n, from_zero, (double*)x,
                       (const double*)rin, (double*)r, (const double*)t, (double*)d,
                       (const double*)dinv, c1, c2);
  else
    hipLaunchKernelGGL(k_cheb_step<float>, dim3(nb(n)), dim3(kT), 0, s, n, from_zero, (float*)x,
                       (const float*)rin, (float*)r, (const float*)t, (float*)d,
                       (const float*)dinv, (float)c1, (float)c2);
  GLLMG_HIP(hipGetLastError());
}
void jacobi_step(int prec, int64_t n, int from_zero, void* x, const void* b, const void* t,
                 const void* dinv, double om, hipStream_t s) {
  if (prec == 0)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_jacobi<double, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, from_zero, (double*)x,
                       (const double*)b, (const double*)t, (const double*)dinv, om, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_jacobi<float, GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, from_zero, (float*)x,
                       (const float*)b, (const float*)t, (const float*)dinv, (float)om, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
}
void dot(int prec, int64_t n, const void* a, const void* b, double* part, double* res,
         hipStream_t s, double* hres) {
  const int g = dot_grid(n);
  if (prec == 0)
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_dot_partial<double, GR>), dim3(g, grp_count()), dim3(kT), 0, s, n, (const double*)a,
                       (const double*)b, part, cur_grp());
    });
  else
    with_gr([&](auto gr) {
      constexpr bool GR = decltype(gr)::value;
      hipLaunchKernelGGL((k_dot_partial<float, GR>), dim3(g, grp_count()), dim3(kT), 0, s, n, (const float*)a,
                       (const float*)b, part, cur_grp());
    });
  GLLMG_HIP(hipGetLastError());
  with_gr([&](auto gr) {
    constexpr bool GR = decltype(gr)::value;
    hipLaunchKernelGGL((k_sum_final<GR>), dim3(1, grp_count()), dim3(kT), 0, s, (const double*)part, g, res,
                       hres, cur_grp());
  });
  GLLMG_HIP(hipGetLastError());
}
void pcg_update_xr(int64_t n, const double* scal, int inum, int iden, double* x, double* r,
                   const double* p, const double* h, double* part, double* rr, hipStream_t s,
                   double* hrr) {
  const int g = dot_grid(n);
  with_gr([&](auto gr) {
    constexpr bool GR = decltype(gr)::value;
    hipLaunchKernelGGL((k_pcg_xr<GR>), dim3(g, grp_count()), dim3(kT), 0, s, n, scal, inum, iden, x, r, p, h, part, cur_grp());
  });
  GLLMG_HIP(hipGetLastError());
  with_gr([&](auto gr) {
    constexpr bool GR = decltype(gr)::value;
    hipLaunchKernelGGL((k_sum_final<GR>), dim3(1, grp_count()), dim3(kT), 0, s, (const double*)part, g, rr, hrr,
                       cur_grp());
  });
  GLLMG_HIP(hipGetLastError());
}
void lanczos_scale_dot(int64_t n, const double* sqd, double* w, const double* v, double* part,
                       hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  hipLaunchKernelGGL(k_lz_scale_dot, dim3(dot_grid(n)), dim3(kT), 0, s, n, sqd, w, v, part);
  GLLMG_HIP(hipGetLastError());
}
void lanczos_axpy2(int64_t n, const double* part, int np, double* alpha, const double* vj,
                   const double* n2, const double* vjm1, double* w, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  GLLMG_CHECK(np >= 1 && np <= kDotBlocks, GLLMG_EINVAL, "partial count out of range");
  hipLaunchKernelGGL(k_lz_axpy2, dim3(dot_grid(n)), dim3(kT), 0, s, n, part, np, alpha, vj, n2, vjm1, w);
  GLLMG_HIP(hipGetLastError());
}
void block_orthogonalize(int64_t n, const double* V, int64_t ld, int c, double* w, double* part,
                         double* coef, double* npart, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  GLLMG_CHECK(c >= 1, GLLMG_EINVAL, "empty basis");
  const int g = (int)std::min<int64_t>(kMdBlocks, std::max<int64_t>(1, (n + kT - 1) / kT));
  hipLaunchKernelGGL(k_multidot, dim3(g, (c + kMdChunk - 1) / kMdChunk), dim3(kT), 0, s, n, V, ld, c,
                     (const double*)w, part);
  GLLMG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_md_final, dim3(c), dim3(kT), 0, s, (const double*)part, g, coef);
  GLLMG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_md_sub_dot, dim3(dot_grid(n)), dim3(kT), 0, s, n, V, ld, c, (const double*)coef, w,
                     npart);
  GLLMG_HIP(hipGetLastError());
}
void lanczos_next(int64_t n, const double* w, const double* part, int np, double* n2,
                  const double* sqd, double* vn, double* t, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  GLLMG_CHECK(np >= 0 && np <= kDotBlocks && (np == 0 || part), GLLMG_EINVAL, "partial count out of range");
  hipLaunchKernelGGL(k_lz_next, dim3(dot_grid(n)), dim3(kT), 0, s, n, w, part, np, n2, sqd, vn, t);
  GLLMG_HIP(hipGetLastError());
}
void sum_partials(const double* part, int np, double* out, hipStream_t s) {
  GLLMG_CHECK(!launch_group(), GLLMG_EINVAL, "kernel without launch-group support");
  hipLaunchKernelGGL((k_sum_final<false>), dim3(1), dim3(kT), 0, s, part, np, out, (double*)nullptr,
                     Grp{nullptr, nullptr});
  GLLMG_HIP(hipGetLastError());
}
void collect_scalars(const double* src, int cnt, double* dst, hipStream_t s) {
  GLLMG_CHECK(cnt >= 1 && cnt <= 64, GLLMG_EINVAL, "scalar count out of range");
  hipLaunchKernelGGL(k_collect, dim3(1, grp_count()), dim3(64), 0, s, src, cnt, dst, cur_grp());
  GLLMG_HIP(hipGetLastError());
}
void pcg_update_p(int64_t n, const double* scal, int inum, int iden, double* p, const double* z,
                  hipStream_t s) {
  with_gr([&](auto gr) {
    constexpr bool GR = decltype(gr)::value;
    hipLaunchKernelGGL((k_pcg_p<GR>), dim3(nb(n), grp_count()), dim3(kT), 0, s, n, scal, inum, iden, p, z, cur_grp());
  });
  GLLMG_HIP(hipGetLastError());
}

}  // namespace gllmg
