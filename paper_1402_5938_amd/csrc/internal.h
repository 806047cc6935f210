// Internal declarations of the gllmg library: level data, kernel launchers, host helpers.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/gllmg.h"

namespace gllmg {

// 2^-e with 2^e within a factor sqrt(2) of sqrt(rr), the norm of a vector r with (r, r) = rr:
// r 2^-e has norm about 1. A power of two scales exactly in FP64 and FP32 while no value leaves
// the normal range, so an FP32 V-cycle of r 2^-e, scaled back by 2^e, equals bitwise the FP32
// V-cycle of r itself wherever that neither overflows nor underflows, and keeps residuals far
// outside FP32's range (below 1e-38 or above 3e38) representable. 1 for rr = 0 or not finite.
__host__ __device__ inline double pow2_inv_norm(double rr) {
  if (!(rr > 0.0) || !(rr <= 1.7976931348623157e308)) return 1.0;
  int k = 0;
  (void)frexp(rr, &k);  // rr in [2^(k-1), 2^k)
  return ldexp(1.0, -(k >> 1));
}

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  gllmg_status status;
  Error(gllmg_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define GLLMG_HIP(call)                                                                   \
  do {                                                                                    \
    hipError_t _e = (call);                                                               \
    if (_e != hipSuccess)                                                                 \
      throw ::gllmg::Error(GLLMG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define GLLMG_CHECK(cond, status, msg)                        \
  do {                                                        \
    if (!(cond)) throw ::gllmg::Error((status), (msg));       \
  } while (0)

// ------------------------------------------------------------------ fields (device view)
struct FieldDev {
  int kind;
  int nmodes;
  double param[12];
  const double* modes;   // device pointer, nmodes x 5
};

// ------------------------------------------------------------------ mesh geometry (device view)
struct Grid {
  int dim;
  int p;             // order
  int ne[3];         // elements per axis (ne[2] = 1 in 2D)
  int nn[3];         // nodes per axis = ne * p + 1 (nn[2] = 1 in 2D)
  int64_t E;         // elements
  int64_t N;         // nodes
  double rnn[2];     // 1 / nn[0], 1 / nn[1] (node index -> grid row -> plane without integer division)
};

// floor(n / d) for n < 2^32, 0 < d < 2^30, with r = 1.0 / d: the FP64 product is within one of
// the quotient (its rounding error is below 2^32 * 2^-52), and one step corrects it.
__host__ __device__ inline uint32_t div_by_recip(uint32_t n, uint32_t d, double r) {
  uint32_t q = (uint32_t)((double)n * r);
  int32_t rem = (int32_t)(n - q * d);
  if (rem < 0) {
    --q;
    rem += (int32_t)d;
  }
  if (rem >= (int32_t)d) ++q;
  return q;
}

// Transfer from a level to the next coarser one: the 1D matrix Pl[child][i][c] (child < nch;
// nch = 1 under p-coarsening, 2 under h-coarsening) evaluating coarse element basis function c
// at fine element node i, the same for every element and axis of the uniform mesh.
struct Xfer {
  int nch = 1;
  double* P64 = nullptr;  // device, nch * n_fine * n_coarse
  float* P32 = nullptr;
};

struct Level {
  Grid g;
  bool gauss = false;     // Gauss quadrature (else collocated GLL)
  int n;                  // p + 1
  int64_t nint;           // interior nodes
  int64_t npts;           // E * n^d quadrature points
  int ncomp;              // unique G entries per point (3 in 2D, 6 in 3D)
  double* G64 = nullptr;  // [E][ncomp][n^d]
  float* G32 = nullptr;
  double* D64 = nullptr;  // n x n derivative matrix, D[i*n + l] = l_l'(xi_i), then its transpose
  float* D32 = nullptr;
  double* xi64 = nullptr; // GLL nodes and weights of the level's order
  double* w64 = nullptr;
  double* Iq64 = nullptr; // Gauss quadrature: basis and derivative at the Gauss points (n x n)
  float* Iq32 = nullptr;
  double* Dq64 = nullptr;
  float* Dq32 = nullptr;
  double* wg64 = nullptr; // Gauss weights
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  double* l1inv64 = nullptr;  // l1-Jacobi smoother: 1 / sum_j |A_ij| (interior), else unused
  float* l1inv32 = nullptr;
  double* Binv64 = nullptr;   // block Jacobi: E inverted padded blocks of p^d x p^d
  float* Binv32 = nullptr;
  double lmax = 0.0;
  // V-cycle scratch in the V-cycle precision (and an FP64 set for FP64 calls)
  void* vb[2] = {nullptr, nullptr};
  void* vx[2] = {nullptr, nullptr};
  void* vr[2] = {nullptr, nullptr};
  void* vd[2] = {nullptr, nullptr};
  void* vd2[2] = {nullptr, nullptr};  // Chebyshev directions alternate between vd and vd2
  void* vd3[2] = {nullptr, nullptr};  // degree 4: the third direction, kept to the last step
  // transfer to the next coarser level (if any)
  bool has_coarse = false;
  Xfer tp;  // to the next coarser level
  // exact solve (coarsest level): dense inverse of the interior block
  const void* zero = nullptr;  // 64 zero bytes in device memory (a load source for masked lanes)
  double* Ainv64 = nullptr;
  float* Ainv32 = nullptr;
  // Chebyshev coefficients on the device: pair 0 = (theta, delta), pair i = (c1, c2) of step i
  double* ctab = nullptr;
  int64_t applies = 0;
};

// bump allocator over one device region
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  bool dry = false;   // only count
  void* take(size_t bytes) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + bytes;
    if (dry) return nullptr;
    if (used > size) throw Error(GLLMG_ENOMEM, "device workspace too small");
    return base + off;
  }
};

// ------------------------------------------------------------------ host reference element (FP64)
struct RefElem {
  int p;
  std::vector<double> xi, w, D;   // D[i*(p+1)+l] = l_l'(xi_i)
  std::vector<double> lam;        // barycentric weights of the nodes xi
  // Gauss-Legendre rule with p+1 points: eta, wg; the basis at the points Iq[q*(p+1)+i] =
  // l_i(eta_q) and its derivative Dq = Iq D (l_i' has degree p, so it equals its interpolant)
  std::vector<double> eta, wg, Iq, Dq;
};
RefElem ref_element(int p);
// fills eta, wg, Iq, Dq of re (after ref_element)
void gauss_rule(RefElem& re);
// Lagrange basis of the order-p GLL nodes evaluated at point y: out[j] = l_j(y).
void lagrange_at(const RefElem& re, double y, double* out);
// Largest eigenvalue of the symmetric tridiagonal matrix (diag a[0..m-1], offdiag b[0..m-2]).
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b);
// In-place inverse of a dense SPD matrix (row-major n x n) via Cholesky; false if not SPD.
bool spd_inverse(std::vector<double>& A, int n);

// ------------------------------------------------------------------ kernel launchers
// precision index: 0 = double, 1 = float
// Geometric factors of a level from the physical coordinates xn (N x dim) and mu (N) at its nodes
void launch_geometry(const Level& L, const double* xn, const double* mun, double* G64,
                     float* G32, double* wdet, int* flag, hipStream_t s);
// nodal coordinates and mu of a grid whose node (i, j, k) is node stride * (i, j, k) of grid g0
void launch_subsample_nodal(const Grid& g0, const Grid& g, int stride, const double* xn0,
                            const double* mu0, double* xn, double* mu, hipStream_t s);
// a field at given physical node coordinates xn (N x dim)
void launch_field_at(const Grid& g, const double* xn, const FieldDev& f, double* out, hipStream_t s);
void launch_gather_full(const Level& L, const double* elem_vals, double* out, hipStream_t s);
void launch_node_coords(const Grid& g, const double* xi, const FieldDev& map, double* out,
                        hipStream_t s);
void launch_eval_field(const Grid& g, const double* xi, const FieldDev& map, const FieldDev& f,
                       double* out, hipStream_t s);
void launch_rhs(const Grid& g, const double* mass, const double* f, double* b, hipStream_t s);
void launch_diag(const Level& L, double* diag, double* F, hipStream_t s);
void launch_dinv(const Grid& g, const double* diag, double* dinv64, float* dinv32, int* flag,
                 hipStream_t s);

// What a product y = A x does with each output value (the update is fused into the product):
//  STORE:    y = A x
//  RESIDUAL: r = b - A x
//  JACOBI:   x = x + (omega dinv) (b - A x)                    (in place; the input is x)
//  CHEB_START: r = b - A x, d = dinv r / c1                    (c1 = theta)
//  CHEB:     with t = A d: x = x + d (or x = d), r = rin - t,
//            d = c1 d + (c2 dinv) r                             (in place; the input is d)
//  CHEB_D:   CHEB without the x update (r and the next d only)
//  CHEB_SUM: the polynomial's last step with the x updates of the CHEB_D steps before it:
//            x = (((x + e0) + e1) + d) + (c1 d + (c2 dinv) (rin - t)), the terms in the order
//            of the step-by-step updates (x omitted when from_zero, e1 when null)
// and, for sums that are not products (the restriction's gather, s = the summed value):
//  STORE_CHEB0:   y = s, d = dinv s / c1      (first Chebyshev step from x = 0, c1 = theta)
//  STORE_JACOBI0: y = s, x = (om dinv) s      (first Jacobi step from x = 0)
// At Dirichlet boundary nodes every output is 0.
enum EpiMode {
  EPI_STORE = 0,
  EPI_RESIDUAL = 1,
  EPI_JACOBI = 2,
  EPI_CHEB = 3,
  EPI_CHEB_START = 4,
  EPI_STORE_CHEB0 = 5,
  EPI_STORE_JACOBI0 = 6,
  EPI_CHEB_D = 7,
  EPI_CHEB_SUM = 8
};
struct Epi {
  int mode = EPI_STORE;
  int from_zero = 0;
  int last = 0;  // CHEB: also add the next d into x; r and d are not written
  void* y = nullptr;
  const void* b = nullptr;
  void* x = nullptr;
  const void* rin = nullptr;
  void* r = nullptr;
  void* d = nullptr;
  const void* dinv = nullptr;
  const void* e0 = nullptr;  // CHEB_SUM: earlier directions
  const void* e1 = nullptr;
  double c1 = 0, c2 = 0, om = 0;
  // when set: c1, c2 are read on the device from cc[0], cc[1] (per problem in a launch group)
  const double* cc = nullptr;
};

// Launch groups: several problems of one shape in each launch (batched solves). Problem k's
// device buffers lie at the same offsets in its workspace as problem 0's, so a kernel reaches
// them by adding dlt[k] bytes to the pointers it was given for problem 0; act[k] == 0 skips
// problem k. Kernels take a Grp argument ({nullptr, nullptr}: one problem) and run problem
// blockIdx.y; launches made while a LaunchGroup is current have gridDim.y = count.
struct Grp {
  const int64_t* dlt;
  const int* act;
};
struct LaunchGroup {
  Grp g;
  int count;
};
const LaunchGroup* launch_group();          // the current group of this thread, or nullptr
void set_launch_group(const LaunchGroup* g);
inline Grp cur_grp() {
  const LaunchGroup* g = launch_group();
  return g ? g->g : Grp{nullptr, nullptr};
}
inline unsigned grp_count() {
  const LaunchGroup* g = launch_group();
  return g ? (unsigned)g->count : 1u;
}
// f(std::true_type) inside a launch group, else f(std::false_type): launchers pick the kernel
// instance with or without the group code
template <class F>
void with_gr(F&& f) {
  if (launch_group())
    f(std::true_type{});
  else
    f(std::false_type{});
}
void launch_apply(const Level& L, int prec, int neumann, const void* x, const Epi& ep, void* F,
                  hipStream_t s);
size_t face_buffer_elems(const Level& L);

// Multicolor Gauss-Seidel (SSOR smoother): x_i += omega dinv_i (b_i - (A x)_i) at every
// interior node of one color (0 <= color < n^2); x must be 0 at boundary nodes
void launch_gs_color(const Level& L, int prec, const void* b, void* x, const void* dinv, int color,
                     double omega, hipStream_t s);
void zero_boundary(const Level& L, int prec, void* v, hipStream_t s);
// l1 row sums of the interior block, sum_j |A_ij| over interior j (0 at boundary rows); FP64
void launch_l1_rowsum(const Level& L, double* out, hipStream_t s);
// Element block Jacobi: P = p^d slots per element; B = E padded P x P blocks (FP64), filled with
// the assembled owned-node blocks and inverted in place (flag bit 8: a non-positive pivot)
int block_slots(const Level& L);
void launch_block_setup(const Level& L, double* B, int* flag, hipStream_t s);
// x += omega Binv^T r per element block (the owned interior nodes)
void launch_block_apply(const Level& L, int prec, const void* Binv, const void* r, void* x,
                        double omega, hipStream_t s);

// The allocation-free product's element-vector buffer: a file-scope device array of this many
// bytes (one per device, shared by every call on that device). static_scratch(dev) returns its
// device address on device dev, looked up once per device.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
void* static_scratch(int dev);

// Node-order sum of element vectors R (layout [e][k][j][i] on level L) followed by the epilogue.
void launch_gather_epi(const Level& L, int prec, const void* R, const Epi& ep, hipStream_t s);
// ... with the product's input xin (read by the in-place epilogues) and the boundary rule
void launch_gather_in(const Level& L, int prec, const void* R, const void* xin, int neumann,
                      const Epi& ep, hipStream_t s);

// Gauss quadrature (k_gauss.hip): the product (element pass + gather), the physical Gauss points
// (E n^d x dim), a field at given points, the geometric factors and w~ detJ, the diagonal and
// the consistent mass on element vectors (FP64)
void launch_apply_gauss(const Level& L, int prec, int neumann, const void* x, const Epi& ep,
                        void* F, hipStream_t s);
void launch_gauss_points(const Level& L, const double* xn, double* xq, hipStream_t s);
void launch_field_pts(int64_t npts, int dim, const double* pts, const FieldDev& f, double* out,
                      hipStream_t s);
void launch_geometry_gauss(const Level& L, const double* xn, const double* muq, double* G64,
                           float* G32, double* wdetq, int* flag, hipStream_t s);
void launch_diag_gauss(const Level& L, double* diag, double* F, hipStream_t s);
void launch_mass_gauss(const Level& L, const double* f, const double* wdetq, double* F,
                       hipStream_t s);

// xf = P xc (or xf += P xc)
void launch_prolong(const Level& fine, const Level& coarse, int prec, const void* xc, void* xf,
                    bool add, hipStream_t s);
// P^T rf summed into the coarse level's epilogue ep (EPI_STORE: ep.y = P^T rf); R is a buffer
// of restrict_buffer_elems elements of the precision
void launch_restrict(const Level& fine, const Level& coarse, int prec, const void* rf,
                     const Epi& ep, void* R, hipStream_t s);
size_t restrict_buffer_elems(const Level& fine, const Level& coarse);

void launch_coarse_solve(const Level& L, int prec, const void* b, void* x, hipStream_t s);

// elementwise vector kernels (prec 0 = double, 1 = float); scalars are passed in FP64
void vec_copy(int prec, int64_t n, const void* a, void* out, hipStream_t s);
void stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);  // bytes % 16 == 0
void vec_zero(int prec, int64_t n, void* out, hipStream_t s);
void vec_sub(int prec, int64_t n, const void* a, const void* b, void* out, hipStream_t s);  // a - b
void vec_axpy(int prec, int64_t n, double alpha, const void* x, void* y, hipStream_t s);   // y += a x
void vec_scale_mul(int prec, int64_t n, double alpha, const void* a, const void* b, void* out,
                   hipStream_t s);                                                          // alpha a*b
void vec_div(int64_t n, const double* a, double den, double* out, hipStream_t s);       // a / den
void vec_sqrt(int64_t n, const double* a, double* out, hipStream_t s);
void vec_recip_masked(int prec, int64_t n, void* v, hipStream_t s);     // v = v ? 1/v : 0
// Casts between the FP64 and FP32 vectors; with rr (the device (r, r) of the FP64 vector that the
// FP32 one stands for) both scale by pow2_inv_norm(*rr): out = float(a * 2^-e), then
// out = double(a) * 2^e.
void cast_64_32(int64_t n, const double* a, float* out, hipStream_t s, const double* rr = nullptr);
void cast_32_64(int64_t n, const float* a, double* out, hipStream_t s, const double* rr = nullptr);
// Chebyshev / Jacobi fused updates
// d = dinv (b - t) / theta (r = b - t when t is given); th, when given, holds theta on the
// device (per problem in a launch group) and replaces the argument
void cheb_start(int prec, int64_t n, const void* b, const void* t, const void* dinv,
                double theta, void* r, void* d, hipStream_t s, const double* th = nullptr);
void cheb_step(int prec, int64_t n, int x_from_zero, void* x, const void* rin, void* r,
               const void* t, void* d, const void* dinv, double c1, double c2, hipStream_t s);
void jacobi_step(int prec, int64_t n, int x_from_zero, void* x, const void* b, const void* t,
                 const void* dinv, double omega, hipStream_t s);
// deterministic dot products (FP64 result written to a device scalar)
constexpr int kDotBlocks = 1024;
constexpr int kDotThreads = 256;  // threads of the dot-product and CG-update blocks
// blocks of the dot products and CG updates for vectors of n entries (a function of n alone, so
// that every reduction over such a vector adds its entries in one fixed order)
__host__ __device__ inline int dot_grid(int64_t n) {
  const int64_t g = (n + kDotThreads - 1) / kDotThreads;
  return (int)(g < kDotBlocks ? (g < 1 ? 1 : g) : kDotBlocks);
}
// hresult: also into this pinned host scalar (or nullptr; ignored in launch groups)
void dot(int prec, int64_t n, const void* a, const void* b, double* partials, double* result,
         hipStream_t s, double* hresult = nullptr);
// scalar(s) in device memory for the PCG iteration
void pcg_update_xr(int64_t n, const double* scal, int i_num, int i_den, double* x, double* r,
                   const double* p, const double* h, double* partials, double* rr, hipStream_t s,
                   double* hrr = nullptr);
// Lanczos: w -= V (V^T w) against the c basis vectors V_v = V + v ld (one classical
// Gram-Schmidt pass: all coefficients from the same w, fixed-order sums), leaving the dot
// product's partials of w . w in npart (dot_grid(n) of them). part holds c kMdBlocks doubles,
// coef c. The multi-dot takes as many workgroups as a dot product: with one per compute unit
// it read a 57M-node basis at 1.6 TB/s.
constexpr int kMdBlocks = kDotBlocks;
void block_orthogonalize(int64_t n, const double* V, int64_t ld, int c, double* w, double* part,
                         double* coef, double* npart, hipStream_t s);
// Fused vector passes of a Lanczos step (the same arithmetic and reduction order as separate
// dot, sum and update kernels; each sum of np partials is formed by every workgroup that needs
// it, in the final-sum kernel's order, and stored by the first): w = sqd w with the partials of
// v . w in part (dot_grid(n) of them); *alpha = the sum of np partials, then w = w - *alpha vj
// - sqrt(*n2) vjm1 (the last term only if vjm1); *n2 = the sum of np partials (np = 0: *n2 is
// given), then vn = w / sqrt(*n2) and t = sqd vn; *out = the sum of np partials.
void lanczos_scale_dot(int64_t n, const double* sqd, double* w, const double* v, double* part,
                       hipStream_t s);
void lanczos_axpy2(int64_t n, const double* part, int np, double* alpha, const double* vj,
                   const double* n2, const double* vjm1, double* w, hipStream_t s);
void lanczos_next(int64_t n, const double* w, const double* part, int np, double* n2,
                  const double* sqd, double* vn, double* t, hipStream_t s);
void sum_partials(const double* part, int np, double* out, hipStream_t s);
// dst[k cnt + i] = scal[i] (src = the first problem's scalars) for every active problem k of
// the current launch group (dst is not shifted: one buffer for the group)
void collect_scalars(const double* src, int cnt, double* dst, hipStream_t s);
// iterative refinement: e += a p, r -= a h with a = scal[num] / scal[den] (FP32 vectors);
// p = z + b p with b = scal[num] / scal[den]; x += e times the power of two that undoes the
// scaling of the residual whose (r, r) is *rr
void ir_update_er(int64_t n, const double* scal, int i_num, int i_den, float* e, float* r,
                  const float* p, const float* h, hipStream_t s);
void ir_update_p(int64_t n, const double* scal, int i_num, int i_den, float* p, const float* z,
                 hipStream_t s);
void ir_add(int64_t n, const float* e, const double* rr, double* x, hipStream_t s);
void pcg_update_p(int64_t n, const double* scal, int i_num, int i_den, double* p,
                  const double* z, hipStream_t s);
// e = 1 at the interior nodes whose interior indices are (ox, oy, oz) mod c, 0 elsewhere
void color_unit_vector(const Grid& g, int c, int ox, int oy, int oz, double* e, hipStream_t s);
void start_vector(const Grid& g, uint64_t seed, int level, double* v, hipStream_t s);

}  // namespace gllmg
