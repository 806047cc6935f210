// Host side of the library: hierarchy planning, workspace layout, setup, smoothers, V-cycle,
// solvers and the C ABI declared in include/gllmg.h.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "batch_desc.h"
#include "internal.h"

namespace gllmg {

namespace {

struct LevelSpec {
  int ne[3];
  int p;
};

int64_t interior_count(int dim, const int ne[3], int p) {
  int64_t c = 1;
  for (int a = 0; a < dim; ++a) c *= (int64_t)ne[a] * p - 1;
  return c;
}

void validate(const gllmg_config& c) {
  GLLMG_CHECK(c.dim == 2 || c.dim == 3, GLLMG_EINVAL, "dim must be 2 or 3");
  GLLMG_CHECK(c.order >= 1 && c.order <= 16, GLLMG_EINVAL, "order must be in [1, 16]");
  for (int a = 0; a < c.dim; ++a)
    GLLMG_CHECK(c.nelem[a] >= 1 && (int64_t)c.nelem[a] * c.order + 1 < (1 << 30), GLLMG_EINVAL,
                "nelem out of range");
  GLLMG_CHECK(c.hierarchy == GLLMG_HIER_H || c.hierarchy == GLLMG_HIER_P ||
                  c.hierarchy == GLLMG_HIER_LOW,
              GLLMG_EINVAL, "hierarchy must be GLLMG_HIER_H, GLLMG_HIER_P or GLLMG_HIER_LOW");
  GLLMG_CHECK(c.hierarchy != GLLMG_HIER_LOW || (c.low_cycles >= 1 && c.low_cycles <= 64),
              GLLMG_EINVAL, "low_cycles must be in [1, 64]");
  GLLMG_CHECK(c.coarse_unknowns >= 0 && c.coarse_unknowns <= 4096, GLLMG_EINVAL,
              "coarse_unknowns must be in [0, 4096]");
  GLLMG_CHECK(c.ir_inner >= 0 && c.ir_inner <= 100, GLLMG_EINVAL, "ir_inner must be in [0, 100]");
  GLLMG_CHECK(c.ir_inner == 0 || c.vcycle_prec == GLLMG_F32, GLLMG_EINVAL,
              "iterative refinement (ir_inner > 0) runs the FP32 V-cycle: vcycle_prec must be F32");
  GLLMG_CHECK(c.hierarchy != GLLMG_HIER_LOW || c.quadrature == GLLMG_QUAD_GLL, GLLMG_EUNSUPPORTED,
              "the first-order hierarchy is built for GLL collocation");
  GLLMG_CHECK(c.smoother == GLLMG_SMOOTH_JACOBI || c.smoother == GLLMG_SMOOTH_CHEBYSHEV ||
                  c.smoother == GLLMG_SMOOTH_SSOR || c.smoother == GLLMG_SMOOTH_L1_JACOBI ||
                  c.smoother == GLLMG_SMOOTH_BLOCK_JACOBI,
              GLLMG_EINVAL, "unknown smoother");
  GLLMG_CHECK(c.quadrature == GLLMG_QUAD_GLL || c.quadrature == GLLMG_QUAD_GAUSS, GLLMG_EINVAL,
              "quadrature must be GLLMG_QUAD_GLL or GLLMG_QUAD_GAUSS");
  GLLMG_CHECK(c.quadrature == GLLMG_QUAD_GLL || c.smoother == GLLMG_SMOOTH_JACOBI ||
                  c.smoother == GLLMG_SMOOTH_CHEBYSHEV,
              GLLMG_EUNSUPPORTED,
              "the Gauss-quadrature operator takes the Jacobi and Chebyshev smoothers");
  if (c.smoother == GLLMG_SMOOTH_BLOCK_JACOBI) {
    int P = 1;
    for (int a = 0; a < c.dim; ++a) P *= c.order;
    GLLMG_CHECK(P <= 1024, GLLMG_EUNSUPPORTED,
                "block Jacobi needs element blocks of at most 1024 unknowns (p^d <= 1024)");
  }
  GLLMG_CHECK(c.nu_pre >= 0 && c.nu_post >= 0 && c.nu_pre <= 64 && c.nu_post <= 64, GLLMG_EINVAL,
              "smoothing steps out of range");
  GLLMG_CHECK(c.omega > 0.0 && c.omega < 2.0, GLLMG_EINVAL, "omega out of range");
  GLLMG_CHECK(c.cheb_lo > 0.0 && c.cheb_lo < 1.0, GLLMG_EINVAL, "cheb_lo must be in (0, 1)");
  GLLMG_CHECK(c.cheb_safety > 0.0, GLLMG_EINVAL, "cheb_safety must be positive");
  GLLMG_CHECK(c.eig_steps >= 1 && c.eig_steps <= 64, GLLMG_EINVAL, "eig_steps out of range");
  GLLMG_CHECK(c.vcycle_prec == GLLMG_F64 || c.vcycle_prec == GLLMG_F32, GLLMG_EINVAL,
              "vcycle_prec must be GLLMG_F64 or GLLMG_F32");
  GLLMG_CHECK(c.max_levels >= 0, GLLMG_EINVAL, "max_levels must be >= 0");
  int64_t nodes = 1;
  for (int a = 0; a < c.dim; ++a) nodes *= (int64_t)c.nelem[a] * c.order + 1;
  GLLMG_CHECK(nodes < (int64_t(1) << 31), GLLMG_EINVAL, "more than 2^31 - 1 nodes");
  int ne[3] = {c.nelem[0], c.nelem[1], c.dim == 3 ? c.nelem[2] : 1};
  GLLMG_CHECK(interior_count(c.dim, ne, c.order) >= 1, GLLMG_EINVAL,
              "the mesh has no interior node");
}

// Levels from fine to coarse (§3.1, §4.3): h-hierarchy keeps p; p-hierarchy takes
// p -> ceil(p/2) down to 1; then elements are halved while every axis is even and the coarser
// mesh keeps an interior node.
std::vector<LevelSpec> plan_levels(const gllmg_config& c) {
  std::vector<LevelSpec> L;
  LevelSpec s{{c.nelem[0], c.nelem[1], c.dim == 3 ? c.nelem[2] : 1}, c.order};
  L.push_back(s);
  if (c.hierarchy == GLLMG_HIER_P)
    while (s.p > 1) {
      s.p = (s.p + 1) / 2;
      L.push_back(s);
    }
  if (c.hierarchy == GLLMG_HIER_LOW && s.p > 1) {  // first-order cells on the order-p nodes
    for (int a = 0; a < c.dim; ++a) s.ne[a] *= s.p;
    s.p = 1;
    L.push_back(s);
  }
  for (;;) {
    if (c.coarse_unknowns > 0 && s.p == 1 && interior_count(c.dim, s.ne, s.p) <= c.coarse_unknowns)
      break;  // the first first-order level small enough for the exact solve
    bool even = true;
    for (int a = 0; a < c.dim; ++a) even = even && (s.ne[a] % 2 == 0);
    if (!even) break;
    LevelSpec t = s;
    for (int a = 0; a < c.dim; ++a) t.ne[a] /= 2;
    if (interior_count(c.dim, t.ne, t.p) < 1) break;
    s = t;
    L.push_back(s);
  }
  if (c.max_levels > 0 && (int)L.size() > c.max_levels) L.resize(c.max_levels);
  return L;
}

Grid make_grid(int dim, const LevelSpec& s) {
  Grid g{};
  g.dim = dim;
  g.p = s.p;
  g.E = 1;
  g.N = 1;
  for (int a = 0; a < 3; ++a) {
    g.ne[a] = a < dim ? s.ne[a] : 1;
    g.nn[a] = a < dim ? s.ne[a] * s.p + 1 : 1;
    g.E *= g.ne[a];
    g.N *= g.nn[a];
  }
  g.rnn[0] = 1.0 / g.nn[0];
  g.rnn[1] = 1.0 / g.nn[1];
  return g;
}

constexpr int64_t kMaxCoarse = 4096;
// problems in one launch group of gllmg_batch_solve (the group's buffers sit in the first
// problem's workspace; a shape with more problems forms several groups)
constexpr int kGroupMax = 256;

}  // namespace

}  // namespace gllmg

using namespace gllmg;

struct gllmg_problem {
  gllmg_config cfg;
  std::vector<Level> L;
  std::vector<RefElem> re;
  FieldDev map{}, mu{};
  gllmg_field_fn map_fn = nullptr, mu_fn = nullptr;  // callback kinds (used during setup only)
  void* map_ctx = nullptr;
  void* mu_ctx = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;
  double* mass = nullptr;
  double* wdetq = nullptr;  // Gauss quadrature: w~ detJ at the finest level's Gauss points
  void* F = nullptr;
  void* zeros = nullptr;
  double* scal = nullptr;
  double* part = nullptr;
  int* flag = nullptr;
  double* map_modes = nullptr;
  double* mu_modes = nullptr;
  double* pr = nullptr;  // FP64 fine-level solve vectors
  double* pz = nullptr;
  double* pp = nullptr;
  double* ph = nullptr;
  double* pt = nullptr;
  float* ir32 = nullptr;     // iterative refinement: FP32 r, z, p, h, e (N0 each), or null
  char* scratch = nullptr;   // start of the region shared by setup temporaries and solve vectors
  size_t scratch_bytes = 0;
  double* hbuf = nullptr;    // pinned host scalars
  int vprec = 0;             // V-cycle precision index
  // the solve's V-cycle (pr -> pz) captured once as a HIP graph and replayed per iteration
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraphExec_t vexec = nullptr;
  std::vector<int64_t> vapplies;
  // state of the solve in progress (gllmg_solve_begin / _poll / _end)
  struct Solve {
    bool active = false, done = false, conv = false, breakdown = false;
    // a V-cycle for the next iteration enqueued before the current residual norm was known, and
    // the products it added to the per-level counts (taken back if it goes unused)
    bool spec = false;
    std::vector<int64_t> spec_applies;
    int mode = 0, maxit = 0, iters = 0, g = 0, phase = 0;
    const double* b = nullptr;
    double* x = nullptr;
    double rtol = 0, n0 = 0, nr = 0, rt = 0;
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<double> hist;
    std::vector<int64_t> a0;
    std::chrono::steady_clock::time_point t0;
  } sv;
  hipStream_t xs = nullptr;  // internal stream for batched solves (default priority)
  BatchProblem* bdev = nullptr;   // descriptor of the persistent batched solver (workspace)
  BatchProblem* bhost = nullptr;  // its pinned host image
  bool persistent = true;         // gllmg_batch_solve may use the persistent solver
  // a launch group led by this problem (gllmg_batch_solve): per member k its workspace offset,
  // active flag and collected scalars in the workspace, their pinned host images, and the
  // events that order the batch's streams; all made at setup, so a batch allocates nothing
  int64_t* gdlt = nullptr;
  int* gact = nullptr;
  double* gsc = nullptr;
  int* ghact = nullptr;
  double* ghsc = nullptr;
  hipEvent_t bev = nullptr;  // the batch's start, recorded on the caller's stream
  hipEvent_t gev = nullptr;  // the end of the group this problem leads
  int dev = -1;                 // the device current at setup
  void* sscratch = nullptr;     // that device's static scratch (gllmg_apply_noalloc)
};

namespace gllmg {
namespace {

// pairs in a level's Chebyshev coefficient table: (theta, delta) and steps 1 .. k - 1
inline int ctab_pairs(const gllmg_config& c) { return std::max(std::max(c.nu_pre, c.nu_post), 1) + 1; }

// Lay out (or only size) the whole device footprint.
size_t layout(gllmg_problem* P, const std::vector<LevelSpec>& specs, Arena& A) {
  const gllmg_config& c = P->cfg;
  const bool f32 = c.vcycle_prec == GLLMG_F32;
  P->L.resize(specs.size());
  size_t face = 0;
  for (size_t l = 0; l < specs.size(); ++l) {
    Level& L = P->L[l];
    L.g = make_grid(c.dim, specs[l]);
    L.gauss = c.quadrature == GLLMG_QUAD_GAUSS;
    L.n = specs[l].p + 1;
    L.nint = interior_count(c.dim, L.g.ne, L.g.p);
    L.ncomp = c.dim == 3 ? 6 : 3;
    L.npts = L.g.E * (c.dim == 3 ? (int64_t)L.n * L.n * L.n : (int64_t)L.n * L.n);
    L.has_coarse = l + 1 < specs.size();
    const int n = L.n;
    L.D64 = (double*)A.take(sizeof(double) * 2 * n * n);
    L.D32 = (float*)A.take(sizeof(float) * 2 * n * n);
    L.xi64 = (double*)A.take(sizeof(double) * n);
    L.w64 = (double*)A.take(sizeof(double) * n);
    if (L.gauss) {
      L.Iq64 = (double*)A.take(sizeof(double) * n * n);
      L.Iq32 = (float*)A.take(sizeof(float) * n * n);
      L.Dq64 = (double*)A.take(sizeof(double) * n * n);
      L.Dq32 = (float*)A.take(sizeof(float) * n * n);
      L.wg64 = (double*)A.take(sizeof(double) * n);
    }
    L.G64 = (double*)A.take(sizeof(double) * L.npts * L.ncomp);
    L.G32 = f32 ? (float*)A.take(sizeof(float) * L.npts * L.ncomp) : nullptr;
    L.ctab = (double*)A.take(sizeof(double) * 2 * ctab_pairs(c));
    L.dinv64 = (double*)A.take(sizeof(double) * L.g.N);
    L.dinv32 = f32 ? (float*)A.take(sizeof(float) * L.g.N) : nullptr;
    if (c.smoother == GLLMG_SMOOTH_L1_JACOBI) {
      L.l1inv64 = (double*)A.take(sizeof(double) * L.g.N);
      L.l1inv32 = f32 ? (float*)A.take(sizeof(float) * L.g.N) : nullptr;
    }
    if (c.smoother == GLLMG_SMOOTH_BLOCK_JACOBI) {
      const size_t PP = (size_t)block_slots(L) * block_slots(L);
      L.Binv64 = (double*)A.take(sizeof(double) * L.g.E * PP);
      L.Binv32 = f32 ? (float*)A.take(sizeof(float) * L.g.E * PP) : nullptr;
    }
    face = std::max(face, face_buffer_elems(L));
    if (!L.has_coarse && L.nint <= kMaxCoarse) {
      // the exact coarse solve exists only up to kMaxCoarse unknowns; a larger coarsest level
      // still supports products and smoothing, and vcycle/solve report EUNSUPPORTED
      L.Ainv64 = (double*)A.take(sizeof(double) * L.nint * L.nint);
      L.Ainv32 = f32 ? (float*)A.take(sizeof(float) * L.nint * L.nint) : nullptr;
    }
  }
  // the first-order hierarchy's levels 0 and 1 share their nodes: no transfer between them
  const bool shares = c.hierarchy == GLLMG_HIER_LOW && specs.size() > 1 && specs[0].p > 1;
  for (size_t l = shares ? 1 : 0; l + 1 < specs.size(); ++l) {
    Level& F = P->L[l];
    Level& C = P->L[l + 1];
    face = std::max(face, restrict_buffer_elems(F, C));
    F.tp.nch = F.g.p == C.g.p ? 2 : 1;
    const size_t np = (size_t)F.tp.nch * F.n * C.n;
    F.tp.P64 = (double*)A.take(sizeof(double) * np);
    F.tp.P32 = (float*)A.take(sizeof(float) * np);
  }
  const int64_t N0 = P->L[0].g.N;
  P->mass = (double*)A.take(sizeof(double) * N0);
  if (c.quadrature == GLLMG_QUAD_GAUSS) P->wdetq = (double*)A.take(sizeof(double) * P->L[0].npts);
  P->F = A.take(sizeof(double) * std::max<size_t>(face, 1));
  P->bdev = (BatchProblem*)A.take(sizeof(BatchProblem));
  P->zeros = A.take(64);
  for (auto& L : P->L) L.zero = P->zeros;
  P->scal = (double*)A.take(sizeof(double) * 64);
  P->part = (double*)A.take(sizeof(double) * kDotBlocks);
  P->flag = (int*)A.take(sizeof(int) * 4);
  P->gdlt = (int64_t*)A.take(sizeof(int64_t) * kGroupMax);
  P->gact = (int*)A.take(sizeof(int) * kGroupMax);
  P->gsc = (double*)A.take(sizeof(double) * 4 * kGroupMax);
  P->map_modes = (double*)A.take(sizeof(double) * 5 * GLLMG_MAX_MODES);
  P->mu_modes = (double*)A.take(sizeof(double) * 5 * GLLMG_MAX_MODES);
  // scratch: solve vectors in steady state, setup temporaries during setup
  const size_t before = A.used;
  P->scratch = (char*)A.take(0);
  P->pr = (double*)A.take(sizeof(double) * N0);
  P->pz = (double*)A.take(sizeof(double) * N0);
  P->pp = (double*)A.take(sizeof(double) * N0);
  P->ph = (double*)A.take(sizeof(double) * N0);
  P->pt = (double*)A.take(sizeof(double) * N0);
  // iterative refinement's FP32 r, z, p, h, e
  if (P->cfg.ir_inner > 0 && P->cfg.vcycle_prec == GLLMG_F32) P->ir32 = (float*)A.take(sizeof(float) * 5 * N0);
  for (auto& L : P->L) {
    const int64_t N = L.g.N;
    for (int pr = 0; pr < (f32 ? 2 : 1); ++pr) {
      const size_t es = pr == 0 ? sizeof(double) : sizeof(float);
      L.vb[pr] = A.take(es * N);
      L.vx[pr] = A.take(es * N);
      L.vr[pr] = A.take(es * N);
      L.vd[pr] = A.take(es * N);
      L.vd2[pr] = A.take(es * N);
      // the third direction of a degree-4 smoother
      L.vd3[pr] = (c.smoother == GLLMG_SMOOTH_CHEBYSHEV && std::max(c.nu_pre, c.nu_post) >= 4)
                      ? A.take(es * N) : nullptr;
    }
  }
  const size_t steady = A.used - before;
  int64_t maxN = 0;
  for (auto& L : P->L) maxN = std::max(maxN, L.g.N);
  const size_t setup = sizeof(double) * (size_t)std::max<int64_t>(
                                            (int64_t)c.eig_steps * maxN + 4 * maxN +
                                                (int64_t)(c.eig_steps + 1) * (3 + kMdBlocks),
                                            5 * P->L[0].npts + 4 * maxN) + 4096;
  if (setup > steady) A.take(setup - steady);
  P->scratch_bytes = A.used - before;
  return A.used + 256;
}

FieldDev to_dev(const gllmg_field* f, double* dev_modes, hipStream_t s, bool is_map) {
  FieldDev d{};
  GLLMG_CHECK(f != nullptr, GLLMG_EINVAL, "field is NULL");
  d.kind = f->kind;
  if (is_map)
    GLLMG_CHECK(f->kind == GLLMG_MAP_IDENTITY || f->kind == GLLMG_MAP_WARP_SINE ||
                    f->kind == GLLMG_MAP_AFFINE || f->kind == GLLMG_MAP_CALLBACK,
                GLLMG_EINVAL, "unknown map kind");
  else
    GLLMG_CHECK((f->kind >= GLLMG_FIELD_CONST && f->kind <= GLLMG_FIELD_COS2_SUM) ||
                    f->kind == GLLMG_FIELD_CALLBACK,
                GLLMG_EINVAL, "unknown field kind");
  if (f->kind == GLLMG_MAP_CALLBACK || f->kind == GLLMG_FIELD_CALLBACK)
    GLLMG_CHECK(f->fn != nullptr, GLLMG_EINVAL, "a callback field needs fn");
  for (int i = 0; i < 12; ++i) d.param[i] = f->param[i];
  d.nmodes = 0;
  d.modes = dev_modes;
  if (!is_map && f->kind == GLLMG_FIELD_EXP_FOURIER) {
    GLLMG_CHECK(f->nmodes >= 1 && f->nmodes <= GLLMG_MAX_MODES && f->modes, GLLMG_EINVAL,
                "EXP_FOURIER needs 1..64 modes");
    d.nmodes = f->nmodes;
    GLLMG_HIP(hipMemcpyAsync(dev_modes, f->modes, sizeof(double) * 5 * f->nmodes,
                             hipMemcpyHostToDevice, s));
    GLLMG_HIP(hipStreamSynchronize(s));
  }
  return d;
}

double read_scalar(gllmg_problem* P, int idx, hipStream_t s) {
  GLLMG_HIP(hipMemcpyAsync(P->hbuf, P->scal + idx, sizeof(double), hipMemcpyDeviceToHost, s));
  GLLMG_HIP(hipStreamSynchronize(s));
  return P->hbuf[0];
}

void read_scalars(gllmg_problem* P, int idx, int cnt, double* out, hipStream_t s) {
  GLLMG_HIP(hipMemcpyAsync(P->hbuf, P->scal + idx, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
  GLLMG_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < cnt; ++i) out[i] = P->hbuf[i];
}

void apply_epi(gllmg_problem* P, int l, int pr, int neumann, const void* x, const Epi& ep,
               hipStream_t s) {
  Level& L = P->L[l];
  launch_apply(L, pr, neumann, x, ep, P->F, s);
  ++L.applies;
}

void apply_level(gllmg_problem* P, int l, int pr, int neumann, const void* x, void* y, hipStream_t s) {
  Epi ep;
  ep.y = y;
  apply_epi(P, l, pr, neumann, x, ep, s);
}

// r = b - A_l x
void residual(gllmg_problem* P, int l, int pr, const void* b, const void* x, void* r, hipStream_t s) {
  Epi ep;
  ep.mode = EPI_RESIDUAL;
  ep.b = b;
  ep.r = r;
  apply_epi(P, l, pr, 0, x, ep, s);
}

// The 1D matrix of the transfer from level l to level l + 1 (paper §2.2): coarse basis
// function c evaluated at fine node i of child `ch`, whose reference coordinate in the coarse
// element is xi_i (p-coarsening: same element) or (xi_i + 2 ch - 1) / 2 (h-coarsening: the
// fine element is half ch of the coarse one along the axis).
// (the host tables go into k64 and k32, which the caller keeps until the stream has copied them)
void build_transfer_tables(gllmg_problem* P, int l, hipStream_t s, std::deque<std::vector<double>>& k64,
                           std::deque<std::vector<float>>& k32) {
  Level& F = P->L[l];
  Level& C = P->L[l + 1];
  const RefElem& rf = P->re[l];
  const RefElem& rc = P->re[l + 1];
  const int nf = F.n, nc = C.n, nch = F.tp.nch;
  auto& Pl = k64.emplace_back((size_t)nch * nf * nc);
  for (int ch = 0; ch < nch; ++ch)
    for (int i = 0; i < nf; ++i) {
      const double xc = nch == 1 ? rf.xi[i] : (rf.xi[i] + 2.0 * ch - 1.0) / 2.0;
      lagrange_at(rc, xc, &Pl[((size_t)ch * nf + i) * nc]);
    }
  const auto& Pl32 = k32.emplace_back(Pl.begin(), Pl.end());
  GLLMG_HIP(hipMemcpyAsync(F.tp.P64, Pl.data(), sizeof(double) * Pl.size(), hipMemcpyHostToDevice, s));
  GLLMG_HIP(hipMemcpyAsync(F.tp.P32, Pl32.data(), sizeof(float) * Pl32.size(), hipMemcpyHostToDevice, s));
}

// lambda_max of D^{-1} A (§3.2.2: a few Arnoldi steps in setup): Lanczos on the symmetric
// S = D^{-1/2} A D^{-1/2} with full reorthogonalization (one classical Gram-Schmidt pass per
// step: one multi-dot and one update against the whole basis),
// m = min(eig_steps, interior unknowns) steps, SplitMix64 start vector; breakdown when
// beta <= 1e-14 ||T||. Returns the largest eigenvalue of the tridiagonal T_m.
double lanczos_lmax(gllmg_problem* P, int l, hipStream_t s) {
  Level& L = P->L[l];
  const int64_t N = L.g.N;
  const int m = (int)std::min<int64_t>(P->cfg.eig_steps, L.nint);
  double* base = (double*)P->scratch;
  std::vector<double*> V(m + 1);
  for (int i = 0; i <= m; ++i) V[i] = base + (size_t)i * N;
  // m+1 basis vectors, w, t and sqrt(dinv): (m + 4) N doubles, then the per-step scalars
  // alpha_j, |w_j|^2 and the orthogonalization's coefficients and partial sums
  double* w = base + (size_t)(m + 1) * N;
  double* t = w + N;
  double* sqd = t + N;
  double* alpha = sqd + N;
  double* n2 = alpha + (m + 1);
  double* coef = n2 + (m + 1);
  double* part = coef + (m + 1);
  vec_sqrt(N, L.dinv64, sqd, s);
  start_vector(L.g, P->cfg.eig_seed, l, V[0], s);
  dot(0, N, V[0], V[0], P->part, P->scal + 8, s);
  lanczos_next(N, V[0], nullptr, 0, P->scal + 8, sqd, V[0], t, s);  // V_0 normalized, t = sqd V_0
  const int np = dot_grid(N);  // partial sums of each dot product (P->part holds them)
  // The whole recurrence is enqueued without reading anything back: beta_j = |w_j| stays on
  // the device. A breakdown (|w_j| ~ 0) is found afterwards on the host, where the
  // coefficients past it are discarded. Per step: w = sqd A t, alpha_j = V_j . w,
  // w -= alpha_j V_j + beta_{j-1} V_{j-1}, w -= V (V^T w), |w|^2, V_{j+1} = w / |w| and the
  // next step's t = sqd V_{j+1}.
  for (int j = 0; j < m; ++j) {
    apply_level(P, l, 0, 0, t, w, s);
    lanczos_scale_dot(N, sqd, w, V[j], P->part, s);
    lanczos_axpy2(N, P->part, np, alpha + j, V[j], j > 0 ? n2 + (j - 1) : nullptr,
                  j > 0 ? V[j - 1] : nullptr, w, s);
    block_orthogonalize(N, V[0], N, j + 1, w, part, coef, P->part, s);
    if (j + 1 < m)
      lanczos_next(N, w, P->part, np, n2 + j, sqd, V[j + 1], t, s);
    else
      sum_partials(P->part, np, n2 + j, s);
  }
  std::vector<double> ha(m), hn(m);
  GLLMG_HIP(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  GLLMG_HIP(hipMemcpyAsync(hn.data(), n2, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  GLLMG_HIP(hipStreamSynchronize(s));
  std::vector<double> al, be;
  double tnorm = 0.0;
  for (int j = 0; j < m; ++j) {
    const double a = ha[j];
    const double bn = std::sqrt(hn[j]);
    al.push_back(a);
    tnorm = std::max(tnorm, std::fabs(a) + (be.empty() ? 0.0 : be.back()) + bn);
    if (j == m - 1 || bn <= 1e-14 * tnorm) break;
    be.push_back(bn);
  }
  be.resize(al.size() - 1);
  return tridiag_max_eig(al, be);
}

// The coarsest operator's interior block, column by column from matrix-free products. Two
// nodes couple only if they share an element, so they lie within p index steps of each other
// along every axis; nodes 2p+1 steps apart along some axis therefore couple to disjoint sets
// of nodes, and one product of the sum of their unit vectors yields all their columns at once
// (each entry bitwise equal to the product of its own unit vector: an element sees at most one
// of the nodes). (2p+1)^d products instead of one per interior node.
void build_coarse_inverse(gllmg_problem* P, hipStream_t s) {
  Level& L = P->L.back();
  const int64_t N = L.g.N, ni = L.nint;
  const int dim = L.g.dim, p = L.g.p, c = 2 * p + 1;
  const int nx = L.g.nn[0], ny = L.g.nn[1];
  const int mx = nx - 2, my = ny - 2, mz = dim == 3 ? L.g.nn[2] - 2 : 1;
  auto node = [&](int jx, int jy, int jz) {
    return (jx + 1) + (int64_t)nx * ((jy + 1) + (int64_t)ny * (dim == 3 ? jz + 1 : 0));
  };
  auto row = [&](int jx, int jy, int jz) { return jx + (int64_t)mx * (jy + (int64_t)my * jz); };
  // the colors (ox, oy, oz); their products go B at a time into the scratch region (the
  // color vector e, then B product columns) and come back in one copy per batch
  std::vector<std::array<int, 3>> colors;
  for (int oz = 0; oz < std::min(c, mz); ++oz)
    for (int oy = 0; oy < std::min(c, my); ++oy)
      for (int ox = 0; ox < std::min(c, mx); ++ox) colors.push_back({ox, oy, oz});
  const int64_t cap = (int64_t)(P->scratch_bytes / sizeof(double)) / N - 1;
  GLLMG_CHECK(cap >= 1, GLLMG_ENOMEM, "scratch region too small for the coarse assembly");
  const int B = (int)std::min<int64_t>(cap, (int64_t)colors.size());
  double* e = (double*)P->scratch;
  double* y = e + N;
  std::vector<double> A((size_t)ni * ni, 0.0), cols((size_t)B * N);
  for (size_t c0 = 0; c0 < colors.size(); c0 += B) {
    const int nb = (int)std::min<size_t>(B, colors.size() - c0);
    for (int b = 0; b < nb; ++b) {
      const auto& o = colors[c0 + b];
      color_unit_vector(L.g, c, o[0], o[1], o[2], e, s);
      apply_level(P, (int)P->L.size() - 1, 0, 0, e, y + (size_t)b * N, s);
    }
    GLLMG_HIP(hipMemcpyAsync(cols.data(), y, sizeof(double) * N * nb, hipMemcpyDeviceToHost, s));
    GLLMG_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) {
      const auto& o = colors[c0 + b];
      const double* col = cols.data() + (size_t)b * N;
      for (int jz = o[2]; jz < mz; jz += c)
        for (int jy = o[1]; jy < my; jy += c)
          for (int jx = o[0]; jx < mx; jx += c) {
            const int64_t j = row(jx, jy, jz);
            for (int iz = std::max(0, jz - p); iz <= std::min(mz - 1, jz + p); ++iz)
              for (int iy = std::max(0, jy - p); iy <= std::min(my - 1, jy + p); ++iy)
                for (int ix = std::max(0, jx - p); ix <= std::min(mx - 1, jx + p); ++ix)
                  A[(size_t)row(ix, iy, iz) * ni + j] = col[node(ix, iy, iz)];
          }
    }
  }
  // symmetrize the rounding of the matrix-free products
  for (int64_t i = 0; i < ni; ++i)
    for (int64_t j = 0; j < i; ++j) {
      const double v = 0.5 * (A[(size_t)i * ni + j] + A[(size_t)j * ni + i]);
      A[(size_t)i * ni + j] = A[(size_t)j * ni + i] = v;
    }
  GLLMG_CHECK(spd_inverse(A, (int)ni), GLLMG_EINVAL, "coarsest operator is not SPD");
  std::vector<float> A32(A.begin(), A.end());
  GLLMG_HIP(hipMemcpyAsync(L.Ainv64, A.data(), sizeof(double) * A.size(), hipMemcpyHostToDevice, s));
  if (L.Ainv32)
    GLLMG_HIP(hipMemcpyAsync(L.Ainv32, A32.data(), sizeof(float) * A32.size(), hipMemcpyHostToDevice, s));
  GLLMG_HIP(hipStreamSynchronize(s));
  L.applies = 0;
}

void check_flag(gllmg_problem* P, hipStream_t s) {
  int f = 0;
  GLLMG_HIP(hipMemcpyAsync(&f, P->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  GLLMG_HIP(hipStreamSynchronize(s));
  GLLMG_CHECK(!(f & 1), GLLMG_EINVAL, "detJ <= 0 at a quadrature point: the map is not a diffeomorphism");
  GLLMG_CHECK(!(f & 2), GLLMG_EINVAL, "mu is not positive and finite at a quadrature point");
  GLLMG_CHECK(!(f & 4), GLLMG_EINVAL, "the operator diagonal is not positive");
  GLLMG_CHECK(!(f & 8), GLLMG_EINVAL, "an element block of the block-Jacobi smoother is not positive definite");
}

// The first-order hierarchy's levels 0 (order p) and 1 (first order) share their nodes.
bool low_first(const gllmg_problem* P) {
  return P->cfg.hierarchy == GLLMG_HIER_LOW && P->L.size() > 1 && P->L[0].g.p > 1;
}

// Phi and mu at every node of level l, into `nodal` (N dim coordinates, then N values of mu):
// the built-in families by the same kernels as gllmg_node_coords and gllmg_eval_field; callback
// kinds by the caller's functions, called once with every node of the level in node order
// (Phi at the reference coordinates, mu at the physical ones) and copied to the device.
void nodal_fields(gllmg_problem* P, int l, double* nodal, hipStream_t s, bool need_mu = true) {
  const Level& L = P->L[l];
  const int dim = L.g.dim;
  const int64_t N = L.g.N;
  double* xn = nodal;
  double* mun = nodal + (size_t)N * dim;
  std::vector<double> x;
  if (P->map_fn) {
    const RefElem& re = P->re[l];
    std::vector<double> X((size_t)N * dim);
    x.resize((size_t)N * dim);
    for (int64_t t = 0; t < N; ++t) {
      const int64_t gc[3] = {t % L.g.nn[0], (t / L.g.nn[0]) % L.g.nn[1],
                             t / ((int64_t)L.g.nn[0] * L.g.nn[1])};
      for (int a = 0; a < dim; ++a) {
        const int p = L.g.p, ne = L.g.ne[a];
        const int e = (int)std::min<int64_t>(gc[a] / p, ne - 1);
        X[(size_t)t * dim + a] = ((double)e + (re.xi[gc[a] - (int64_t)e * p] + 1.0) * 0.5) / (double)ne;
      }
    }
    P->map_fn(X.data(), N, dim, x.data(), P->map_ctx);
    GLLMG_HIP(hipMemcpyAsync(xn, x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice, s));
    GLLMG_HIP(hipStreamSynchronize(s));
  } else {
    launch_node_coords(L.g, L.xi64, P->map, xn, s);
  }
  if (!need_mu) return;
  if (P->mu_fn) {
    if (x.empty()) {
      x.resize((size_t)N * dim);
      GLLMG_HIP(hipMemcpyAsync(x.data(), xn, sizeof(double) * x.size(), hipMemcpyDeviceToHost, s));
      GLLMG_HIP(hipStreamSynchronize(s));
    }
    std::vector<double> m((size_t)N);
    P->mu_fn(x.data(), N, dim, m.data(), P->mu_ctx);
    GLLMG_HIP(hipMemcpyAsync(mun, m.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    GLLMG_HIP(hipStreamSynchronize(s));  // the host values go out of scope
  } else if (P->map_fn) {
    launch_field_at(L.g, xn, P->mu, mun, s);
  } else {
    launch_eval_field(L.g, L.xi64, P->map, P->mu, mun, s);
  }
}

void setup_impl(gllmg_problem* P, const gllmg_field* map, const gllmg_field* mu, hipStream_t s) {
  const gllmg_config& c = P->cfg;
  const bool f32 = c.vcycle_prec == GLLMG_F32;
  P->map = to_dev(map, P->map_modes, s, true);
  P->mu = to_dev(mu, P->mu_modes, s, false);
  P->map_fn = map->kind == GLLMG_MAP_CALLBACK ? map->fn : nullptr;
  P->map_ctx = map->ctx;
  P->mu_fn = mu->kind == GLLMG_FIELD_CALLBACK ? mu->fn : nullptr;
  P->mu_ctx = mu->ctx;
  GLLMG_HIP(hipMemsetAsync(P->flag, 0, sizeof(int) * 4, s));
  GLLMG_HIP(hipMemsetAsync(P->zeros, 0, 64, s));
  P->re.clear();
  P->re.reserve(P->L.size());
  // host images of the per-level tables, alive until the stream has copied them (one
  // synchronization after the loop)
  std::deque<std::vector<double>> keep64;
  std::deque<std::vector<float>> keep32;
  struct SyncFirst {  // destroyed before the images, also when setup throws
    hipStream_t s;
    ~SyncFirst() { (void)hipStreamSynchronize(s); }
  } sync_first{s};
  for (auto& L : P->L) {
    P->re.push_back(ref_element(L.g.p));
    RefElem& r = P->re.back();
    if (L.gauss) {
      gauss_rule(r);
      const auto& I32 = keep32.emplace_back(r.Iq.begin(), r.Iq.end());
      const auto& Dq32 = keep32.emplace_back(r.Dq.begin(), r.Dq.end());
      GLLMG_HIP(hipMemcpyAsync(L.Iq64, r.Iq.data(), sizeof(double) * r.Iq.size(), hipMemcpyHostToDevice, s));
      GLLMG_HIP(hipMemcpyAsync(L.Iq32, I32.data(), sizeof(float) * I32.size(), hipMemcpyHostToDevice, s));
      GLLMG_HIP(hipMemcpyAsync(L.Dq64, r.Dq.data(), sizeof(double) * r.Dq.size(), hipMemcpyHostToDevice, s));
      GLLMG_HIP(hipMemcpyAsync(L.Dq32, Dq32.data(), sizeof(float) * Dq32.size(), hipMemcpyHostToDevice, s));
      GLLMG_HIP(hipMemcpyAsync(L.wg64, r.wg.data(), sizeof(double) * r.wg.size(), hipMemcpyHostToDevice, s));
    }
    const int n = L.n;
    auto& DDt = keep64.emplace_back(r.D);  // D, then its transpose
    DDt.resize((size_t)2 * n * n);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) DDt[(size_t)n * n + a * n + b] = r.D[(size_t)b * n + a];
    const auto& D32 = keep32.emplace_back(DDt.begin(), DDt.end());
    GLLMG_HIP(hipMemcpyAsync(L.D64, DDt.data(), sizeof(double) * DDt.size(), hipMemcpyHostToDevice, s));
    GLLMG_HIP(hipMemcpyAsync(L.D32, D32.data(), sizeof(float) * D32.size(), hipMemcpyHostToDevice, s));
    GLLMG_HIP(hipMemcpyAsync(L.xi64, r.xi.data(), sizeof(double) * r.xi.size(), hipMemcpyHostToDevice, s));
    GLLMG_HIP(hipMemcpyAsync(L.w64, r.w.data(), sizeof(double) * r.w.size(), hipMemcpyHostToDevice, s));
  }
  GLLMG_HIP(hipStreamSynchronize(s));  // the per-level tables are on the device
  for (size_t l = 0; l < P->L.size(); ++l) {
    Level& L = P->L[l];
    double* wdet = l == 0 ? (double*)P->scratch : nullptr;
    double* nodal = (double*)P->scratch + P->L[0].npts;
    if (L.gauss) {
      // the physical Gauss points (isoparametric interpolant of the mapped nodes), mu there
      // (built-in family on the device, or the caller's callback), then the factors
      nodal_fields(P, (int)l, nodal, s, false);
      double* xq = nodal + 4 * (size_t)L.g.N;
      double* muq = xq + (size_t)L.npts * c.dim;
      launch_gauss_points(L, nodal, xq, s);
      if (P->mu_fn) {
        std::vector<double> xh((size_t)L.npts * c.dim), mh((size_t)L.npts);
        GLLMG_HIP(hipMemcpyAsync(xh.data(), xq, sizeof(double) * xh.size(), hipMemcpyDeviceToHost, s));
        GLLMG_HIP(hipStreamSynchronize(s));
        P->mu_fn(xh.data(), L.npts, c.dim, mh.data(), P->mu_ctx);
        GLLMG_HIP(hipMemcpyAsync(muq, mh.data(), sizeof(double) * mh.size(), hipMemcpyHostToDevice, s));
        GLLMG_HIP(hipStreamSynchronize(s));
      } else {
        launch_field_pts(L.npts, c.dim, xq, P->mu, muq, s);
      }
      launch_geometry_gauss(L, nodal, muq, L.G64, f32 ? L.G32 : nullptr, l == 0 ? P->wdetq : nullptr,
                            P->flag, s);
    } else if (l >= 1 && low_first(P)) {
      // first-order levels: the vertices are the order-p nodes (every stride-th one per axis),
      // whose Phi and mu level 0 left in `nodal`
      double* nl = nodal + 4 * (size_t)P->L[0].g.N;
      const int stride = (P->L[0].g.nn[0] - 1) / (L.g.nn[0] - 1);
      launch_subsample_nodal(P->L[0].g, L.g, stride, nodal, nodal + (size_t)P->L[0].g.N * c.dim,
                             nl, nl + (size_t)L.g.N * c.dim, s);
      launch_geometry(L, nl, nl + (size_t)L.g.N * c.dim, L.G64, f32 ? L.G32 : nullptr, wdet,
                      P->flag, s);
    } else {
      nodal_fields(P, (int)l, nodal, s);
      launch_geometry(L, nodal, nodal + (size_t)L.g.N * c.dim, L.G64, f32 ? L.G32 : nullptr, wdet,
                      P->flag, s);
      if (l == 0) launch_gather_full(L, wdet, P->mass, s);
    }
    double* diag = (double*)P->scratch;
    launch_diag(L, diag, (double*)P->F, s);
    launch_dinv(L.g, diag, L.dinv64, f32 ? L.dinv32 : nullptr, P->flag, s);
    if (c.smoother == GLLMG_SMOOTH_L1_JACOBI) {
      launch_l1_rowsum(L, diag, s);
      launch_dinv(L.g, diag, L.l1inv64, f32 ? L.l1inv32 : nullptr, P->flag, s);
    }
    if (c.smoother == GLLMG_SMOOTH_BLOCK_JACOBI) {
      launch_block_setup(L, L.Binv64, P->flag, s);
      if (f32) cast_64_32(L.g.E * (int64_t)block_slots(L) * block_slots(L), L.Binv64, L.Binv32, s);
    }
  }
  // the checks of every level at once (the flag bits accumulate; the kernels above run to the
  // end on invalid values without harm, and check_flag reports the first kind of failure)
  check_flag(P, s);
  for (size_t l = low_first(P) ? 1 : 0; l + 1 < P->L.size(); ++l)
    build_transfer_tables(P, (int)l, s, keep64, keep32);
  for (size_t l = 0; l < P->L.size(); ++l)
    if (P->L[l].has_coarse || !P->L[l].Ainv64)
      P->L[l].lmax = c.cheb_safety * lanczos_lmax(P, (int)l, s);
  if (P->L.back().Ainv64) build_coarse_inverse(P, s);
  for (auto& L : P->L) L.applies = 0;
  GLLMG_HIP(hipStreamSynchronize(s));  // (also the end of the transfer tables' copies)
}

// ------------------------------------------------------------------ smoothers and cycles
const void* dinv_of(const Level& L, int pr) { return pr == 0 ? (const void*)L.dinv64 : (const void*)L.dinv32; }

// The inverse diagonal a Jacobi-type smoother scales residuals by: D^{-1}, or D_l1^{-1} for
// l1-Jacobi (§3.2.3).
const void* jacobi_dinv(const gllmg_problem* P, const Level& L, int pr) {
  if (P->cfg.smoother == GLLMG_SMOOTH_L1_JACOBI)
    return pr == 0 ? (const void*)L.l1inv64 : (const void*)L.l1inv32;
  return dinv_of(L, pr);
}

bool jacobi_type(const gllmg_config& c) {
  return c.smoother == GLLMG_SMOOTH_JACOBI || c.smoother == GLLMG_SMOOTH_L1_JACOBI;
}

// Chebyshev interval [cheb_lo lambda, lambda]: its center theta and half-width delta
void cheb_interval(const gllmg_problem* P, const Level& L, double* theta, double* delta) {
  const double lam = L.lmax, alpha = P->cfg.cheb_lo * lam;
  *theta = 0.5 * (lam + alpha);
  *delta = 0.5 * (lam - alpha);
}

// The Chebyshev coefficients of every level as smooth_impl forms them, into the levels'
// device tables (read by launch groups). Stream-ordered on s (never the legacy stream, which
// would conflict with another thread's graph capture) and complete on return.
void fill_ctab(gllmg_problem* P, hipStream_t s) {
  const int np = ctab_pairs(P->cfg);
  std::vector<double> t(2 * (size_t)np);
  for (auto& L : P->L) {
    double theta, delta;
    cheb_interval(P, L, &theta, &delta);
    std::fill(t.begin(), t.end(), 0.0);
    t[0] = theta;
    t[1] = delta;
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    for (int i = 1; i < np; ++i) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      t[2 * i] = rn * rho;
      t[2 * i + 1] = 2.0 * rn / delta;
      rho = rn;
    }
    GLLMG_HIP(hipMemcpyAsync(L.ctab, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, s));
    GLLMG_HIP(hipStreamSynchronize(s));
  }
}

// k smoothing steps on level l. zero: x starts at 0 (not read). started (with zero): the first
// step from x = 0 has been done already by the restriction's epilogue (Jacobi: x written;
// Chebyshev: d = dinv b / theta written).
void smooth_impl(gllmg_problem* P, int l, int pr, const void* b, void* x, int k, bool zero,
                 hipStream_t s, bool started = false) {
  Level& L = P->L[l];
  const int64_t N = L.g.N;
  if (k <= 0) {
    if (zero) vec_zero(pr, N, x, s);
    return;
  }
  void* r = L.vr[pr];
  void* d = L.vd[pr];
  void* d2 = L.vd2[pr];
  const void* dinv = dinv_of(L, pr);
  if (P->cfg.smoother == GLLMG_SMOOTH_SSOR) {
    // k SSOR steps: colors 0..C-1, then C-1..0, each a launch updating its nodes in place
    if (zero)
      vec_zero(pr, N, x, s);
    else
      zero_boundary(L, pr, x, s);
    const int C = L.n * L.n;
    for (int it = 0; it < k; ++it) {
      for (int c = 0; c < C; ++c) launch_gs_color(L, pr, b, x, dinv, c, P->cfg.omega, s);
      for (int c = C - 1; c >= 0; --c) launch_gs_color(L, pr, b, x, dinv, c, P->cfg.omega, s);
      L.applies += 2;  // a forward and a backward sweep: about two products' arithmetic
    }
    return;
  }
  if (P->cfg.smoother == GLLMG_SMOOTH_BLOCK_JACOBI) {
    // k steps x += omega B^{-1} (b - A x): the residual product, then the element-block update
    const void* Binv = pr == 0 ? (const void*)L.Binv64 : (const void*)L.Binv32;
    if (zero)
      vec_zero(pr, N, x, s);
    else
      zero_boundary(L, pr, x, s);
    for (int it = 0; it < k; ++it) {
      if (it == 0 && zero) {
        launch_block_apply(L, pr, Binv, b, x, P->cfg.omega, s);  // r = b
      } else {
        residual(P, l, pr, b, x, r, s);
        launch_block_apply(L, pr, Binv, r, x, P->cfg.omega, s);
      }
    }
    return;
  }
  if (jacobi_type(P->cfg)) {
    dinv = jacobi_dinv(P, L, pr);
    for (int it = 0; it < k; ++it) {
      if (it == 0 && zero) {
        if (!started) jacobi_step(pr, N, 1, x, b, nullptr, dinv, P->cfg.omega, s);
      } else {
        Epi ep;  // x = x + (omega dinv) (b - A x), fused into the product
        ep.mode = EPI_JACOBI;
        ep.x = x;
        ep.b = b;
        ep.dinv = dinv;
        ep.om = P->cfg.omega;
        apply_epi(P, l, pr, 0, x, ep, s);
      }
    }
    return;
  }
  // Chebyshev acceleration of Jacobi on [cheb_lo lambda, lambda] (Saad, Alg. 12.1 with D^{-1})
  double theta, delta;
  cheb_interval(P, L, &theta, &delta);
  // in a launch group each problem takes its own coefficients from its table (same values as
  // computed here for the first problem, from each problem's lambda_max)
  const bool grp = launch_group() != nullptr;
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  const void* rin;
  if (zero) {
    if (!started) cheb_start(pr, N, b, nullptr, dinv, theta, r, d, s, grp ? L.ctab : nullptr);  // d = dinv b / theta
    rin = b;
  } else {
    Epi ep;  // r = b - A x, d = dinv r / theta
    ep.mode = EPI_CHEB_START;
    ep.b = b;
    ep.r = r;
    ep.d = d;
    ep.dinv = dinv;
    ep.c1 = theta;
    if (grp) ep.cc = L.ctab;
    apply_epi(P, l, pr, 0, x, ep, s);
    rin = r;
  }
  // Degrees 3 and 4: the steps before the last leave x alone and keep their directions in
  // buffers of their own; the last step adds them all to x in the order of the step-by-step
  // updates (same values to the bit, two vector passes fewer per step)
  const bool defer = k == 3 || (k == 4 && L.vd3[pr] != nullptr);
  void* dirs[3] = {d, d2, L.vd3[pr]};
  for (int i = 1; i <= k; ++i) {
    const bool first_zero = zero && i == 1;
    if (defer && i < k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      Epi ep;
      ep.mode = i < k - 1 ? EPI_CHEB_D : EPI_CHEB_SUM;
      ep.from_zero = zero ? 1 : 0;
      ep.x = x;
      ep.rin = rin;
      ep.r = r;
      ep.d = i < k - 1 ? dirs[i] : nullptr;
      ep.e0 = dirs[0];
      ep.e1 = k == 4 ? dirs[1] : nullptr;
      ep.dinv = dinv;
      ep.c1 = rn * rho;
      ep.c2 = 2.0 * rn / delta;
      if (grp) ep.cc = L.ctab + 2 * i;
      apply_epi(P, l, pr, 0, dirs[i - 1], ep, s);
      rin = r;
      rho = rn;
    } else if (i < k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      Epi ep;  // with t = A d: x += d; r = rin - t; d = rn rho d + (2 rn / delta) dinv r
      ep.mode = EPI_CHEB;
      ep.from_zero = first_zero ? 1 : 0;
      ep.last = i == k - 1 ? 1 : 0;  // ... and then x += d, the polynomial's final update
      ep.x = x;
      ep.rin = rin;
      ep.r = r;
      ep.d = d2;  // the next direction goes to the other buffer: d is the product's input
      ep.dinv = dinv;
      ep.c1 = rn * rho;
      ep.c2 = 2.0 * rn / delta;
      if (grp) ep.cc = L.ctab + 2 * i;
      apply_epi(P, l, pr, 0, d, ep, s);
      std::swap(d, d2);
      rin = r;
      rho = rn;
    } else if (k == 1) {  // a degree-1 polynomial has no product to fuse the update into
      if (first_zero)
        vec_copy(pr, N, d, x, s);
      else
        vec_axpy(pr, N, 1.0, d, x, s);
    }
  }
}

// started: the first pre-smoothing step from x = 0 has been done by the restriction
void vcycle_level(gllmg_problem* P, int l, int pr, const void* b, void* x, hipStream_t s,
                  bool started = false) {
  Level& L = P->L[l];
  if (!L.has_coarse) {
    GLLMG_CHECK(L.Ainv64 != nullptr, GLLMG_EUNSUPPORTED,
                "the coarsest level is too large for the dense exact solve; allow more levels");
    launch_coarse_solve(L, pr, b, x, s);
    return;
  }
  Level& C = P->L[l + 1];
  smooth_impl(P, l, pr, b, x, P->cfg.nu_pre, true, s, started);
  residual(P, l, pr, b, x, L.vr[pr], s);
  // b_c = P^T r, and with it the coarse level's first smoothing step from x_c = 0
  Epi ep;
  ep.y = C.vb[pr];
  // the coarse level's first pre-smoothing step from zero rides on the restriction's gather
  // (Jacobi and Chebyshev; the Gauss-Seidel sweeps start from a cleared vector instead)
  const bool fuse = C.has_coarse && P->cfg.nu_pre > 0 &&
                    (jacobi_type(P->cfg) || P->cfg.smoother == GLLMG_SMOOTH_CHEBYSHEV);
  if (fuse && jacobi_type(P->cfg)) {
    ep.mode = EPI_STORE_JACOBI0;
    ep.x = C.vx[pr];
    ep.dinv = jacobi_dinv(P, C, pr);
    ep.om = P->cfg.omega;
  } else if (fuse) {
    double theta, delta;
    cheb_interval(P, C, &theta, &delta);
    ep.mode = EPI_STORE_CHEB0;
    ep.d = C.vd[pr];
    ep.dinv = dinv_of(C, pr);
    ep.c1 = theta;
    if (launch_group()) ep.cc = C.ctab;
  }
  launch_restrict(L, C, pr, L.vr[pr], ep, P->F, s);
  vcycle_level(P, l + 1, pr, C.vb[pr], C.vx[pr], s, fuse);
  launch_prolong(L, C, pr, C.vx[pr], x, true, s);
  smooth_impl(P, l, pr, b, x, P->cfg.nu_post, false, s);
}

// First-order hierarchy: z = low_cycles sweeps x <- x + V_1 (r - A_1 x) from x = 0 at level 1
// (whose nodes are level 0's), in precision pr; level 1's b and x vectors hold the residual and
// the correction (the V-cycle from level 1 takes r and z as its own b and x).
void low_sweeps(gllmg_problem* P, int pr, const void* r, void* z, hipStream_t s) {
  Level& L1 = P->L[1];
  vcycle_level(P, 1, pr, r, z, s);
  for (int it = 1; it < P->cfg.low_cycles; ++it) {
    residual(P, 1, pr, r, z, L1.vb[pr], s);
    vcycle_level(P, 1, pr, L1.vb[pr], L1.vx[pr], s);
    vec_axpy(pr, L1.g.N, 1.0, L1.vx[pr], z, s);
  }
}

// The preconditioner in precision pr on vectors of that precision: the V-cycle, or the
// first-order sweeps.
void precond_level0(gllmg_problem* P, int pr, const void* r, void* z, hipStream_t s) {
  if (low_first(P))
    low_sweeps(P, pr, r, z, s);
  else
    vcycle_level(P, 0, pr, r, z, s);
}

// device scalars of a solve in P->scal: (r, r), (p, A p), the two (z, r), (b - A x, b - A x);
// the inner CG of the iterative refinement: its two (z, r) and (p, A p)
enum { S_RR = 0, S_PH = 1, S_G0 = 2, S_G1 = 3, S_B = 4, S_IG0 = 10, S_IG1 = 11, S_IPH = 12 };

// z = V r for the solve's FP64 residual r = P->pr, with (r, r) in scal[S_RR], into z on the
// finest level, in the problem's V-cycle precision. An FP32 preconditioner sees r scaled by a
// power of two to norm about 1 and its result is scaled back (pow2_inv_norm).
void precond_eager(gllmg_problem* P, const double* r, double* z, hipStream_t s) {
  GLLMG_CHECK(r == P->pr, GLLMG_EINVAL, "the preconditioner runs on the solve's residual vector");
  Level& L = P->L[0];
  const double* rr = P->scal + S_RR;
  if (P->vprec == 0) {
    precond_level0(P, 0, r, z, s);
  } else {
    cast_64_32(L.g.N, r, (float*)L.vb[1], s, rr);
    precond_level0(P, 1, L.vb[1], L.vx[1], s);
    cast_32_64(L.g.N, (const float*)L.vx[1], z, s, rr);
  }
}

void drop_graph(gllmg_problem* P) {
  if (P->vexec) (void)hipGraphExecDestroy(P->vexec);
  P->vexec = nullptr;
}

// Capture the launch sequence of one V-cycle from P->pr to P->pz (kernels only: no copies,
// memsets or synchronization) on a private stream of default priority. Relaxed mode: other
// threads of the process (a server's setup thread, say) may keep issuing synchronous HIP
// calls while the capture is open.
void capture_vcycle(gllmg_problem* P) {
  GLLMG_CHECK(P->cap != nullptr, GLLMG_EDEVICE, "no capture stream");
  std::vector<int64_t> a0;
  for (auto& L : P->L) a0.push_back(L.applies);
  GLLMG_HIP(hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed));
  hipGraph_t g = nullptr;
  try {
    precond_eager(P, P->pr, P->pz, P->cap);
  } catch (...) {
    (void)hipStreamEndCapture(P->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  GLLMG_HIP(hipStreamEndCapture(P->cap, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) throw Error(GLLMG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  P->vexec = ex;
  P->vapplies.assign(P->L.size(), 0);
  for (size_t l = 0; l < P->L.size(); ++l) {
    P->vapplies[l] = P->L[l].applies - a0[l];
    P->L[l].applies = a0[l];
  }
}

// (Re)capture the V-cycle graph if the problem uses one; if capture fails the same kernels are
// launched one by one instead.
void recapture(gllmg_problem* P) {
  drop_graph(P);
  if (!P->use_graph || !P->L.back().Ainv64) return;
  try {
    capture_vcycle(P);
  } catch (const Error&) {
    (void)hipGetLastError();
    P->use_graph = false;
  }
}

void precond(gllmg_problem* P, const double* r, double* z, hipStream_t s) {
  if (!P->use_graph || !P->vexec || r != P->pr || z != P->pz) {
    precond_eager(P, r, z, s);
    return;
  }
  GLLMG_HIP(hipGraphLaunch(P->vexec, s));
  for (size_t l = 0; l < P->L.size(); ++l) P->L[l].applies += P->vapplies[l];
}

enum { PH_INIT = 0, PH_ITER = 1, PH_FINAL = 2 };

// Host-visible scalars of the solve arrive in the pinned buffer hbuf through stream-ordered
// copies followed by an event; the state machine advances only when that event has completed,
// so the host never blocks inside solve_poll.
void post_scalars(gllmg_problem* P, int src, int cnt, int dst) {
  auto& v = P->sv;
  GLLMG_HIP(hipMemcpyAsync(P->hbuf + dst, P->scal + src, sizeof(double) * cnt,
                           hipMemcpyDeviceToHost, v.s));
  GLLMG_HIP(hipEventRecord(v.ev, v.s));
}
// the reductions wrote their results to hbuf themselves: only the event
void post_event(gllmg_problem* P) { GLLMG_HIP(hipEventRecord(P->sv.ev, P->sv.s)); }

// One PCG iteration up to its convergence data: h = A p; (p, h); x += alpha p; r -= alpha h;
// (r, r). One MG iteration: z = V r; x += z; r = b - A x; (r, r).
void enqueue_iteration(gllmg_problem* P) {
  auto& v = P->sv;
  const int64_t N = P->L[0].g.N;
  if (v.mode == GLLMG_MODE_PCG) {
    apply_level(P, 0, 0, 0, P->pp, P->ph, v.s);
    dot(0, N, P->pp, P->ph, P->part, P->scal + S_PH, v.s, P->hbuf + 1);
    pcg_update_xr(N, P->scal, v.g, S_PH, v.x, P->pr, P->pp, P->ph, P->part, P->scal + S_RR, v.s,
                  P->hbuf);
  } else {
    precond(P, P->pr, P->pz, v.s);
    vec_axpy(0, N, 1.0, P->pz, v.x, v.s);
    residual(P, 0, 0, v.b, v.x, P->pr, v.s);
    dot(0, N, P->pr, P->pr, P->part, P->scal + S_RR, v.s, P->hbuf);
  }
  post_event(P);
  v.phase = PH_ITER;
  // PCG: unless this iteration may well be the last (its residual norm, extrapolated from the
  // last two, within 10x of the target, or maxit next), the next V-cycle is enqueued now, so
  // that the GPU does not wait for the host to read the norm; the same kernels in the same
  // order as without it. If the solve ends here after all, its result is simply not used.
  v.spec = false;
  const size_t h = v.hist.size();
  if (v.mode == GLLMG_MODE_PCG && v.iters + 1 < v.maxit && h >= 2 && v.hist[h - 2] > 0.0) {
    const double pred = v.hist[h - 1] * (v.hist[h - 1] / v.hist[h - 2]);
    if (std::isfinite(pred) && pred > 10.0 * v.rtol * v.n0) {
      v.spec_applies.resize(P->L.size());
      for (size_t l = 0; l < P->L.size(); ++l) v.spec_applies[l] = P->L[l].applies;
      precond(P, P->pr, P->pz, v.s);
      for (size_t l = 0; l < P->L.size(); ++l) v.spec_applies[l] = P->L[l].applies - v.spec_applies[l];
      v.spec = true;
    }
  }
}

// the speculative V-cycle goes unused: its products leave the counts
void drop_spec(gllmg_problem* P) {
  auto& v = P->sv;
  if (!v.spec) return;
  for (size_t l = 0; l < P->L.size() && l < v.spec_applies.size(); ++l) P->L[l].applies -= v.spec_applies[l];
  v.spec = false;
}

void enqueue_final(gllmg_problem* P) {
  auto& v = P->sv;
  const int64_t N = P->L[0].g.N;
  if (v.n0 > 0.0 && std::isfinite(v.n0)) {
    residual(P, 0, 0, v.b, v.x, P->pt, v.s);
    dot(0, N, P->pt, P->pt, P->part, P->scal + S_B, v.s, P->hbuf + 2);
    post_event(P);
  } else {
    post_scalars(P, S_B, 1, 2);
  }
  v.phase = PH_FINAL;
}

void solve_begin(gllmg_problem* P, int mode, const double* b, double* x, double rtol, int maxit,
                 hipStream_t s) {
  auto& v = P->sv;
  GLLMG_CHECK(!v.active, GLLMG_EINVAL, "a solve is already in progress on this problem");
  hipEvent_t ev = v.ev;  // made at setup
  v = gllmg_problem::Solve{};
  v.ev = ev;
  v.active = true;
  v.mode = mode;
  v.b = b;
  v.x = x;
  v.rtol = rtol;
  v.maxit = maxit;
  v.s = s;
  v.t0 = std::chrono::steady_clock::now();
  for (auto& lv : P->L) v.a0.push_back(lv.applies);
  const int64_t N = P->L[0].g.N;
  residual(P, 0, 0, b, x, P->pr, s);
  dot(0, N, P->pr, P->pr, P->part, P->scal + S_RR, s, P->hbuf);
  post_event(P);
  v.phase = PH_INIT;
}

bool solve_poll_impl(gllmg_problem* P);

// Advance without blocking; returns true when the solve has finished. A failure while
// advancing ends the solve: the stream is drained (so b, x and the internal vectors are no
// longer in use) and the problem accepts a new solve.
bool solve_poll(gllmg_problem* P) {
  auto& v = P->sv;
  GLLMG_CHECK(v.active, GLLMG_EINVAL, "no solve in progress");
  try {
    return solve_poll_impl(P);
  } catch (...) {
    (void)hipStreamSynchronize(v.s);
    (void)hipGetLastError();
    v.active = false;
    throw;
  }
}

bool solve_poll_impl(gllmg_problem* P) {
  auto& v = P->sv;
  while (!v.done) {
    const hipError_t q = hipEventQuery(v.ev);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess) throw Error(GLLMG_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(q));
    const int64_t N = P->L[0].g.N;
    if (v.phase == PH_INIT) {
      v.n0 = std::sqrt(P->hbuf[0]);
      v.nr = v.n0;
      v.hist.assign(1, v.n0);
      v.conv = v.n0 == 0.0;
      v.breakdown = !std::isfinite(v.n0);
      if (v.conv || v.breakdown) {
        enqueue_final(P);
        continue;
      }
      if (v.mode == GLLMG_MODE_PCG) {
        precond(P, P->pr, P->pz, v.s);
        dot(0, N, P->pz, P->pr, P->part, P->scal + S_G0, v.s);
        vec_copy(0, N, P->pz, P->pp, v.s);
        v.g = S_G0;
      }
      enqueue_iteration(P);
    } else if (v.phase == PH_ITER) {
      const double rr = P->hbuf[0], ph = P->hbuf[1];
      ++v.iters;
      v.nr = std::sqrt(rr);
      v.hist.push_back(v.nr);
      if ((v.mode == GLLMG_MODE_PCG && !(ph > 0.0)) || !std::isfinite(v.nr)) {
        v.breakdown = true;
        drop_spec(P);
        enqueue_final(P);
      } else if (v.nr <= v.rtol * v.n0) {
        v.conv = true;
        drop_spec(P);
        enqueue_final(P);
      } else if (v.iters >= v.maxit) {
        drop_spec(P);
        enqueue_final(P);
      } else {
        if (v.mode == GLLMG_MODE_PCG) {
          if (!v.spec) precond(P, P->pr, P->pz, v.s);
          v.spec = false;
          const int gn = v.g == S_G0 ? S_G1 : S_G0;
          dot(0, N, P->pz, P->pr, P->part, P->scal + gn, v.s);
          pcg_update_p(N, P->scal, gn, v.g, P->pp, P->pz, v.s);
          v.g = gn;
        }
        enqueue_iteration(P);
      }
    } else {
      v.rt = (v.n0 > 0.0 && std::isfinite(v.n0)) ? std::sqrt(P->hbuf[2]) / v.n0 : 0.0;
      v.done = true;
    }
  }
  return true;
}

gllmg_status solve_end(gllmg_problem* P, gllmg_solve_stats* st) {
  auto& v = P->sv;
  GLLMG_CHECK(v.active, GLLMG_EINVAL, "no solve in progress");
  while (!solve_poll(P)) GLLMG_HIP(hipEventSynchronize(v.ev));
  v.active = false;
  if (st) {
    st->iters = v.iters;
    st->converged = v.conv ? 1 : 0;
    st->relres = v.n0 > 0.0 ? v.nr / v.n0 : 0.0;
    st->relres_true = v.rt;
    for (int i = 0; i < 16; ++i) st->applies[i] = 0;
    for (size_t i = 0; i < P->L.size() && i < 16; ++i) st->applies[i] = P->L[i].applies - v.a0[i];
    if (st->history)
      for (size_t i = 0; i < v.hist.size() && i <= (size_t)v.maxit; ++i) st->history[i] = v.hist[i];
    st->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - v.t0).count();
  }
  if (v.breakdown) throw Error(GLLMG_EBREAKDOWN, "breakdown: non-finite residual or p^T A p <= 0");
  if (!v.conv) return GLLMG_ENOTCONV;
  return GLLMG_OK;
}

// Iterative refinement (GLLMG_MODE_IR): FP64 residuals outside, cfg.ir_inner steps of FP32 CG
// preconditioned by the FP32 V-cycle inside, on the residual scaled by a power of two; the inner
// steps run on the device without host round trips (their scalars stay in P->scal), one
// read-back per refinement step.
gllmg_status ir_solve(gllmg_problem* P, const double* b, double* x, double rtol, int maxit,
                      gllmg_solve_stats* st, hipStream_t s) {
  GLLMG_CHECK(P->ir32 != nullptr, GLLMG_EUNSUPPORTED,
              "iterative refinement needs ir_inner > 0 and the FP32 V-cycle at setup");
  GLLMG_CHECK(!P->sv.active, GLLMG_EINVAL, "a solve is already in progress on this problem");
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<int64_t> a0;
  for (auto& L : P->L) a0.push_back(L.applies);
  const int64_t N = P->L[0].g.N;
  float* r32 = P->ir32;
  float* z32 = r32 + N;
  float* p32 = z32 + N;
  float* h32 = p32 + N;
  float* e32 = h32 + N;
  auto residual_norm = [&]() {
    residual(P, 0, 0, b, x, P->pr, s);
    dot(0, N, P->pr, P->pr, P->part, P->scal + S_RR, s);
    GLLMG_HIP(hipMemcpyAsync(P->hbuf, P->scal + S_RR, sizeof(double), hipMemcpyDeviceToHost, s));
    GLLMG_HIP(hipStreamSynchronize(s));
    return std::sqrt(P->hbuf[0]);
  };
  const double n0 = residual_norm();
  std::vector<double> hist{n0};
  double nr = n0;
  int iters = 0;
  bool conv = n0 == 0.0, breakdown = !std::isfinite(n0);
  // inner length: k for the first step; after it, the mean rate per CG step of the previous
  // refinement step (its residual reduction to the power 1/length) predicts how many steps
  // reach the tolerance, and a step runs that many (at most k) instead of k
  double rate = 0.0;
  while (!conv && !breakdown && iters < maxit) {
    int m = std::min(P->cfg.ir_inner, maxit - iters);
    if (rate > 0.0 && rate < 1.0) {
      const double need = rtol * n0 / nr;
      const double q = need < 1.0 ? std::ceil(std::log(need) / std::log(rate)) : 1.0;
      if (q < (double)m) m = std::max(1, (int)q);  // compared as doubles: q may exceed int range
    }
    cast_64_32(N, P->pr, r32, s, P->scal + S_RR);
    vec_zero(1, N, e32, s);
    precond_level0(P, 1, r32, z32, s);
    dot(1, N, z32, r32, P->part, P->scal + S_IG0, s);
    vec_copy(1, N, z32, p32, s);
    int g = S_IG0;
    for (int it = 0; it < m; ++it) {
      apply_level(P, 0, 1, 0, p32, h32, s);
      dot(1, N, p32, h32, P->part, P->scal + S_IPH, s);
      ir_update_er(N, P->scal, g, S_IPH, e32, r32, p32, h32, s);
      if (it + 1 == m) break;
      precond_level0(P, 1, r32, z32, s);
      const int gn = g == S_IG0 ? S_IG1 : S_IG0;
      dot(1, N, z32, r32, P->part, P->scal + gn, s);
      ir_update_p(N, P->scal, gn, g, p32, z32, s);
      g = gn;
    }
    iters += m;
    ir_add(N, e32, P->scal + S_RR, x, s);  // S_RR still holds the scaled residual's (r, r)
    const double before = nr;
    nr = residual_norm();
    hist.push_back(nr);
    rate = nr > 0.0 && nr < before ? std::pow(nr / before, 1.0 / m) : 0.0;
    breakdown = !std::isfinite(nr);
    conv = !breakdown && nr <= rtol * n0;
  }
  if (st) {
    st->iters = iters;
    st->converged = conv ? 1 : 0;
    st->relres = n0 > 0.0 ? nr / n0 : 0.0;
    st->relres_true = st->relres;
    for (int i = 0; i < 16; ++i) st->applies[i] = 0;
    for (size_t i = 0; i < P->L.size() && i < 16; ++i) st->applies[i] = P->L[i].applies - a0[i];
    if (st->history) {
      for (size_t i = 0; i < hist.size() && i <= (size_t)maxit; ++i) st->history[i] = hist[i];
      if (hist.size() <= (size_t)maxit) st->history[hist.size()] = -1.0;  // end of the list
    }
    st->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (breakdown) throw Error(GLLMG_EBREAKDOWN, "breakdown: non-finite residual");
  if (!conv) return GLLMG_ENOTCONV;
  return GLLMG_OK;
}

gllmg_status solve_impl(gllmg_problem* P, int mode, const double* b, double* x, double rtol,
                        int maxit, gllmg_solve_stats* st, hipStream_t s) {
  if (mode == GLLMG_MODE_IR) return ir_solve(P, b, x, rtol, maxit, st, s);
  solve_begin(P, mode, b, x, rtol, maxit, s);
  return solve_end(P, st);
}

// ------------------------------------------------------------------ persistent batched solver
// Problems it takes: 3D, FP32 V-cycle, at most kBatchMaxLevels levels and kBatchMaxNodes fine
// nodes, an exact coarse solve, orders along the chain n0, n0/2 + 1, ..., 2 (h-coarsening at
// n0 or at 2), and maxit below the history capacity.
bool batch_eligible(const gllmg_problem* P, int maxit) {
  if (!P->persistent || P->cfg.dim != 3 || P->vprec != 1) return false;
  if (P->cfg.hierarchy == GLLMG_HIER_LOW) return false;
  if (P->cfg.quadrature != GLLMG_QUAD_GLL) return false;
  if (P->cfg.smoother != GLLMG_SMOOTH_JACOBI && P->cfg.smoother != GLLMG_SMOOTH_CHEBYSHEV) return false;
  if (P->L.size() > (size_t)kBatchMaxLevels || !P->L.back().Ainv64) return false;
  if (maxit >= kBatchHist || P->L[0].g.N > kBatchMaxNodes) return false;
  const int n0 = P->L[0].n;
  if (n0 < 2 || n0 > 17) return false;
  auto in_chain = [&](int n) {
    for (int m = n0;; m = m / 2 + 1) {
      if (m == n) return true;
      if (m <= 2) return false;
    }
  };
  for (size_t l = 0; l < P->L.size(); ++l) {
    const Level& L = P->L[l];
    if (!in_chain(L.n)) return false;
    if (l + 1 < P->L.size() && L.tp.nch == 2 && L.n != n0 && L.n != 2) return false;
  }
  return true;
}

void batch_fill(const gllmg_problem* P, BatchProblem& d) {
  d.nlev = (int)P->L.size();
  d.smoother = P->cfg.smoother;
  d.nu_pre = P->cfg.nu_pre;
  d.nu_post = P->cfg.nu_post;
  d.vprec = P->vprec;
  d.omega = P->cfg.omega;
  d.F = P->F;
  d.zero = P->zeros;
  d.pr = P->pr;
  d.pz = P->pz;
  d.pp = P->pp;
  d.ph = P->ph;
  d.pt = P->pt;
  for (size_t l = 0; l < P->L.size(); ++l) {
    const Level& L = P->L[l];
    BatchLevel& b = d.L[l];
    b.g = L.g;
    b.n = L.n;
    b.has_coarse = L.has_coarse ? 1 : 0;
    b.nch = L.tp.nch;
    b.nint = L.nint;
    const double lam = L.lmax, alpha = P->cfg.cheb_lo * lam;
    b.theta = 0.5 * (lam + alpha);
    b.delta = 0.5 * (lam - alpha);
    b.G64 = L.G64;
    b.G32 = L.G32;
    b.D64 = L.D64;
    b.D32 = L.D32;
    b.dinv64 = L.dinv64;
    b.dinv32 = L.dinv32;
    b.P64 = L.tp.P64;
    b.P32 = L.tp.P32;
    b.Ainv64 = L.Ainv64;
    b.Ainv32 = L.Ainv32;
    for (int q = 0; q < 2; ++q) {
      b.vb[q] = L.vb[q];
      b.vx[q] = L.vx[q];
      b.vr[q] = L.vr[q];
      b.vd[q] = L.vd[q];
      b.vd2[q] = L.vd2[q];
    }
  }
}

thread_local const LaunchGroup* g_launch_group = nullptr;

// ------------------------------------------------------------------ launch groups of a batch
// Smoothers whose kernels take launch groups (the Gauss-Seidel passes do not).
bool groupable_smoother(int sm) {
  return sm == GLLMG_SMOOTH_JACOBI || sm == GLLMG_SMOOTH_CHEBYSHEV || sm == GLLMG_SMOOTH_L1_JACOBI;
}

// Problems that a launch group can take together: the same levels, smoother and V-cycle
// precision, and every device buffer at the same offset in its workspace (the layout is a
// function of the configuration, so equal configurations give equal offsets).
bool same_shape(const gllmg_problem* A, const gllmg_problem* B) {
  const gllmg_config &a = A->cfg, &b = B->cfg;
  if (a.dim != b.dim || a.smoother != b.smoother || a.nu_pre != b.nu_pre ||
      a.nu_post != b.nu_post || a.omega != b.omega || A->vprec != B->vprec ||
      A->L.size() != B->L.size())
    return false;
  auto collect = [](const gllmg_problem* P, std::vector<int64_t>& o) {
    auto off = [P](const void* q) { return q ? (int64_t)((const char*)q - P->ws) : (int64_t)-1; };
    for (const auto& L : P->L) {
      o.insert(o.end(), {L.g.ne[0], L.g.ne[1], L.g.ne[2], L.g.p, (int64_t)L.has_coarse,
                         (int64_t)L.tp.nch, off(L.G64), off(L.G32), off(L.D64), off(L.D32),
                         off(L.dinv64), off(L.dinv32), off(L.tp.P64), off(L.tp.P32), off(L.Ainv64),
                         off(L.Ainv32), off(L.ctab), off(L.zero), off(L.l1inv64), off(L.l1inv32)});
      for (int q = 0; q < 2; ++q)
        o.insert(o.end(), {off(L.vb[q]), off(L.vx[q]), off(L.vr[q]), off(L.vd[q]), off(L.vd2[q]),
                           off(L.vd3[q])});
    }
    o.insert(o.end(), {off(P->F), off(P->scal), off(P->part), off(P->pr), off(P->pz), off(P->pp),
                       off(P->ph), off(P->pt), off(P->zeros)});
  };
  std::vector<int64_t> oa, ob;
  collect(A, oa);
  collect(B, ob);
  return oa == ob;
}

// Result of one problem of a group solve.
struct GroupOut {
  int iters = 0;
  bool conv = false, breakdown = false;
  double n0 = 0, nr = 0, rt = 0;
  std::vector<double> hist;
};

// Makes a launch group current for this thread while it lives.
struct GroupScope {
  explicit GroupScope(const LaunchGroup* g) { set_launch_group(g); }
  ~GroupScope() { set_launch_group(nullptr); }
};

// PCG (Alg. 1 of the paper with the V-cycle preconditioner) on K problems of one shape in
// lockstep: every kernel of an iteration runs once for all problems still iterating (a
// problem leaves the launches when it has converged, broken down or reached maxit). Each
// problem follows exactly the arithmetic of its own solve (same kernels, same reduction
// trees), so the results equal gllmg_solve's bit for bit. The group's buffers are the first
// problem's (its workspace and pinned images, made at setup), so at most kGroupMax problems.
// Synchronous on s.
void group_solve(const std::vector<gllmg_problem*>& G, const std::vector<const double*>& bu,
                 const std::vector<double*>& xu, double rtol, int maxit, hipStream_t s,
                 std::vector<GroupOut>& out) {
  const int K = (int)G.size();
  gllmg_problem* P0 = G[0];
  GLLMG_CHECK(K >= 1 && K <= kGroupMax, GLLMG_EINVAL, "launch group size out of range");
  struct {
    int64_t* dlt;
    int* act;
    double* sc;
    int* hact;
    double* hsc;
  } m{P0->gdlt, P0->gact, P0->gsc, P0->ghact, P0->ghsc};
  const int64_t N = P0->L[0].g.N;
  std::vector<int64_t> hd(K);
  for (int k = 0; k < K; ++k) hd[k] = G[k]->ws - P0->ws;
  GLLMG_HIP(hipMemcpyAsync(m.dlt, hd.data(), sizeof(int64_t) * K, hipMemcpyHostToDevice, s));
  GLLMG_HIP(hipStreamSynchronize(s));
  // b and x in workspace vectors unused by the FP64 solve on level 0 (every buffer a group
  // kernel touches must lie in the workspaces)
  double* bw = (double*)P0->L[0].vb[0];
  double* xw = (double*)P0->L[0].vx[0];
  for (int k = 0; k < K; ++k) {
    GLLMG_HIP(hipMemcpyAsync((char*)bw + hd[k], bu[k], sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    GLLMG_HIP(hipMemcpyAsync((char*)xw + hd[k], xu[k], sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  }
  out.assign(K, GroupOut{});
  std::vector<char> on(K, 1);
  auto any = [](const std::vector<char>& v) { return std::find(v.begin(), v.end(), 1) != v.end(); };
  {
    const LaunchGroup lg{{m.dlt, m.act}, K};
    GroupScope scope(&lg);
    auto set_act = [&](const std::vector<char>& a) {
      GLLMG_HIP(hipStreamSynchronize(s));  // the pinned image is no longer being read
      for (int k = 0; k < K; ++k) m.hact[k] = a[k];
      GLLMG_HIP(hipMemcpyAsync(m.act, m.hact, sizeof(int) * K, hipMemcpyHostToDevice, s));
    };
    auto collect = [&](int src, int cnt) {
      collect_scalars(P0->scal + src, cnt, m.sc, s);
      GLLMG_HIP(hipMemcpyAsync(m.hsc, m.sc, sizeof(double) * cnt * K, hipMemcpyDeviceToHost, s));
      GLLMG_HIP(hipStreamSynchronize(s));
    };
    // the first problem's product counters advance once per launch; each phase's count goes
    // to the problems that took part in it
    std::vector<int64_t> c0(P0->L.size());
    auto mark = [&]() {
      for (size_t l = 0; l < P0->L.size(); ++l) c0[l] = P0->L[l].applies;
    };
    auto credit = [&](const std::vector<char>& who) {
      for (size_t l = 0; l < P0->L.size(); ++l) {
        const int64_t d = P0->L[l].applies - c0[l];
        P0->L[l].applies = c0[l];
        for (int k = 0; k < K; ++k)
          if (who[k]) G[k]->L[l].applies += d;
      }
    };
    set_act(on);
    mark();
    residual(P0, 0, 0, bw, xw, P0->pr, s);
    dot(0, N, P0->pr, P0->pr, P0->part, P0->scal + S_RR, s);
    credit(on);
    collect(S_RR, 1);
    for (int k = 0; k < K; ++k) {
      GroupOut& o = out[k];
      o.n0 = o.nr = std::sqrt(m.hsc[k]);
      o.hist.assign(1, o.n0);
      o.conv = o.n0 == 0.0;
      o.breakdown = !std::isfinite(o.n0);
      if (o.conv || o.breakdown) on[k] = 0;
    }
    int g = S_G0;
    if (any(on)) {
      set_act(on);
      mark();
      precond_eager(P0, P0->pr, P0->pz, s);
      dot(0, N, P0->pz, P0->pr, P0->part, P0->scal + S_G0, s);
      vec_copy(0, N, P0->pz, P0->pp, s);
      credit(on);
    }
    while (any(on)) {
      mark();
      apply_level(P0, 0, 0, 0, P0->pp, P0->ph, s);
      dot(0, N, P0->pp, P0->ph, P0->part, P0->scal + S_PH, s);
      pcg_update_xr(N, P0->scal, g, S_PH, xw, P0->pr, P0->pp, P0->ph, P0->part, P0->scal + S_RR, s);
      credit(on);
      collect(S_RR, 2);
      for (int k = 0; k < K; ++k) {
        if (!on[k]) continue;
        GroupOut& o = out[k];
        const double rr = m.hsc[2 * k], ph = m.hsc[2 * k + 1];
        ++o.iters;
        o.nr = std::sqrt(rr);
        o.hist.push_back(o.nr);
        if (!(ph > 0.0) || !std::isfinite(o.nr)) {
          o.breakdown = true;
          on[k] = 0;
        } else if (o.nr <= rtol * o.n0) {
          o.conv = true;
          on[k] = 0;
        } else if (o.iters >= maxit) {
          on[k] = 0;
        }
      }
      if (!any(on)) break;
      set_act(on);
      mark();
      precond_eager(P0, P0->pr, P0->pz, s);
      const int gn = g == S_G0 ? S_G1 : S_G0;
      dot(0, N, P0->pz, P0->pr, P0->part, P0->scal + gn, s);
      pcg_update_p(N, P0->scal, gn, g, P0->pp, P0->pz, s);
      credit(on);
      g = gn;
    }
    // the true residual b - A x of every problem with a finite, nonzero initial residual
    std::vector<char> fin(K);
    for (int k = 0; k < K; ++k) fin[k] = out[k].n0 > 0.0 && std::isfinite(out[k].n0);
    if (any(fin)) {
      set_act(fin);
      mark();
      residual(P0, 0, 0, bw, xw, P0->pt, s);
      dot(0, N, P0->pt, P0->pt, P0->part, P0->scal + S_B, s);
      credit(fin);
      collect(S_B, 1);
      for (int k = 0; k < K; ++k)
        if (fin[k]) out[k].rt = std::sqrt(m.hsc[k]) / out[k].n0;
    }
  }
  for (int k = 0; k < K; ++k)
    GLLMG_HIP(hipMemcpyAsync(xu[k], (char*)xw + hd[k], sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  GLLMG_HIP(hipStreamSynchronize(s));
}

thread_local std::string g_err;

template <class Fn>
gllmg_status guard(Fn&& fn) {
  try {
    return fn();
  } catch (const Error& e) {
    g_err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return GLLMG_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return GLLMG_EINVAL;
  }
}

// Everything gllmg_setup made besides the host object itself.
// Host-side resources of one problem: pinned scalar and descriptor images, two private
// streams, three events. Freeing pinned memory synchronizes the whole device, so problems
// return them to a per-device pool when destroyed and later setups on that device take them
// from there: past the first problems of a process, setup and destroy neither allocate host
// resources nor wait for other work on the device (a server creating and destroying
// problems while others solve). The pool lives until the process ends.
struct HostRes {
  double* hbuf = nullptr;
  BatchProblem* bhost = nullptr;
  int* ghact = nullptr;
  double* ghsc = nullptr;
  hipStream_t xs = nullptr, cap = nullptr;
  hipEvent_t ev = nullptr, bev = nullptr, gev = nullptr;
};
std::mutex g_host_pool_mu;
std::map<int, std::vector<HostRes>> g_host_pool;

HostRes take_host_res(int dev) {
  {
    std::lock_guard<std::mutex> lk(g_host_pool_mu);
    std::vector<HostRes>& v = g_host_pool[dev];
    if (!v.empty()) {
      HostRes r = v.back();
      v.pop_back();
      return r;
    }
  }
  HostRes r;
  try {
    GLLMG_HIP(hipHostMalloc((void**)&r.hbuf, sizeof(double) * 64, hipHostMallocDefault));
    GLLMG_HIP(hipHostMalloc((void**)&r.bhost, sizeof(BatchProblem), hipHostMallocDefault));
    GLLMG_HIP(hipHostMalloc((void**)&r.ghact, sizeof(int) * kGroupMax, hipHostMallocDefault));
    GLLMG_HIP(hipHostMalloc((void**)&r.ghsc, sizeof(double) * 4 * kGroupMax, hipHostMallocDefault));
    GLLMG_HIP(hipStreamCreateWithFlags(&r.xs, hipStreamNonBlocking));
    GLLMG_HIP(hipStreamCreateWithFlags(&r.cap, hipStreamNonBlocking));
    GLLMG_HIP(hipEventCreateWithFlags(&r.ev, hipEventDisableTiming));
    GLLMG_HIP(hipEventCreateWithFlags(&r.bev, hipEventDisableTiming));
    GLLMG_HIP(hipEventCreateWithFlags(&r.gev, hipEventDisableTiming));
  } catch (...) {  // a partly made set is freed at once (setup's own failure path)
    if (r.cap) (void)hipStreamDestroy(r.cap);
    if (r.xs) (void)hipStreamDestroy(r.xs);
    for (hipEvent_t e : {r.ev, r.bev, r.gev})
      if (e) (void)hipEventDestroy(e);
    for (void* h : {(void*)r.hbuf, (void*)r.bhost, (void*)r.ghact, (void*)r.ghsc})
      if (h) (void)hipHostFree(h);
    throw;
  }
  return r;
}

// Back to the pool once everything of the problem that uses them has finished: its own
// streams and its last recorded events (a solve's scalar copies into hbuf, a batch's
// descriptors and group scalars); waits on nothing else.
void give_host_res(int dev, const HostRes& r) {
  (void)hipStreamSynchronize(r.xs);
  (void)hipStreamSynchronize(r.cap);
  for (hipEvent_t e : {r.ev, r.bev, r.gev}) (void)hipEventSynchronize(e);
  (void)hipGetLastError();
  std::lock_guard<std::mutex> lk(g_host_pool_mu);
  g_host_pool[dev].push_back(r);
}

void release_resources(gllmg_problem* P) {
  drop_graph(P);
  if (P->owns_ws) (void)hipFree(P->ws);
  if (P->hbuf) {
    HostRes r;
    r.hbuf = P->hbuf;
    r.bhost = P->bhost;
    r.ghact = P->ghact;
    r.ghsc = P->ghsc;
    r.xs = P->xs;
    r.cap = P->cap;
    r.ev = P->sv.ev;
    r.bev = P->bev;
    r.gev = P->gev;
    give_host_res(P->dev, r);
  }
  P->cap = P->xs = nullptr;
  P->sv.ev = P->bev = P->gev = nullptr;
  P->hbuf = nullptr;
  P->bhost = nullptr;
  P->ghact = nullptr;
  P->ghsc = nullptr;
  if (P->owns_ws) P->ws = nullptr;
}

const Level& level_of(const gllmg_problem* P, int l) {
  GLLMG_CHECK(P != nullptr, GLLMG_EINVAL, "problem is NULL");
  GLLMG_CHECK(l >= 0 && l < (int)P->L.size(), GLLMG_EINVAL, "level out of range");
  return P->L[l];
}

int prec_index(const gllmg_problem* P, int prec) {
  GLLMG_CHECK(prec == GLLMG_F64 || prec == GLLMG_F32, GLLMG_EINVAL, "bad precision");
  if (prec == GLLMG_F32)
    GLLMG_CHECK(P->cfg.vcycle_prec == GLLMG_F32, GLLMG_EUNSUPPORTED,
                "FP32 data needs a problem set up with vcycle_prec = GLLMG_F32");
  return prec == GLLMG_F64 ? 0 : 1;
}

void check_ptr(const void* p, size_t align, const char* what) {
  GLLMG_CHECK(p != nullptr, GLLMG_EINVAL, std::string(what) + " is NULL");
  GLLMG_CHECK(((uintptr_t)p % align) == 0, GLLMG_EINVAL, std::string(what) + " is misaligned");
}

}  // namespace

const LaunchGroup* launch_group() { return g_launch_group; }
void set_launch_group(const LaunchGroup* g) { g_launch_group = g; }

}  // namespace gllmg

extern "C" {

const char* gllmg_last_error(void) { return gllmg::g_err.c_str(); }

void gllmg_config_default(gllmg_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->dim = 3;
  c->nelem[0] = c->nelem[1] = c->nelem[2] = 1;
  c->order = 1;
  c->hierarchy = GLLMG_HIER_P;
  c->max_levels = 0;
  c->smoother = GLLMG_SMOOTH_CHEBYSHEV;
  c->nu_pre = 4;
  c->nu_post = 4;
  c->omega = 2.0 / 3.0;
  c->cheb_lo = 0.25;
  c->cheb_safety = 1.0;
  c->eig_steps = 10;
  c->vcycle_prec = GLLMG_F64;
  c->eig_seed = 0;
  c->quadrature = GLLMG_QUAD_GLL;
  c->low_cycles = 1;
  c->coarse_unknowns = 0;
  c->ir_inner = 0;
}

gllmg_status gllmg_plan(const gllmg_config* cfg, int32_t* nlevels, size_t* bytes) {
  return guard([&]() {
    GLLMG_CHECK(cfg != nullptr, GLLMG_EINVAL, "config is NULL");
    validate(*cfg);
    gllmg_problem tmp;
    tmp.cfg = *cfg;
    auto specs = plan_levels(*cfg);
    Arena A;
    A.dry = true;
    const size_t tot = layout(&tmp, specs, A);
    if (nlevels) *nlevels = (int32_t)specs.size();
    if (bytes) *bytes = tot;
    return GLLMG_OK;
  });
}

gllmg_status gllmg_setup(const gllmg_config* cfg, const gllmg_field* map, const gllmg_field* mu,
                         void* ws, size_t ws_bytes, void* stream, gllmg_problem** out) {
  return guard([&]() {
    GLLMG_CHECK(cfg != nullptr && out != nullptr, GLLMG_EINVAL, "NULL argument");
    validate(*cfg);
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<gllmg_problem> P(new gllmg_problem());
    P->cfg = *cfg;
    P->vprec = cfg->vcycle_prec == GLLMG_F32 ? 1 : 0;
    auto specs = plan_levels(*cfg);
    Arena dry;
    dry.dry = true;
    const size_t need = layout(P.get(), specs, dry);
    if (ws) {
      GLLMG_CHECK(ws_bytes >= need, GLLMG_ENOMEM, "workspace smaller than gllmg_plan's size");
      GLLMG_CHECK(((uintptr_t)ws % 256) == 0, GLLMG_EINVAL, "workspace must be 256-byte aligned");
      P->ws = (char*)ws;
      P->ws_bytes = ws_bytes;
    } else {
      void* m = nullptr;
      if (hipMalloc(&m, need) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(GLLMG_ENOMEM, "device allocation of the workspace failed");
      }
      P->ws = (char*)m;
      P->ws_bytes = need;
      P->owns_ws = true;
    }
    struct Free {
      gllmg_problem* p;
      bool armed = true;
      ~Free() {
        if (armed) release_resources(p);
      }
    } guard_free{P.get()};
    Arena A;
    A.base = P->ws;
    A.size = P->ws_bytes;
    layout(P.get(), specs, A);
    // every host-side resource of the problem's later calls (pinned images, internal streams,
    // events) is taken here, from the device's pool or newly made: no later call allocates
    GLLMG_HIP(hipGetDevice(&P->dev));
    {
      const HostRes r = take_host_res(P->dev);
      P->hbuf = r.hbuf;
      P->bhost = r.bhost;
      P->ghact = r.ghact;
      P->ghsc = r.ghsc;
      P->xs = r.xs;
      P->cap = r.cap;
      P->sv.ev = r.ev;
      P->bev = r.bev;
      P->gev = r.gev;
    }
    P->sscratch = static_scratch(P->dev);
    setup_impl(P.get(), map, mu, s);
    fill_ctab(P.get(), s);
    // capture the solve's V-cycle now, while nothing else of this problem is in flight
    recapture(P.get());
    guard_free.armed = false;
    *out = P.release();
    return GLLMG_OK;
  });
}

gllmg_status gllmg_destroy(gllmg_problem* P) {
  return guard([&]() {
    if (!P) return GLLMG_OK;
    release_resources(P);
    delete P;
    return GLLMG_OK;
  });
}

gllmg_status gllmg_num_levels(const gllmg_problem* P, int32_t* n) {
  return guard([&]() {
    GLLMG_CHECK(P && n, GLLMG_EINVAL, "NULL argument");
    *n = (int32_t)P->L.size();
    return GLLMG_OK;
  });
}

gllmg_status gllmg_level_info(const gllmg_problem* P, int32_t level, int64_t* nnodes,
                              int64_t* ninterior, int32_t* order, int32_t nelem[3], double* lmax) {
  return guard([&]() {
    const Level& L = level_of(P, level);
    if (nnodes) *nnodes = L.g.N;
    if (ninterior) *ninterior = L.nint;
    if (order) *order = L.g.p;
    if (nelem)
      for (int a = 0; a < 3; ++a) nelem[a] = a < L.g.dim ? L.g.ne[a] : 0;
    if (lmax) *lmax = L.lmax;
    return GLLMG_OK;
  });
}

gllmg_status gllmg_set_lmax(gllmg_problem* P, int32_t level, double lmax) {
  return guard([&]() {
    level_of(P, level);
    GLLMG_CHECK(lmax > 0.0 && std::isfinite(lmax), GLLMG_EINVAL, "lmax must be positive");
    P->L[level].lmax = lmax;
    fill_ctab(P, P->xs);
    // the captured V-cycle holds the old Chebyshev coefficients: capture it again now, so that
    // the next solve replays a graph without building one
    recapture(P);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_set_persistent(gllmg_problem* P, int32_t enable) {
  return guard([&]() {
    GLLMG_CHECK(P != nullptr, GLLMG_EINVAL, "problem is NULL");
    P->persistent = enable != 0;
    return GLLMG_OK;
  });
}

gllmg_status gllmg_set_graphs(gllmg_problem* P, int32_t enable) {
  return guard([&]() {
    GLLMG_CHECK(P != nullptr, GLLMG_EINVAL, "problem is NULL");
    P->use_graph = enable != 0;
    if (!P->use_graph) drop_graph(P);
    else if (!P->vexec) recapture(P);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_node_coords(const gllmg_problem* P, int32_t level, double* out, void* stream) {
  return guard([&]() {
    const Level& L = level_of(P, level);
    check_ptr(out, 8, "out");
    GLLMG_CHECK(P->map.kind != GLLMG_MAP_CALLBACK, GLLMG_EUNSUPPORTED,
                "node coordinates of a callback map are the caller's own Phi");
    launch_node_coords(L.g, L.xi64, P->map, out, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_eval_field(const gllmg_problem* P, int32_t level, const gllmg_field* f,
                              double* out, void* stream) {
  return guard([&]() {
    const Level& L = level_of(P, level);
    check_ptr(out, 8, "out");
    GLLMG_CHECK(f != nullptr, GLLMG_EINVAL, "field is NULL");
    GLLMG_CHECK(f->kind != GLLMG_FIELD_EXP_FOURIER, GLLMG_EUNSUPPORTED,
                "EXP_FOURIER fields are evaluated only as the coefficient");
    FieldDev d{};
    d.kind = f->kind;
    for (int i = 0; i < 12; ++i) d.param[i] = f->param[i];
    GLLMG_CHECK(f->kind >= GLLMG_FIELD_CONST && f->kind <= GLLMG_FIELD_COS2_SUM, GLLMG_EINVAL,
                "unknown field kind (callback fields are evaluated at setup only)");
    GLLMG_CHECK(P->map.kind != GLLMG_MAP_CALLBACK, GLLMG_EUNSUPPORTED,
                "fields on a callback map are evaluated by the caller");
    launch_eval_field(L.g, L.xi64, P->map, d, out, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_rhs(const gllmg_problem* P, const double* f, double* b, void* stream) {
  return guard([&]() {
    const Level& L = level_of(P, 0);
    check_ptr(f, 8, "f_nodal");
    check_ptr(b, 8, "b");
    if (L.gauss) {  // consistent mass: element vectors, then the node-order sum (boundary 0)
      launch_mass_gauss(L, f, P->wdetq, (double*)P->F, (hipStream_t)stream);
      Epi ep;
      ep.y = b;
      launch_gather_in(L, 0, P->F, nullptr, 0, ep, (hipStream_t)stream);
      return GLLMG_OK;
    }
    launch_rhs(L.g, P->mass, f, b, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_diag(const gllmg_problem* P, int32_t level, gllmg_prec prec, void* d, void* stream) {
  return guard([&]() {
    const Level& L = level_of(P, level);
    const int pr = prec_index(P, prec);
    check_ptr(d, pr == 0 ? 8 : 4, "d");
    hipStream_t s = (hipStream_t)stream;
    // diag = 1 / dinv on the interior
    vec_copy(pr, L.g.N, dinv_of(L, pr), d, s);
    vec_recip_masked(pr, L.g.N, d, s);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_apply(const gllmg_problem* P, int32_t level, gllmg_prec prec, int32_t neumann,
                         const void* x, void* y, void* stream) {
  return guard([&]() {
    level_of(P, level);
    const int pr = prec_index(P, prec);
    check_ptr(x, pr == 0 ? 8 : 4, "x");
    check_ptr(y, pr == 0 ? 8 : 4, "y");
    GLLMG_CHECK(x != y, GLLMG_EINVAL, "x and y must not alias");
    apply_level(const_cast<gllmg_problem*>(P), level, pr, neumann ? 1 : 0, x, y, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_apply_noalloc(const gllmg_problem* P, int32_t level, gllmg_prec prec,
                                 int32_t neumann, const void* x, void* y, void* stream) {
  return guard([&]() {
    const Level& L = level_of(P, level);
    const int pr = prec_index(P, prec);
    check_ptr(x, pr == 0 ? 8 : 4, "x");
    check_ptr(y, pr == 0 ? 8 : 4, "y");
    GLLMG_CHECK(x != y, GLLMG_EINVAL, "x and y must not alias");
    const size_t need = face_buffer_elems(L) * (pr == 0 ? sizeof(double) : sizeof(float));
    GLLMG_CHECK(need <= kStaticScratchBytes, GLLMG_EINVAL,
                "the level's element vectors (" + std::to_string(need) +
                    " bytes) exceed the static scratch of gllmg_apply_noalloc (" +
                    std::to_string(kStaticScratchBytes) + " bytes)");
    GLLMG_CHECK(P->sscratch != nullptr, GLLMG_EDEVICE, "no static scratch on the problem's device");
    Epi ep;
    ep.y = y;
    Level& Lw = const_cast<gllmg_problem*>(P)->L[level];
    launch_apply(Lw, pr, neumann ? 1 : 0, x, ep, P->sscratch, (hipStream_t)stream);
    ++Lw.applies;
    return GLLMG_OK;
  });
}

gllmg_status gllmg_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  return guard([&]() {
    check_ptr(src, 16, "src");
    check_ptr(dst, 16, "dst");
    GLLMG_CHECK(bytes % 16 == 0, GLLMG_EINVAL, "bytes must be a multiple of 16");
    const char* a = (const char*)src;
    const char* b = (const char*)dst;
    GLLMG_CHECK(a + bytes <= b || b + bytes <= a, GLLMG_EINVAL, "src and dst overlap");
    stream_copy(src, dst, bytes, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_smooth(const gllmg_problem* P, int32_t level, gllmg_prec prec, const void* b,
                          void* x, int32_t steps, int32_t zero_guess, void* stream) {
  return guard([&]() {
    level_of(P, level);
    const int pr = prec_index(P, prec);
    check_ptr(b, pr == 0 ? 8 : 4, "b");
    check_ptr(x, pr == 0 ? 8 : 4, "x");
    GLLMG_CHECK(steps >= 0 && steps <= 64, GLLMG_EINVAL, "steps out of range");
    GLLMG_CHECK(P->cfg.smoother != GLLMG_SMOOTH_CHEBYSHEV || P->L[level].lmax > 0.0,
                GLLMG_EUNSUPPORTED, "no Chebyshev bound on this level (coarsest level)");
    smooth_impl(const_cast<gllmg_problem*>(P), level, pr, b, x, steps, zero_guess != 0,
                (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_prolong(const gllmg_problem* P, int32_t fl, gllmg_prec prec, const void* xc,
                           void* xf, void* stream) {
  return guard([&]() {
    level_of(P, fl);
    level_of(P, fl + 1);
    GLLMG_CHECK(!(fl == 0 && low_first(P)), GLLMG_EUNSUPPORTED,
                "levels 0 and 1 of the first-order hierarchy share their nodes (no transfer)");
    const int pr = prec_index(P, prec);
    check_ptr(xc, pr == 0 ? 8 : 4, "xc");
    check_ptr(xf, pr == 0 ? 8 : 4, "xf");
    GLLMG_CHECK(xc != xf, GLLMG_EINVAL, "xc and xf must not alias");
    launch_prolong(P->L[fl], P->L[fl + 1], pr, xc, xf, false, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_restrict(const gllmg_problem* P, int32_t fl, gllmg_prec prec, const void* rf,
                            void* rc, void* stream) {
  return guard([&]() {
    level_of(P, fl);
    level_of(P, fl + 1);
    GLLMG_CHECK(!(fl == 0 && low_first(P)), GLLMG_EUNSUPPORTED,
                "levels 0 and 1 of the first-order hierarchy share their nodes (no transfer)");
    const int pr = prec_index(P, prec);
    check_ptr(rf, pr == 0 ? 8 : 4, "rf");
    check_ptr(rc, pr == 0 ? 8 : 4, "rc");
    GLLMG_CHECK(rf != rc, GLLMG_EINVAL, "rf and rc must not alias");
    Epi ep;
    ep.y = rc;
    launch_restrict(P->L[fl], P->L[fl + 1], pr, rf, ep, P->F, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_vcycle(const gllmg_problem* P, gllmg_prec prec, const void* r, void* e, void* stream) {
  return guard([&]() {
    level_of(P, 0);
    const int pr = prec_index(P, prec);
    check_ptr(r, pr == 0 ? 8 : 4, "r");
    check_ptr(e, pr == 0 ? 8 : 4, "e");
    GLLMG_CHECK(r != e, GLLMG_EINVAL, "r and e must not alias");
    precond_level0(const_cast<gllmg_problem*>(P), pr, r, e, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_solve(const gllmg_problem* P, int32_t mode, const double* b, double* x,
                         double rtol, int32_t maxit, gllmg_solve_stats* st, void* stream) {
  return guard([&]() {
    level_of(P, 0);
    GLLMG_CHECK(mode == GLLMG_MODE_PCG || mode == GLLMG_MODE_MG || mode == GLLMG_MODE_IR,
                GLLMG_EINVAL, "unknown mode");
    check_ptr(b, 8, "b");
    check_ptr(x, 8, "x");
    GLLMG_CHECK(rtol > 0.0 && maxit >= 1, GLLMG_EINVAL, "rtol must be > 0 and maxit >= 1");
    GLLMG_CHECK(P->L.back().Ainv64 != nullptr, GLLMG_EUNSUPPORTED,
                "the coarsest level is too large for the dense exact solve");
    gllmg_status r = solve_impl(const_cast<gllmg_problem*>(P), mode, b, x, rtol, maxit, st,
                                (hipStream_t)stream);
    if (r == GLLMG_ENOTCONV) g_err = "maximum number of iterations reached";
    return r;
  });
}

gllmg_status gllmg_solve_begin(gllmg_problem* P, int32_t mode, const double* b, double* x,
                               double rtol, int32_t maxit, void* stream) {
  return guard([&]() {
    level_of(P, 0);
    GLLMG_CHECK(mode != GLLMG_MODE_IR, GLLMG_EUNSUPPORTED,
                "iterative refinement runs through gllmg_solve only");
    GLLMG_CHECK(mode == GLLMG_MODE_PCG || mode == GLLMG_MODE_MG, GLLMG_EINVAL, "unknown mode");
    check_ptr(b, 8, "b");
    check_ptr(x, 8, "x");
    GLLMG_CHECK(rtol > 0.0 && maxit >= 1, GLLMG_EINVAL, "rtol must be > 0 and maxit >= 1");
    GLLMG_CHECK(P->L.back().Ainv64 != nullptr, GLLMG_EUNSUPPORTED,
                "the coarsest level is too large for the dense exact solve");
    solve_begin(P, mode, b, x, rtol, maxit, (hipStream_t)stream);
    return GLLMG_OK;
  });
}

gllmg_status gllmg_solve_poll(gllmg_problem* P, int32_t* done) {
  return guard([&]() {
    GLLMG_CHECK(P && done, GLLMG_EINVAL, "NULL argument");
    *done = solve_poll(P) ? 1 : 0;
    return GLLMG_OK;
  });
}

gllmg_status gllmg_solve_end(gllmg_problem* P, gllmg_solve_stats* st) {
  return guard([&]() {
    GLLMG_CHECK(P != nullptr, GLLMG_EINVAL, "problem is NULL");
    gllmg_status r = solve_end(P, st);
    if (r == GLLMG_ENOTCONV) g_err = "maximum number of iterations reached";
    return r;
  });
}

gllmg_status gllmg_batch_solve(gllmg_problem* const* probs, const double* const* b,
                               double* const* x, int32_t count, int32_t mode, double rtol,
                               int32_t maxit, gllmg_solve_stats* stats, gllmg_status* status,
                               void* stream) {
  return guard([&]() {
    GLLMG_CHECK(count >= 0 && (count == 0 || (probs && b && x)), GLLMG_EINVAL, "NULL argument");
    hipStream_t cs = (hipStream_t)stream;
    if (count == 0) return GLLMG_OK;
    std::vector<int> live;
    gllmg_status worst = GLLMG_OK;
    auto fail = [&](int i, gllmg_status st) {
      if (status) status[i] = st;
      if (worst == GLLMG_OK || worst == GLLMG_ENOTCONV) worst = st;
    };
    {
      std::vector<const gllmg_problem*> seen(probs, probs + count);
      for (auto* P : seen) GLLMG_CHECK(P != nullptr, GLLMG_EINVAL, "problem is NULL");
      std::sort(seen.begin(), seen.end());
      GLLMG_CHECK(std::adjacent_find(seen.begin(), seen.end()) == seen.end(), GLLMG_EINVAL,
                  "a problem appears twice in the batch");
    }
    hipEvent_t start = probs[0]->bev;
    GLLMG_HIP(hipEventRecord(start, cs));
    const auto t0 = std::chrono::steady_clock::now();
    const bool args_ok = (mode == GLLMG_MODE_PCG || mode == GLLMG_MODE_MG) && rtol > 0.0 && maxit >= 1;
    // Problems of one shape (two or more) are solved in lockstep by launch groups, one group at
    // a time on the first problem's internal stream; measured faster than the one-workgroup
    // solver at every size of the 4^3-element batch (729 nodes: 3.7 vs 4.4 ms for 65 problems;
    // 4913 nodes: 6.0 vs 21.8 ms for 67). A shape with more than kGroupMax problems forms
    // several groups.
    std::vector<std::vector<int>> shapes;
    std::vector<char> in_group(count, 0);
    if (args_ok && mode == GLLMG_MODE_PCG) {
      for (int i = 0; i < count; ++i) {
        gllmg_problem* P = probs[i];
        if (P->sv.active || !P->persistent || !P->L.back().Ainv64) continue;
        if (!groupable_smoother(P->cfg.smoother) || P->cfg.quadrature != GLLMG_QUAD_GLL ||
            P->cfg.hierarchy == GLLMG_HIER_LOW)
          continue;
        if (!b[i] || !x[i] || ((uintptr_t)b[i] % 8) || ((uintptr_t)x[i] % 8)) continue;
        bool placed = false;
        for (auto& sh : shapes)
          if ((int)sh.size() < kGroupMax && same_shape(probs[sh[0]], P)) {
            sh.push_back(i);
            placed = true;
            break;
          }
        if (!placed) shapes.push_back({i});
      }
      shapes.erase(std::remove_if(shapes.begin(), shapes.end(),
                                  [](const std::vector<int>& v) { return v.size() < 2; }),
                   shapes.end());
      for (const auto& sh : shapes)
        for (int i : sh) in_group[i] = 1;
    }
    // small problems without a same-shape partner: one persistent launch per finest order, one
    // workgroup per problem, on the caller's stream (overlapping the groups)
    std::vector<char> pers(count, 0);
    std::vector<int> groups[18];
    for (int i = 0; i < count; ++i) {
      gllmg_problem* P = probs[i];
      if (in_group[i] || !args_ok || P->sv.active || !batch_eligible(P, maxit)) continue;
      if (!b[i] || !x[i] || ((uintptr_t)b[i] % 8) || ((uintptr_t)x[i] % 8)) continue;
      pers[i] = 1;
      groups[P->L[0].n].push_back(i);
    }
    for (int n0 = 2; n0 <= 17; ++n0) {
      const auto& idx = groups[n0];
      for (size_t c0 = 0; c0 < idx.size(); c0 += kBatchMaxProbs) {
        const int cnt = (int)std::min<size_t>(kBatchMaxProbs, idx.size() - c0);
        BatchArgs args{};
        for (int k = 0; k < cnt; ++k) {
          const int i = idx[c0 + k];
          gllmg_problem* P = probs[i];
          BatchProblem& h = *P->bhost;
          batch_fill(P, h);
          h.b = b[i];
          h.x = x[i];
          h.rtol = rtol;
          h.maxit = maxit;
          h.mode = mode;
          GLLMG_HIP(hipMemcpyAsync(P->bdev, &h, offsetof(BatchProblem, iters),
                                   hipMemcpyHostToDevice, cs));
          args.p[k] = P->bdev;
        }
        launch_batch(n0, args, cnt, cs);
      }
    }
    for (int i = 0; i < count; ++i)
      if (pers[i]) {
        gllmg_problem* P = probs[i];
        GLLMG_HIP(hipMemcpyAsync(&P->bhost->iters, &P->bdev->iters,
                                 offsetof(BatchProblem, hist) - offsetof(BatchProblem, iters) +
                                     sizeof(double) * (size_t)(maxit + 1),
                                 hipMemcpyDeviceToHost, cs));
      }
    // each group on a host thread of its own (its launches on its own stream), concurrently
    // with each other, the persistent launch and the streams below
    struct GroupRun {
      std::vector<gllmg_problem*> G;
      std::vector<const double*> gb;
      std::vector<double*> gx;
      std::vector<std::vector<int64_t>> a0;
      std::vector<GroupOut> res;
      hipStream_t s = nullptr;
      double el = 0.0;
      std::exception_ptr err;
    };
    std::vector<GroupRun> runs(shapes.size());
    for (size_t q = 0; q < shapes.size(); ++q) {
      GroupRun& r = runs[q];
      gllmg_problem* P0 = probs[shapes[q][0]];
      GLLMG_HIP(hipStreamWaitEvent(P0->xs, start, 0));
      r.s = P0->xs;
      for (int i : shapes[q]) {
        r.G.push_back(probs[i]);
        r.gb.push_back(b[i]);
        r.gx.push_back(x[i]);
        r.a0.emplace_back();
        for (auto& L : probs[i]->L) r.a0.back().push_back(L.applies);
      }
    }
    std::vector<std::thread> workers;
    for (size_t q = 0; q < runs.size(); ++q)
      workers.emplace_back([&, q]() {
        GroupRun& r = runs[q];
        try {
          group_solve(r.G, r.gb, r.gx, rtol, maxit, r.s, r.res);
        } catch (...) {
          r.err = std::current_exception();
        }
        r.el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      });
    struct Joiner {
      std::vector<std::thread>& w;
      ~Joiner() {
        for (auto& t : w)
          if (t.joinable()) t.join();
      }
    } joiner{workers};
    const std::vector<char>& grouped = in_group;
    // the others: their own streams, iteration-level interleaving
    for (int i = 0; i < count; ++i) {
      if (pers[i] || grouped[i]) continue;
      gllmg_problem* P = probs[i];
      GLLMG_HIP(hipStreamWaitEvent(P->xs, start, 0));
      const gllmg_status st = gllmg_solve_begin(P, mode, b[i], x[i], rtol, maxit, P->xs);
      if (st != GLLMG_OK) {
        fail(i, st);
        continue;
      }
      live.push_back(i);
    }
    // iteration-level interleaving: every live problem advances as soon as its last
    // iteration's scalars have arrived
    std::vector<char> fin(count, 0);
    size_t left = live.size();
    while (left > 0) {
      bool progressed = false;
      for (int i : live) {
        if (fin[i]) continue;
        bool finished = false;
        try {
          finished = solve_poll(probs[i]);
        } catch (const Error& e) {
          // this problem's solve has ended with the error; the others go on
          fin[i] = 1;
          --left;
          progressed = true;
          g_err = e.what();
          fail(i, e.status);
          continue;
        }
        if (finished) {
          fin[i] = 1;
          --left;
          progressed = true;
          const gllmg_status st = gllmg_solve_end(probs[i], stats ? &stats[i] : nullptr);
          if (status) status[i] = st;
          if (st != GLLMG_OK) fail(i, st);
        }
      }
      if (!progressed && left > 0) std::this_thread::yield();
    }
    for (int i : live) {
      GLLMG_HIP(hipEventRecord(probs[i]->sv.ev, probs[i]->xs));
      GLLMG_HIP(hipStreamWaitEvent(cs, probs[i]->sv.ev, 0));
    }
    for (auto& t : workers) t.join();
    for (size_t q = 0; q < runs.size(); ++q) {
      GroupRun& r = runs[q];
      if (r.err) std::rethrow_exception(r.err);
      for (size_t k = 0; k < r.G.size(); ++k) {
        const int i = shapes[q][k];
        const GroupOut& o = r.res[k];
        if (stats) {
          gllmg_solve_stats& st = stats[i];
          st.iters = o.iters;
          st.converged = o.conv ? 1 : 0;
          st.relres = o.n0 > 0.0 ? o.nr / o.n0 : 0.0;
          st.relres_true = o.rt;
          st.t_solve_s = r.el;
          for (int l = 0; l < 16; ++l)
            st.applies[l] = l < (int)r.G[k]->L.size() ? r.G[k]->L[l].applies - r.a0[k][l] : 0;
          if (st.history)
            for (size_t j = 0; j < o.hist.size() && j <= (size_t)maxit; ++j) st.history[j] = o.hist[j];
        }
        const gllmg_status si = o.breakdown ? GLLMG_EBREAKDOWN : (o.conv ? GLLMG_OK : GLLMG_ENOTCONV);
        if (status) status[i] = si;
        if (si != GLLMG_OK) fail(i, si);
        if (si == GLLMG_EBREAKDOWN) g_err = "breakdown: non-finite residual or p^T A p <= 0";
      }
      hipEvent_t e = r.G[0]->gev;
      GLLMG_HIP(hipEventRecord(e, r.s));
      GLLMG_HIP(hipStreamWaitEvent(cs, e, 0));
    }

    if (std::find(pers.begin(), pers.end(), 1) != pers.end()) {
      GLLMG_HIP(hipStreamSynchronize(cs));
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (int i = 0; i < count; ++i) {
        if (!pers[i]) continue;
        gllmg_problem* P = probs[i];
        const BatchProblem& r = *P->bhost;
        for (size_t l = 0; l < P->L.size(); ++l) P->L[l].applies += r.applies[l];
        if (stats) {
          gllmg_solve_stats& st = stats[i];
          st.iters = r.iters;
          st.converged = r.status == 0 ? 1 : 0;
          st.relres = r.n0 > 0.0 ? r.nr / r.n0 : 0.0;
          st.relres_true = r.relres_true;
          st.t_solve_s = el;
          for (int l = 0; l < 16; ++l) st.applies[l] = l < (int)P->L.size() ? r.applies[l] : 0;
          if (st.history)
            for (int k = 0; k <= r.iters && k <= maxit; ++k) st.history[k] = r.hist[k];
        }
        const gllmg_status si = r.status == 0 ? GLLMG_OK : (r.status == 1 ? GLLMG_ENOTCONV : GLLMG_EBREAKDOWN);
        if (status) status[i] = si;
        if (si != GLLMG_OK) fail(i, si);
        if (si == GLLMG_EBREAKDOWN) g_err = "breakdown: non-finite residual or p^T A p <= 0";
      }
    }
    if (worst == GLLMG_ENOTCONV) g_err = "maximum number of iterations reached in a problem";
    return worst;
  });
}

}  // extern "C"
