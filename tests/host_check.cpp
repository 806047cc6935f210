// Host-side checks of the library's setup code under AddressSanitizer and UndefinedBehavior-
// Sanitizer, with no GPU call: configuration validation and level planning with the workspace
// footprint for every family of configurations (and the errors of invalid ones), argument
// checks of the entry points, the reference element at every order (GLL nodes, weights,
// derivative matrix, Lagrange evaluation), the Gauss rule, the dense SPD inverse used by the
// exact coarse solve, and the tridiagonal eigenvalue of the Lanczos estimate. Exit status 0
// when every check holds; the sanitizers abort on the first error they find.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../paper_1402_5938_amd/csrc/internal.h"

static int fails = 0;
#define EXPECT(c)                                                         \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);  \
      ++fails;                                                            \
    }                                                                     \
  } while (0)

using namespace gllmg;

static void check_ref_elements() {
  for (int p = 1; p <= 16; ++p) {
    RefElem re = ref_element(p);
    const int n = p + 1;
    EXPECT((int)re.xi.size() == n && (int)re.w.size() == n && (int)re.D.size() == n * n);
    EXPECT(re.xi[0] == -1.0 && re.xi[p] == 1.0);
    double ws = 0.0;
    for (int i = 0; i < n; ++i) {
      ws += re.w[i];
      if (i > 0) EXPECT(re.xi[i] > re.xi[i - 1]);
      EXPECT(std::fabs(re.xi[i] + re.xi[p - i]) <= 1e-15);
      double rs = 0.0, mx = 0.0;
      for (int j = 0; j < n; ++j) {
        rs += re.D[i * n + j];
        mx = std::max(mx, std::fabs(re.D[i * n + j]));
      }
      EXPECT(std::fabs(rs) <= 1e-12 * mx);  // derivative of the constant 1
    }
    EXPECT(std::fabs(ws - 2.0) <= 1e-14);
    std::vector<double> l(n);
    lagrange_at(re, re.xi[p / 2], l.data());
    for (int j = 0; j < n; ++j) EXPECT(l[j] == (j == p / 2 ? 1.0 : 0.0));
    lagrange_at(re, 0.3, l.data());
    double ls = 0.0;
    for (double v : l) ls += v;
    EXPECT(std::fabs(ls - 1.0) <= 1e-13);
    gauss_rule(re);
    EXPECT((int)re.eta.size() == n && (int)re.Iq.size() == n * n && (int)re.Dq.size() == n * n);
    double gs = 0.0;
    for (int q = 0; q < n; ++q) {
      gs += re.wg[q];
      EXPECT(re.eta[q] > -1.0 && re.eta[q] < 1.0);
      double is = 0.0, ds = 0.0, dm = 0.0;
      for (int i = 0; i < n; ++i) {
        is += re.Iq[q * n + i];
        ds += re.Dq[q * n + i];
        dm = std::max(dm, std::fabs(re.Dq[q * n + i]));
      }
      EXPECT(std::fabs(is - 1.0) <= 1e-13);
      EXPECT(std::fabs(ds) <= 1e-12 * dm);
    }
    EXPECT(std::fabs(gs - 2.0) <= 1e-14);
  }
}

static void check_spd_inverse() {
  std::mt19937_64 g(5);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (int n : {1, 2, 9, 70, 150}) {
    std::vector<double> B((size_t)n * n), A((size_t)n * n, 0.0);
    for (double& v : B) v = U(g);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double t = i == j ? n : 0.0;
        for (int k = 0; k < n; ++k) t += B[(size_t)i * n + k] * B[(size_t)j * n + k];
        A[(size_t)i * n + j] = t;
      }
    std::vector<double> Ai = A;
    EXPECT(spd_inverse(Ai, n));
    double err = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double t = 0.0;
        for (int k = 0; k < n; ++k) t += A[(size_t)i * n + k] * Ai[(size_t)k * n + j];
        err = std::max(err, std::fabs(t - (i == j ? 1.0 : 0.0)));
        EXPECT(Ai[(size_t)i * n + j] == Ai[(size_t)j * n + i]);
      }
    EXPECT(err <= 1e-12);
  }
  std::vector<double> bad = {1.0, 2.0, 2.0, 1.0};  // eigenvalues 3 and -1
  EXPECT(!spd_inverse(bad, 2));
}

static void check_tridiag() {
  for (int m : {1, 2, 10, 40}) {
    std::vector<double> a(m, 2.0), b(m > 0 ? m - 1 : 0, -1.0);
    const double ex = 2.0 - 2.0 * std::cos(m * M_PI / (m + 1));
    EXPECT(std::fabs(tridiag_max_eig(a, b) - ex) <= 1e-12);
  }
}

static gllmg_config base(int dim, int ne, int p) {
  gllmg_config c;
  gllmg_config_default(&c);
  c.dim = dim;
  c.nelem[0] = c.nelem[1] = c.nelem[2] = ne;
  c.order = p;
  return c;
}

static void check_plans() {
  int ok = 0, rejected = 0;
  for (int dim = 2; dim <= 3; ++dim)
    for (int p = 1; p <= 16; ++p)
      for (int ne : {1, 3, 8})
        for (int hier : {GLLMG_HIER_H, GLLMG_HIER_P, GLLMG_HIER_LOW})
          for (int sm = GLLMG_SMOOTH_JACOBI; sm <= GLLMG_SMOOTH_BLOCK_JACOBI; ++sm)
            for (int quad : {GLLMG_QUAD_GLL, GLLMG_QUAD_GAUSS})
              for (int ml : {0, 1, 3})
                for (int cu : {0, 512}) {
                  if (dim == 3 && ne == 8 && p > 8) continue;  // plan sizes only; keep it quick
                  gllmg_config c = base(dim, ne, p);
                  c.hierarchy = hier;
                  c.smoother = sm;
                  c.quadrature = quad;
                  c.max_levels = ml;
                  c.coarse_unknowns = cu;
                  c.vcycle_prec = (p + ne) % 2 ? GLLMG_F32 : GLLMG_F64;
                  int32_t nl = -1;
                  size_t bytes = 0;
                  const gllmg_status st = gllmg_plan(&c, &nl, &bytes);
                  if (st == GLLMG_OK) {
                    ++ok;
                    EXPECT(nl >= 1 && bytes > 0);
                    if (ml > 0) EXPECT(nl <= ml);
                  } else {
                    ++rejected;
                    EXPECT(st == GLLMG_EINVAL || st == GLLMG_EUNSUPPORTED);  // combinations not built
                    EXPECT(std::strlen(gllmg_last_error()) > 0);
                  }
                }
  EXPECT(ok > 1000 && rejected > 0);
  // invalid configurations, each with its own error
  gllmg_config c = base(3, 2, 4);
  int32_t nl = 0;
  size_t bytes = 0;
  EXPECT(gllmg_plan(nullptr, &nl, &bytes) == GLLMG_EINVAL);
  c.order = 0;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c.order = 17;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c = base(4, 2, 4);
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c = base(3, 0, 4);
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c = base(3, 2, 4);
  c.smoother = 99;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c = base(3, 2, 4);
  c.nu_pre = -1;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c = base(3, 2, 4);
  c.hierarchy = GLLMG_HIER_LOW;
  c.low_cycles = 0;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c = base(3, 2, 4);
  c.ir_inner = 4;  // refinement needs the FP32 V-cycle
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c.vcycle_prec = GLLMG_F32;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_OK);
  c.ir_inner = 101;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c = base(3, 2, 4);
  c.coarse_unknowns = -1;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  c.coarse_unknowns = 4097;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_EINVAL);
  // the literal reading of the 16^3 p = 8 hierarchy: four levels down to 16^3 at p = 1, by
  // truncation or by the coarse-unknowns limit
  c = base(3, 16, 8);
  c.max_levels = 4;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_OK && nl == 4);
  c = base(3, 16, 8);
  c.coarse_unknowns = 4096;
  EXPECT(gllmg_plan(&c, &nl, &bytes) == GLLMG_OK && nl == 4);
}

static void check_entry_points() {
  gllmg_problem* P = nullptr;
  gllmg_config c = base(3, 2, 4);
  EXPECT(gllmg_setup(nullptr, nullptr, nullptr, nullptr, 0, nullptr, &P) == GLLMG_EINVAL);
  EXPECT(gllmg_setup(&c, nullptr, nullptr, nullptr, 0, nullptr, nullptr) == GLLMG_EINVAL);
  EXPECT(P == nullptr);
  int32_t nl = 0;
  EXPECT(gllmg_num_levels(nullptr, &nl) == GLLMG_EINVAL);
  EXPECT(gllmg_destroy(nullptr) == GLLMG_OK);
}

int main() {
  check_ref_elements();
  check_spd_inverse();
  check_tridiag();
  check_plans();
  check_entry_points();
  std::printf("host checks: %s\n", fails ? "FAILED" : "ok");
  return fails ? 1 : 0;
}
