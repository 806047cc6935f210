// Host reference element in FP64: GLL nodes and weights, the 1D derivative matrix, Lagrange
// evaluation; plus the small dense/tridiagonal helpers of the setup phase.
//
// GLL points of order p (paper §1, §2.3, Fig. 1): -1, 1 and the p-1 zeros of P_p', which are
// the zeros of the Jacobi polynomial P^{(1,1)}_{p-1}. Those are the eigenvalues of the
// symmetric tridiagonal Jacobi matrix of P^{(1,1)} (Golub-Welsch): zero diagonal and
// off-diagonal b_k = sqrt(k (k+2) / ((2k+1)(2k+3))), k = 1..p-2. They are found by Sturm
// bisection and polished by Newton's method on P_{p-1} - x P_p. Weights: 2 / (p (p+1) P_p^2).
// Derivative matrix D_ij = l_j'(x_i) in barycentric form from the computed nodes (off-diagonal
// (lam_j / lam_i) / (x_i - x_j), diagonal minus the row's other entries; see ref_element).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

#include "internal.h"

namespace gllmg {

static void legendre_pp(int p, double x, double* Pp, double* Pm1) {
  double a = 1.0, b = x;  // P_0, P_1
  for (int k = 1; k < p; ++k) {
    double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
    a = b;
    b = c;
  }
  *Pp = b;
  *Pm1 = a;
}

// Number of eigenvalues < x of the symmetric tridiagonal (a, b) by the Sturm sequence.
static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  const size_t m = a.size();
  for (size_t i = 0; i < m; ++i) {
    double bb = (i == 0) ? 0.0 : b[i - 1] * b[i - 1];
    q = (a[i] - x) - (i == 0 ? 0.0 : bb / q);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// k-th smallest eigenvalue (0-based) by bisection on [lo, hi].
static double tridiag_eig_k(const std::vector<double>& a, const std::vector<double>& b, int k,
                            double lo, double hi) {
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, mid) > k)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  if (m == 0) return 0.0;
  double r = 0.0;  // Gershgorin bound
  for (int i = 0; i < m; ++i) {
    double s = std::fabs(a[i]);
    if (i > 0) s += std::fabs(b[i - 1]);
    if (i < m - 1) s += std::fabs(b[i]);
    r = std::max(r, s);
  }
  r = r * (1.0 + 1e-12) + 1e-300;
  return tridiag_eig_k(a, b, m - 1, -r, r);
}

RefElem ref_element(int p) {
  GLLMG_CHECK(p >= 1 && p <= 32, GLLMG_EINVAL, "order out of range");
  RefElem re;
  re.p = p;
  const int n = p + 1;
  re.xi.assign(n, 0.0);
  re.xi[0] = -1.0;
  re.xi[p] = 1.0;
  if (p >= 2) {
    const int m = p - 1;
    std::vector<double> a(m, 0.0), b(std::max(m - 1, 0));
    for (int k = 1; k <= m - 1; ++k)
      b[k - 1] = std::sqrt((double)k * (k + 2) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)));
    for (int k = 0; k < m; ++k) {
      double x = tridiag_eig_k(a, b, k, -1.0, 1.0);
      for (int it = 0; it < 3; ++it) {  // Newton on q(x) = P_{p-1} - x P_p, q' = -(p+1) P_p
        double P, Pm1;
        legendre_pp(p, x, &P, &Pm1);
        x += (Pm1 - x * P) / ((p + 1.0) * P);
      }
      re.xi[k + 1] = x;
    }
    for (int k = 0; k < n / 2; ++k) {  // the rule is symmetric
      double s = 0.5 * (re.xi[p - k] - re.xi[k]);
      re.xi[k] = -s;
      re.xi[p - k] = s;
    }
    if (p % 2 == 0) re.xi[p / 2] = 0.0;
  }
  re.w.resize(n);
  for (int i = 0; i < n; ++i) {
    double P, Pm1;
    legendre_pp(p, re.xi[i], &P, &Pm1);
    re.w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
  // Barycentric weights of the computed (rounded) nodes, lam_j = 1 / prod_{k != j}(xi_j - xi_k).
  // The derivative matrix is built from them rather than from the Legendre closed form
  // P_p(xi_i) / (P_p(xi_j)(xi_i - xi_j)), which presumes exact nodes: with nodes off by an ulp
  // it no longer differentiates linear functions exactly (at p = 16, D xi - 1 reaches 3e-13),
  // and the isoparametric Jacobian D x amplifies that by |x| / |J|, i.e. by the element count.
  re.lam.resize(n);
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) prod *= (re.xi[j] - re.xi[k]);
    re.lam[j] = 1.0 / prod;
  }
  // D_ij = (lam_j / lam_i) / (xi_i - xi_j) off the diagonal; each diagonal entry is minus the
  // sum of its row's others, so that D annihilates constants to rounding (Baltensperger and
  // Trummer, SIAM J. Sci. Comput. 2003).
  re.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j)
      if (i != j) {
        re.D[i * n + j] = (re.lam[j] / re.lam[i]) / (re.xi[i] - re.xi[j]);
        rs += re.D[i * n + j];
      }
    re.D[i * n + i] = -rs;
  }
  return re;
}

// Gauss-Legendre rule of q = p + 1 points: the zeros of P_q are the eigenvalues of the
// symmetric tridiagonal Jacobi matrix of the Legendre polynomials (Golub-Welsch), zero diagonal
// and off-diagonal k / sqrt(4 k^2 - 1), found by Sturm bisection and polished by Newton's method
// on P_q; weights 2 / ((1 - x^2) P_q'(x)^2) with P_q' = q (x P_q - P_{q-1}) / (x^2 - 1).
// The basis of the GLL nodes at those points by barycentric evaluation, its derivative as Iq D.
void gauss_rule(RefElem& re) {
  const int q = re.p + 1, n = re.p + 1;
  std::vector<double> a(q, 0.0), b(std::max(q - 1, 0));
  for (int k = 1; k <= q - 1; ++k) b[k - 1] = (double)k / std::sqrt(4.0 * k * k - 1.0);
  re.eta.assign(q, 0.0);
  re.wg.assign(q, 0.0);
  for (int k = 0; k < q; ++k) {
    double x = tridiag_eig_k(a, b, k, -1.0, 1.0);
    for (int it = 0; it < 3; ++it) {
      double P, Pm1;
      legendre_pp(q, x, &P, &Pm1);
      const double dP = q * (x * P - Pm1) / (x * x - 1.0);
      x -= P / dP;
    }
    re.eta[k] = x;
  }
  for (int k = 0; k < q / 2; ++k) {  // the rule is symmetric
    const double s = 0.5 * (re.eta[q - 1 - k] - re.eta[k]);
    re.eta[k] = -s;
    re.eta[q - 1 - k] = s;
  }
  if (q % 2 == 1) re.eta[q / 2] = 0.0;
  for (int k = 0; k < q; ++k) {
    const double x = re.eta[k];
    double P, Pm1;
    legendre_pp(q, x, &P, &Pm1);
    const double dP = q * (x * P - Pm1) / (x * x - 1.0);
    re.wg[k] = 2.0 / ((1.0 - x * x) * dP * dP);
  }
  re.Iq.assign((size_t)q * n, 0.0);
  for (int k = 0; k < q; ++k) lagrange_at(re, re.eta[k], &re.Iq[(size_t)k * n]);
  re.Dq.assign((size_t)q * n, 0.0);
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int i = 0; i < n; ++i) v += re.Iq[(size_t)k * n + i] * re.D[(size_t)i * n + j];
      re.Dq[(size_t)k * n + j] = v;
    }
}

// Barycentric Lagrange evaluation (Berrut and Trefethen, SIAM Review 2004, "second form").
void lagrange_at(const RefElem& re, double y, double* out) {
  const int n = re.p + 1;
  for (int j = 0; j < n; ++j)
    if (y == re.xi[j]) {
      for (int k = 0; k < n; ++k) out[k] = (k == j) ? 1.0 : 0.0;
      return;
    }
  const std::vector<double>& lam = re.lam;
  double den = 0.0;
  for (int j = 0; j < n; ++j) den += lam[j] / (y - re.xi[j]);
  for (int j = 0; j < n; ++j) out[j] = (lam[j] / (y - re.xi[j])) / den;
}

namespace {
// Host threads for the dense setup loops: up to 16, about one per 64 rows.
int host_threads(int n) {
  return std::max(1, std::min({16, (int)std::thread::hardware_concurrency(), n / 64}));
}

// Runs body(t) on T host threads (t = 0..T-1) and joins them.
template <class F>
void run_threads(int T, F body) {
  if (T == 1) return body(0);
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) th.emplace_back([&, t] { body(t); });
  for (std::thread& x : th) x.join();
}

// Barrier of T spinning host threads; what a thread wrote before wait() is visible to every
// thread after it.
class SpinBarrier {
 public:
  explicit SpinBarrier(int T) : T_(T) {}
  void wait() {
    const int g = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) == T_ - 1) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_release);
      return;
    }
    for (int spin = 0; gen_.load(std::memory_order_acquire) == g; ++spin)
      if (spin > 1024) std::this_thread::yield();
  }

 private:
  const int T_;
  std::atomic<int> count_{0};
  std::atomic<int> gen_{0};
};
}  // namespace

// Inverse of a dense SPD matrix by Cholesky: A = L L^T, L^{-1} column by column, then
// A^{-1} = L^{-T} L^{-1}. Every inner product runs in increasing k; independent rows and
// columns are spread over host threads and interleaved, which leaves each sum's order alone.
// The result is exactly symmetric.
bool spd_inverse(std::vector<double>& A, int n) {
  const int T = host_threads(n);
  // Cholesky, column j from columns < j (lower triangle, in place). The rows of one column
  // are formed eight at a time, each with its own running sum; blocks of eight rows go to the
  // threads in turn, and a barrier ends each column.
  constexpr int R = 8;
  std::atomic<bool> spd{true};
  SpinBarrier bar(T);
  run_threads(T, [&](int th) {
    for (int j = 0; j < n; ++j) {
      const double* Lj = &A[(size_t)j * n];
      double s = Lj[j];
      for (int k = 0; k < j; ++k) s -= Lj[k] * Lj[k];
      if (!(s > 0.0)) {  // every thread sees the same s and leaves at the same column
        spd.store(false);
        return;
      }
      const double ljj = std::sqrt(s);
      for (int i = j + 1 + th * R; i < n; i += T * R) {
        const int m = std::min(R, n - i);
        double t[R];
        const double* Li[R];
        for (int r = 0; r < R; ++r) {
          Li[r] = &A[(size_t)(i + std::min(r, m - 1)) * n];
          t[r] = Li[r][j];
        }
        for (int k = 0; k < j; ++k) {
          const double l = Lj[k];
          for (int r = 0; r < R; ++r) t[r] -= Li[r][k] * l;
        }
        for (int r = 0; r < m; ++r) A[(size_t)(i + r) * n + j] = t[r] / ljj;
      }
      bar.wait();
      if (th == 0) A[(size_t)j * n + j] = ljj;  // no thread reads A[j][j] in later columns
    }
  });
  if (!spd.load()) return false;
  // W = L^{-T} stored by rows: W[j][k] = (L^{-1})_{kj}, k >= j; the columns of L^{-1} are
  // independent of each other
  std::vector<double> W((size_t)n * n, 0.0);
  run_threads(T, [&](int th) {
    for (int j = th; j < n; j += T) {
      double* Wj = &W[(size_t)j * n];
      Wj[j] = 1.0 / A[(size_t)j * n + j];
      for (int i = j + 1; i < n; ++i) {
        const double* Li = &A[(size_t)i * n];
        double t = 0.0;
        for (int k = j; k < i; ++k) t += Li[k] * Wj[k];
        Wj[i] = -t / Li[i];
      }
    }
  });
  // (A^{-1})_{ij} = sum over k >= i of (L^{-1})_{ki} (L^{-1})_{kj}, for j <= i
  run_threads(T, [&](int th) {
    for (int i = th; i < n; i += T) {
      const double* Wi = &W[(size_t)i * n];
      for (int j = 0; j <= i; ++j) {
        const double* Wj = &W[(size_t)j * n];
        double t = 0.0;
        for (int k = i; k < n; ++k) t += Wi[k] * Wj[k];
        A[(size_t)i * n + j] = t;
      }
    }
  });
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)j * n + i] = A[(size_t)i * n + j];
  return true;
}

}  // namespace gllmg
