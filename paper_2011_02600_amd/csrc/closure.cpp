// Boundary closures of the upwind dual-pair SBP operators (Sec. 4.1).
//
// The paper fixes the properties -- H D+ + (H D-)^T = B (eq. upw_SBP),
// H (D+ - D-) symmetric negative semi-definite, the accuracy conditions
// eq. acc (order p at the boundary for interior order 2p) and the interior
// stencils of Table tab:upwind -- but not the closure coefficients.  They are
// constructed here as
//   h D+- = H^{-1} (A + B/2 +- S/2),   S = -kappa Dp^T Dp  (P-th undivided
//   difference, P = q), A skew with the interior antisymmetric part of alpha
//   outside a free m x m corner block, H = diag(w_0..w_{m-1}, 1, ...),
// where the corner block and the weights solve the accuracy conditions of the
// first m rows (a linear least-squares problem that is consistent and has a
// unique solution for orders 2 and 4).  Orders 3, 5 and 6 leave entries of the
// corner block free; they are fixed where the one-dimensional elastic operator
// with characteristic penalties has the smallest spectral radius (no larger
// than the interior stencil's) with positive weights, at the simplest
// rational of equal radius: order 3 A[1][2] = 1/2, order 5 A[2][4] = 1/4 and
// A[3][4] = 1/2, order 6 A[4][5] = 101/125, order 7 A[5][6] = 2/3,
// A[4][6] = A[3][6] = 0, A[4][5] = 3/5, order 8 A[6][7] = 5/6, A[5][7] = -1/5,
// A[5][6] = 3/4 (spectral radius 2.35 against the interior 2.10 at N = 80;
// the radius depends sharply on these entries and its minimum lies at
// irrational values).  For interior order 2p + 1 the
// boundary accuracy is p, as for 2p.  The system is solved with Householder
// QR in long double.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace sbp {
namespace {

struct Row {
  int order, r;
  int num[10], den[10];
  int n;
};

// Table tab:upwind, orders 2 to 8: alpha_{-r} .. alpha_{q}.  Order 8's
// alpha_4 is printed +1/28; -1/28 makes the coefficients sum to zero (a
// consistent difference) and the stencil eighth-order accurate.
const Row kTable[] = {
    {2, 0, {-3, 2, -1}, {2, 1, 2}, 3},
    {3, 1, {-1, -1, 1, -1}, {3, 2, 1, 6}, 4},
    {4, 1, {-1, -5, 3, -1, 1}, {4, 6, 2, 2, 12}, 5},
    {5, 2, {1, -1, -1, 1, -1, 1}, {20, 2, 3, 1, 4, 30}, 6},
    {6, 2, {1, -2, -7, 4, -1, 2, -1}, {30, 5, 12, 3, 2, 15, 60}, 7},
    {7, 3, {-1, 1, -3, -1, 1, -3, 1, -1}, {105, 10, 5, 4, 1, 10, 15, 140}, 8},
    {8, 3, {-1, 1, -1, -9, 5, -1, 1, -1, 1}, {168, 14, 2, 20, 4, 2, 6, 28, 280}, 9},
};

// Corner-block entries A[i][j] = num/den left free by the accuracy conditions.
struct FreeEntry {
  int order, i, j, num, den;
};
const FreeEntry kFree[] = {
    {3, 1, 2, 1, 2},
    {5, 2, 4, 1, 4},
    {5, 3, 4, 1, 2},
    {6, 4, 5, 101, 125},
    {7, 5, 6, 2, 3},
    {7, 4, 6, 0, 1},
    {7, 3, 6, 0, 1},
    {7, 4, 5, 3, 5},
    {8, 6, 7, 5, 6},
    {8, 5, 7, -1, 5},
    {8, 5, 6, 3, 4},
};

long double binom(int n, int k) {
  long double v = 1;
  for (int i = 1; i <= k; ++i) v = v * (n - k + i) / i;
  return v;
}

// Least squares min |Ax - b| by Householder QR; A is rows x cols, row-major.
// Returns false if A is rank deficient.
bool lstsq(std::vector<long double> A, std::vector<long double> b, int rows, int cols,
           std::vector<long double>* x) {
  for (int k = 0; k < cols; ++k) {
    long double nrm = 0;
    for (int i = k; i < rows; ++i) nrm += A[i * cols + k] * A[i * cols + k];
    nrm = std::sqrt(nrm);
    if (nrm < 1e-30L) return false;
    long double alpha = A[k * cols + k] > 0 ? -nrm : nrm;
    std::vector<long double> v(rows, 0);
    for (int i = k; i < rows; ++i) v[i] = A[i * cols + k];
    v[k] -= alpha;
    long double vn = 0;
    for (int i = k; i < rows; ++i) vn += v[i] * v[i];
    if (vn == 0) continue;
    for (int j = k; j < cols; ++j) {
      long double d = 0;
      for (int i = k; i < rows; ++i) d += v[i] * A[i * cols + j];
      d = 2 * d / vn;
      for (int i = k; i < rows; ++i) A[i * cols + j] -= d * v[i];
    }
    long double d = 0;
    for (int i = k; i < rows; ++i) d += v[i] * b[i];
    d = 2 * d / vn;
    for (int i = k; i < rows; ++i) b[i] -= d * v[i];
  }
  x->assign(cols, 0);
  for (int k = cols - 1; k >= 0; --k) {
    long double s = b[k];
    for (int j = k + 1; j < cols; ++j) s -= A[k * cols + j] * (*x)[j];
    if (std::fabs(A[k * cols + k]) < 1e-24L) return false;
    (*x)[k] = s / A[k * cols + k];
  }
  return true;
}

}  // namespace

bool build_closure(int order, Closure* out, const char** err) {
  const Row* row = nullptr;
  for (const Row& t : kTable)
    if (t.order == order) row = &t;
  if (!row) {
    *err = "unsupported order (2 to 8)";
    return false;
  }
  const int r = row->r;
  const int q = row->n - 1 - r;
  const int p = order / 2;
  const int m = order;
  const int P = q;
  std::vector<long double> alpha(row->n);
  for (int i = 0; i < row->n; ++i) alpha[i] = (long double)row->num[i] / row->den[i];
  auto al = [&](int j) -> long double { return (j >= -r && j <= q) ? alpha[j + r] : 0.0L; };
  std::vector<long double> a(q + 1, 0), s(q + 1, 0);
  for (int j = 0; j <= q; ++j) {
    a[j] = j ? 0.5L * (al(j) - al(-j)) : 0.0L;
    s[j] = 0.5L * (al(j) + al(-j));
  }
  const long double kappa = -2.0L * s[0] / binom(2 * P, P);

  // unknowns: w_0..w_{m-1}, A[i][j] (i < j < m)
  std::vector<int> pi, pj;
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) { pi.push_back(i); pj.push_back(j); }
  const int nunk = m + (int)pi.size();
  auto uidx = [&](int i, int j) {
    for (size_t k = 0; k < pi.size(); ++k)
      if (pi[k] == i && pj[k] == j) return m + (int)k;
    return -1;
  };
  auto Atoep = [&](int i, int j) -> long double {
    int d = j - i;
    if (d > 0 && d <= q) return a[d];
    if (d < 0 && -d <= q) return -a[-d];
    return 0.0L;
  };
  const int ncol = m + q;
  std::vector<long double> M, b;
  int neq = 0;
  for (int k = 0; k <= p; ++k) {
    for (int i = 0; i < m; ++i) {
      std::vector<long double> eq(nunk, 0);
      long double rhs = 0;
      for (int j = 0; j < ncol; ++j) {
        long double xk = (k == 0) ? 1.0L : std::pow((long double)j, k);
        if (j < m) {
          if (i < j) eq[uidx(i, j)] += xk;
          else if (j < i) eq[uidx(j, i)] -= xk;
        } else {
          rhs -= Atoep(i, j) * xk;
        }
      }
      if (i == 0 && k == 0) rhs += 0.5L;  // -(B/2)_{00} * x_0^0
      if (k >= 1) eq[i] -= k * ((k == 1) ? 1.0L : std::pow((long double)i, k - 1));
      M.insert(M.end(), eq.begin(), eq.end());
      b.push_back(rhs);
      ++neq;
    }
  }
  for (const FreeEntry& f : kFree) {
    if (f.order != order) continue;
    std::vector<long double> eq(nunk, 0);
    eq[uidx(f.i, f.j)] = 1;
    M.insert(M.end(), eq.begin(), eq.end());
    b.push_back((long double)f.num / f.den);
    ++neq;
  }
  std::vector<long double> x;
  if (!lstsq(M, b, neq, nunk, &x)) {
    *err = "closure system is rank deficient";
    return false;
  }
  // consistency: the least-squares solution must solve every equation
  for (int e = 0; e < neq; ++e) {
    long double res = -b[e];
    for (int u = 0; u < nunk; ++u) res += M[e * nunk + u] * x[u];
    if (std::fabs(res) > 1e-15L) {
      *err = "closure system is inconsistent";
      return false;
    }
  }
  Closure c;
  c.order = order;
  c.m = m;
  c.q = q;
  c.r = r;
  c.ncol = ncol;
  for (int i = 0; i < row->n; ++i) c.alpha[i] = (double)alpha[i];
  std::vector<long double> Ablk(m * m, 0);
  for (size_t k = 0; k < pi.size(); ++k) {
    Ablk[pi[k] * m + pj[k]] = x[m + k];
    Ablk[pj[k] * m + pi[k]] = -x[m + k];
  }
  auto Delta = [&](int k, int j) -> long double {  // row k of the P-th difference
    int d = j - k;
    if (d < 0 || d > P) return 0.0L;
    return ((P - d) % 2 ? -1.0L : 1.0L) * binom(P, d);
  };
  for (int i = 0; i < m; ++i) {
    if (x[i] <= 0) {
      *err = "closure norm is not positive";
      return false;
    }
    c.w[i] = (double)x[i];
    for (int col = 0; col < ncol; ++col) {
      long double A = (col < m) ? Ablk[i * m + col] : Atoep(i, col);
      long double S = 0;
      for (int k = 0; k <= i && k <= col; ++k) S += Delta(k, i) * Delta(k, col);
      S *= -kappa;
      long double B = (i == 0 && col == 0) ? -1.0L : 0.0L;
      c.dp[i][col] = (double)((A + 0.5L * B + 0.5L * S) / x[i]);
      c.dm[i][col] = (double)((A + 0.5L * B - 0.5L * S) / x[i]);
    }
  }
  *out = c;
  return true;
}

}  // namespace sbp
