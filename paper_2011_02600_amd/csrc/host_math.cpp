// Host-side numerics of the set-up (see host_math.hpp).
#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace sbp {

void apply_axis(const Closure& c, const Grid3& g, const double* in, double* out, int ax, int kind) {
  const int N = g.len(ax);
  const std::size_t stride = ax == 0 ? 1 : (ax == 1 ? (std::size_t)g.nq : (std::size_t)g.nq * g.nr);
  const double ih = N - 1;
  const int R = c.r, m = c.m, nt = c.r + c.q + 1;
  // every line along ax
  const int n1 = ax == 0 ? g.nr : g.nq;
  const int n2 = ax == 2 ? g.nr : g.ns;
  for (int b = 0; b < n2; ++b) {
    for (int a = 0; a < n1; ++a) {
      std::size_t base;
      if (ax == 0) base = g.idx(0, a, b);
      else if (ax == 1) base = g.idx(a, 0, b);
      else base = g.idx(a, b, 0);
      const double* f = in + base;
      double* o = out + base;
      for (int i = 0; i < N; ++i) {
        double vp = 0, vm = 0;
        if (i >= m && i < N - m) {
          for (int s = 0; s < nt; ++s) {
            vp += c.alpha[s] * f[(std::size_t)(i - R + s) * stride];
            vm -= c.alpha[s] * f[(std::size_t)(i + R - s) * stride];
          }
        } else if (i < m) {
          for (int cc = 0; cc < c.ncol; ++cc) {
            vp += c.dp[i][cc] * f[(std::size_t)cc * stride];
            vm += c.dm[i][cc] * f[(std::size_t)cc * stride];
          }
        } else {
          // right end: D+ = -flip(D-), D- = -flip(D+)
          const int row = N - 1 - i;
          for (int cc = 0; cc < c.ncol; ++cc) {
            vp -= c.dm[row][cc] * f[(std::size_t)(N - 1 - cc) * stride];
            vm -= c.dp[row][cc] * f[(std::size_t)(N - 1 - cc) * stride];
          }
        }
        o[(std::size_t)i * stride] = ih * (kind == 0 ? vp : (kind == 1 ? vm : 0.5 * (vp + vm)));
      }
    }
  }
}

long long metric_terms(const Closure& cl, const Grid3& g, const double* X, double* J, double* M) {
  const std::size_t n = g.n;
  std::vector<double> d(9 * n);  // d[3 c + xi] = D0_xi x_c
  for (int c = 0; c < 3; ++c)
    for (int xi = 0; xi < 3; ++xi) apply_axis(cl, g, X + c * n, d.data() + (3 * c + xi) * n, xi, 2);
  long long bad = -1;
  for (std::size_t o = 0; o < n; ++o) {
    const double xq = d[0 * n + o], xr = d[1 * n + o], xs = d[2 * n + o];
    const double yq = d[3 * n + o], yr = d[4 * n + o], ys = d[5 * n + o];
    const double zq = d[6 * n + o], zr = d[7 * n + o], zs = d[8 * n + o];
    J[o] = xq * (yr * zs - zr * ys) - yq * (xr * zs - zr * xs) + zq * (xr * ys - yr * xs);
    if (!(J[o] > 0) && bad < 0) bad = (long long)o;
  }
  std::vector<double> tmp(n), t2(n);
  for (int xi = 0; xi < 3; ++xi) {
    const int eta = (xi + 1) % 3, zeta = (xi + 2) % 3;
    for (int c = 0; c < 3; ++c) {
      const int dd = (c + 1) % 3, e = (c + 2) % 3;
      double* t1 = M + (std::size_t)(3 * xi + c) * n;
      for (std::size_t o = 0; o < n; ++o) tmp[o] = X[e * n + o] * d[(3 * dd + eta) * n + o];
      apply_axis(cl, g, tmp.data(), t1, zeta, 1);
      for (std::size_t o = 0; o < n; ++o) tmp[o] = X[e * n + o] * d[(3 * dd + zeta) * n + o];
      apply_axis(cl, g, tmp.data(), t2.data(), eta, 1);
      for (std::size_t o = 0; o < n; ++o) t1[o] -= t2[o];
    }
  }
  return bad;
}

int delta_window(int N, int width, double u) {
  int s0 = (int)std::floor(u) - width / 2 + 1;
  return std::min(std::max(s0, 0), N - width);
}

void lagrange_basis(int width, int start, double u, double* phi, double* dphi) {
  for (int a = 0; a < width; ++a) {
    double num = 1, den = 1, dnum = 0;
    for (int b = 0; b < width; ++b) {
      if (b == a) continue;
      const double f = u - (start + b);
      dnum = dnum * f + num;  // product rule, accumulated factor by factor
      num *= f;
      den *= (double)(a - b);
    }
    phi[a] = num / den;
    if (dphi) dphi[a] = dnum / den;
  }
}

namespace {

// tensor-product interpolant of the node coordinates at u (node units) and
// its derivative in u: Xu[c], Ju[c][axis]
void interpolate_map(const Grid3& g, const double* X, int width, const double u[3], double Xu[3],
                     double Ju[3][3]) {
  double phi[3][kMaxSrcWidth], dphi[3][kMaxSrcWidth];
  int st[3];
  for (int a = 0; a < 3; ++a) {
    st[a] = delta_window(g.len(a), width, u[a]);
    lagrange_basis(width, st[a], u[a], phi[a], dphi[a]);
  }
  for (int c = 0; c < 3; ++c) {
    Xu[c] = 0;
    for (int a = 0; a < 3; ++a) Ju[c][a] = 0;
  }
  for (int k = 0; k < width; ++k)
    for (int j = 0; j < width; ++j)
      for (int i = 0; i < width; ++i) {
        const std::size_t o = g.idx(st[0] + i, st[1] + j, st[2] + k);
        const double w = phi[0][i] * phi[1][j] * phi[2][k];
        const double wq = dphi[0][i] * phi[1][j] * phi[2][k];
        const double wr = phi[0][i] * dphi[1][j] * phi[2][k];
        const double ws = phi[0][i] * phi[1][j] * dphi[2][k];
        for (int c = 0; c < 3; ++c) {
          const double v = X[c * g.n + o];
          Xu[c] += w * v;
          Ju[c][0] += wq * v;
          Ju[c][1] += wr * v;
          Ju[c][2] += ws * v;
        }
      }
}

// solves A x = b (3 x 3) by Gaussian elimination with partial pivoting;
// false if A is singular to working precision
bool solve3(double A[3][3], double b[3], double x[3]) {
  int p[3] = {0, 1, 2};
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (std::fabs(A[p[r]][col]) > std::fabs(A[p[piv]][col])) piv = r;
    std::swap(p[col], p[piv]);
    const double d = A[p[col]][col];
    if (!(std::fabs(d) > 1e-300)) return false;
    for (int r = col + 1; r < 3; ++r) {
      const double f = A[p[r]][col] / d;
      for (int cc = col; cc < 3; ++cc) A[p[r]][cc] -= f * A[p[col]][cc];
      b[p[r]] -= f * b[p[col]];
    }
  }
  for (int col = 2; col >= 0; --col) {
    double s = b[p[col]];
    for (int cc = col + 1; cc < 3; ++cc) s -= A[p[col]][cc] * x[cc];
    x[col] = s / A[p[col]][col];
  }
  return true;
}

}  // namespace

int locate_point(const Grid3& g, const double* X, int width, const double x[3], double xi[3], double* resid) {
  const std::size_t n = g.n;
  // length scale of the block (for the residual test) and the nearest node
  double lo[3] = {X[0], X[n], X[2 * n]}, hi[3] = {X[0], X[n], X[2 * n]};
  std::size_t best = 0;
  double bd = -1;
  for (std::size_t o = 0; o < n; ++o) {
    double d2 = 0;
    for (int c = 0; c < 3; ++c) {
      const double v = X[c * n + o];
      lo[c] = std::min(lo[c], v);
      hi[c] = std::max(hi[c], v);
      d2 += (v - x[c]) * (v - x[c]);
    }
    if (bd < 0 || d2 < bd) {
      bd = d2;
      best = o;
    }
  }
  const double scale = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                 (hi[2] - lo[2]) * (hi[2] - lo[2]));
  for (int c = 0; c < 3; ++c)
    if (x[c] < lo[c] - 1e-9 * scale || x[c] > hi[c] + 1e-9 * scale) return 1;
  double u[3] = {(double)(best % g.nq), (double)((best / g.nq) % g.nr), (double)(best / ((std::size_t)g.nq * g.nr))};
  bool conv = false;
  for (int it = 0; it < 100 && !conv; ++it) {
    double Xu[3], Ju[3][3], r[3], du[3];
    interpolate_map(g, X, width, u, Xu, Ju);
    for (int c = 0; c < 3; ++c) r[c] = x[c] - Xu[c];
    if (!solve3(Ju, r, du)) return 2;
    // damped step: at most two cells per iteration
    double m = 0;
    for (int a = 0; a < 3; ++a) m = std::max(m, std::fabs(du[a]));
    const double f = m > 2.0 ? 2.0 / m : 1.0;
    for (int a = 0; a < 3; ++a) {
      u[a] += f * du[a];
      u[a] = std::min(std::max(u[a], -1.0), (double)(g.len(a) - 1) + 1.0);
    }
    conv = f == 1.0 && m < 1e-12;
  }
  if (!conv) return 2;
  for (int a = 0; a < 3; ++a) {
    const double N1 = g.len(a) - 1;
    if (u[a] < -1e-9 || u[a] > N1 + 1e-9) return 1;
    u[a] = std::min(std::max(u[a], 0.0), N1);
  }
  double Xu[3], Ju[3][3];
  interpolate_map(g, X, width, u, Xu, Ju);
  const double res = std::sqrt((Xu[0] - x[0]) * (Xu[0] - x[0]) + (Xu[1] - x[1]) * (Xu[1] - x[1]) +
                               (Xu[2] - x[2]) * (Xu[2] - x[2]));
  if (resid) *resid = res;
  if (res > 1e-9 * scale) return 1;
  for (int a = 0; a < 3; ++a) xi[a] = u[a] / (double)(g.len(a) - 1);
  return 0;
}

}  // namespace sbp
