// CPU-only check of the library's host-side set-up code, built with the
// address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py:
// the SBP closures of every supported order, the metric terms of a warped
// mesh, the discrete delta's window and basis, and the inversion of the map
// at physical points (inside, on a face, outside).  Prints one line per check
// and returns non-zero on a failed check; the sanitizers abort on any memory
// or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2011_02600_amd/csrc/host_math.hpp"

using namespace sbp;

int main() {
  int bad = 0;
  for (int order = 2; order <= 9; ++order) {
    Closure c;
    const char* err = "";
    const bool ok = build_closure(order, &c, &err);
    std::printf("closure order %d: %s %s\n", order, ok ? "built" : "rejected", ok ? "" : err);
    if (ok) {
      // H D+ + (H D-)^T = B on the closure block: row sums of D+ vanish
      for (int i = 0; i < c.m; ++i) {
        double s = 0;
        for (int j = 0; j < c.ncol; ++j) s += c.dp[i][j];
        if (std::fabs(s) > 1e-12) {
          std::printf("  row %d of D+ does not annihilate constants (%g)\n", i, s);
          ++bad;
        }
      }
    }
  }
  Closure c;
  const char* err = "";
  if (!build_closure(6, &c, &err)) return 1;
  Grid3 g;
  g.nq = 19;
  g.nr = 17;
  g.ns = 21;
  g.n = (std::size_t)g.nq * g.nr * g.ns;
  std::vector<double> X(3 * g.n), J(g.n), M(9 * g.n);
  for (int k = 0; k < g.ns; ++k)
    for (int j = 0; j < g.nr; ++j)
      for (int i = 0; i < g.nq; ++i) {
        const double u = (double)i / (g.nq - 1), v = (double)j / (g.nr - 1), w = (double)k / (g.ns - 1);
        const std::size_t o = g.idx(i, j, k);
        X[o] = u + 0.04 * std::sin(6.2831853 * v) * std::sin(6.2831853 * w);
        X[g.n + o] = v + 0.03 * std::sin(6.2831853 * u + 1.0) * w;
        X[2 * g.n + o] = w + 0.05 * u * v * (1 - u);
      }
  const long long neg = metric_terms(c, g, X.data(), J.data(), M.data());
  std::printf("metric terms: first non-positive J at %lld\n", neg);
  if (neg >= 0) ++bad;
  const int width = 2 * (6 / 2 + 1);
  double phi[kMaxSrcWidth], dphi[kMaxSrcWidth];
  for (double u : {0.0, 0.3, 7.5, 17.9, 18.0}) {
    const int st = delta_window(g.nq, width, u);
    lagrange_basis(width, st, u, phi, dphi);
    double s = 0, ds = 0;
    for (int a = 0; a < width; ++a) {
      s += phi[a];
      ds += dphi[a];
    }
    if (st < 0 || st + width > g.nq || std::fabs(s - 1) > 1e-12 || std::fabs(ds) > 1e-10) {
      std::printf("delta window/basis wrong at u = %g\n", u);
      ++bad;
    }
  }
  // a node, a point between nodes, a point on the top face, a point outside
  struct P {
    double x[3];
    int expect;
  };
  const std::size_t a = g.idx(5, 6, 7), b = g.idx(6, 7, 8), t = g.idx(3, 4, g.ns - 1);
  P pts[] = {{{X[a], X[g.n + a], X[2 * g.n + a]}, 0},
             {{0.5 * (X[a] + X[b]), 0.5 * (X[g.n + a] + X[g.n + b]), 0.5 * (X[2 * g.n + a] + X[2 * g.n + b])}, 0},
             {{X[t], X[g.n + t], X[2 * g.n + t]}, 0},
             {{0.5, 0.5, 1.4}, 1}};
  for (const P& p : pts) {
    double xi[3] = {0, 0, 0}, res = -1;
    const int r = locate_point(g, X.data(), width, p.x, xi, &res);
    std::printf("locate (%g, %g, %g): code %d xi (%g, %g, %g) residual %g\n", p.x[0], p.x[1], p.x[2], r, xi[0],
                xi[1], xi[2], res);
    if ((r == 0) != (p.expect == 0)) ++bad;
  }
  std::printf("%s\n", bad ? "FAILED" : "OK");
  return bad ? 1 : 0;
}
