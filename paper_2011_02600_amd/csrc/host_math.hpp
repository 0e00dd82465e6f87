// Host-side numerics of the set-up, in double precision and plain C++ (no
// HIP): one-dimensional SBP operators applied along an axis, the metric
// terms, the one-dimensional discrete delta of a point source and the
// inversion of the curvilinear map at a physical point.  Kept free of the
// runtime so that it can also be built and checked on the CPU alone.
#pragma once

#include <cstddef>

#include "internal.hpp"

namespace sbp {

// Points along q, r, s of a block; dense grid functions in (s, r, q) order,
// q fastest.
struct Grid3 {
  int nq = 0, nr = 0, ns = 0;
  std::size_t n = 0;
  std::size_t idx(int i, int j, int k) const { return ((std::size_t)k * nr + j) * nq + i; }
  int len(int ax) const { return ax == 0 ? nq : (ax == 1 ? nr : ns); }
};

// out = (h * D) in along axis ax (0 q, 1 r, 2 s) for D = D+ (kind 0),
// D- (kind 1) or D0 = (D+ + D-) / 2 (kind 2), with 1 / h = N - 1 (Sec. 4.1).
void apply_axis(const Closure& c, const Grid3& g, const double* in, double* out, int ax, int kind);

// Metric terms of Sec. 2.2 from the node coordinates X (3 grid functions x,
// y, z): x_xi = D0_xi x, J = det, and the conservative cofactor form
// M[xi][c] = D-_zeta(e D0_eta d) - D-_eta(e D0_zeta d), (xi, eta, zeta) and
// (c, d, e) cyclic, written to M (9 grid functions, M[3 xi + c]) and J.
// Returns the index of the first node with J <= 0, or -1.
long long metric_terms(const Closure& c, const Grid3& g, const double* X, double* J, double* M);

// First node of the `width` nodes nearest to reference position u (in node
// units, 0 .. N-1) along an axis of N points, clamped inside the axis.
int delta_window(int N, int width, double u);

// Lagrange basis of the nodes start .. start+width-1 at u: phi[a] and, if
// dphi is not null, its derivative in u.
void lagrange_basis(int width, int start, double u, double* phi, double* dphi);

// Reference coordinates (q, r, s in [0, 1]) of the physical point x for the
// block with node coordinates X: Newton iteration on the tensor-product
// Lagrange interpolant of X over the `width` nearest nodes per axis (the
// window of the discrete delta), started at the nearest node.  Returns 0 and
// writes xi on success, 1 if the point lies outside the block, 2 if the
// iteration does not converge.  *resid (may be null) receives the distance
// |X(xi) - x| of the result.
int locate_point(const Grid3& g, const double* X, int width, const double x[3], double xi[3], double* resid);

}  // namespace sbp
