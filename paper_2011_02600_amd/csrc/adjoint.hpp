// Kernels of the discrete adjoint (misfit gradient with respect to the
// material): argument block and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "internal.hpp"

namespace sbp {

// One pass over every node of a grid.  Fields are in the NodeMap layout of
// the solver; every buffer holds 9 fields unless noted.
template <typename T>
struct AdjArgs {
  NodeMap nm;
  std::size_t field;
  int nq, nr, ns, m;
  T w[kMaxM];       // boundary norm weights w_0 .. w_{m-1} (the rest are 1)
  T h[3];           // grid spacings 1 / (n - 1) along q, r, s
  const T* coef;    // 12 fields: M[xi][c], lambda/J, mu/J, 1/(rho J)
  const T* face;    // workspace base of the face coefficient arrays
  std::size_t face_off[6], face_n[6];
  T gamma[6];
  int traction[6];
  T* qb;            // adjoint state
  T* dqb;           // adjoint Runge-Kutta register
  T* y;             // W^{-1} dqb
  const T* r;       // volume right-hand side of y (adj_post) or, with unit
                    // material, of the forward stage input (adj_grad)
  const T* qs;      // forward stage input
  const T* jac;     // 1 field: J
  T* grad;          // 3 fields: d chi / d (rho, lambda, mu)
  T a, b, dt;
};

template <typename T>
hipError_t launch_adj_pre(const AdjArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_adj_post(const AdjArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_adj_grad(const AdjArgs<T>& a, hipStream_t st);
// qb[c][off[r]] += res[r][c] for the nrec receivers (velocity components)
template <typename T>
hipError_t launch_adj_inject(T* qb, std::size_t field, const long long* off, int nrec, const T* res,
                             hipStream_t st);
// n values of dst = v
template <typename T>
hipError_t launch_fill(T* dst, std::size_t n, T v, hipStream_t st);

}  // namespace sbp
