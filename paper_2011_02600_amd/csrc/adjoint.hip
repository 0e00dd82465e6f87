// HIP kernels (gfx950) of the discrete adjoint: the transposed operator and
// the misfit gradient with respect to the nodal material.
//
// The transposed semi-discrete operator is built from the forward one.  With
// W the energy weights H J diag(rho I_3, C^{-1}) (per node; H the tensor
// norm), the volume operator L_v satisfies the energy identity of the scheme
// (summation by parts along each axis, H D+ + (H D-)^T = B):
//   W L_v + L_v^T W = Bd,
//   Q^T Bd Q' = sum_xi sum_i [v_i^T B_xi F_xi,i(sigma') + v'_i^T B_xi F_xi,i(sigma)],
// B_xi = +-(norm weights of the two other axes) on the faces xi = 0, 1 and F
// the stress flux with the metric row M_xi.  Hence
//   L^T l = -W L_v(W^{-1} l) + Bd W^{-1} l + P^T l,
// P the face-local penalty blocks.  L_v(W^{-1} l) is one forward
// right-hand-side evaluation with the penalties off (the stage kernel); the
// kernels here apply W^{-1} (adj_pre), -W (adj_post, every node) and Bd and
// P^T (adj_face, face nodes only, one launch per axis).
//
// The material enters the right-hand side pointwise: 1/(rho J) times the
// flux divergence dv, lambda/J and mu/J times the velocity gradient terms,
// and the penalty coefficients of the node's faces.  adj_grad takes dv and
// the gradient terms from a forward evaluation with unit material
// (lambda/J = 0, mu/J = 1, 1/(rho J) = 1, penalties off) and differentiates
// the penalties on dual numbers.
#include <hip/hip_runtime.h>

#include "adjoint.hpp"
#include "penalty.hpp"

namespace sbp {
namespace {

// value and derivative along one direction
template <typename T>
struct Dual {
  T v, d;
  Dual() = default;
  __device__ Dual(double x) : v(T(x)), d(T(0)) {}
  __device__ Dual(T x, T dx) : v(x), d(dx) {}
};
template <typename T>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return Dual<T>(a.v + b.v, a.d + b.d); }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return Dual<T>(a.v - b.v, a.d - b.d); }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return Dual<T>(-a.v, -a.d); }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
  return Dual<T>(a.v * b.v, a.d * b.v + a.v * b.d);
}
template <typename T>
__device__ __forceinline__ Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { return a = a + b; }
template <typename T>
__device__ __forceinline__ Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { return a = a - b; }

template <typename T>
__device__ __forceinline__ T norm_w(const AdjArgs<T>& A, int i, int n) {
  if (i < A.m) return A.w[i];
  if (i >= n - A.m) return A.w[n - 1 - i];
  return T(1);
}

struct Node {
  int i, j, k;
  long long o;
};

template <typename T>
__device__ __forceinline__ Node node_of(const AdjArgs<T>& A, long long n) {
  Node d;
  d.i = (int)(n % A.nq);
  const long long t = n / A.nq;
  d.j = (int)(t % A.nr);
  d.k = (int)(t / A.nr);
  d.o = A.nm(d.i, d.j, d.k);
  return d;
}

template <typename T>
__global__ void adj_pre_kernel(const AdjArgs<T> A) {
  const long long N = (long long)A.nq * A.nr * A.ns;
  const std::size_t F = A.field;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const Node nd = node_of(A, n);
    const long long o = nd.o;
    T d[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const T prev = A.a != T(0) ? A.a * A.dqb[c * F + o] : T(0);
      d[c] = prev + A.b * A.qb[c * F + o];
      A.dqb[c * F + o] = d[c];
    }
    const T iH = T(1) / (A.h[0] * norm_w(A, nd.i, A.nq) * A.h[1] * norm_w(A, nd.j, A.nr) * A.h[2] *
                         norm_w(A, nd.k, A.ns));
    const T lamJ = A.coef[9 * F + o], muJ = A.coef[10 * F + o], rJ = A.coef[11 * F + o];
    // W^{-1}: v / (H rho J), and C / (H J) on the stress (engineering shear)
    const T tr = d[3] + d[4] + d[5];
    T y[9];
    y[0] = rJ * d[0] * iH;
    y[1] = rJ * d[1] * iH;
    y[2] = rJ * d[2] * iH;
    y[3] = (lamJ * tr + T(2) * muJ * d[3]) * iH;
    y[4] = (lamJ * tr + T(2) * muJ * d[4]) * iH;
    y[5] = (lamJ * tr + T(2) * muJ * d[5]) * iH;
    y[6] = muJ * d[6] * iH;
    y[7] = muJ * d[7] * iH;
    y[8] = muJ * d[8] * iH;
#pragma unroll
    for (int c = 0; c < 9; ++c) A.y[c * F + o] = y[c];
  }
}

template <typename T>
__global__ void adj_post_kernel(const AdjArgs<T> A) {
  const long long N = (long long)A.nq * A.nr * A.ns;
  const std::size_t F = A.field;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const Node nd = node_of(A, n);
    const long long o = nd.o;
    const T wq = norm_w(A, nd.i, A.nq), wr = norm_w(A, nd.j, A.nr), ws = norm_w(A, nd.k, A.ns);
    const T Hn = A.h[0] * wq * A.h[1] * wr * A.h[2] * ws;
    const T lamJ = A.coef[9 * F + o], muJ = A.coef[10 * F + o], rJ = A.coef[11 * F + o];
    T r[9], out[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) r[c] = A.r[c * F + o];
    // -W r: -H rho J r_v and -H J C^{-1} r_sigma
    out[0] = -Hn * r[0] / rJ;
    out[1] = -Hn * r[1] / rJ;
    out[2] = -Hn * r[2] / rJ;
    const T trr = r[3] + r[4] + r[5];
    const T cl = lamJ / (T(3) * lamJ + T(2) * muJ);
    const T i2m = T(1) / (T(2) * muJ);
    out[3] = -Hn * (r[3] - cl * trr) * i2m;
    out[4] = -Hn * (r[4] - cl * trr) * i2m;
    out[5] = -Hn * (r[5] - cl * trr) * i2m;
    out[6] = -Hn * r[6] / muJ;
    out[7] = -Hn * r[7] / muJ;
    out[8] = -Hn * r[8] / muJ;
#pragma unroll
    for (int c = 0; c < 9; ++c) A.qb[c * F + o] += A.dt * out[c];
  }
}

template <typename T>
__global__ void adj_grad_kernel(const AdjArgs<T> A) {
  const long long N = (long long)A.nq * A.nr * A.ns;
  const std::size_t F = A.field;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const Node nd = node_of(A, n);
    const long long o = nd.o;
    T ru[9], l[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      ru[c] = A.r[c * F + o];
      l[c] = A.dqb[c * F + o];
    }
    const T J = A.jac[o];
    const T rJ = A.coef[11 * F + o];
    const T iJ = T(1) / J;
    // volume terms: d(1/(rho J))/d rho = -rJ^2 J, d(lambda/J)/d lambda = d(mu/J)/d mu = 1/J
    T g0 = -rJ * rJ * J * (l[0] * ru[0] + l[1] * ru[1] + l[2] * ru[2]);
    const T div = T(0.5) * (ru[3] + ru[4] + ru[5]);
    T g1 = iJ * div * (l[3] + l[4] + l[5]);
    T g2 = iJ * (l[3] * ru[3] + l[4] * ru[4] + l[5] * ru[5] + l[6] * ru[6] + l[7] * ru[7] + l[8] * ru[8]);
    A.grad[0 * F + o] += A.dt * g0;
    A.grad[1 * F + o] += A.dt * g1;
    A.grad[2 * F + o] += A.dt * g2;
  }
}

// Face terms of one axis xi: the nodes of faces 2 xi and 2 xi + 1 (disjoint,
// so one launch per axis has no two threads on one node).  GRAD = false:
// Bd y + P^T dqb added to qb (times dt); GRAD = true: the derivative of the
// penalty with respect to the node's rho, lambda, mu (dual numbers, seeded
// with the derivatives of the face coefficients) against dqb, added to grad.
template <typename T, bool GRAD>
__global__ void adj_face_kernel(const AdjArgs<T> A, int xi) {
  const std::size_t F = A.field;
  const std::size_t fn = xi == 0 ? (std::size_t)A.nr * A.ns : (xi == 1 ? (std::size_t)A.nq * A.ns
                                                                        : (std::size_t)A.nq * A.nr);
  const std::size_t t = blockIdx.x * (std::size_t)blockDim.x + threadIdx.x;
  if (t >= 2 * fn) return;
  const int side = t >= fn ? 1 : 0;
  const int f = 2 * xi + side;
  const std::size_t idx = t - side * fn;
  Node nd;
  if (xi == 0) {
    nd.i = side ? A.nq - 1 : 0;
    nd.j = (int)(idx % A.nr);
    nd.k = (int)(idx / A.nr);
  } else if (xi == 1) {
    nd.i = (int)(idx % A.nq);
    nd.j = side ? A.nr - 1 : 0;
    nd.k = (int)(idx / A.nq);
  } else {
    nd.i = (int)(idx % A.nq);
    nd.j = (int)(idx / A.nq);
    nd.k = side ? A.ns - 1 : 0;
  }
  const long long o = A.nm(nd.i, nd.j, nd.k);
  T fc[kNumFaceCoef];
#pragma unroll
  for (int kk = 0; kk < kNumFaceCoef; ++kk) fc[kk] = A.face[A.face_off[f] + idx + (std::size_t)kk * A.face_n[f]];
  const T sgn = side ? T(1) : T(-1);
  T l[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) l[c] = A.dqb[c * F + o];
  if constexpr (!GRAD) {
    T y[9], out[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) y[c] = A.y[c * F + o];
    const T wq = norm_w(A, nd.i, A.nq), wr = norm_w(A, nd.j, A.nr), ws = norm_w(A, nd.k, A.ns);
    // B_xi: sign times the norm weights of the two other axes
    const T bw = xi == 0 ? A.h[1] * wr * A.h[2] * ws : (xi == 1 ? A.h[0] * wq * A.h[2] * ws : A.h[0] * wq * A.h[1] * wr);
    const T b = sgn * bw;
    const T m0 = A.coef[(3 * xi) * F + o], m1 = A.coef[(3 * xi + 1) * F + o], m2 = A.coef[(3 * xi + 2) * F + o];
    // Bd y: velocity rows take the flux of y_sigma, stress rows the
    // transposed flux map of y_v
    out[0] = b * (m0 * y[3] + m1 * y[6] + m2 * y[7]);
    out[1] = b * (m0 * y[6] + m1 * y[4] + m2 * y[8]);
    out[2] = b * (m0 * y[7] + m1 * y[8] + m2 * y[5]);
    const T z0 = b * y[0], z1 = b * y[1], z2 = b * y[2];
    out[3] = m0 * z0;
    out[4] = m1 * z1;
    out[5] = m2 * z2;
    out[6] = m1 * z0 + m0 * z1;
    out[7] = m2 * z0 + m0 * z2;
    out[8] = m2 * z1 + m1 * z2;
    // P^T l: column kk of the penalty block is its response to unit vector kk
    for (int kk = 0; kk < 9; ++kk) {
      T ev[3] = {T(0), T(0), T(0)}, es[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
      if (kk < 3) ev[kk] = T(1);
      else es[kk - 3] = T(1);
      T rate[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) rate[c] = T(0);
      face_penalty(fc, A.gamma[f], sgn, A.traction[f] != 0, ev, es, rate);
      T s = T(0);
#pragma unroll
      for (int c = 0; c < 9; ++c) s += rate[c] * l[c];
      out[kk] += s;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) A.qb[c * F + o] += A.dt * out[c];
  } else {
    using D = Dual<T>;
    D v[3], sg[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = D(A.qs[c * F + o], T(0));
#pragma unroll
    for (int c = 0; c < 6; ++c) sg[c] = D(A.qs[(3 + c) * F + o], T(0));
    const T rho = T(1) / (A.coef[11 * F + o] * A.jac[o]);
    const T zp = fc[F_ZP], zs = fc[F_ZS], izp = fc[F_IZP], izs = fc[F_IZS], kr = fc[F_KR];
    const T kap = kr * rho;
    // derivatives of the face coefficients (Z_p = sqrt(rho (lambda + 2 mu)),
    // Z_s = sqrt(rho mu), their inverses, kappa/rho, kappa lambda, kappa mu)
    // with respect to rho, lambda, mu
    T seed[3][kNumFaceCoef] = {};
    seed[0][F_ZP] = zp / (T(2) * rho);
    seed[0][F_ZS] = zs / (T(2) * rho);
    seed[0][F_IZP] = -izp / (T(2) * rho);
    seed[0][F_IZS] = -izs / (T(2) * rho);
    seed[0][F_KR] = -kr / rho;
    seed[1][F_ZP] = T(0.5) * rho * izp;
    seed[1][F_IZP] = -T(0.5) * rho * izp * izp * izp;
    seed[1][F_KL] = kap;
    seed[2][F_ZP] = rho * izp;
    seed[2][F_ZS] = T(0.5) * rho * izs;
    seed[2][F_IZP] = -rho * izp * izp * izp;
    seed[2][F_IZS] = -T(0.5) * rho * izs * izs * izs;
    seed[2][F_KM] = kap;
    for (int p = 0; p < 3; ++p) {
      D dfc[kNumFaceCoef], rate[9];
#pragma unroll
      for (int kk = 0; kk < kNumFaceCoef; ++kk) dfc[kk] = D(fc[kk], seed[p][kk]);
#pragma unroll
      for (int c = 0; c < 9; ++c) rate[c] = D(T(0), T(0));
      face_penalty(dfc, D(A.gamma[f], T(0)), D(sgn, T(0)), A.traction[f] != 0, v, sg, rate);
      T s = T(0);
#pragma unroll
      for (int c = 0; c < 9; ++c) s += rate[c].d * l[c];
      A.grad[p * F + o] += A.dt * s;
    }
  }
}

template <typename T>
__global__ void adj_inject_kernel(T* qb, std::size_t field, const long long* off, int nrec, const T* res) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrec) return;
  const long long o = off[r];
#pragma unroll
  for (int c = 0; c < 3; ++c) atomicAdd(qb + c * field + o, res[3 * r + c]);
}

template <typename T>
__global__ void fill_kernel(T* dst, std::size_t n, T v) {
  for (std::size_t e = blockIdx.x * (std::size_t)blockDim.x + threadIdx.x; e < n; e += (std::size_t)gridDim.x * blockDim.x)
    dst[e] = v;
}

template <typename T>
int node_blocks(const AdjArgs<T>& a) {
  const long long N = (long long)a.nq * a.nr * a.ns;
  return (int)std::min<long long>((N + 255) / 256, 1 << 16);
}

}  // namespace

template <typename T>
hipError_t launch_adj_pre(const AdjArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(adj_pre_kernel<T>, dim3(node_blocks(a)), dim3(256), 0, st, a);
  return hipGetLastError();
}
template <typename T, bool GRAD>
hipError_t launch_faces(const AdjArgs<T>& a, hipStream_t st) {
  const std::size_t fn[3] = {(std::size_t)a.nr * a.ns, (std::size_t)a.nq * a.ns, (std::size_t)a.nq * a.nr};
  for (int xi = 0; xi < 3; ++xi) {
    hipLaunchKernelGGL((adj_face_kernel<T, GRAD>), dim3((unsigned)((2 * fn[xi] + 255) / 256)), dim3(256), 0, st, a,
                       xi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template <typename T>
hipError_t launch_adj_post(const AdjArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(adj_post_kernel<T>, dim3(node_blocks(a)), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_faces<T, false>(a, st);
}
template <typename T>
hipError_t launch_adj_grad(const AdjArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(adj_grad_kernel<T>, dim3(node_blocks(a)), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_faces<T, true>(a, st);
}
template <typename T>
hipError_t launch_adj_inject(T* qb, std::size_t field, const long long* off, int nrec, const T* res,
                             hipStream_t st) {
  if (nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(adj_inject_kernel<T>, dim3((nrec + 255) / 256), dim3(256), 0, st, qb, field, off, nrec, res);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(T* dst, std::size_t n, T v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int nb = (int)std::min<std::size_t>((n + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(fill_kernel<T>, dim3(nb), dim3(256), 0, st, dst, n, v);
  return hipGetLastError();
}

template hipError_t launch_adj_pre<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adj_pre<double>(const AdjArgs<double>&, hipStream_t);
template hipError_t launch_adj_post<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adj_post<double>(const AdjArgs<double>&, hipStream_t);
template hipError_t launch_adj_grad<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adj_grad<double>(const AdjArgs<double>&, hipStream_t);
template hipError_t launch_adj_inject<float>(float*, std::size_t, const long long*, int, const float*, hipStream_t);
template hipError_t launch_adj_inject<double>(double*, std::size_t, const long long*, int, const double*,
                                              hipStream_t);
template hipError_t launch_fill<float>(float*, std::size_t, float, hipStream_t);
template hipError_t launch_fill<double>(double*, std::size_t, double, hipStream_t);

}  // namespace sbp
