// HIP kernels (gfx950) for one Runge-Kutta stage of the upwind-SBP elastic
// solver, plus source injection, receiver gather and the energy reduction.
//
// Stage kernel (fused; one launch per stage):
//   for every node: RHS = volume terms (D+ on the velocities in the
//   non-conservative term, D- on the conservative stress flux, metric and
//   material weights; eq. gen_hyp_transformed_discrete) + boundary penalties
//   (eq. SAT_General / eq. SAT_free_surface), then
//   dQ <- A_k dQ + dt RHS,  Q_out <- Q_in + B_k dQ.
// Q_in and Q_out are different buffers (ping-pong), so neighbours are never
// read after being overwritten.
//
// Work decomposition: a thread block owns a tile of up to 64 (q) x TY (r)
// columns and marches along s over a chunk of planes.  For each plane it
// stages v, the q-flux and the r-flux of the tile plus a halo into LDS (the
// cross-axis stencils read LDS); along s it keeps register queues of v and of
// the s-flux (the interior s-stencils read registers).  The first and last m
// planes (SBP closure rows along s) read their s-neighbours from global memory.
// Boundary closure rows along q and r read wider LDS windows; tiles are laid
// out on the host so that each closure row lives in a tile whose window covers
// the columns it needs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "kernels.hpp"

namespace sbp {

template <int ORDER>
struct Stencil;
// Table tab:upwind: interior forward stencils alpha_{-r} .. alpha_{q}.
template <>
struct Stencil<2> {
  static constexpr int R = 0, Q = 2, M = 2;
  static constexpr double a[3] = {-3.0 / 2, 2.0, -1.0 / 2};
};
template <>
struct Stencil<4> {
  static constexpr int R = 1, Q = 3, M = 4;
  static constexpr double a[5] = {-1.0 / 4, -5.0 / 6, 3.0 / 2, -1.0 / 2, 1.0 / 12};
};
template <>
struct Stencil<6> {
  static constexpr int R = 2, Q = 4, M = 6;
  static constexpr double a[7] = {1.0 / 30, -2.0 / 5, -7.0 / 12, 4.0 / 3, -1.0 / 2, 2.0 / 15, -1.0 / 60};
};

// ---------------------------------------------------------------------------
// boundary penalty at one face node, accumulated into rate[9]
template <typename T>
__device__ __forceinline__ void face_penalty(const T* __restrict__ fc, std::size_t fstride,
                                             T gamma, T eps, bool traction, const T v[3],
                                             const T sg[6], T rate[9]) {
  const T nx = fc[FN_X * fstride], ny = fc[FN_Y * fstride], nz = fc[FN_Z * fstride];
  const T kr = fc[F_KR * fstride];
  // traction T = sigma n
  const T Tx = sg[0] * nx + sg[3] * ny + sg[4] * nz;
  const T Ty = sg[3] * nx + sg[1] * ny + sg[5] * nz;
  const T Tz = sg[4] * nx + sg[5] * ny + sg[2] * nz;
  if (traction) {
    rate[0] -= eps * kr * Tx;
    rate[1] -= eps * kr * Ty;
    rate[2] -= eps * kr * Tz;
    return;
  }
  const T zp = fc[F_ZP * fstride], zs = fc[F_ZS * fstride];
  const T izp = fc[F_IZP * fstride], izs = fc[F_IZS * fstride];
  const T kl = fc[F_KL * fstride], km = fc[F_KM * fstride];
  const T vn = v[0] * nx + v[1] * ny + v[2] * nz;
  const T Tn = Tx * nx + Ty * ny + Tz * nz;
  const T cv = T(0.5) * (T(1) - gamma);
  const T ct = T(0.5) * eps * (T(1) + gamma);
  // G_eta = 1/2 [(1 - gamma) Z_eta v_eta + eps (1 + gamma) T_eta], split into
  // the normal part and the tangential plane (Z_m = Z_l = Z_s)
  const T Gn = cv * zp * vn + ct * Tn;
  const T gtx = cv * zs * (v[0] - vn * nx) + ct * (Tx - Tn * nx);
  const T gty = cv * zs * (v[1] - vn * ny) + ct * (Ty - Tn * ny);
  const T gtz = cv * zs * (v[2] - vn * nz) + ct * (Tz - Tn * nz);
  rate[0] -= kr * (Gn * nx + gtx);
  rate[1] -= kr * (Gn * ny + gty);
  rate[2] -= kr * (Gn * nz + gtz);
  const T gn = Gn * izp;
  const T Gx = gn * nx + gtx * izs, Gy = gn * ny + gty * izs, Gz = gn * nz + gtz * izs;
  const T sxx = nx * Gx, syy = ny * Gy, szz = nz * Gz;
  const T tr = sxx + syy + szz;
  const T e = -eps;
  rate[3] += e * (kl * tr + T(2) * km * sxx);
  rate[4] += e * (kl * tr + T(2) * km * syy);
  rate[5] += e * (kl * tr + T(2) * km * szz);
  rate[6] += e * km * (ny * Gx + nx * Gy);
  rate[7] += e * km * (nz * Gx + nx * Gz);
  rate[8] += e * km * (nz * Gy + ny * Gz);
}

// ---------------------------------------------------------------------------
// the fused stage kernel
template <typename T, int ORDER, int TY>
__global__ __launch_bounds__(64 * TY) void stage_kernel(StageArgs<T> A) {
  using S = Stencil<ORDER>;
  constexpr int R = S::R, Q = S::Q, M = S::M;
  constexpr int H = Q;            // LDS halo width (Q >= R)
  constexpr int WX = 64 + 2 * H;  // LDS window
  constexpr int WY = TY + 2 * H;
  constexpr int WN = WX * WY;
  constexpr int QD = R + Q + 1;   // register queue depth
  constexpr int NT = 64 * TY;
  __shared__ T lds[9 * WN];  // v (3), q-flux (3), r-flux (3)

  // XCD-aware tile order: consecutive tiles land on the same XCD
  const int nb = gridDim.x;
  const int per = nb >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= A.ntiles) return;
  const int xt = tile % A.nxt;
  const int yt = (tile / A.nxt) % A.nyt;
  const int zc = tile / (A.nxt * A.nyt);
  const int* __restrict__ xb = A.bounds;
  const int* __restrict__ yb = A.bounds + A.nxt + 1;
  const int* __restrict__ zb = A.bounds + A.nxt + A.nyt + 2;
  const int x0 = xb[xt], x1 = xb[xt + 1];
  const int y0 = yb[yt], y1 = yb[yt + 1];
  const int z0 = zb[zc], z1 = zb[zc + 1];

  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * 64 + tx;
  const int i = x0 + tx, j = y0 + ty;
  const bool act = (i < x1) && (j < y1);
  const int nq = A.nq, nr = A.nr, ns = A.ns;
  const std::size_t px = A.px, plane = A.plane, field = A.field;
  const std::size_t col = (std::size_t)j * px + i;  // offset of (i, j) in a plane

  const T* __restrict__ qin = A.qin;
  const T* __restrict__ cf = A.coef;

  // s-flux F_s,i = sum_c M[s][c] sigma_ic at (i, j, k)
  auto sflux = [&](int k, T f[3]) {
    const std::size_t o = (std::size_t)k * plane + col;
    const T m0 = cf[6 * field + o], m1 = cf[7 * field + o], m2 = cf[8 * field + o];
    const T sxx = qin[3 * field + o], syy = qin[4 * field + o], szz = qin[5 * field + o];
    const T sxy = qin[6 * field + o], sxz = qin[7 * field + o], syz = qin[8 * field + o];
    f[0] = m0 * sxx + m1 * sxy + m2 * sxz;
    f[1] = m0 * sxy + m1 * syy + m2 * syz;
    f[2] = m0 * sxz + m1 * syz + m2 * szz;
  };

  // register queues: vq[s] = v(a - R + s), fq[t] = F_s(a - Q + t)
  T vq[3][QD], fq[3][QD];
#pragma unroll
  for (int s = 0; s < QD; ++s) {
#pragma unroll
    for (int c = 0; c < 3; ++c) { vq[c][s] = T(0); fq[c][s] = T(0); }
  }
  if (act) {
#pragma unroll
    for (int s = 0; s < QD; ++s) {
      const int kv = z0 - R + s;
      if (kv >= 0 && kv < ns) {
        const std::size_t o = (std::size_t)kv * plane + col;
#pragma unroll
        for (int c = 0; c < 3; ++c) vq[c][s] = qin[c * field + o];
      }
      const int kf = z0 - Q + s;
      if (kf >= 0 && kf < ns) {
        T f[3];
        sflux(kf, f);
#pragma unroll
        for (int c = 0; c < 3; ++c) fq[c][s] = f[c];
      }
    }
  }

  const int lx = tx + H, ly = ty + H;  // own LDS position
  const T ihq = A.inv_h[0], ihr = A.inv_h[1], ihs = A.inv_h[2];

  for (int a = z0; a < z1; ++a) {
    const std::size_t pa = (std::size_t)a * plane;
    // ---- stage v, q-flux, r-flux of plane a (tile + halo) into LDS
    for (int p = tid; p < WN; p += NT) {
      const int wy = p / WX, wx = p - wy * WX;
      const int gx = x0 - H + wx, gy = y0 - H + wy;
      T vals[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) vals[c] = T(0);
      if (gx >= 0 && gx < nq && gy >= 0 && gy < nr) {
        const std::size_t o = pa + (std::size_t)gy * px + gx;
        const T sxx = qin[3 * field + o], syy = qin[4 * field + o], szz = qin[5 * field + o];
        const T sxy = qin[6 * field + o], sxz = qin[7 * field + o], syz = qin[8 * field + o];
        const T q0 = cf[0 * field + o], q1 = cf[1 * field + o], q2 = cf[2 * field + o];
        const T r0 = cf[3 * field + o], r1 = cf[4 * field + o], r2 = cf[5 * field + o];
        vals[0] = qin[o];
        vals[1] = qin[field + o];
        vals[2] = qin[2 * field + o];
        vals[3] = q0 * sxx + q1 * sxy + q2 * sxz;
        vals[4] = q0 * sxy + q1 * syy + q2 * syz;
        vals[5] = q0 * sxz + q1 * syz + q2 * szz;
        vals[6] = r0 * sxx + r1 * sxy + r2 * sxz;
        vals[7] = r0 * sxy + r1 * syy + r2 * syz;
        vals[8] = r0 * sxz + r1 * syz + r2 * szz;
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) lds[c * WN + p] = vals[c];
    }
    __syncthreads();

    if (act) {
      T u[3][3];   // u[xi][c] = D+_xi v_c (times 1/h_xi applied below)
      T dv[3];     // sum_xi D-_xi F_xi,c
      const T* lv = lds;
      const T* lfq = lds + 3 * WN;
      const T* lfr = lds + 6 * WN;
      const int me = ly * WX + lx;
      // ---- q direction (LDS row)
      if (i >= M && i < nq - M) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sp = T(0), sm = T(0);
#pragma unroll
          for (int s = 0; s < QD; ++s) {
            sp += T(S::a[s]) * lv[c * WN + me - R + s];
            sm += T(S::a[s]) * lfq[c * WN + me + R - s];
          }
          u[0][c] = sp * ihq;
          dv[c] = -sm * ihq;
        }
      } else {
        const bool left = i < M;
        const int row = left ? i : nq - 1 - i;
        const int rowbase = ly * WX;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sp = T(0), sm = T(0);
          for (int cc = 0; cc < A.ncol; ++cc) {
            const int gcol = left ? cc : nq - 1 - cc;
            const int w = rowbase + gcol - x0 + H;
            if (left) {
              sp += A.dp[row][cc] * lv[c * WN + w];
              sm += A.dm[row][cc] * lfq[c * WN + w];
            } else {
              sp -= A.dm[row][cc] * lv[c * WN + w];
              sm -= A.dp[row][cc] * lfq[c * WN + w];
            }
          }
          u[0][c] = sp * ihq;
          dv[c] = sm * ihq;
        }
      }
      // ---- r direction (LDS column)
      if (j >= M && j < nr - M) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sp = T(0), sm = T(0);
#pragma unroll
          for (int s = 0; s < QD; ++s) {
            sp += T(S::a[s]) * lv[c * WN + me + (s - R) * WX];
            sm += T(S::a[s]) * lfr[c * WN + me + (R - s) * WX];
          }
          u[1][c] = sp * ihr;
          dv[c] -= sm * ihr;
        }
      } else {
        const bool left = j < M;
        const int row = left ? j : nr - 1 - j;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sp = T(0), sm = T(0);
          for (int cc = 0; cc < A.ncol; ++cc) {
            const int grow = left ? cc : nr - 1 - cc;
            const int w = (grow - y0 + H) * WX + lx;
            if (left) {
              sp += A.dp[row][cc] * lv[c * WN + w];
              sm += A.dm[row][cc] * lfr[c * WN + w];
            } else {
              sp -= A.dm[row][cc] * lv[c * WN + w];
              sm -= A.dp[row][cc] * lfr[c * WN + w];
            }
          }
          u[1][c] = sp * ihr;
          dv[c] += sm * ihr;
        }
      }
      // ---- s direction
      if (a >= M && a < ns - M) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sp = T(0), sm = T(0);
#pragma unroll
          for (int s = 0; s < QD; ++s) {
            sp += T(S::a[s]) * vq[c][s];
            sm += T(S::a[s]) * fq[c][R + Q - s];
          }
          u[2][c] = sp * ihs;
          dv[c] -= sm * ihs;
        }
      } else {
        const bool left = a < M;
        const int row = left ? a : ns - 1 - a;
        T sp[3] = {T(0), T(0), T(0)}, sm[3] = {T(0), T(0), T(0)};
        for (int cc = 0; cc < A.ncol; ++cc) {
          const int k = left ? cc : ns - 1 - cc;
          const std::size_t o = (std::size_t)k * plane + col;
          T f[3];
          sflux(k, f);
          const T cp = left ? A.dp[row][cc] : -A.dm[row][cc];
          const T cm = left ? A.dm[row][cc] : -A.dp[row][cc];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            sp[c] += cp * qin[c * field + o];
            sm[c] += cm * f[c];
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          u[2][c] = sp[c] * ihs;
          dv[c] += sm[c] * ihs;
        }
      }

      // ---- pointwise: stress rates (non-conservative metric form + Hooke)
      const std::size_t o = pa + col;
      T Mm[3][3];
#pragma unroll
      for (int xi = 0; xi < 3; ++xi)
#pragma unroll
        for (int c = 0; c < 3; ++c) Mm[xi][c] = cf[(3 * xi + c) * field + o];
      const T lamJ = cf[9 * field + o], muJ = cf[10 * field + o], rJ = cf[11 * field + o];
      T G[3][3];  // G[c][i] = sum_xi M[xi][c] u[xi][i]  (= J dv_i/dx_c)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
          G[c][ii] = Mm[0][c] * u[0][ii] + Mm[1][c] * u[1][ii] + Mm[2][c] * u[2][ii];
      const T div = G[0][0] + G[1][1] + G[2][2];
      T rate[9];
      rate[0] = rJ * dv[0];
      rate[1] = rJ * dv[1];
      rate[2] = rJ * dv[2];
      rate[3] = lamJ * div + T(2) * muJ * G[0][0];
      rate[4] = lamJ * div + T(2) * muJ * G[1][1];
      rate[5] = lamJ * div + T(2) * muJ * G[2][2];
      rate[6] = muJ * (G[1][0] + G[0][1]);
      rate[7] = muJ * (G[2][0] + G[0][2]);
      rate[8] = muJ * (G[2][1] + G[1][2]);

      T v[3] = {vq[0][R], vq[1][R], vq[2][R]};
      T sg[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] = qin[(3 + c) * field + o];

      // ---- boundary penalties (faces q0, q1, r0, r1, s0, s1)
      if (i == 0 || i == nq - 1 || j == 0 || j == nr - 1 || a == 0 || a == ns - 1) {
        if (i == 0)
          face_penalty(A.face + A.face_off[0] + ((std::size_t)a * nr + j), A.face_n[0], A.gamma[0],
                       T(-1), A.traction[0], v, sg, rate);
        if (i == nq - 1)
          face_penalty(A.face + A.face_off[1] + ((std::size_t)a * nr + j), A.face_n[1], A.gamma[1],
                       T(1), A.traction[1], v, sg, rate);
        if (j == 0)
          face_penalty(A.face + A.face_off[2] + ((std::size_t)a * nq + i), A.face_n[2], A.gamma[2],
                       T(-1), A.traction[2], v, sg, rate);
        if (j == nr - 1)
          face_penalty(A.face + A.face_off[3] + ((std::size_t)a * nq + i), A.face_n[3], A.gamma[3],
                       T(1), A.traction[3], v, sg, rate);
        if (a == 0)
          face_penalty(A.face + A.face_off[4] + ((std::size_t)j * nq + i), A.face_n[4], A.gamma[4],
                       T(-1), A.traction[4], v, sg, rate);
        if (a == ns - 1)
          face_penalty(A.face + A.face_off[5] + ((std::size_t)j * nq + i), A.face_n[5], A.gamma[5],
                       T(1), A.traction[5], v, sg, rate);
      }

      // ---- Runge-Kutta stage update
      T* __restrict__ dq = A.dq;
      T* __restrict__ qout = A.qout;
      const T dt = A.dt, Ak = A.Ak, Bk = A.Bk;
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        T d = dt * rate[c];
        if (A.read_dq) d += Ak * dq[c * field + o];
        dq[c * field + o] = d;
        const T q0 = (c < 3) ? v[c] : sg[c - 3];
        qout[c * field + o] = q0 + Bk * d;
      }
    }

    // ---- advance the s queues to plane a + 1
    if (act) {
#pragma unroll
      for (int s = 0; s < QD - 1; ++s) {
#pragma unroll
        for (int c = 0; c < 3; ++c) { vq[c][s] = vq[c][s + 1]; fq[c][s] = fq[c][s + 1]; }
      }
      const int kv = a + 1 + Q;
      if (kv < ns) {
        const std::size_t oo = (std::size_t)kv * plane + col;
#pragma unroll
        for (int c = 0; c < 3; ++c) vq[c][QD - 1] = qin[c * field + oo];
      }
      const int kf = a + 1 + R;
      if (kf < ns) {
        T f[3];
        sflux(kf, f);
#pragma unroll
        for (int c = 0; c < 3; ++c) fq[c][QD - 1] = f[c];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// point sources: dQ += gdt * w M, Q_out += Bk * gdt * w M on the source stencil
template <typename T>
__global__ void source_kernel(SourceArgs<T> S) {
  const int s = blockIdx.x;
  const int w = S.width;
  const int n = w * w * w;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int a = t % w, b = (t / w) % w, c = t / (w * w);
    const std::size_t o = (std::size_t)(S.k0[s] + c) * S.plane + (std::size_t)(S.j0[s] + b) * S.px +
                          (S.i0[s] + a);
    const T* wm = S.wm + ((std::size_t)s * kMaxSrcWidth * kMaxSrcWidth * kMaxSrcWidth + t) * 6;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const T add = S.gdt[s] * wm[f];
      S.dq[(3 + f) * S.field + o] += add;
      if (S.qout) S.qout[(3 + f) * S.field + o] += S.Bk * add;
    }
  }
}

// receivers: out[(step * nrec + r) * 3 + c] = v_c(node_r)
template <typename T>
__global__ void record_kernel(const T* __restrict__ q, std::size_t field, const long long* __restrict__ off,
                              int nrec, T* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrec) return;
  const long long o = off[r];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[(std::size_t)r * 3 + c] = q[c * field + o];
}

// energy: partial sums of 1/2 H J (rho |v|^2 + sigma^T C^{-1} sigma) per block
template <typename T>
__global__ void energy_kernel(EnergyArgs<T> E) {
  __shared__ double red[256];
  double acc = 0.0;
  const long long n = (long long)E.nq * E.nr * E.ns;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const int i = idx % E.nq;
    const int j = (idx / E.nq) % E.nr;
    const int k = idx / ((long long)E.nq * E.nr);
    auto wgt = [&](int ii, int nn, const double* w, int m, double h) {
      if (ii < m) return h * w[ii];
      if (ii >= nn - m) return h * w[nn - 1 - ii];
      return h;
    };
    const double H = wgt(i, E.nq, E.w, E.m, E.h[0]) * wgt(j, E.nr, E.w, E.m, E.h[1]) *
                     wgt(k, E.ns, E.w, E.m, E.h[2]);
    const std::size_t o = (std::size_t)k * E.plane + (std::size_t)j * E.px + i;
    const double vx = E.q[o], vy = E.q[E.field + o], vz = E.q[2 * E.field + o];
    const double sxx = E.q[3 * E.field + o], syy = E.q[4 * E.field + o], szz = E.q[5 * E.field + o];
    const double sxy = E.q[6 * E.field + o], sxz = E.q[7 * E.field + o], syz = E.q[8 * E.field + o];
    const double lam = E.coef[9 * E.field + o], mu = E.coef[10 * E.field + o];
    const double rJ = E.coef[11 * E.field + o];
    const double tr = sxx + syy + szz;
    const double strain = (sxx * sxx + syy * syy + szz * szz - lam / (3 * lam + 2 * mu) * tr * tr) / (2 * mu) +
                          (sxy * sxy + sxz * sxz + syz * syz) / mu;
    acc += 0.5 * H * ((vx * vx + vy * vy + vz * vz) / rJ + strain);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) E.part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// launchers
template <typename T, int ORDER, int TY>
static hipError_t launch_stage_t(const StageArgs<T>& a, hipStream_t st) {
  const int nb = ((a.ntiles + 7) / 8) * 8;
  hipLaunchKernelGGL((stage_kernel<T, ORDER, TY>), dim3(nb), dim3(64, TY), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stage(int order, int ty, const StageArgs<T>& a, hipStream_t st) {
  if (ty == 8) {
    if (order == 2) return launch_stage_t<T, 2, 8>(a, st);
    if (order == 4) return launch_stage_t<T, 4, 8>(a, st);
    if (order == 6) return launch_stage_t<T, 6, 8>(a, st);
  } else if (ty == 4) {
    if (order == 2) return launch_stage_t<T, 2, 4>(a, st);
    if (order == 4) return launch_stage_t<T, 4, 4>(a, st);
    if (order == 6) return launch_stage_t<T, 6, 4>(a, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_source(const SourceArgs<T>& s, int nsrc, hipStream_t st) {
  hipLaunchKernelGGL(source_kernel<T>, dim3(nsrc), dim3(256), 0, st, s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_record(const T* q, std::size_t field, const long long* off, int nrec, T* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(record_kernel<T>, dim3((nrec + 255) / 256), dim3(256), 0, st, q, field, off, nrec, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_energy(const EnergyArgs<T>& e, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(energy_kernel<T>, dim3(nblocks), dim3(256), 0, st, e);
  return hipGetLastError();
}

template hipError_t launch_stage<float>(int, int, const StageArgs<float>&, hipStream_t);
template hipError_t launch_stage<double>(int, int, const StageArgs<double>&, hipStream_t);
template hipError_t launch_source<float>(const SourceArgs<float>&, int, hipStream_t);
template hipError_t launch_source<double>(const SourceArgs<double>&, int, hipStream_t);
template hipError_t launch_record<float>(const float*, std::size_t, const long long*, int, float*, hipStream_t);
template hipError_t launch_record<double>(const double*, std::size_t, const long long*, int, double*,
                                          hipStream_t);
template hipError_t launch_energy<float>(const EnergyArgs<float>&, int, hipStream_t);
template hipError_t launch_energy<double>(const EnergyArgs<double>&, int, hipStream_t);

}  // namespace sbp
