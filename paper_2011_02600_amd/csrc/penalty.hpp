// Boundary penalty of one face node (shared by the stage, edge and adjoint
// kernels).  Written for any arithmetic type T with +, -, * and construction
// from a constant, so that the adjoint can evaluate it on dual numbers.
#pragma once

#include "internal.hpp"

namespace sbp {

// boundary penalty at one face node, accumulated into rate[9]
template <typename T>
__device__ __forceinline__ void face_penalty(const T fc[kNumFaceCoef], T gamma, T eps, bool traction,
                                             const T v[3], const T sg[6], T rate[9]) {
  const T nx = fc[FN_X], ny = fc[FN_Y], nz = fc[FN_Z];
  const T kr = fc[F_KR];
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
  const T zp = fc[F_ZP], zs = fc[F_ZS];
  const T izp = fc[F_IZP], izs = fc[F_IZS];
  const T kl = fc[F_KL], km = fc[F_KM];
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

}  // namespace sbp
