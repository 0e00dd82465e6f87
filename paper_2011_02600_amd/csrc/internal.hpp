// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>

namespace sbp {

// Largest closure block (interior order 8: 8 rows x 13 columns).
constexpr int kMaxM = 8;
constexpr int kMaxCols = 13;
constexpr int kMaxSources = 4;
constexpr int kMaxSrcWidth = 10;  // 2 (p + 1) for p = 4
constexpr int kNumFaceCoef = 10;  // per face node, see FaceCoef
constexpr int kNumCoef = 12;      // per node: M[3][3], lambda/J, mu/J, 1/(rho J)

// Closure data of one interior order (Sec. 4.1): the first m rows of h*D+ and
// h*D- (columns 0 .. m+q-1) and the norm weights w_0..w_{m-1}.  The right
// end follows from D+ = -flip(D-) and D- = -flip(D+).
struct Closure {
  int order = 0;
  int m = 0;        // closure rows
  int q = 0;        // forward reach of the interior D+ stencil
  int r = 0;        // backward reach of the interior D+ stencil
  int ncol = 0;     // m + q
  double w[kMaxM] = {};
  double dp[kMaxM][kMaxCols] = {};
  double dm[kMaxM][kMaxCols] = {};
  double alpha[10] = {};  // interior D+ stencil alpha_{-r..q} (Table tab:upwind)
};

// Builds the closure for orders 2 to 7; returns false on failure (message
// in *err).
bool build_closure(int order, Closure* out, const char** err);

// Per-face penalty coefficients, in this order, for every face node:
// nx, ny, nz, Zp, Zs, 1/Zp, 1/Zs, kappa/rho, kappa*lambda, kappa*mu,
// kappa = |M_xi| / (J h_xi w_0).
enum FaceCoef { FN_X = 0, FN_Y, FN_Z, F_ZP, F_ZS, F_IZP, F_IZS, F_KR, F_KL, F_KM };

// Position of node (i, j, k) in a field (element offset).  The first nq - 1
// columns of every (j, k) row lie in rows of pitch px (a multiple of the
// 128-byte line, so that rows and 64-point tiles start on lines); column
// nq - 1 of all rows is stored after them, compactly in (k, j) order, where
// its values fill whole lines instead of one value per line.
struct NodeMap {
  long long plane = 0;  // px * nr
  long long cbase = 0;  // offset of the last-column array: plane * ns
  int px = 0, nr = 0, nqm = 0;  // nqm = nq - 1
#if defined(__HIPCC__)
  __host__ __device__
#endif
  long long operator()(int i, int j, int k) const {
    return i < nqm ? (long long)k * plane + (long long)j * px + i : cbase + (long long)k * nr + j;
  }
};

}  // namespace sbp
