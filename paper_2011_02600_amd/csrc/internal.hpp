// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>

namespace sbp {

// Largest closure block (interior order 6: 6 rows x 10 columns).
constexpr int kMaxM = 6;
constexpr int kMaxCols = 10;
constexpr int kMaxSources = 4;
constexpr int kMaxSrcWidth = 8;   // 2 (p + 1) for p = 3
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

// Builds the closure for order 2, 4 or 6; returns false on failure (message
// in *err).
bool build_closure(int order, Closure* out, const char** err);

// Per-face penalty coefficients, in this order, for every face node:
// nx, ny, nz, Zp, Zs, 1/Zp, 1/Zs, kappa/rho, kappa*lambda, kappa*mu,
// kappa = |M_xi| / (J h_xi w_0).
enum FaceCoef { FN_X = 0, FN_Y, FN_Z, F_ZP, F_ZS, F_IZP, F_IZS, F_KR, F_KL, F_KM };

// Element layout of the device arrays of one handle (all counts in elements
// of the handle's dtype, relative to the start of the workspace).
struct Layout {
  int nq = 0, nr = 0, ns = 0;
  int px = 0;             // x pitch (elements), multiple of 16
  std::size_t plane = 0;  // px * nr
  std::size_t field = 0;  // plane * ns
  std::size_t q_a = 0, q_b = 0, dq = 0, coef = 0;  // 9, 9, 9, 12 fields
  std::size_t face[6] = {};   // kNumFaceCoef arrays of face size each
  std::size_t face_n[6] = {}; // nodes per face
  std::size_t face_na[6] = {};// fast extent of the face array
  std::size_t src = 0;        // kMaxSources * (kMaxSrcWidth^3 * 6) weights
  std::size_t part = 0;       // energy partial sums (double, bytes offset)
  std::size_t bounds = 0;     // int tile bounds (bytes offset)
  std::size_t total_bytes = 0;
};

}  // namespace sbp
