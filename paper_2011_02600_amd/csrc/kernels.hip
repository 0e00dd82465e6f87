// HIP kernels (gfx950) for one Runge-Kutta stage of the upwind-SBP elastic
// solver, plus source injection, receiver gather and the energy reduction.
//
// Stage kernel (fused; one launch per stage):
//   for every node: RHS = volume terms (D+ on the velocities in the
//   non-conservative term, D- on the conservative stress flux, metric and
//   material weights; eq. gen_hyp_transformed_discrete), then
//   dQ <- A_k dQ + dt RHS,  Q_out <- Q_in + B_k dQ.
// Penalty kernel (after the stage and edge kernels): at every node of the
//   block's surface, the boundary penalties of its faces (eq. SAT_General /
//   eq. SAT_free_surface) enter the same update, dQ += dt P, Q_out += B_k dt P
//   (the update is linear in the right-hand side).  Keeping them out of the
//   stage kernel's plane loop keeps that loop's registers for its own data.
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
#include "penalty.hpp"

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
struct Stencil<3> {
  static constexpr int R = 1, Q = 2, M = 3;
  static constexpr double a[4] = {-1.0 / 3, -1.0 / 2, 1.0, -1.0 / 6};
};
template <>
struct Stencil<4> {
  static constexpr int R = 1, Q = 3, M = 4;
  static constexpr double a[5] = {-1.0 / 4, -5.0 / 6, 3.0 / 2, -1.0 / 2, 1.0 / 12};
};
template <>
struct Stencil<5> {
  static constexpr int R = 2, Q = 3, M = 5;
  static constexpr double a[6] = {1.0 / 20, -1.0 / 2, -1.0 / 3, 1.0, -1.0 / 4, 1.0 / 30};
};
template <>
struct Stencil<6> {
  static constexpr int R = 2, Q = 4, M = 6;
  static constexpr double a[7] = {1.0 / 30, -2.0 / 5, -7.0 / 12, 4.0 / 3, -1.0 / 2, 2.0 / 15, -1.0 / 60};
};
template <>
struct Stencil<7> {
  static constexpr int R = 3, Q = 4, M = 7;
  static constexpr double a[8] = {-1.0 / 105, 1.0 / 10, -3.0 / 5, -1.0 / 4, 1.0, -3.0 / 10, 1.0 / 15, -1.0 / 140};
};
// (alpha_4 printed +1/28; -1/28 sums the coefficients to zero)
template <>
struct Stencil<8> {
  static constexpr int R = 3, Q = 5, M = 8;
  static constexpr double a[9] = {-1.0 / 168, 1.0 / 14, -1.0 / 2,  -9.0 / 20,  5.0 / 4,
                                  -1.0 / 2,   1.0 / 6,  -1.0 / 28, 1.0 / 280};
};

// ---------------------------------------------------------------------------
// element `off` of the field starting at the uniform address `base`: the byte
// offset is formed in 32 bits so that the load uses a scalar base address plus
// a 32-bit vector offset (fields are smaller than 4 GiB)
template <typename T>
__device__ __forceinline__ T ldf(const T* base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (unsigned)(off * sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void stf(T* base, unsigned off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (unsigned)(off * sizeof(T))) = v;
}

// Field array accessor: BUF = true uses a buffer resource (one descriptor per
// array, the field offset in a scalar register, the element offset as a
// 32-bit vector offset; the array must be smaller than 4 GiB); BUF = false
// uses plain pointers.  ldn / st mark the access non-temporal (cache policy
// bit NT): data that no other block reads during the launch (the Runge-Kutta
// register, the material, every store) then does not push the halo lines
// that neighbouring tiles are about to read out of L2.
template <typename T, bool BUF>
struct Arr;

template <typename T>
struct Arr<T, true> {
  __amdgpu_buffer_rsrc_t r;
  unsigned fbytes;
  __device__ Arr(const T* p, std::size_t field)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, -1, 0x00020000)),
        fbytes((unsigned)(field * sizeof(T))) {}
  static constexpr int kNT = 2;  // cache policy: non-temporal
  template <int POL = 0>
  __device__ __forceinline__ T ldp(int c, unsigned off) const {
    if constexpr (sizeof(T) == 4) {
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(off * 4u), (int)(c * fbytes), POL));
    } else {
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(off * 8u), (int)(c * fbytes), POL));
    }
  }
  __device__ __forceinline__ T ld(int c, unsigned off) const { return ldp<0>(c, off); }
  __device__ __forceinline__ T ldn(int c, unsigned off) const { return ldp<kNT>(c, off); }
  __device__ __forceinline__ void st(int c, unsigned off, T v) const {
    if constexpr (sizeof(T) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)(off * 4u), (int)(c * fbytes), kNT);
    } else {
      using u2 = unsigned __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)(off * 8u), (int)(c * fbytes), kNT);
    }
  }
};

template <typename T>
struct Arr<T, false> {
  T* p;
  std::size_t field;
  __device__ Arr(const T* p_, std::size_t f) : p(const_cast<T*>(p_)), field(f) {}
  __device__ __forceinline__ T ld(int c, unsigned off) const { return ldf(p + c * field, off); }
  __device__ __forceinline__ T ldn(int c, unsigned off) const { return ldf(p + c * field, off); }
  __device__ __forceinline__ void st(int c, unsigned off, T v) const { stf(p + c * field, off, v); }
};

// Flux e . sigma_i for the three components i, with e = (m0, m1, m2) a metric
// row: explicit fused multiply-adds in a fixed order, so that every site that
// forms the flux of a node (own point, halo point, s-queue) rounds identically
// and results do not depend on the tiling.
template <typename T>
__device__ __forceinline__ void flux3(T m0, T m1, T m2, T sxx, T syy, T szz, T sxy, T sxz, T syz, T f[3]) {
  f[0] = fma(m2, sxz, fma(m1, sxy, m0 * sxx));
  f[1] = fma(m2, syz, fma(m1, syy, m0 * sxy));
  f[2] = fma(m2, szz, fma(m1, syz, m0 * sxz));
}

// In double precision the scheduler's hoisting of every stencil load of a
// derivative (three components, value and flux) ahead of its arithmetic
// takes more registers than a thread has: a fence between components keeps
// one component's loads in flight at a time.
template <typename T>
__device__ __forceinline__ void sched_fence() {
  if constexpr (sizeof(T) == 8) __builtin_amdgcn_sched_barrier(0);
}

// ---------------------------------------------------------------------------
// pointwise part of the right-hand side at one node: stress rates from the
// velocity derivatives u[xi][i] = D+_xi v_i (non-conservative metric form
// and Hooke's law) and momentum rates from dv[i] = sum_xi D-_xi F_xi,i
template <typename T>
__device__ __forceinline__ void node_rates(const T u[3][3], const T dv[3], const T mq[3], const T mr[3],
                                           const T ms[3], T lamJ, T muJ, T rJ, T rate[9]) {
  T G[3][3];  // G[c][ii] = sum_xi M[xi][c] u[xi][ii]  (= J dv_ii/dx_c)
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) G[c][ii] = mq[c] * u[0][ii] + mr[c] * u[1][ii] + ms[c] * u[2][ii];
  const T div = G[0][0] + G[1][1] + G[2][2];
  rate[0] = rJ * dv[0];
  rate[1] = rJ * dv[1];
  rate[2] = rJ * dv[2];
  rate[3] = lamJ * div + T(2) * muJ * G[0][0];
  rate[4] = lamJ * div + T(2) * muJ * G[1][1];
  rate[5] = lamJ * div + T(2) * muJ * G[2][2];
  rate[6] = muJ * (G[1][0] + G[0][1]);
  rate[7] = muJ * (G[2][0] + G[0][2]);
  rate[8] = muJ * (G[2][1] + G[1][2]);
}

// ---------------------------------------------------------------------------
// the fused stage kernel
//
// Per plane a of the block's chunk:
//   phase 1  load plane a: own sigma and q/r metric rows (q/r fluxes), the
//            y-halo and x-halo points of the tile, the s-flux of the lead
//            plane a+1+R (into the LDS ring) and the lead velocity a+1+Q;
//            stage v, F_q, F_r in LDS
//   phase 2  derivatives (LDS along q and r, the v register queue and the
//            F_s LDS ring along s), rates, penalties, stage update, stores
// LDS: v window (64+2H) x (TY+2H), F_q window (64+2H) x TY, F_r window
// 64 x (TY+2H), and a per-thread ring of QD planes of F_s.
// All offsets inside one field are 32-bit; field bases are uniform.
#ifndef SBP_STAGE_MIN_WAVES
#define SBP_STAGE_MIN_WAVES 1  // minimum waves per SIMD the register allocation must allow
#endif
constexpr std::size_t kLdsBytes = 160 * 1024;

// LDS of stage_body<T, ORDER, TY> (element offsets of its arrays in one
// buffer): v window (64+2H) x (TY+2H), F_q window (64+2H) x TY, F_r window
// 64 x (TY+2H), the per-thread ring of QD planes of F_s; sigma (6) and M_s
// (3) of planes a .. a+R, read once from memory as the s-flux lead and kept
// until the plane is the output plane (when the budget allows it; otherwise
// plane a reloads them); the closure rows (D+, D- and their mirror images)
template <typename T, int ORDER, int TY>
struct StageLds {
  using S = Stencil<ORDER>;
  static constexpr int R = S::R, Q = S::Q, H = Q, NT = 64 * TY;
  static constexpr int QD = R + Q + 1, SD = R + 1;
  // q derivatives: every lane sums NC = M + Q taps (a closure row's width;
  // the interior stencil padded with zero weights), so the windows along q
  // hold NC - QD zero columns beyond the halo
  static constexpr int NC = S::M + S::Q, PADQ = NC - QD;
  static constexpr int VX = 64 + 2 * H + PADQ, VY = TY + 2 * H, QX = 64 + 2 * H + PADQ, RX = 64;
  static constexpr int TABN = kMaxM * kMaxCols;
  // rows of q weights: interior, left closure rows 0..M-1, right closure rows
  // 0..M-1 (columns nq-NC .. nq-1 ascending); D+ rows, then D- rows
  static constexpr int QROWS = 2 * S::M + 1;
  static constexpr std::size_t n_tq = 2 * QROWS * NC;
  static constexpr std::size_t n_lv = 3 * VX * VY, n_lq = 3 * QX * TY, n_lr = 3 * RX * VY;
  // s-flux ring: F_s of the QD planes a - Q .. a + R that D-_s at plane a
  // reads.  Where that ring leaves the LDS short (double precision, orders 7
  // and 8), the NL newest planes stay in registers and the ring keeps the
  // QD - NL older ones
  static constexpr std::size_t fixed = n_lv + n_lq + n_lr + kClosureTab * kMaxM * kMaxCols + n_tq + kNumFaceCoef * TY;
  static constexpr int NL = (sizeof(T) != 8 || TY != 8) ? 0
                            : sizeof(T) * (fixed + (std::size_t)QD * 3 * NT) <= kLdsBytes ? 0
                            : sizeof(T) * (fixed + (std::size_t)(QD - 1) * 3 * NT) <= kLdsBytes ? 1
                            : sizeof(T) * (fixed + (std::size_t)(QD - 2) * 3 * NT) <= kLdsBytes ? 2
                                                                                           : 3;
  static constexpr int NR = QD - NL;
  static constexpr std::size_t n_ring = (std::size_t)NR * 3 * NT;
  static constexpr std::size_t base_bytes = sizeof(T) * (n_lv + n_lq + n_lr + n_ring);
  static constexpr bool SR = base_bytes + sizeof(T) * SD * 9 * NT <= kLdsBytes;
  static constexpr std::size_t n_sring = SR ? SD * 9 * NT : 1;
  static constexpr std::size_t n_tab = kClosureTab * TABN;
  static constexpr std::size_t o_lv = 0, o_lq = o_lv + n_lv, o_lr = o_lq + n_lq, o_ring = o_lr + n_lr,
                               o_sring = o_ring + n_ring, o_tab = o_sring + n_sring, o_tq = o_tab + n_tab,
                               o_fq = o_tq + n_tq, total = o_fq + kNumFaceCoef * TY;
  static constexpr std::size_t bytes = total * sizeof(T);
};

// whether stage_body<T, ORDER, TY> is built: its LDS fits
template <typename T, int ORDER, int TY>
constexpr bool stage_built() {
  return StageLds<T, ORDER, TY>::bytes <= kLdsBytes;
}

// EQ: the copies for the edge kernel (StageArgs::eqc) are built in (the
// single-grid kernel; batched launches gather instead)
// the point-source increments dt g(t) w M of node (i, j, k) (stress
// components), summed over the sources whose stencil holds it
template <typename T>
__device__ __forceinline__ void source_add(const StageArgs<T>& A, int i, int j, int k, T add[6]) {
  const int w = A.src_w;
  for (int s = 0; s < A.nsrc; ++s) {
    const int dk = k - A.src_k0[s], dj = j - A.src_j0[s], di = i - A.src_i0[s];
    if ((unsigned)dk < (unsigned)w && (unsigned)dj < (unsigned)w && (unsigned)di < (unsigned)w) {
      const T gdt = A.src_clock
                        ? static_cast<const T*>(A.src_clock->gtab)[((std::size_t)A.src_clock->step * 5 + A.src_stage) *
                                                                       kMaxSources + s]
                        : A.src_gdt[s];
      const T* wm =
          A.src_wm + ((std::size_t)s * kMaxSrcWidth * kMaxSrcWidth * kMaxSrcWidth + (dk * w + dj) * w + di) * 6;
#pragma unroll
      for (int f = 0; f < 6; ++f) add[f] += gdt * wm[f];
    }
  }
}

template <typename T, int ORDER, int TY, bool BUF, bool EQ = false>
__device__ __forceinline__ void stage_body(const StageArgs<T>& A, const int tile, char* lds) {
  using S = Stencil<ORDER>;
  using L = StageLds<T, ORDER, TY>;
  constexpr int R = S::R, Q = S::Q, M = S::M;
  constexpr int H = Q;            // halo width (Q >= R)
  constexpr int NT = 64 * TY;     // threads
  constexpr int VX = L::VX, VY = L::VY;  // v window
  constexpr int QX = L::QX;              // F_q window (TY rows)
  constexpr int RX = L::RX;              // F_r window (VY rows)
  constexpr int QD = L::QD;       // s queue depth
  constexpr int NYH = 2 * H * 64; // y-halo points
  constexpr int NXH = 2 * H * TY; // x-halo points
  constexpr int TABN = L::TABN;
  // one y-halo point per thread; halo rows beyond the first NT / 64 (order
  // 8: 10 rows for 8-row tiles) are upper rows past the flux's reach r,
  // which need v only and take a second point in the first threads
  constexpr int NYH2 = NYH > NT ? NYH - NT : 0;
  static_assert(NYH2 <= NT && (NYH2 == 0 || NT / 64 >= H + R), "y halo");
  static_assert(TY >= M, "r closure rows must fit in one tile");
  static_assert(L::bytes <= kLdsBytes, "stage tile exceeds the LDS");
  T* const lv = reinterpret_cast<T*>(lds) + L::o_lv;
  T* const lq = reinterpret_cast<T*>(lds) + L::o_lq;
  T* const lr = reinterpret_cast<T*>(lds) + L::o_lr;
  T* const ring = reinterpret_cast<T*>(lds) + L::o_ring;
  constexpr int SD = L::SD;
  constexpr bool SR = L::SR;
  T* const sring = reinterpret_cast<T*>(lds) + L::o_sring;
  T* const ltab = reinterpret_cast<T*>(lds) + L::o_tab;
  T* const tq = reinterpret_cast<T*>(lds) + L::o_tq;
  constexpr int NC = L::NC, QROWS = L::QROWS;

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
  const int nq = A.nq, nr = A.nr, ns = A.ns;
  const bool act = (i < x1) && (j < y1);    // node computed by this block
  const bool ing = (i < x1) && (j < nr);    // node staged in LDS (own or halo of the tile)
  const unsigned px = A.px, plane = A.plane;
  const std::size_t field = A.field;
  const unsigned col = (unsigned)j * px + (unsigned)i;

  const Arr<T, BUF> gq(A.qin, field), gc(A.coef, field), gd(A.dq, field), go(A.qout, field);
  for (int e = threadIdx.y * 64 + threadIdx.x; e < kClosureTab * TABN; e += NT) ltab[e] = A.tab[e];
  // q = 0 face coefficients of the plane, one row of kNumFaceCoef per wave
  T* const lfq = reinterpret_cast<T*>(lds) + L::o_fq;
  // the q weight rows (from the closure table in memory, the right-end rows
  // reversed so that every row runs over ascending columns; D- interior
  // weights with the sign of the difference folded in) and zeroed q windows
  for (int e = threadIdx.y * 64 + threadIdx.x; e < 2 * QROWS * NC; e += NT) {
    const int pm = e / (QROWS * NC), rem = e - pm * QROWS * NC, row = rem / NC, t = rem - row * NC;
    T w = T(0);
    if (row == 0) {
      if (t < QD) w = pm == 0 ? T(S::a[t]) : -T(S::a[R + Q - t]);
    } else if (row <= M) {
      w = A.tab[pm * TABN + (row - 1) * kMaxCols + t];
    } else {
      w = A.tab[(2 + pm) * TABN + (row - 1 - M) * kMaxCols + (NC - 1 - t)];
    }
    tq[e] = w;
  }
  // Window positions that no load fills are read with zero weights (the
  // padded q taps; closure rows along r that end before the row range does,
  // as order 8's flux rows beyond r above the first tile): they must hold
  // finite values, whatever an earlier kernel left in this LDS
  for (int e = threadIdx.y * 64 + threadIdx.x; e < 3 * VX * VY; e += NT) lv[e] = T(0);
  for (int e = threadIdx.y * 64 + threadIdx.x; e < 3 * QX * TY; e += NT) lq[e] = T(0);
  for (int e = threadIdx.y * 64 + threadIdx.x; e < 3 * RX * VY; e += NT) lr[e] = T(0);

  // y halo: rows y0-H..y0-1 and y0+TY..y0+TY+H-1, columns x0..x1-1
  const int yh_r = tid >> 6;
  const int yh_gy = (yh_r < H) ? (y0 - H + yh_r) : (y0 + TY + yh_r - H);
  const int yh_gx = x0 + (tid & 63);
  const bool yh_in = tid < NYH && yh_gx < x1 && yh_gy >= 0 && yh_gy < nr;
  const int yh_ly = (yh_r < H) ? yh_r : TY + yh_r;   // row in the v / F_r windows
  const unsigned yh_col = yh_in ? (unsigned)yh_gy * px + (unsigned)yh_gx : 0u;
  // D+ reads v at R rows below and Q rows above a node, D- reads the flux at
  // Q below and R above: only those halo rows are loaded.  The last tile
  // along r (also when an edge row follows it) keeps every lower v row,
  // which its boundary closure rows read.
  const bool yh_v = yh_in && (yh_r >= H - R || y1 >= nr - 1);
  // (with an edge row after the last tile, the boundary closure rows of that
  // tile also read the flux of the edge row, which may lie beyond R)
  const bool yh_f = yh_in && (yh_r < H + R || y1 == nr - 1);
  // the second point: halo row NT / 64 + (tid >> 6), an upper row
  const int yh2_r = NT / 64 + (tid >> 6);
  const int yh2_gy = y0 + TY + yh2_r - H;
  const bool yh2_v = NYH2 > 0 && tid < NYH2 && yh_gx < x1 && yh2_gy < nr;
  const int yh2_ly = TY + yh2_r;
  const unsigned yh2_col = yh2_v ? (unsigned)yh2_gy * px + (unsigned)yh_gx : 0u;
  // x halo: columns x0-H..x0-1 and x1..x1+H-1, rows y0..y0+TY-1.  Column
  // nq-1 (the right halo of the last tile) is read from the last-column
  // array of the fields.
  const int xh_c = tid / TY;
  const int xh_r = tid - xh_c * TY;
  const int xh_gx = (xh_c < H) ? (x0 - H + xh_c) : (x1 + xh_c - H);
  const int xh_gy = y0 + xh_r;
  const bool xh_in = tid < NXH && xh_gx >= 0 && xh_gx < nq && xh_gy < nr;
  const int xh_lx = (xh_c < H) ? xh_c : (x1 - x0) + xh_c;  // column in the v / F_q windows
  const bool xh_edge = xh_in && xh_gx == A.nm.nqm;
  const unsigned xh_col = (xh_in && !xh_edge) ? (unsigned)xh_gy * px + (unsigned)xh_gx : 0u;
  // waves holding x-halo lanes (a wave-uniform condition)
  const bool xh_wave = __builtin_amdgcn_readfirstlane(ty) * 64 < NXH;

  // s-flux F_s,i = sum_c M[s][c] sigma_ic
  auto sflux = [&](unsigned o, T f[3]) {
    const T m0 = gc.ld(6, o), m1 = gc.ld(7, o), m2 = gc.ld(8, o);
    const T sxx = gq.ld(3, o), syy = gq.ld(4, o), szz = gq.ld(5, o);
    const T sxy = gq.ld(6, o), sxz = gq.ld(7, o), syz = gq.ld(8, o);
    flux3(m0, m1, m2, sxx, syy, szz, sxy, sxz, syz, f);
  };
  // ring slot of plane k (k >= -Q)
  constexpr int NR = L::NR, NL = L::NL;
  auto slot = [&](int k) { return (k + 7 * NR) % NR; };

  __syncthreads();  // closure and weight rows written, windows zeroed

  // s closure rows.  The terms h D+_s v and h D-_s F_s of a closure plane
  // gather its row's NC planes; gathered plane by plane, the M closure planes
  // would read those planes M times.  The block forms the terms of all
  // closure rows of its planes here, in one pass over the NC planes, keeps
  // them in the workspace (A.scl) and reads them back at the plane.
  {
    const unsigned cl = act ? col : 0u;
    constexpr int PU = sizeof(T) == 4 ? NC : 5;
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
      // planes with a closure row on this side (left rows take precedence)
      const int lo = side == 0 ? z0 : max(z0, max(ns - M, M));
      const int hi = side == 0 ? min(z1, M) : z1;
      if (lo >= hi) continue;
      const int zt = side == 0 ? 0 : 2 * TABN;
      // pass 0: h D+_s v from v; pass 1: h D-_s F_s from sigma and M_s
#pragma unroll 1
      for (int pass = 0; pass < 2; ++pass) {
        T acc[M][3];
#pragma unroll
        for (int r = 0; r < M; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r][c] = T(0);
#pragma unroll PU
        for (int cc = 0; cc < NC; ++cc) {
          const int k = side == 0 ? cc : ns - 1 - cc;
          const unsigned ok = (unsigned)k * plane + cl;
          T x[3];
          if (pass == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) x[c] = gq.ld(c, ok);
          } else {
            sflux(ok, x);
          }
#pragma unroll
          for (int r = 0; r < M; ++r) {
            const T w = ltab[zt + pass * TABN + r * kMaxCols + cc];
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][c] += w * x[c];
          }
        }
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const int ar = side == 0 ? r : ns - 1 - r;
          if (act && ar >= lo && ar < hi) {
            T* dst = A.scl + (std::size_t)((side * kMaxM + r) * 6 + 3 * pass) * plane + col;
#pragma unroll
            for (int c = 0; c < 3; ++c) dst[(std::size_t)c * plane] = acc[r][c];
          }
        }
      }
    }
  }

  // register queue vq[s] = v(a - R + s); ring holds F_s(a - Q .. a + R)
  // (with NL lead planes in registers: a - Q .. a + R - NL, and flead[k]
  // = F_s(a + R - NL + 1 + k))
  T vq[3][QD];
  T flead[NL > 0 ? NL : 1][3] = {};
#pragma unroll
  for (int s = 0; s < QD; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) vq[c][s] = T(0);
  if (ing) {
#pragma unroll
    for (int s = 0; s < QD; ++s) {
      const int kv = z0 - R + s;
      if (kv >= 0 && kv < ns) {
        const unsigned o = (unsigned)kv * plane + col;
#pragma unroll
        for (int c = 0; c < 3; ++c) vq[c][s] = gq.ld(c, o);
      }
    }
    for (int s = 0; s < QD; ++s) {
      const int kf = z0 - Q + s;
      T f[3] = {T(0), T(0), T(0)};
      if (kf >= 0 && kf < ns) {
        const unsigned o = (unsigned)kf * plane + col;
        T r[9];
#pragma unroll
        for (int c = 0; c < 6; ++c) r[c] = gq.ld(3 + c, o);
#pragma unroll
        for (int c = 0; c < 3; ++c) r[6 + c] = gc.ld(6 + c, o);
        flux3(r[6], r[7], r[8], r[0], r[1], r[2], r[3], r[4], r[5], f);
        if (SR && kf >= z0) {
#pragma unroll
          for (int c = 0; c < 9; ++c) sring[((kf % SD) * 9 + c) * NT + tid] = r[c];
        }
      }
      if (NL > 0 && s >= QD - NL) {
#pragma unroll
        for (int c = 0; c < 3; ++c) flead[NL > 0 ? s - (QD - NL) : 0][c] = f[c];
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) ring[(slot(kf) * 3 + c) * NT + tid] = f[c];
      }
    }
  }

  const int vme = (ty + H) * VX + tx + H;   // own position in the v window
  const int qme = ty * QX + tx + H;         // ... F_q window
  // q weight row of the lane and the window columns its taps start at
  const int qrow = (i < M) ? 1 + i : (i >= nq - M ? 1 + M + (nq - 1 - i) : 0);
  const int qv0 = (ty + H) * VX + (qrow == 0 ? tx + H - R : (i < M ? H - x0 : H - x0 + nq - NC));
  const int qf0 = ty * QX + (qrow == 0 ? tx + H - Q : (i < M ? H - x0 : H - x0 + nq - NC));
  // FP32 keeps the lane's weights in registers; FP64 reads them from LDS
  constexpr bool QWREG = sizeof(T) == 4;
  T wqp[QWREG ? NC : 1], wqm[QWREG ? NC : 1];
  if constexpr (QWREG) {
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      wqp[t] = tq[qrow * NC + t];
      wqm[t] = tq[(QROWS + qrow) * NC + t];
    }
  }
  const int rme = (ty + H) * RX + tx;       // ... F_r window
  const T ihq = A.inv_h[0], ihr = A.inv_h[1], ihs = A.inv_h[2];
  const bool yin = j >= M && j < nr - M;
  const int yrow = (j < M) ? j : nr - 1 - j;
  const int ytab = (j < M) ? 0 : 2 * TABN;
  // closure rows along r (LDS reads): unrolled in single precision; in
  // double precision the registers are not there.  The s closure rows
  // (memory gathers over NC planes) take one column at a time: issuing
  // every column's loads together measured slower.
  constexpr int RU = sizeof(T) == 4 ? NC : 1;
  // the q = 0 face penalty in this kernel (single precision): blocks of the
  // first tile column, lane 0 of each row
  constexpr bool Q0S = q0_in_stage<T>();
  const bool q0pen = Q0S && A.sat != 0 && x0 == 0;
  // single precision: lanes of the columns nq-NC .. nq-2 copy v and F_q of
  // their node from LDS to A.eqc for the edge kernel's last-column q closure
  // rows (after the plane's loads are issued, like the deferred stores), so
  // that the edge kernel does not gather those columns, a line per row and
  // field (in double precision that gather costs the edge kernel about as
  // much as the copies cost this kernel)
  constexpr bool EQC = EQ && sizeof(T) == 4;
  const bool eql = EQC && A.eqc != nullptr && act && i >= nq - NC;

  // prefetch registers: everything plane a needs from memory (own sigma, M,
  // material, Runge-Kutta register; the y-halo and x-halo points of the
  // thread), loaded one plane ahead so that the loads of plane a+1 overlap
  // the arithmetic of plane a
  constexpr int NSG = SR ? 1 : 6, NMS = SR ? 6 : 9;
  T p_sg[NSG], p_m[NMS], p_mat[3], p_dq[9], p_hy[12], p_hx[12], p_hy2[NYH2 > 0 ? 3 : 1];
  const bool rdq = A.read_dq != 0;
  // the halo points of a plane are loaded with the plane's other data one
  // plane ahead; in double precision their registers do not fit beside the
  // rest, and each plane loads its halo points when it starts
  constexpr bool HALO_AHEAD = sizeof(T) == 4;
  // the material and the Runge-Kutta register are needed only by the stage
  // update at the end of the plane: in double precision they are loaded when
  // the plane starts (their latency hidden by the derivatives), not a plane
  // ahead, which would keep two planes' copies live through the derivatives
  constexpr bool LATE_AHEAD = sizeof(T) == 4;
  auto load_halo = [&](int a) {
    const unsigned pa = (unsigned)a * plane;
    const unsigned ohv = pa + (yh_v ? yh_col : 0u);
    const unsigned ohf = pa + (yh_f ? yh_col : 0u);
#pragma unroll
    for (int c = 0; c < 3; ++c) p_hy[c] = gq.ld(c, ohv);
#pragma unroll
    for (int c = 3; c < 9; ++c) p_hy[c] = gq.ld(c, ohf);
#pragma unroll
    for (int c = 0; c < 3; ++c) p_hy[9 + c] = gc.ld(3 + c, ohf);
    if constexpr (NYH2 > 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) p_hy2[c] = gq.ld(c, pa + yh2_col);
    }
    if (xh_wave) {
      const unsigned ox = xh_edge ? (unsigned)(A.nm.cbase + (long long)a * nr + xh_gy) : pa + xh_col;
#pragma unroll
      for (int c = 0; c < 9; ++c) p_hx[c] = gq.ld(c, ox);
#pragma unroll
      for (int c = 0; c < 3; ++c) p_hx[9 + c] = gc.ld(c, ox);
    }
  };
  auto load_late = [&](int a) {
    const unsigned pa = (unsigned)a * plane;
    const unsigned oa = pa + (act ? col : 0u);
#pragma unroll
    for (int c = 0; c < 3; ++c) p_mat[c] = gc.ldn(9 + c, oa);
    const unsigned od = rdq ? oa : 0u;   // unused (and masked below) in the first stage
#pragma unroll
    for (int c = 0; c < 9; ++c) p_dq[c] = gd.ldn(c, od);
  };
  auto load_plane = [&](int a) {
    const unsigned pa = (unsigned)a * plane;
    // Every lane loads; a lane that needs no value reads element 0 of the
    // plane (or of the array).  Loads under a mask or a branch would make the
    // compiler merge old and new register values, and the merge waits for
    // the loads in flight.
    const unsigned oi = pa + (ing ? col : 0u);
    const unsigned oa = pa + (act ? col : 0u);
    if constexpr (!SR) {
#pragma unroll
      for (int c = 0; c < 6; ++c) p_sg[c] = gq.ld(3 + c, oi);
#pragma unroll
      for (int c = 6; c < 9; ++c) p_m[c] = gc.ld(c, oa);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) p_m[c] = gc.ld(c, oi);
    if constexpr (LATE_AHEAD) load_late(a);
    if constexpr (HALO_AHEAD) load_halo(a);
  };
#pragma unroll
  for (int c = 0; c < NSG; ++c) p_sg[c] = T(0);
#pragma unroll
  for (int c = 0; c < NMS; ++c) p_m[c] = T(0);
#pragma unroll
  for (int c = 0; c < 9; ++c) p_dq[c] = T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) p_mat[c] = T(0);
  // with lead planes of the s-flux ring in registers (double precision,
  // order 8) the plane's own values are loaded when it starts, not a plane
  // ahead
  constexpr bool PF = NL < 2;
  if constexpr (PF) load_plane(z0);

  // results of the previous plane, stored after the next plane's loads have
  // been issued: loads and stores share one counter, and a wait for a load
  // while stores are in flight waits for the stores as well, so stores issued
  // at the end of a plane would put one write round trip on every plane.  In
  // double precision the 18 held values do not fit the register budget
  // beside the prefetch: there each plane stores its results at once.
  constexpr bool DEFER = sizeof(T) == 4;
  T st_d[DEFER ? 9 : 1], st_q[DEFER ? 9 : 1];
  unsigned st_o = 0;
  bool st_pend = false;
  auto flush_stores = [&]() {
    if (DEFER && st_pend && act) {
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        gd.st(c, st_o, st_d[c]);
        go.st(c, st_o, st_q[c]);
      }
    }
  };

  for (int a = z0; a < z1; ++a) {
    const unsigned pa = (unsigned)a * plane;
    const unsigned o = pa + col;
    if constexpr (!PF) load_plane(a);
    if constexpr (!HALO_AHEAD) load_halo(a);
    if constexpr (!LATE_AHEAD && PF) load_late(a);
    // s closure terms of a closure plane: loaded when the plane starts in
    // single precision, where they are used in double precision
    constexpr bool SCL_EARLY = sizeof(T) == 4;
    const bool sclose = !(a >= M && a < ns - M);
    auto scl_at = [&](unsigned c) -> const T* {
      const int side = a < M ? 0 : 1, r = side == 0 ? a : ns - 1 - a;
      return A.scl + (std::size_t)((side * kMaxM + r) * 6 + c) * plane;
    };
    T pscl[SCL_EARLY ? 6 : 1];
    if constexpr (SCL_EARLY) {
      if (sclose) {
        const unsigned cl = act ? col : 0u;
#pragma unroll
        for (int c = 0; c < 6; ++c) pscl[c] = scl_at(c)[cl];
      }
    }
    // coefficients of the q = 0 face at the wave's row, loaded when the plane
    // starts, one per lane (lane kk: coefficient kk), and passed through LDS
    // to lane 0, which adds the penalty before the stage update
    T fq_lane = T(0);
    if constexpr (Q0S) {
      if (q0pen) {
        const std::size_t fo = A.face_off[0] + (std::size_t)a * nr + (std::size_t)min(j, nr - 1);
        fq_lane = A.face[fo + (std::size_t)min(tx, kNumFaceCoef - 1) * A.face_n[0]];
      }
    }
    // ---------------- phase 1: stage plane a in LDS from the prefetched registers
    T sg[6], mq[3], mr[3], ms[3], dqo[9];
    if constexpr (SR) {
      const int sl = a % SD;
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] = sring[(sl * 9 + c) * NT + tid];
#pragma unroll
      for (int c = 0; c < 3; ++c) ms[c] = sring[(sl * 9 + 6 + c) * NT + tid];
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] = p_sg[c];
#pragma unroll
      for (int c = 0; c < 3; ++c) ms[c] = p_m[6 + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) { mq[c] = p_m[c]; mr[c] = p_m[3 + c]; }
    T lamJ = T(0), muJ = T(0), rJ = T(0);
    if constexpr (LATE_AHEAD) {  // copies before the prefetch of plane a + 1
#pragma unroll
      for (int c = 0; c < 9; ++c) dqo[c] = rdq ? p_dq[c] : T(0);
      lamJ = p_mat[0];
      muJ = p_mat[1];
      rJ = p_mat[2];
    }
    if (ing) {
      lv[0 * VX * VY + vme] = vq[0][R];
      lv[1 * VX * VY + vme] = vq[1][R];
      lv[2 * VX * VY + vme] = vq[2][R];
      T f[3];
      flux3(mq[0], mq[1], mq[2], sg[0], sg[1], sg[2], sg[3], sg[4], sg[5], f);
      lq[0 * QX * TY + qme] = f[0];
      lq[1 * QX * TY + qme] = f[1];
      lq[2 * QX * TY + qme] = f[2];
      flux3(mr[0], mr[1], mr[2], sg[0], sg[1], sg[2], sg[3], sg[4], sg[5], f);
      lr[0 * RX * VY + rme] = f[0];
      lr[1 * RX * VY + rme] = f[1];
      lr[2 * RX * VY + rme] = f[2];
    }
    if (yh_v) {  // v of the y-halo point
      const T* h = p_hy;
      const int wv = yh_ly * VX + (tid & 63) + H;
      lv[0 * VX * VY + wv] = h[0];
      lv[1 * VX * VY + wv] = h[1];
      lv[2 * VX * VY + wv] = h[2];
    }
    if constexpr (NYH2 > 0) {
      if (yh2_v) {  // v of the second y-halo point
        const int wv = yh2_ly * VX + (tid & 63) + H;
        lv[0 * VX * VY + wv] = p_hy2[0];
        lv[1 * VX * VY + wv] = p_hy2[1];
        lv[2 * VX * VY + wv] = p_hy2[2];
      }
    }
    if (yh_f) {  // r-flux of the y-halo point
      const T* h = p_hy;
      const int wr = yh_ly * RX + (tid & 63);
      T f[3];
      flux3(h[9], h[10], h[11], h[3], h[4], h[5], h[6], h[7], h[8], f);
      lr[0 * RX * VY + wr] = f[0];
      lr[1 * RX * VY + wr] = f[1];
      lr[2 * RX * VY + wr] = f[2];
    }
    if constexpr (Q0S) {
      if (q0pen && tx < kNumFaceCoef) lfq[ty * kNumFaceCoef + tx] = fq_lane;
    }
    if (xh_in) {  // v and q-flux of the x-halo point
      const T* h = p_hx;
      const int wv = (xh_r + H) * VX + xh_lx;
      const int wq = xh_r * QX + xh_lx;
      lv[0 * VX * VY + wv] = h[0];
      lv[1 * VX * VY + wv] = h[1];
      lv[2 * VX * VY + wv] = h[2];
      T f[3];
      flux3(h[9], h[10], h[11], h[3], h[4], h[5], h[6], h[7], h[8], f);
      lq[0 * QX * TY + wq] = f[0];
      lq[1 * QX * TY + wq] = f[1];
      lq[2 * QX * TY + wq] = f[2];
    }
    __syncthreads();

    // s-queue lead planes, then the prefetch of plane a+1.  The lead values
    // stay raw until the end of the plane: forming the flux here would make
    // the compiler wait for every load issued so far (vmcnt retires in order).
    // Plane indices are clamped so that the loads need no branch; clamped
    // values belong to planes >= ns, which no interior plane reads.
    T lead_v[3], lead_raw[9];
    // (without prefetch the same loads are issued at the end of the plane,
    // so that their values do not hold registers through the derivatives)
    auto load_lead = [&]() {
      const unsigned cl = ing ? col : 0u;
      const unsigned ov = (unsigned)min(a + 1 + Q, ns - 1) * plane + cl;
      const unsigned of = (unsigned)min(a + 1 + R, ns - 1) * plane + cl;
#pragma unroll
      for (int c = 0; c < 3; ++c) lead_v[c] = gq.ld(c, ov);
#pragma unroll
      for (int c = 0; c < 6; ++c) lead_raw[c] = gq.ld(3 + c, of);
#pragma unroll
      for (int c = 0; c < 3; ++c) lead_raw[6 + c] = gc.ld(6 + c, of);
    };
    if constexpr (PF) {
      const unsigned cl = ing ? col : 0u;
      const unsigned ov = (unsigned)min(a + 1 + Q, ns - 1) * plane + cl;
      const unsigned of = (unsigned)min(a + 1 + R, ns - 1) * plane + cl;
#pragma unroll
      for (int c = 0; c < 3; ++c) lead_v[c] = gq.ld(c, ov);
#pragma unroll
      for (int c = 0; c < 6; ++c) lead_raw[c] = gq.ld(3 + c, of);
#pragma unroll
      for (int c = 0; c < 3; ++c) lead_raw[6 + c] = gc.ld(6 + c, of);
    }
    if constexpr (PF) load_plane(min(a + 1, ns - 1));   // the last plane's prefetch is unused
    flush_stores();                   // after every load of the plane
    if constexpr (EQC) {
      if (eql) {  // the last column's q closure inputs, from LDS
        T* const e = A.eqc + 8 * (((std::size_t)a * nr + j) * (NC - 1) + (std::size_t)(i - (nq - NC)));
        const float4 w0 = make_float4(lv[vme], lv[VX * VY + vme], lv[2 * VX * VY + vme], lq[qme]);
        const float2 w1 = make_float2(lq[QX * TY + qme], lq[2 * QX * TY + qme]);
        *reinterpret_cast<float4*>(e) = w0;
        *reinterpret_cast<float2*>(e + 4) = w1;
      }
    }

    // ---------------- phase 2
    if (act) {
      T u[3][3];   // u[xi][c] = D+_xi v_c
      T dv[3];     // sum_xi D-_xi F_xi,c
      // q direction: the same NC taps for interior and closure lanes (no
      // divergence within a wave); zero weights on the padding taps
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T sp = T(0), sm = T(0);
#pragma unroll
        for (int t = 0; t < NC; ++t) {
          const T cp = QWREG ? wqp[QWREG ? t : 0] : tq[qrow * NC + t];
          const T cm = QWREG ? wqm[QWREG ? t : 0] : tq[(QROWS + qrow) * NC + t];
          sp += cp * lv[c * VX * VY + qv0 + t];
          sm += cm * lq[c * QX * TY + qf0 + t];
        }
        u[0][c] = sp * ihq;
        dv[c] = sm * ihq;
        sched_fence<T>();
      }
      // r direction
      if (__builtin_expect(yin, 1)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sp = T(0), sm = T(0);
#pragma unroll
          for (int s = 0; s < QD; ++s) {
            sp += T(S::a[s]) * lv[c * VX * VY + vme + (s - R) * VX];
            sm += T(S::a[s]) * lr[c * RX * VY + rme + (R - s) * RX];
          }
          u[1][c] = sp * ihr;
          dv[c] -= sm * ihr;
          sched_fence<T>();
        }
      } else {
        T sp[3] = {T(0), T(0), T(0)}, sm[3] = {T(0), T(0), T(0)};
        const bool left = j < M;
        const int rowv = H - y0 + (left ? 0 : nr - 1);
        const int stepr = left ? 1 : -1;
#pragma unroll RU
        for (int cc = 0; cc < NC; ++cc) {
          const T cp = ltab[ytab + yrow * kMaxCols + cc];
          const T cm = ltab[ytab + TABN + yrow * kMaxCols + cc];
          const int rw = rowv + stepr * cc;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            sp[c] += cp * lv[c * VX * VY + rw * VX + tx + H];
            sm[c] += cm * lr[c * RX * VY + rw * RX + tx];
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          u[1][c] = sp[c] * ihr;
          dv[c] += sm[c] * ihr;
        }
      }
      // s direction
      if (__builtin_expect(!sclose, 1)) {
        const int s0 = slot(a - Q);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sp = T(0), sm = T(0);
#pragma unroll
          for (int s = 0; s < QD; ++s) {
            sp += T(S::a[s]) * vq[c][s];
            if constexpr (NL > 0) {
              if (s < NL) {
                sm += T(S::a[s]) * flead[NL > 0 ? NL - 1 - s : 0][c];
              } else {
                int t = s0 + R + Q - s;
                t = t >= NR ? t - NR : t;
                sm += T(S::a[s]) * ring[(t * 3 + c) * NT + tid];
              }
            } else {
              int t = s0 + R + Q - s;
              t = t >= QD ? t - QD : t;
              sm += T(S::a[s]) * ring[(t * 3 + c) * NT + tid];
            }
          }
          u[2][c] = sp * ihs;
          dv[c] -= sm * ihs;
          sched_fence<T>();
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          u[2][c] = (SCL_EARLY ? pscl[SCL_EARLY ? c : 0] : scl_at(c)[col]) * ihs;
          dv[c] += (SCL_EARLY ? pscl[SCL_EARLY ? 3 + c : 0] : scl_at(3 + c)[col]) * ihs;
        }
      }

      if constexpr (!PF) load_late(a);   // without prefetch: loaded where used
      if constexpr (!LATE_AHEAD) {
#pragma unroll
        for (int c = 0; c < 9; ++c) dqo[c] = rdq ? p_dq[c] : T(0);
        lamJ = p_mat[0];
        muJ = p_mat[1];
        rJ = p_mat[2];
      }
      T rate[9];
      node_rates(u, dv, mq, mr, ms, lamJ, muJ, rJ, rate);

      const T v[3] = {vq[0][R], vq[1][R], vq[2][R]};

      // the penalty of the q = 0 face at its nodes (single precision); the
      // other boundary penalties are added by penalty_kernel after the launch
      if constexpr (Q0S) {
        if (q0pen && tx == 0) {
          T fcq[kNumFaceCoef];
#pragma unroll
          for (int kk = 0; kk < kNumFaceCoef; ++kk) fcq[kk] = lfq[ty * kNumFaceCoef + kk];
          face_penalty(fcq, A.gamma[0], T(-1), A.traction[0] != 0, v, sg, rate);
        }
      }

      // point sources whose stencil holds the node (single precision, one grid)
      T sadd[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
      if constexpr (EQC) {
        if (A.nsrc > 0) source_add(A, i, j, a, sadd);
      }

      // Runge-Kutta stage update
      const T dt = A.dt, Ak = A.Ak, Bk = A.Bk;
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        T d = dt * rate[c] + Ak * dqo[c];
        if constexpr (EQC) {
          if (c >= 3) d += sadd[c - 3];
        }
        const T q0 = (c < 3) ? v[c] : sg[c - 3];
        if constexpr (DEFER) {
          st_d[c] = d;
          st_q[c] = q0 + Bk * d;
        } else {
          gd.st(c, o, d);
          go.st(c, o, q0 + Bk * d);
        }
      }
      st_o = o;
    }
    st_pend = true;
    __syncthreads();
    if constexpr (!PF) load_lead();

    // advance the s queues to plane a + 1 (the ring slot of plane a - Q
    // becomes that of plane a + 1 + R; each thread touches only its own slots)
#pragma unroll
    for (int s = 0; s < QD - 1; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) vq[c][s] = vq[c][s + 1];
#pragma unroll
    for (int c = 0; c < 3; ++c) vq[c][QD - 1] = lead_v[c];
    {
      const T* r = lead_raw;  // sigma (6), M_s (3) of plane a + 1 + R
      T f[3];
      flux3(r[6], r[7], r[8], r[0], r[1], r[2], r[3], r[4], r[5], f);
      if constexpr (NL > 0) {  // the oldest lead plane joins the ring in the slot of plane a - Q
        const int sl = slot(a + R - NL + 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ring[(sl * 3 + c) * NT + tid] = flead[0][c];
#pragma unroll
          for (int k = 0; k + 1 < NL; ++k) flead[k][c] = flead[k + 1][c];
          flead[NL > 0 ? NL - 1 : 0][c] = f[c];
        }
      } else {
        const int sl = slot(a + 1 + R);
#pragma unroll
        for (int c = 0; c < 3; ++c) ring[(sl * 3 + c) * NT + tid] = f[c];
      }
      if constexpr (SR) {  // plane a's slot is free now: it takes plane a + 1 + R
        const int ss = (a + 1 + R) % SD;
#pragma unroll
        for (int c = 0; c < 9; ++c) sring[(ss * 9 + c) * NT + tid] = r[c];
      }
    }
  }
  flush_stores();
}

// ---------------------------------------------------------------------------
// Edge nodes: when the tiles of the stage kernel cover [0, nq-1) x [0, nr-1)
// exactly, the last q column (ex: nodes (nq-1, j, k)) and the last r row (ey:
// nodes (i, nr-1, k), i < nq - ex) are computed here.  Each is a 2D strip
// with a tangential axis (r for the column, q for the row) and the s axis;
// its normal axis (q for the column, r for the row) is at the boundary.
// A block owns 64 strip points x KZ planes: it stages v and the tangential
// and s fluxes of the strip, with halos, in LDS, and takes the interior rows
// of the tangential and s derivatives from there; boundary closure rows of
// every axis (always the case along the normal axis) gather their columns
// from memory.  Same arithmetic as the stage kernel: interior rows from the
// interior stencil, boundary rows from the closure table, fluxes by flux3,
// rates by node_rates, then the Runge-Kutta update (the penalties of its
// face nodes follow in penalty_kernel).
// LDS of edge_body<T, ORDER, KZ>: the closure rows, the patch (v, the
// tangential flux and the s flux of 64 + 2H strip points x KZ + 2H planes)
// and, for the column strip, the partial sums of its q closure row over
// columns nq-2 .. nq-NC (D+ part 3, D- part 3) per node of the block
template <typename T, int ORDER, int KZ>
struct EdgeLds {
  static constexpr int H = Stencil<ORDER>::Q, NT = 64 * KZ;
  static constexpr int PT = 64 + 2 * H, PK = KZ + 2 * H, NP = PT * PK;
  static constexpr std::size_t o_tab = 0, o_lp = o_tab + kClosureTab * kMaxM * kMaxCols, o_lqc = o_lp + 9 * NP,
                               total = o_lqc + 6 * NT;
  static constexpr std::size_t bytes = total * sizeof(T);
};

// PEN: the boundary penalties of the strip's nodes are added here (before
// the stage update) instead of by penalty_kernel
template <typename T, int ORDER, int KZ, bool EQ = false, bool PEN = false>
__device__ __forceinline__ void edge_body(const StageArgs<T>& A, int b, char* lds) {
  using S = Stencil<ORDER>;
  using L = EdgeLds<T, ORDER, KZ>;
  constexpr int R = S::R, Q = S::Q, M = S::M;
  constexpr int QD = R + Q + 1;
  constexpr int NC = M + Q;  // columns of a closure row
  static_assert(NC <= kMaxCols, "closure width");
  constexpr int TABN = kMaxM * kMaxCols;
  constexpr int H = Q;
  constexpr int NT = 64 * KZ;
  constexpr int PT = L::PT, NP = L::NP;
  static_assert(L::bytes <= kLdsBytes, "edge patch exceeds the LDS");
  T* const ltab = reinterpret_cast<T*>(lds) + L::o_tab;
  T* const lp = reinterpret_cast<T*>(lds) + L::o_lp;    // v (3), tangential flux (3), s flux (3)
  T* const lqc = reinterpret_cast<T*>(lds) + L::o_lqc;

  const int nq = A.nq, nr = A.nr, ns = A.ns;
  const int ex = A.ex, ey = A.ey;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  for (int e = tid; e < kClosureTab * TABN; e += NT) ltab[e] = A.tab[e];
  // the column strip's partial sums below read the table: every wave's part
  // of it must be written first (what an earlier block left in this LDS is
  // another layout's data when blocks of several orders share the launch)
  __syncthreads();

  // block -> strip, tangential tile, s tile
  const int nkt = (ns + KZ - 1) / KZ;
  const int ntc = ex ? (nr + 63) / 64 : 0;               // column strip tiles along r
  const int nrow = nq - (ex ? 1 : 0);                     // row strip points along q
  const int ntr = ey ? (nrow + 63) / 64 : 0;
  if (b >= (ntc + ntr) * nkt) return;
  const int st = b < ntc * nkt ? 0 : 1;                   // 0: column strip, 1: row strip
  if (st == 1) b -= ntc * nkt;
  const int tt = b % (st == 0 ? ntc : ntr), kt = b / (st == 0 ? ntc : ntr);
  const int t0 = tt * 64, k0 = kt * KZ;
  const int La = st == 0 ? nr : nq;                       // tangential axis length
  const int Ln = st == 0 ? nr : nrow;                     // strip points computed
  const int Nn = st == 0 ? nq : nr;                       // normal axis length
  const int mt = st == 0 ? 3 : 0;                         // metric row of the tangential axis
  const int mn = st == 0 ? 0 : 3;                         // metric row of the normal axis
  const long long field = (long long)A.field;
  // the node map's fields as scalars, both offsets formed before the
  // select: a select between the fields of a local NodeMap (or a closure
  // holding them) becomes a select of their addresses and keeps the object
  // in scratch memory
  const long long nm_plane = A.nm.plane, nm_cbase = A.nm.cbase;
  const int nm_px = A.nm.px, nm_nr = A.nm.nr, nm_nqm = A.nm.nqm;
  auto nm = [&](int i, int j, int k) -> long long {
    const long long in = (long long)k * nm_plane + (long long)j * nm_px + i;
    const long long last = nm_cbase + (long long)k * nm_nr + j;
    return i < nm_nqm ? in : last;
  };
  // element offset of the point (tangential t, s k) displaced dn along the normal axis
  auto at = [&](int dn, int t, int k) -> long long {
    const int i = st == 0 ? nq - 1 + dn : t, j = st == 0 ? t : nr - 1 + dn;
    return nm(i, j, k);
  };
  const T iht = st == 0 ? A.inv_h[1] : A.inv_h[0];
  const T ihn = st == 0 ? A.inv_h[0] : A.inv_h[1];
  const T ihs = A.inv_h[2];
  const T* __restrict__ qin = A.qin;
  const T* __restrict__ cf = A.coef;

  // stage the patch
  for (int e = tid; e < NP; e += NT) {
    const int pk = e / PT, pt = e - pk * PT;
    const int t = t0 - H + pt, k = k0 - H + pk;
    if (t < 0 || t >= La || k < 0 || k >= ns) continue;
    const long long o = at(0, t, k);
    T sg[6], f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) lp[c * NP + e] = qin[c * field + o];
#pragma unroll
    for (int c = 0; c < 6; ++c) sg[c] = qin[(3 + c) * field + o];
    flux3(cf[mt * field + o], cf[(mt + 1) * field + o], cf[(mt + 2) * field + o], sg[0], sg[1], sg[2], sg[3], sg[4],
          sg[5], f);
#pragma unroll
    for (int c = 0; c < 3; ++c) lp[(3 + c) * NP + e] = f[c];
    flux3(cf[6 * field + o], cf[7 * field + o], cf[8 * field + o], sg[0], sg[1], sg[2], sg[3], sg[4], sg[5], f);
#pragma unroll
    for (int c = 0; c < 3; ++c) lp[(6 + c) * NP + e] = f[c];
  }
  if (st == 0) {
    // The q closure row of a column node reads columns nq-NC .. nq-1 of the
    // node's row.  Sixteen lanes per node (lane l: column nq-16+l) load them
    // together, so that a load touches a few lines instead of one per lane,
    // and sum in a fixed butterfly; column nq-1 is added by the node itself.
    // In the rows the stage tiles compute, v and F_q of those columns come
    // from the stage kernel's copies (A.eqc), contiguous per row.
    const int grp = tid >> 4, l = tid & 15;
    const int col = nq - 16 + l, cc = 15 - l;  // cc: column index of the closure row
    const T cp = (cc >= 1 && cc < NC) ? ltab[2 * TABN + cc] : T(0);
    const T cm = (cc >= 1 && cc < NC) ? ltab[3 * TABN + cc] : T(0);
#pragma unroll 2
    for (int nd = grp; nd < NT; nd += NT / 16) {
      const int tq = t0 + (nd & 63), kq = k0 + nd / 64;
      T pv[3] = {T(0), T(0), T(0)}, pf[3] = {T(0), T(0), T(0)};
      if (tq < Ln && kq < ns && cc >= 1 && cc < NC && col >= 0) {
        if (EQ && A.eqc != nullptr && tq < nr - ey) {
          const T* const e = A.eqc + 8 * (((std::size_t)kq * nr + tq) * (NC - 1) + (std::size_t)(NC - 1 - cc));
          T w[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) w[c] = e[c];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            pv[c] = cp * w[c];
            pf[c] = cm * w[3 + c];
          }
        } else {
          const long long op = nm(col, tq, kq);
          T f[3];
          flux3(cf[op], cf[field + op], cf[2 * field + op], qin[3 * field + op], qin[4 * field + op],
                qin[5 * field + op], qin[6 * field + op], qin[7 * field + op], qin[8 * field + op], f);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            pv[c] = cp * qin[c * field + op];
            pf[c] = cm * f[c];
          }
        }
      }
#pragma unroll
      for (int w = 8; w >= 1; w >>= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pv[c] += __shfl_xor(pv[c], w, 16);
          pf[c] += __shfl_xor(pf[c], w, 16);
        }
      }
      if (l == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lqc[c * NT + nd] = pv[c];
          lqc[(3 + c) * NT + nd] = pf[c];
        }
      }
    }
  }
  __syncthreads();

  const int t = t0 + threadIdx.x, k = k0 + threadIdx.y;
  if (t >= Ln || k >= ns) return;
  const long long o = at(0, t, k);
  const int pme = (threadIdx.y + H) * PT + threadIdx.x + H;  // own patch point

  // derivatives along one axis at position p of n: D+ of v into uo, D- of
  // the flux added to dv; gv(d, c) / gf(d, f) return v and the flux at the
  // point d positions away along the axis (interior rows), cv / cflux the
  // same from memory (closure rows)
  T dv[3] = {T(0), T(0), T(0)};
  auto derivs = [&](int p, int n, T ih, auto gv, auto gf, auto cvf, auto cflux, T uo[3]) {
    T sp[3] = {T(0), T(0), T(0)}, sm[3] = {T(0), T(0), T(0)};
    if (p >= M && p < n - M) {
#pragma unroll
      for (int s = 0; s < QD; ++s) {
        T f[3];
        gf(R - s, f);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          sp[c] += T(S::a[s]) * gv(s - R, c);
          sm[c] += T(S::a[s]) * f[c];
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        uo[c] = sp[c] * ih;
        dv[c] -= sm[c] * ih;
      }
    } else {
      const bool left = p < M;
      const int row = left ? p : n - 1 - p;
      const int tb = left ? 0 : 2 * TABN;
      // in double precision a fully unrolled row keeps every column's loads
      // in flight at once, more registers than the kernel has
      constexpr int CU = sizeof(T) == 4 ? NC : 2;
#pragma unroll CU
      for (int cc = 0; cc < NC; ++cc) {
        const int d = (left ? cc : n - 1 - cc) - p;
        const T cp = ltab[tb + row * kMaxCols + cc];
        const T cm = ltab[tb + TABN + row * kMaxCols + cc];
        T f[3];
        cflux(d, f);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          sp[c] += cp * cvf(d, c);
          sm[c] += cm * f[c];
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        uo[c] = sp[c] * ih;
        dv[c] += sm[c] * ih;
      }
    }
  };
  // v and the flux of metric row m at the point d steps away along axis ax
  // (0 normal, 1 tangential, 2 s), read from memory
  auto pt_off = [=](int ax, int d) { return at(ax == 0 ? d : 0, ax == 1 ? t + d : t, ax == 2 ? k + d : k); };
  auto mem_v = [&](int ax) { return [=](int d, int c) { return qin[c * field + pt_off(ax, d)]; }; };
  auto mem_f = [&](int ax, int m) {
    return [=](int d, T f[3]) {
      const long long od = pt_off(ax, d);
      flux3(cf[m * field + od], cf[(m + 1) * field + od], cf[(m + 2) * field + od], qin[3 * field + od],
            qin[4 * field + od], qin[5 * field + od], qin[6 * field + od], qin[7 * field + od], qin[8 * field + od],
            f);
    };
  };
  T un[3], ut[3], us[3];
  // normal axis: closure row of the far boundary
  if (st == 0) {
    T f[3];
    mem_f(0, mn)(0, f);
    const T cp = ltab[2 * TABN], cm = ltab[3 * TABN];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      un[c] = (lqc[c * NT + tid] + cp * lp[c * NP + pme]) * ihn;
      dv[c] += (lqc[(3 + c) * NT + tid] + cm * f[c]) * ihn;
    }
  } else {
    derivs(Nn - 1, Nn, ihn, mem_v(0), mem_f(0, mn), mem_v(0), mem_f(0, mn), un);
  }
  // tangential axis and s axis: interior rows from the patch
  derivs(t, La, iht, [&](int d, int c) { return lp[c * NP + pme + d]; },
         [&](int d, T f[3]) {
#pragma unroll
           for (int c = 0; c < 3; ++c) f[c] = lp[(3 + c) * NP + pme + d];
         },
         mem_v(1), mem_f(1, mt), ut);
  derivs(k, ns, ihs, [&](int d, int c) { return lp[c * NP + pme + d * PT]; },
         [&](int d, T f[3]) {
#pragma unroll
           for (int c = 0; c < 3; ++c) f[c] = lp[(6 + c) * NP + pme + d * PT];
         },
         mem_v(2), mem_f(2, 6), us);

  T u[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u[0][c] = st == 0 ? un[c] : ut[c];  // q
    u[1][c] = st == 0 ? ut[c] : un[c];  // r
    u[2][c] = us[c];                    // s
  }
  const int i = st == 0 ? nq - 1 : t, j = st == 0 ? t : nr - 1;
  T mq[3], mr[3], ms[3], v[3], sg[6];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    mq[c] = cf[c * field + o];
    mr[c] = cf[(3 + c) * field + o];
    ms[c] = cf[(6 + c) * field + o];
    v[c] = lp[c * NP + pme];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) sg[c] = qin[(3 + c) * field + o];
  T rate[9];
  node_rates(u, dv, mq, mr, ms, cf[9 * field + o], cf[10 * field + o], cf[11 * field + o], rate);

  // the boundary penalties of every face the node lies on (with PEN; else
  // penalty_kernel adds them after the launch)
  if constexpr (PEN) {
    if (A.sat) {
      T fc[kNumFaceCoef];
      auto face = [&](int f, std::size_t idx, T eps) {
#pragma unroll
        for (int kk = 0; kk < kNumFaceCoef; ++kk) fc[kk] = A.face[A.face_off[f] + idx + (std::size_t)kk * A.face_n[f]];
        face_penalty(fc, A.gamma[f], eps, A.traction[f] != 0, v, sg, rate);
      };
      if (i == 0) face(0, (std::size_t)k * nr + j, T(-1));
      if (i == nq - 1) face(1, (std::size_t)k * nr + j, T(1));
      if (j == 0) face(2, (std::size_t)k * nq + i, T(-1));
      if (j == nr - 1) face(3, (std::size_t)k * nq + i, T(1));
      if (k == 0) face(4, (std::size_t)j * nq + i, T(-1));
      if (k == ns - 1) face(5, (std::size_t)j * nq + i, T(1));
    }
  }

  T sadd[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  if constexpr (EQ && sizeof(T) == 4) {
    if (A.nsrc > 0) source_add(A, i, j, k, sadd);
  }
  const T dt = A.dt, Ak = A.Ak, Bk = A.Bk;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const long long oc = (long long)c * field + o;
    const T dqo = A.read_dq ? A.dq[oc] : T(0);
    T d = dt * rate[c] + Ak * dqo;
    if constexpr (EQ && sizeof(T) == 4) {
      if (c >= 3) d += sadd[c - 3];
    }
    const T q0 = (c < 3) ? v[c] : sg[c - 3];
    A.dq[oc] = d;
    A.qout[oc] = q0 + Bk * d;
  }
}

// ---------------------------------------------------------------------------
// launch wrappers: one grid with its arguments passed by value (stage_kernel,
// edge_kernel), or the blocks of many grids in one launch (the _batch
// kernels: block -> (grid, local block) through the prefix sums of the
// per-grid block counts; the grid's arguments are read from a device table)
template <typename T, int ORDER, int TY, bool BUF>
__global__ __launch_bounds__(64 * TY, SBP_STAGE_MIN_WAVES) void stage_kernel(const StageArgs<T> A) {
  __shared__ __align__(16) char lds[StageLds<T, ORDER, TY>::bytes];
  // XCD-aware tile order: consecutive tiles land on the same XCD
  const int per = gridDim.x >> 3;
  stage_body<T, ORDER, TY, BUF, true>(A, (blockIdx.x & 7) * per + (blockIdx.x >> 3), lds);
}

template <typename T, int ORDER, int KZ>
__global__ __launch_bounds__(64 * KZ) void edge_kernel(const StageArgs<T> A) {
  __shared__ __align__(16) char lds[EdgeLds<T, ORDER, KZ>::bytes];
  edge_body<T, ORDER, KZ, true>(A, blockIdx.x, lds);
}

// penalty_part and penalty_body are defined further down
template <typename T>
__device__ __forceinline__ long long penalty_part(const StageArgs<T>& A, long long e);
template <typename T>
__device__ __forceinline__ void penalty_body(const StageArgs<T>& A, long long e);

// single precision: the edge blocks, with the penalties of their own nodes,
// then the boundary penalties of the nodes the stage tiles computed (the
// penalty part of those) in the same launch, so that the penalty blocks fill
// the compute units the edge blocks leave idle
template <typename T, int ORDER, int KZ>
__global__ __launch_bounds__(64 * KZ) void edge_penalty_kernel(const StageArgs<T> A, const int eblocks) {
  __shared__ __align__(16) char lds[EdgeLds<T, ORDER, KZ>::bytes];
  if ((int)blockIdx.x < eblocks) {
    edge_body<T, ORDER, KZ, true, true>(A, blockIdx.x, lds);
  } else {
    const long long e =
        penalty_part(A, (long long)(blockIdx.x - eblocks) * (64 * KZ) + threadIdx.y * 64 + threadIdx.x);
    if (e >= 0) penalty_body(A, e);
  }
}

// last entry of first[0 .. n-1] (non-decreasing, first[0] = 0) that is <= item
__device__ __forceinline__ int batch_find(const int* __restrict__ first, int n, int item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int ORDER, int TY, bool BUF>
__global__ __launch_bounds__(64 * TY, SBP_STAGE_MIN_WAVES) void stage_kernel_batch(const BatchArgs<T> B) {
  const int per = gridDim.x >> 3;
  const int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (item >= B.total) return;
  const int g = batch_find(B.first, B.n, item);
  // a private copy: loaded once, and no store of the kernel can alias it
  const StageArgs<T> A = B.args[g];
  __shared__ __align__(16) char lds[StageLds<T, ORDER, TY>::bytes];
  stage_body<T, ORDER, TY, BUF>(A, item - B.first[g], lds);
}

template <typename T, int ORDER, int KZ>
__global__ __launch_bounds__(64 * KZ) void edge_kernel_batch(const BatchArgs<T> B) {
  const int item = blockIdx.x;
  if (item >= B.total) return;
  const int g = batch_find(B.first, B.n, item);
  const StageArgs<T> A = B.args[g];
  __shared__ __align__(16) char lds[EdgeLds<T, ORDER, KZ>::bytes];
  edge_body<T, ORDER, KZ>(A, item - B.first[g], lds);
}

// ---------------------------------------------------------------------------
// Batched stage: one launch per Runge-Kutta stage for the stage tiles and
// edge blocks of every grid of a batch, whatever their interior order, with
// the same kernel bodies as stage_kernel / edge_kernel.  The LDS buffer is
// sized for the largest body of the orders the kernel serves.
template <typename T>
struct PersistOrders;
template <>
struct PersistOrders<float> {
  static constexpr int lo = 2, hi = 7;
};
template <>
struct PersistOrders<double> {
  // order 7 takes grouped launches: its tile fills the LDS, which would
  // then be the size of every block of the kernel
  static constexpr int lo = 2, hi = 6;
};

// the orders a kernel serves: bit o of MASK
template <typename T, unsigned MASK, int O>
constexpr std::size_t persist_lds_upto() {
  if constexpr (O < PersistOrders<T>::lo) {
    return 0;
  } else {
    const std::size_t a = StageLds<T, O, 8>::bytes, b = EdgeLds<T, O, 8>::bytes;
    const std::size_t m = ((MASK >> O) & 1u) ? (a > b ? a : b) : 0;
    const std::size_t r = persist_lds_upto<T, MASK, O - 1>();
    return m > r ? m : r;
  }
}

template <typename T, unsigned MASK, int O>
__device__ __forceinline__ void persist_dispatch(const StageArgs<T>& A, const BatchItem& w, char* lds) {
  if constexpr (O >= PersistOrders<T>::lo) {
    if constexpr ((MASK >> O) & 1u) {
      if (w.order == O) {
        if (w.kind == 0)
          stage_body<T, O, 8, true>(A, w.local, lds);
        else
          edge_body<T, O, 8>(A, w.local, lds);
        return;
      }
    }
    persist_dispatch<T, MASK, O - 1>(A, w, lds);
  }
}

// One launch over the whole work list: block b takes item (b & 7) of the
// interleaved list, so that the hardware, dispatching blocks in order and
// round-robin over the 8 XCDs, hands each XCD its own segment, longest
// items first; a slot past the end of its segment is an empty block.
template <typename T, unsigned MASK>
__global__ __launch_bounds__(512, SBP_STAGE_MIN_WAVES) void stage_kernel_worklist(const PersistArgs<T> P) {
  __shared__ __align__(16) char lds[persist_lds_upto<T, MASK, PersistOrders<T>::hi>()];
  const int sg = blockIdx.x & 7;
  const int item = P.seg[sg] + (int)(blockIdx.x >> 3);
  if (item >= P.seg[sg + 1]) return;
  const BatchItem w = P.items[item];
  const StageArgs<T> A = P.args[w.grid];
  persist_dispatch<T, MASK, PersistOrders<T>::hi>(A, w, lds);
}

// ---------------------------------------------------------------------------
// Boundary penalties: one thread per node of the block's surface, which is
// enumerated once: the q faces (all j, k), the r faces (interior i, all k),
// the s faces (interior i and j).  Each node sums the penalties of every face
// it lies on, in the face order (q0, q1, r0, r1, s0, s1), and adds them to
// the stage update: dQ += dt P, Q_out += B_k dt P (Q_in is the stage input).
template <typename T>
__device__ __forceinline__ void penalty_body(const StageArgs<T>& A, long long e) {
  const int nq = A.nq, nr = A.nr, ns = A.ns;
  constexpr bool Q0S = q0_in_stage<T>();
  // q faces (both, or only q = nq-1), r faces (i in [i0, nq-1-i0)), s faces
  // (the same i, 0 < j < nr-1)
  const int i0 = Q0S ? 0 : 1, ni = nq - 1 - i0;
  const long long nA = (Q0S ? 1LL : 2LL) * nr * ns, nB = 2LL * ni * ns, nC = 2LL * ni * (nr - 2);
  int i, j, k;
  if (e < nA) {
    const long long per = (long long)nr * ns, r = e % per;
    i = (Q0S || e >= per) ? nq - 1 : 0;
    j = (int)(r % nr);
    k = (int)(r / nr);
  } else if ((e -= nA) < nB) {
    const long long per = (long long)ni * ns, r = e % per;
    j = e < per ? 0 : nr - 1;
    i = i0 + (int)(r % ni);
    k = (int)(r / ni);
  } else if ((e -= nB) < nC) {
    const long long per = (long long)ni * (nr - 2), r = e % per;
    k = e < per ? 0 : ns - 1;
    i = i0 + (int)(r % ni);
    j = 1 + (int)(r / ni);
  } else {
    return;
  }
  const long long o = A.nm(i, j, k);
  const std::size_t field = A.field;
  T v[3], sg[6], rate[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = A.qin[c * field + o];
#pragma unroll
  for (int c = 0; c < 6; ++c) sg[c] = A.qin[(3 + c) * field + o];
#pragma unroll
  for (int c = 0; c < 9; ++c) rate[c] = T(0);
  T fc[kNumFaceCoef];
  auto face = [&](int f, std::size_t idx, T eps) {
#pragma unroll
    for (int kk = 0; kk < kNumFaceCoef; ++kk) fc[kk] = A.face[A.face_off[f] + idx + (std::size_t)kk * A.face_n[f]];
    face_penalty(fc, A.gamma[f], eps, A.traction[f], v, sg, rate);
  };
  // (with the q = 0 face in the stage kernel: only at the nodes of the edge
  // row, which the stage tiles do not compute)
  if (i == 0 && (!Q0S || (A.ey && j == nr - 1))) face(0, (std::size_t)k * nr + j, T(-1));
  if (i == nq - 1) face(1, (std::size_t)k * nr + j, T(1));
  if (j == 0) face(2, (std::size_t)k * nq + i, T(-1));
  if (j == nr - 1) face(3, (std::size_t)k * nq + i, T(1));
  if (k == 0) face(4, (std::size_t)j * nq + i, T(-1));
  if (k == ns - 1) face(5, (std::size_t)j * nq + i, T(1));
  const T dt = A.dt, Bk = A.Bk;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const T d = dt * rate[c];
    A.dq[c * field + o] += d;
    A.qout[c * field + o] += Bk * d;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void penalty_kernel(const StageArgs<T> A) {
  penalty_body(A, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// With the q = 0 face in the stage kernel, penalty_body's enumeration is the
// q = nq-1 face [0, nA), the r = 0 face [nA, nA + P), the r = nr-1 face
// [nA + P, nA + 2P), the s faces after (P = (nq-1) ns).  Its part that the
// stage tiles compute: r = 0, the s faces, and r = nr-1 when there is no
// edge row.  Index e of that part -> index of the enumeration, or -1 past
// the part's end.
template <typename T>
__device__ __forceinline__ long long penalty_part(const StageArgs<T>& A, long long e) {
  const long long nA = (long long)A.nr * A.ns, P = (long long)(A.nq - 1) * A.ns;
  const long long nC = 2LL * (A.nq - 1) * (A.nr - 2);
  const long long nrf = A.ey ? P : 2 * P;
  if (e < nrf) return nA + e;
  e -= nrf;
  return e < nC ? nA + 2 * P + e : -1;
}

// number of nodes of that part (host and device)
template <typename T>
__host__ __device__ inline long long penalty_part_nodes(const StageArgs<T>& A) {
  const long long P = (long long)(A.nq - 1) * A.ns, nC = 2LL * (A.nq - 1) * (A.nr - 2);
  return (A.ey ? P : 2 * P) + nC;
}

// surface nodes of several grids: thread -> grid by the prefix sums in first
template <typename T>
__global__ __launch_bounds__(256) void penalty_kernel_batch(const BatchArgs<T> B) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= B.total) return;
  const int g = batch_find(B.first, B.n, item);
  penalty_body(B.args[g], item - B.first[g]);
}

// ---------------------------------------------------------------------------
// point sources: dQ += gdt * w M, Q_out += Bk * gdt * w M on the source stencil.
// One block per source; the stencils of two sources may overlap, so the
// updates are atomic additions.
template <typename T>
__device__ __forceinline__ void source_body(const SourceArgs<T>& S, const int s) {
  const int w = S.width;
  const int n = w * w * w;
  const int stride = S.tab_stride ? S.tab_stride : kMaxSources;
  const T gdt = S.clock ? static_cast<const T*>(S.clock->gtab)[((std::size_t)S.clock->step * 5 + S.stage) * stride +
                                                             S.tab_off + s]
                        : S.gdt[s];
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int a = t % w, b = (t / w) % w, c = t / (w * w);
    const std::size_t o = (std::size_t)S.nm(S.i0[s] + a, S.j0[s] + b, S.k0[s] + c);
    const T* wm = S.wm + ((std::size_t)s * kMaxSrcWidth * kMaxSrcWidth * kMaxSrcWidth + t) * 6;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const T add = gdt * wm[f];
      atomicAdd(&S.dq[(3 + f) * S.field + o], add);
      if (S.qout) atomicAdd(&S.qout[(3 + f) * S.field + o], S.Bk * add);
    }
  }
}

template <typename T>
__global__ void source_kernel(SourceArgs<T> S) {
  source_body(S, blockIdx.x);
}

template <typename T>
__global__ void source_kernel_batch(const SourceBatch<T> B) {
  const int item = blockIdx.x;
  if (item >= B.total) return;
  const int g = batch_find(B.first, B.n, item);
  source_body(B.args[g], item - B.first[g]);
}

// receivers of several grids: one thread per receiver
template <typename T>
__global__ void record_kernel_batch(const RecordBatch<T> B) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= B.total) return;
  const int g = batch_find(B.first, B.n, item);
  const RecordArgs<T>& R = B.args[g];
  const int r = item - B.first[g];
  const long long o = R.off[r];
  std::size_t at = (std::size_t)r * 3;
  if (B.clock) {
    const int nrec = B.first[g + 1] - B.first[g];
    at += (std::size_t)(R.base + B.clock->rec0 + B.clock->step) * nrec * 3;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) R.out[at + c] = R.q[c * R.field + o];
}

// receivers: out[(slot * nrec + r) * 3 + c] = v_c(node_r), slot = the clock's
// receiver slot of the current step (or 0 without a clock: out is the slot)
template <typename T>
__global__ void record_kernel(const T* __restrict__ q, std::size_t field, const long long* __restrict__ off,
                              int nrec, T* __restrict__ out, const StepClock* __restrict__ clock) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrec) return;
  const long long o = off[r];
  const std::size_t slot = clock ? (std::size_t)(clock->rec0 + clock->step) : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) out[(slot * nrec + r) * 3 + c] = q[c * field + o];
}

__global__ void clock_set_kernel(StepClock* c, const void* gtab, long long rec0) {
  c->gtab = gtab;
  c->rec0 = rec0;
  c->step = 0;
}

__global__ void clock_tick_kernel(StepClock* c) { c->step += 1; }

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
    const std::size_t o = (std::size_t)E.nm(i, j, k);
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
// launchers (a stage body whose LDS does not fit is not built: 16-row tiles
// in double, order 8 with 16-row tiles)
template <typename T, int ORDER, int TY>
static hipError_t launch_stage_t(const StageArgs<T>& a, hipStream_t st) {
  if constexpr (!stage_built<T, ORDER, TY>()) {
    return hipErrorInvalidValue;
  } else {
    const int nb = ((a.ntiles + 7) / 8) * 8;
    // buffer addressing needs every array (at most 12 fields) below 4 GiB
    if (!a.plain && 12.0 * (double)a.field * sizeof(T) < 4294967296.0)
      hipLaunchKernelGGL((stage_kernel<T, ORDER, TY, true>), dim3(nb), dim3(64, TY), 0, st, a);
    else
      hipLaunchKernelGGL((stage_kernel<T, ORDER, TY, false>), dim3(nb), dim3(64, TY), 0, st, a);
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_stage(int order, int ty, const StageArgs<T>& a, hipStream_t st) {
  // 16-row tiles only for 4-byte types (LDS capacity)
  if (ty == 16 && sizeof(T) == 4) {
    if (order == 2) return launch_stage_t<T, 2, 16>(a, st);
    if (order == 3) return launch_stage_t<T, 3, 16>(a, st);
    if (order == 4) return launch_stage_t<T, 4, 16>(a, st);
    if (order == 5) return launch_stage_t<T, 5, 16>(a, st);
    if (order == 6) return launch_stage_t<T, 6, 16>(a, st);
    if (order == 7) return launch_stage_t<T, 7, 16>(a, st);
    if (order == 8) return launch_stage_t<T, 8, 16>(a, st);
  } else {
    if (order == 2) return launch_stage_t<T, 2, 8>(a, st);
    if (order == 3) return launch_stage_t<T, 3, 8>(a, st);
    if (order == 4) return launch_stage_t<T, 4, 8>(a, st);
    if (order == 5) return launch_stage_t<T, 5, 8>(a, st);
    if (order == 6) return launch_stage_t<T, 6, 8>(a, st);
    if (order == 7) return launch_stage_t<T, 7, 8>(a, st);
    if (order == 8) return launch_stage_t<T, 8, 8>(a, st);
  }
  return hipErrorInvalidValue;
}

// largest private (scratch) segment, bytes per lane, of the kernels one
// step of `order` launches (stage kernel of tile height ty in both
// addressings, edge, penalty, source and receiver kernels)
template <typename T, int ORDER, int TY>
static std::size_t step_scratch_t() {
  if constexpr (!stage_built<T, ORDER, TY>()) {
    return 0;
  } else {
    std::size_t m = 0;
    const void* fns[] = {reinterpret_cast<const void*>(&stage_kernel<T, ORDER, TY, true>),
                         reinterpret_cast<const void*>(&stage_kernel<T, ORDER, TY, false>),
                         reinterpret_cast<const void*>(&edge_kernel<T, ORDER, 8>),
                         reinterpret_cast<const void*>(&penalty_kernel<T>),
                         reinterpret_cast<const void*>(&source_kernel<T>),
                         reinterpret_cast<const void*>(&record_kernel<T>)};
    for (const void* f : fns) {
      hipFuncAttributes at{};
      if (hipFuncGetAttributes(&at, f) != hipSuccess) return (std::size_t)-1;
      m = std::max<std::size_t>(m, at.localSizeBytes);
    }
    if constexpr (sizeof(T) == 4) {
      const void* fe[] = {reinterpret_cast<const void*>(&edge_penalty_kernel<T, ORDER, 8>)};
      for (const void* f : fe) {
        hipFuncAttributes at{};
        if (hipFuncGetAttributes(&at, f) != hipSuccess) return (std::size_t)-1;
        m = std::max<std::size_t>(m, at.localSizeBytes);
      }
    }
    return m;
  }
}

template <typename T>
std::size_t step_scratch(int order, int ty) {
  if (ty == 16 && sizeof(T) == 4) {
    if (order == 2) return step_scratch_t<T, 2, 16>();
    if (order == 3) return step_scratch_t<T, 3, 16>();
    if (order == 4) return step_scratch_t<T, 4, 16>();
    if (order == 5) return step_scratch_t<T, 5, 16>();
    if (order == 6) return step_scratch_t<T, 6, 16>();
    if (order == 7) return step_scratch_t<T, 7, 16>();
    if (order == 8) return step_scratch_t<T, 8, 16>();
  } else {
    if (order == 2) return step_scratch_t<T, 2, 8>();
    if (order == 3) return step_scratch_t<T, 3, 8>();
    if (order == 4) return step_scratch_t<T, 4, 8>();
    if (order == 5) return step_scratch_t<T, 5, 8>();
    if (order == 6) return step_scratch_t<T, 6, 8>();
    if (order == 7) return step_scratch_t<T, 7, 8>();
    if (order == 8) return step_scratch_t<T, 8, 8>();
  }
  return (std::size_t)-1;
}

// the same for the batched step's kernels (work-list stage kernel for the
// set of orders, penalty, source and receiver kernels)
template <typename T>
std::size_t batch_step_scratch(unsigned orders) {
  constexpr unsigned kAll = ((1u << (PersistOrders<T>::hi + 1)) - 1) & ~3u;
  const void* st = nullptr;
  if ((orders & ~(1u << 4)) == 0) st = reinterpret_cast<const void*>(&stage_kernel_worklist<T, 1u << 4>);
  else if ((orders & ~(1u << 6)) == 0) st = reinterpret_cast<const void*>(&stage_kernel_worklist<T, 1u << 6>);
  else if ((orders & ~((1u << 4) | (1u << 6))) == 0)
    st = reinterpret_cast<const void*>(&stage_kernel_worklist<T, (1u << 4) | (1u << 6)>);
  else if ((orders & ~kAll) == 0) st = reinterpret_cast<const void*>(&stage_kernel_worklist<T, kAll>);
  if (!st) return (std::size_t)-1;
  std::size_t m = 0;
  const void* fns[] = {st, reinterpret_cast<const void*>(&penalty_kernel_batch<T>),
                       reinterpret_cast<const void*>(&source_kernel_batch<T>),
                       reinterpret_cast<const void*>(&record_kernel_batch<T>)};
  for (const void* f : fns) {
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, f) != hipSuccess) return (std::size_t)-1;
    m = std::max<std::size_t>(m, at.localSizeBytes);
  }
  return m;
}

template <typename T>
int edge_blocks(const StageArgs<T>& a) {
  constexpr int KZ = 8;
  const int nkt = (a.ns + KZ - 1) / KZ;
  return ((a.ex ? (a.nr + 63) / 64 : 0) + (a.ey ? (a.nq - (a.ex ? 1 : 0) + 63) / 64 : 0)) * nkt;
}

template <typename T>
hipError_t launch_edge(int order, const StageArgs<T>& a, hipStream_t st) {
  constexpr int KZ = 8;
  const int nb = edge_blocks(a);
  if (nb == 0) return hipSuccess;
  if (order == 2)
    hipLaunchKernelGGL((edge_kernel<T, 2, KZ>), dim3(nb), dim3(64, KZ), 0, st, a);
  else if (order == 3)
    hipLaunchKernelGGL((edge_kernel<T, 3, KZ>), dim3(nb), dim3(64, KZ), 0, st, a);
  else if (order == 4)
    hipLaunchKernelGGL((edge_kernel<T, 4, KZ>), dim3(nb), dim3(64, KZ), 0, st, a);
  else if (order == 5)
    hipLaunchKernelGGL((edge_kernel<T, 5, KZ>), dim3(nb), dim3(64, KZ), 0, st, a);
  else if (order == 6)
    hipLaunchKernelGGL((edge_kernel<T, 6, KZ>), dim3(nb), dim3(64, KZ), 0, st, a);
  else if (order == 7)
    hipLaunchKernelGGL((edge_kernel<T, 7, KZ>), dim3(nb), dim3(64, KZ), 0, st, a);
  else if (order == 8)
    hipLaunchKernelGGL((edge_kernel<T, 8, KZ>), dim3(nb), dim3(64, KZ), 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T, int ORDER, int TY>
static hipError_t launch_stage_batch_t(const BatchArgs<T>& b, bool buf, hipStream_t st) {
  if constexpr (!stage_built<T, ORDER, TY>()) {
    return hipErrorInvalidValue;
  } else {
    const int nb = ((b.total + 7) / 8) * 8;
    if (buf)
      hipLaunchKernelGGL((stage_kernel_batch<T, ORDER, TY, true>), dim3(nb), dim3(64, TY), 0, st, b);
    else
      hipLaunchKernelGGL((stage_kernel_batch<T, ORDER, TY, false>), dim3(nb), dim3(64, TY), 0, st, b);
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_stage_batch(int order, int ty, const BatchArgs<T>& b, bool buf, hipStream_t st) {
  if (b.total == 0) return hipSuccess;
  if (ty == 16 && sizeof(T) == 4) {
    if (order == 2) return launch_stage_batch_t<T, 2, 16>(b, buf, st);
    if (order == 3) return launch_stage_batch_t<T, 3, 16>(b, buf, st);
    if (order == 4) return launch_stage_batch_t<T, 4, 16>(b, buf, st);
    if (order == 5) return launch_stage_batch_t<T, 5, 16>(b, buf, st);
    if (order == 6) return launch_stage_batch_t<T, 6, 16>(b, buf, st);
    if (order == 7) return launch_stage_batch_t<T, 7, 16>(b, buf, st);
    if (order == 8) return launch_stage_batch_t<T, 8, 16>(b, buf, st);
  } else {
    if (order == 2) return launch_stage_batch_t<T, 2, 8>(b, buf, st);
    if (order == 3) return launch_stage_batch_t<T, 3, 8>(b, buf, st);
    if (order == 4) return launch_stage_batch_t<T, 4, 8>(b, buf, st);
    if (order == 5) return launch_stage_batch_t<T, 5, 8>(b, buf, st);
    if (order == 6) return launch_stage_batch_t<T, 6, 8>(b, buf, st);
    if (order == 7) return launch_stage_batch_t<T, 7, 8>(b, buf, st);
    if (order == 8) return launch_stage_batch_t<T, 8, 8>(b, buf, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_edge_batch(int order, const BatchArgs<T>& b, hipStream_t st) {
  constexpr int KZ = 8;
  if (b.total == 0) return hipSuccess;
  if (order == 2)
    hipLaunchKernelGGL((edge_kernel_batch<T, 2, KZ>), dim3(b.total), dim3(64, KZ), 0, st, b);
  else if (order == 3)
    hipLaunchKernelGGL((edge_kernel_batch<T, 3, KZ>), dim3(b.total), dim3(64, KZ), 0, st, b);
  else if (order == 4)
    hipLaunchKernelGGL((edge_kernel_batch<T, 4, KZ>), dim3(b.total), dim3(64, KZ), 0, st, b);
  else if (order == 5)
    hipLaunchKernelGGL((edge_kernel_batch<T, 5, KZ>), dim3(b.total), dim3(64, KZ), 0, st, b);
  else if (order == 6)
    hipLaunchKernelGGL((edge_kernel_batch<T, 6, KZ>), dim3(b.total), dim3(64, KZ), 0, st, b);
  else if (order == 7)
    hipLaunchKernelGGL((edge_kernel_batch<T, 7, KZ>), dim3(b.total), dim3(64, KZ), 0, st, b);
  else if (order == 8)
    hipLaunchKernelGGL((edge_kernel_batch<T, 8, KZ>), dim3(b.total), dim3(64, KZ), 0, st, b);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_source_batch(const SourceBatch<T>& b, hipStream_t st) {
  if (b.total == 0) return hipSuccess;
  hipLaunchKernelGGL(source_kernel_batch<T>, dim3(b.total), dim3(256), 0, st, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_record_batch(const RecordBatch<T>& b, hipStream_t st) {
  if (b.total == 0) return hipSuccess;
  hipLaunchKernelGGL(record_kernel_batch<T>, dim3((b.total + 255) / 256), dim3(256), 0, st, b);
  return hipGetLastError();
}

// one kernel per set of orders that batches commonly mix (the register
// allocation of a kernel is that of its most demanding body), and one for
// every order
template <typename T>
hipError_t launch_stage_worklist(const PersistArgs<T>& p, unsigned orders, int blocks, hipStream_t st) {
  constexpr unsigned kAll = ((1u << (PersistOrders<T>::hi + 1)) - 1) & ~3u;
  if ((orders & ~(1u << 4)) == 0)
    hipLaunchKernelGGL((stage_kernel_worklist<T, 1u << 4>), dim3(blocks), dim3(64, 8), 0, st, p);
  else if ((orders & ~(1u << 6)) == 0)
    hipLaunchKernelGGL((stage_kernel_worklist<T, 1u << 6>), dim3(blocks), dim3(64, 8), 0, st, p);
  else if ((orders & ~((1u << 4) | (1u << 6))) == 0)
    hipLaunchKernelGGL((stage_kernel_worklist<T, (1u << 4) | (1u << 6)>), dim3(blocks), dim3(64, 8), 0, st, p);
  else if ((orders & ~kAll) == 0)
    hipLaunchKernelGGL((stage_kernel_worklist<T, kAll>), dim3(blocks), dim3(64, 8), 0, st, p);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
bool worklist_order_ok(int order) {
  return order >= PersistOrders<T>::lo && order <= PersistOrders<T>::hi;
}

template <typename T>
hipError_t launch_penalty(const StageArgs<T>& a, hipStream_t st) {
  const long long n = surface_nodes(a.nq, a.nr, a.ns, q0_in_stage<T>());
  hipLaunchKernelGGL(penalty_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_edge_penalty(int order, const StageArgs<T>& a, hipStream_t st) {
  if constexpr (sizeof(T) != 4) {
    return hipErrorInvalidValue;
  } else {
    constexpr int KZ = 8;
    const int ne = edge_blocks(a);
    const long long np = penalty_part_nodes(a);
    const int nb = ne + (int)((np + 64 * KZ - 1) / (64 * KZ));
    if (nb == 0) return hipSuccess;
    if (order == 2)
      hipLaunchKernelGGL((edge_penalty_kernel<T, 2, KZ>), dim3(nb), dim3(64, KZ), 0, st, a, ne);
    else if (order == 3)
      hipLaunchKernelGGL((edge_penalty_kernel<T, 3, KZ>), dim3(nb), dim3(64, KZ), 0, st, a, ne);
    else if (order == 4)
      hipLaunchKernelGGL((edge_penalty_kernel<T, 4, KZ>), dim3(nb), dim3(64, KZ), 0, st, a, ne);
    else if (order == 5)
      hipLaunchKernelGGL((edge_penalty_kernel<T, 5, KZ>), dim3(nb), dim3(64, KZ), 0, st, a, ne);
    else if (order == 6)
      hipLaunchKernelGGL((edge_penalty_kernel<T, 6, KZ>), dim3(nb), dim3(64, KZ), 0, st, a, ne);
    else if (order == 7)
      hipLaunchKernelGGL((edge_penalty_kernel<T, 7, KZ>), dim3(nb), dim3(64, KZ), 0, st, a, ne);
    else if (order == 8)
      hipLaunchKernelGGL((edge_penalty_kernel<T, 8, KZ>), dim3(nb), dim3(64, KZ), 0, st, a, ne);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_penalty_batch(const BatchArgs<T>& b, hipStream_t st) {
  if (b.total == 0) return hipSuccess;
  hipLaunchKernelGGL(penalty_kernel_batch<T>, dim3((b.total + 255) / 256), dim3(256), 0, st, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_source(const SourceArgs<T>& s, int nsrc, hipStream_t st) {
  hipLaunchKernelGGL(source_kernel<T>, dim3(nsrc), dim3(256), 0, st, s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_record(const T* q, std::size_t field, const long long* off, int nrec, T* out,
                         const StepClock* clock, hipStream_t st) {
  hipLaunchKernelGGL(record_kernel<T>, dim3((nrec + 255) / 256), dim3(256), 0, st, q, field, off, nrec, out, clock);
  return hipGetLastError();
}

hipError_t launch_clock_set(StepClock* c, const void* gtab, long long rec0, hipStream_t st) {
  hipLaunchKernelGGL(clock_set_kernel, dim3(1), dim3(1), 0, st, c, gtab, rec0);
  return hipGetLastError();
}

hipError_t launch_clock_tick(StepClock* c, hipStream_t st) {
  hipLaunchKernelGGL(clock_tick_kernel, dim3(1), dim3(1), 0, st, c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_energy(const EnergyArgs<T>& e, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(energy_kernel<T>, dim3(nblocks), dim3(256), 0, st, e);
  return hipGetLastError();
}

template hipError_t launch_stage<float>(int, int, const StageArgs<float>&, hipStream_t);
template hipError_t launch_stage<double>(int, int, const StageArgs<double>&, hipStream_t);
template hipError_t launch_edge<float>(int, const StageArgs<float>&, hipStream_t);
template hipError_t launch_edge<double>(int, const StageArgs<double>&, hipStream_t);
template std::size_t step_scratch<float>(int, int);
template std::size_t step_scratch<double>(int, int);
template std::size_t batch_step_scratch<float>(unsigned);
template std::size_t batch_step_scratch<double>(unsigned);
template int edge_blocks<float>(const StageArgs<float>&);
template int edge_blocks<double>(const StageArgs<double>&);
template hipError_t launch_stage_batch<float>(int, int, const BatchArgs<float>&, bool, hipStream_t);
template hipError_t launch_stage_batch<double>(int, int, const BatchArgs<double>&, bool, hipStream_t);
template hipError_t launch_edge_batch<float>(int, const BatchArgs<float>&, hipStream_t);
template hipError_t launch_edge_batch<double>(int, const BatchArgs<double>&, hipStream_t);
template hipError_t launch_source_batch<float>(const SourceBatch<float>&, hipStream_t);
template hipError_t launch_source_batch<double>(const SourceBatch<double>&, hipStream_t);
template hipError_t launch_record_batch<float>(const RecordBatch<float>&, hipStream_t);
template hipError_t launch_record_batch<double>(const RecordBatch<double>&, hipStream_t);
template hipError_t launch_stage_worklist<float>(const PersistArgs<float>&, unsigned, int, hipStream_t);
template hipError_t launch_stage_worklist<double>(const PersistArgs<double>&, unsigned, int, hipStream_t);
template bool worklist_order_ok<float>(int);
template bool worklist_order_ok<double>(int);
template hipError_t launch_penalty<float>(const StageArgs<float>&, hipStream_t);
template hipError_t launch_penalty<double>(const StageArgs<double>&, hipStream_t);
template hipError_t launch_edge_penalty<float>(int, const StageArgs<float>&, hipStream_t);
template hipError_t launch_edge_penalty<double>(int, const StageArgs<double>&, hipStream_t);
template hipError_t launch_penalty_batch<float>(const BatchArgs<float>&, hipStream_t);
template hipError_t launch_penalty_batch<double>(const BatchArgs<double>&, hipStream_t);
template hipError_t launch_source<float>(const SourceArgs<float>&, int, hipStream_t);
template hipError_t launch_source<double>(const SourceArgs<double>&, int, hipStream_t);
template hipError_t launch_record<float>(const float*, std::size_t, const long long*, int, float*,
                                         const StepClock*, hipStream_t);
template hipError_t launch_record<double>(const double*, std::size_t, const long long*, int, double*,
                                          const StepClock*, hipStream_t);
template hipError_t launch_energy<float>(const EnergyArgs<float>&, int, hipStream_t);
template hipError_t launch_energy<double>(const EnergyArgs<double>&, int, hipStream_t);

}  // namespace sbp
