// Host side of the C ABI declared in include/sbp.h: validation, workspace
// layout, metric terms and material coefficients (double precision on the
// host), point-source stencils, and the per-stage kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sbp.h"
#include "internal.hpp"
#include "adjoint.hpp"
#include "host_math.hpp"
#include "kernels.hpp"

using namespace sbp;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(SBP_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Five-stage 2N-storage fourth-order Runge-Kutta coefficients (Carpenter &
// Kennedy 1994, the integrator named in Sec. 7).
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};
const double kRkC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                        2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

constexpr int kMaxRec = 65536;
// sbp_step_batch: at most kMaxBatch handles and kMaxItems work items; the
// source-time table is uploaded for kBatchTabSteps steps at a time (two
// parts); with plain addressing the handles are grouped by interior order
constexpr int kMaxBatch = 64;
constexpr int kBatchTabSteps = 64;
constexpr int kMaxItems = 65536;
constexpr int kMaxGroups = 6;  // six orders

constexpr int kMaxPart = 1024;
constexpr double kPi = 3.14159265358979323846;
// sbp_step: the source-time table is uploaded for kTabSteps steps at a time,
// into one of kTabParts parts (pinned host staging, device copy)
constexpr int kTabSteps = 512;
constexpr int kTabParts = 4;

std::size_t align256(std::size_t b) { return (b + 255) & ~std::size_t(255); }

using Geometry = Grid3;

struct Src {
  int i0, j0, k0;
  double M[6];
  int stf;
  double param, t0;
};

}  // namespace

struct sbp_ctx {
  int order = 0, dtype = 0, esize = 0;
  Geometry g{};
  Closure cl;
  double gamma[6] = {};
  int sat_variant = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  std::size_t ws_bytes = 0;
  // byte offsets in the workspace
  std::size_t off_qa = 0, off_qb = 0, off_dq = 0, off_coef = 0, off_face[6] = {}, off_src = 0,
              off_rec = 0, off_part = 0, off_bounds = 0, off_tab = 0, off_scl = 0, off_eqc = 0, off_batch = 0,
              total = 0;
  std::size_t face_n[6] = {};
  int px = 0;
  std::size_t plane = 0, field = 0;
  NodeMap nm{};   // node -> element offset in a field
  // host copies kept for the material and source set-up
  std::vector<double> J;           // Jacobian (dense)
  std::vector<double> Mface[6];    // M[xi][0..2] on face f (3 * face_n)
  bool have_material = false;
  int cur = 0;  // 0: state in q_a, 1: in q_b
  double t = 0.0;
  long long steps = 0;
  std::vector<Src> src;
  int width = 0;  // source stencil width 2(p+1)
  int nrec = 0, rec_max = 0;
  long long rec_step = 0;
  void* rec_out = nullptr;
  int ty = 8, zchunk = 0;
  bool plain = false;   // plain pointers even where buffer addressing fits (sbp_set_addressing)
  int nxt = 0, nyt = 0, nzc = 0;
  int ex = 0, ey = 0;   // last q column / last r row computed by the edge kernel
  bool bounds_dirty = true;
  // launch timing (sbp_set_profiling)
  bool prof = false;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  double prof_stage_ms = 0.0, prof_edge_ms = 0.0;
  long long prof_n = 0;
  // checkpoints of the last sbp_step_checkpointed (valid until the state,
  // the medium, the sources or the receivers change); ck_id names them
  bool ck_valid = false;
  const char* ck_ws = nullptr;
  int ck_nsteps = 0, ck_every = 0;
  double ck_dt = 0.0, ck_t0 = 0.0;
  long long ck_steps = 0;
  long long ck_id = 0, ck_next = 0;
  // node coordinates (host, 3 grid functions), for sbp_add_source_at
  std::vector<double> X;
  // source-time tables of sbp_step: pinned host staging parts, the event of
  // each part's last upload, the next part to use
  char* tab_host = nullptr;
  hipEvent_t tab_ev[kTabParts] = {};
  bool tab_used[kTabParts] = {};
  int tab_next = 0;
  std::size_t off_clock = 0, off_gtab = 0, tab_part_bytes = 0;
  // graphs of one step (index: starting ping-pong parity), captured on a
  // private stream and launched on the handle's stream; valid while the
  // launch settings (gen) and dt are those they were captured with
  bool graphs = true;
  int batch_L = 0;  // s-chunk length for sbp_step_batch (0: cost model), from sbp_autotune_batch
  // pinned staging of the batch source-time table (first handle of a batch)
  char* btab_host = nullptr;
  hipEvent_t btab_ev[2] = {};
  bool btab_used[2] = {};
  int btab_next = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  long long gx_gen[2] = {-1, -1};
  double gx_dt[2] = {0.0, 0.0};
  long long gen = 0;  // bumped by every change of what the step's launches bake in
};

namespace {

// The first nq - 1 columns in rows starting on 128-byte lines (the memory
// request size); column nq - 1 in a compact array after them (NodeMap).
std::size_t row_pitch(int nq, std::size_t es) {
  const std::size_t line = 128 / es;
  return ((std::size_t)nq - 1 + line - 1) / line * line;
}

// elements of one field
std::size_t field_elems(int nq, int nr, int ns, std::size_t es) {
  const std::size_t line = 128 / es, ncol = (std::size_t)nr * ns;
  return row_pitch(nq, es) * ncol + (ncol + line - 1) / line * line;
}

int check_dims(int nq, int nr, int ns, int order, int dtype) {
  if (order == 9)
    return fail(SBP_EINVAL, "order 9 is not supported: no boundary closure is constructed for it");
  if (order < 2 || order > 8) return fail(SBP_EINVAL, "order must be 2 to 8 (got %d)", order);
  if (dtype != SBP_F32 && dtype != SBP_F64) return fail(SBP_EINVAL, "dtype must be SBP_F32 or SBP_F64");
  const int mn = 2 * order;
  if (nq < mn || nr < mn || ns < mn)
    return fail(SBP_EINVAL, "every axis needs at least %d points for order %d (got %d x %d x %d)", mn, order, nq,
                nr, ns);
  if (nq > 1 << 20 || nr > 1 << 20 || ns > 1 << 20) return fail(SBP_EINVAL, "axis too long");
  // the kernels address a field with 32-bit byte offsets: one field of the
  // layout must stay below 4 GiB
  const std::size_t es = dtype == SBP_F32 ? 4 : 8;
  const std::size_t bytes = field_elems(nq, nr, ns, es) * es;
  if (bytes >= ((std::size_t)1 << 32))
    return fail(SBP_EINVAL, "grid too large: one field takes %zu bytes, the kernels address at most 4 GiB per field",
                bytes);
  return SBP_OK;
}

// Tables of sbp_step_batch, in the workspace of the first handle of a batch
// (sized for double, the larger argument blocks): stage arguments of every
// (stage, parity) and handle, group block prefixes (grouped launches), source
// arguments of every (stage, parity), receiver arguments of both step
// parities, the work list and its segments, the clock, the source-time table
// (two parts).
struct BatchRegion {
  std::size_t stage, first, src, src_first, rec, rec_first, pen_first, items, seg, clock, gtab, gtab_part, total;
};
BatchRegion batch_region() {
  BatchRegion r{};
  std::size_t o = 0;
  auto take = [&](std::size_t bytes) {
    std::size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  r.stage = take((std::size_t)10 * kMaxBatch * sizeof(StageArgs<double>));
  r.first = take((std::size_t)2 * kMaxGroups * (kMaxBatch + 1) * sizeof(int));
  r.src = take((std::size_t)10 * kMaxBatch * sizeof(SourceArgs<double>));
  r.src_first = take((std::size_t)(kMaxBatch + 1) * sizeof(int));
  r.rec = take((std::size_t)2 * kMaxBatch * sizeof(RecordArgs<double>));
  r.rec_first = take((std::size_t)(kMaxBatch + 1) * sizeof(int));
  r.pen_first = take((std::size_t)(kMaxBatch + 1) * sizeof(int));
  r.items = take((std::size_t)kMaxItems * sizeof(BatchItem));
  r.seg = take(9 * sizeof(int));
  r.clock = take(sizeof(StepClock));
  r.gtab_part = align256((std::size_t)kBatchTabSteps * 5 * kMaxBatch * kMaxSources * sizeof(double));
  r.gtab = take(2 * r.gtab_part);
  r.total = o;
  return r;
}
std::size_t batch_region_bytes() { return batch_region().total; }

// elements of the single-precision copies of the last column's q closure
// inputs: 8 values x ns planes x nr rows x (kMaxCols - 1) columns
std::size_t eqc_elems(int nr, int ns) { return (std::size_t)8 * ns * nr * (kMaxCols - 1); }

void layout(sbp_ctx* h) {
  const int es = h->esize;
  const Geometry& g = h->g;
  h->px = (int)row_pitch(g.nq, es);
  h->plane = (std::size_t)h->px * g.nr;
  h->field = field_elems(g.nq, g.nr, g.ns, es);
  h->nm.plane = (long long)h->plane;
  h->nm.cbase = (long long)(h->plane * g.ns);
  h->nm.px = h->px;
  h->nm.nr = g.nr;
  h->nm.nqm = g.nq - 1;
  std::size_t o = 0;
  auto take = [&](std::size_t bytes) {
    std::size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  h->off_qa = take(9 * h->field * es);
  h->off_qb = take(9 * h->field * es);
  h->off_dq = take(9 * h->field * es);
  h->off_coef = take(kNumCoef * h->field * es);
  const std::size_t fn[6] = {(std::size_t)g.nr * g.ns, (std::size_t)g.nr * g.ns, (std::size_t)g.nq * g.ns,
                             (std::size_t)g.nq * g.ns, (std::size_t)g.nq * g.nr, (std::size_t)g.nq * g.nr};
  for (int f = 0; f < 6; ++f) {
    h->face_n[f] = fn[f];
    h->off_face[f] = take(kNumFaceCoef * fn[f] * es);
  }
  h->off_src = take((std::size_t)kMaxSources * kMaxSrcWidth * kMaxSrcWidth * kMaxSrcWidth * 6 * es);
  h->off_rec = take((std::size_t)kMaxRec * sizeof(long long));
  h->off_part = take(kMaxPart * sizeof(double));
  h->off_bounds = take((std::size_t)(g.nq + g.nr + g.ns + 16) * sizeof(int));
  h->off_tab = take((std::size_t)kClosureTab * kMaxM * kMaxCols * es);
  h->off_scl = take((std::size_t)2 * kMaxM * 6 * h->plane * es);
  // single precision: the stage kernel's copies of the last column's q
  // closure inputs (StageArgs::eqc), sized for the widest closure row
  h->off_eqc = take(es == 4 ? eqc_elems(g.nr, g.ns) * es : 0);
  h->off_batch = take(batch_region_bytes());
  h->tab_part_bytes = align256((std::size_t)kTabSteps * 5 * kMaxSources * es);
  h->off_clock = take(sizeof(StepClock));
  h->off_gtab = take(kTabParts * h->tab_part_bytes);
  h->total = o;
}

// Copies of nf fields between a dense (ns, nr, nq) array and device fields in
// the NodeMap layout: the first nq - 1 columns as pitched rows, column nq - 1
// into the compact array.
int copy_in(sbp_ctx* h, char* dst, const void* src, int nf, hipMemcpyKind kind) {
  const Geometry& g = h->g;
  const std::size_t es = h->esize, rows = (std::size_t)g.nr * g.ns;
  if (kind == hipMemcpyHostToDevice) {
    // from pageable host memory: lay the fields out on the host and copy them
    // in one piece (a 2D copy from pageable memory moves row by row)
    std::vector<char> tmp((std::size_t)nf * h->field * es, 0);
    for (int f = 0; f < nf; ++f) {
      char* d = tmp.data() + (std::size_t)f * h->field * es;
      const char* sf = (const char*)src + (std::size_t)f * g.n * es;
      for (std::size_t r = 0; r < rows; ++r) {
        const char* sr = sf + r * g.nq * es;
        std::memcpy(d + r * h->px * es, sr, (g.nq - 1) * es);
        std::memcpy(d + ((std::size_t)h->nm.cbase + r) * es, sr + (g.nq - 1) * es, es);
      }
    }
    HIPCHK(hipMemcpyAsync(dst, tmp.data(), tmp.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SBP_OK;
  }
  for (int f = 0; f < nf; ++f) {
    char* d = dst + (std::size_t)f * h->field * es;
    const char* s = (const char*)src + (std::size_t)f * g.n * es;
    HIPCHK(hipMemcpy2DAsync(d, h->px * es, s, g.nq * es, (g.nq - 1) * es, rows, kind, h->stream));
    HIPCHK(hipMemcpy2DAsync(d + (std::size_t)h->nm.cbase * es, es, s + (g.nq - 1) * es, g.nq * es, es, rows, kind,
                            h->stream));
  }
  return SBP_OK;
}

int copy_out(sbp_ctx* h, void* dst, const char* src, int nf, hipMemcpyKind kind) {
  const Geometry& g = h->g;
  const std::size_t es = h->esize, rows = (std::size_t)g.nr * g.ns;
  for (int f = 0; f < nf; ++f) {
    char* d = (char*)dst + (std::size_t)f * g.n * es;
    const char* s = src + (std::size_t)f * h->field * es;
    HIPCHK(hipMemcpy2DAsync(d, g.nq * es, s, h->px * es, (g.nq - 1) * es, rows, kind, h->stream));
    HIPCHK(hipMemcpy2DAsync(d + (g.nq - 1) * es, g.nq * es, s + (std::size_t)h->nm.cbase * es, es, es, rows, kind,
                            h->stream));
  }
  return SBP_OK;
}

template <typename T>
int upload_field(sbp_ctx* h, std::size_t off, const double* src) {
  const Geometry& g = h->g;
  std::vector<T> tmp(g.n);
  for (std::size_t n = 0; n < g.n; ++n) tmp[n] = (T)src[n];
  int rc = copy_in(h, h->ws + off, tmp.data(), 1, hipMemcpyHostToDevice);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  return SBP_OK;
}

int upload(sbp_ctx* h, std::size_t off, const double* src) {
  return h->dtype == SBP_F32 ? upload_field<float>(h, off, src) : upload_field<double>(h, off, src);
}

template <typename T>
int upload_raw(sbp_ctx* h, std::size_t off, const std::vector<double>& src) {
  std::vector<T> tmp(src.size());
  for (std::size_t n = 0; n < src.size(); ++n) tmp[n] = (T)src[n];
  HIPCHK(hipMemcpyAsync(h->ws + off, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return SBP_OK;
}

int upload_vec(sbp_ctx* h, std::size_t off, const std::vector<double>& src) {
  return h->dtype == SBP_F32 ? upload_raw<float>(h, off, src) : upload_raw<double>(h, off, src);
}

// Metric terms (Sec. 2.2, computed by metric_terms on the host): uploads M,
// keeps J, the face values of M and the node coordinates.
int compute_metrics(sbp_ctx* h, const double* xyz) {
  const Geometry& g = h->g;
  const std::size_t n = g.n;
  h->X.assign(3 * n, 0.0);
  if (xyz) {
    std::memcpy(h->X.data(), xyz, 3 * n * sizeof(double));
  } else {
    for (int k = 0; k < g.ns; ++k)
      for (int j = 0; j < g.nr; ++j)
        for (int i = 0; i < g.nq; ++i) {
          const std::size_t o = g.idx(i, j, k);
          h->X[o] = (double)i / (g.nq - 1);
          h->X[n + o] = (double)j / (g.nr - 1);
          h->X[2 * n + o] = (double)k / (g.ns - 1);
        }
  }
  h->J.assign(n, 0.0);
  std::vector<double> M(9 * n);
  const long long bad = metric_terms(h->cl, g, h->X.data(), h->J.data(), M.data());
  if (bad >= 0) return fail(SBP_EINVAL, "non-positive Jacobian at node %lld", bad);
  for (int xi = 0; xi < 3; ++xi)
    for (int c = 0; c < 3; ++c) {
      const double* t1 = M.data() + (std::size_t)(3 * xi + c) * n;
      int rc = upload(h, h->off_coef + (std::size_t)(3 * xi + c) * h->field * h->esize, t1);
      if (rc) return rc;
      // keep the face values of M[xi][.] for the penalties of faces 2 xi, 2 xi + 1
      for (int side = 0; side < 2; ++side) {
        const int f = 2 * xi + side;
        auto& Mf = h->Mface[f];
        if (Mf.empty()) Mf.assign(3 * h->face_n[f], 0.0);
        std::size_t a = 0;
        if (xi == 0) {
          const int i = side ? g.nq - 1 : 0;
          for (int k = 0; k < g.ns; ++k)
            for (int j = 0; j < g.nr; ++j) Mf[c * h->face_n[f] + a++] = t1[g.idx(i, j, k)];
        } else if (xi == 1) {
          const int j = side ? g.nr - 1 : 0;
          for (int k = 0; k < g.ns; ++k)
            for (int i = 0; i < g.nq; ++i) Mf[c * h->face_n[f] + a++] = t1[g.idx(i, j, k)];
        } else {
          const int k = side ? g.ns - 1 : 0;
          for (int j = 0; j < g.nr; ++j)
            for (int i = 0; i < g.nq; ++i) Mf[c * h->face_n[f] + a++] = t1[g.idx(i, j, k)];
        }
      }
    }
  return SBP_OK;
}

// balanced split of [0, N) into tiles of width <= W whose first and last tile
// hold at least m points (so SBP closure rows never straddle a tile edge)
std::vector<int> tile_bounds(int N, int W, int m) {
  std::vector<int> b;
  if (N <= W) return {0, N};
  int T = (N + W - 1) / W;
  for (int t = 0; t <= T; ++t) b.push_back((int)((long long)t * N / T));
  if (b[1] - b[0] >= m && b[T] - b[T - 1] >= m) return b;
  // fall back: full first and last tiles, balanced middle
  b.assign(1, 0);
  b.push_back(W);
  const int mid = N - 2 * W;
  if (mid > 0) {
    const int Tm = (mid + W - 1) / W;
    for (int t = 1; t <= Tm; ++t) b.push_back(W + (int)((long long)t * mid / Tm));
  }
  if (b.back() != N - W) b.push_back(N - W);
  b.push_back(N);
  return b;
}

// split of [0, N) along q into tiles of width <= 64 whose starts are
// multiples of `align` points (128-byte lines), the first and last tile
// holding at least m points
std::vector<int> tile_bounds_aligned(int N, int align, int m) {
  std::vector<int> b{0};
  while (N - b.back() > 64) b.push_back(b.back() + 64);
  b.push_back(N);
  // a last tile narrower than m: move its start back by one line at a time
  while (b.size() > 2 && b[b.size() - 1] - b[b.size() - 2] < m) {
    const int s = b[b.size() - 2] - align;
    if (s <= b[b.size() - 3]) break;
    b[b.size() - 2] = s;
  }
  bool ok = b.size() >= 2;
  for (std::size_t t = 0; t + 1 < b.size(); ++t) ok = ok && b[t + 1] - b[t] <= 64 && b[t + 1] > b[t];
  ok = ok && (b.size() == 2 || (b[1] - b[0] >= m && b[b.size() - 1] - b[b.size() - 2] >= m));
  return ok ? b : tile_bounds(N, 64, m);
}

int prepare_bounds(sbp_ctx* h) {
  if (!h->bounds_dirty) return SBP_OK;
  const Geometry& g = h->g;
  const int line = 128 / h->esize;  // points per 128-byte line
  // The tiles cover the first nq - 1 columns (the layout keeps column nq - 1
  // apart, NodeMap); the edge kernel computes column nq - 1 and, when nr - 1
  // is a multiple of the tile height, also row nr - 1 so that no tile along
  // r is shorter than ty (for nq = 64 k + 1, nr = ty k + 1 every tile is full).
  h->ex = 1;
  h->ey = ((g.nr - 1) % h->ty == 0 && g.nr - 1 >= 2 * h->ty) ? 1 : 0;
  std::vector<int> xb = tile_bounds_aligned(g.nq - h->ex, line, h->cl.m);
  std::vector<int> yb = tile_bounds(g.nr - h->ey, h->ty, h->cl.m);
  h->nxt = (int)xb.size() - 1;
  h->nyt = (int)yb.size() - 1;
  int zc = h->zchunk;
  if (zc <= 0) {
    // chunks along s: the s queues of a chunk start with r + q + 1 planes
    // of warm-up, and the blocks run in waves of one block per compute unit;
    // take the number of chunks that minimises waves x (planes + warm-up)
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      int v = 0;
      if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    const long long cols = (long long)h->nxt * h->nyt;
    const int warm = h->cl.r + h->cl.q + 1;
    const int nzmax = std::max(1, g.ns / 8);
    long long best = -1;
    int bestnz = 1;
    for (int nz = 1; nz <= nzmax; ++nz) {
      const long long waves = (cols * nz + cus - 1) / cus;
      const long long cost = waves * ((g.ns + nz - 1) / nz + warm);
      if (best < 0 || cost < best) {
        best = cost;
        bestnz = nz;
      }
    }
    zc = (g.ns + bestnz - 1) / bestnz;
  }
  zc = std::max(1, std::min(zc, g.ns));
  h->nzc = (g.ns + zc - 1) / zc;
  std::vector<int> all(xb);
  all.insert(all.end(), yb.begin(), yb.end());
  for (int t = 0; t <= h->nzc; ++t) all.push_back((int)((long long)t * g.ns / h->nzc));
  HIPCHK(hipMemcpyAsync(h->ws + h->off_bounds, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->bounds_dirty = false;
  ++h->gen;
  return SBP_OK;
}

double stf_value(const Src& s, double t) {
  if (s.stf == SBP_STF_RICKER) {
    const double a = kPi * s.param * (t - s.t0);
    const double a2 = a * a;
    return (1.0 - 2.0 * a2) * std::exp(-a2);
  }
  const double tt = t - s.t0;
  return tt >= 0 ? tt / (s.param * s.param) * std::exp(-tt / s.param) : 0.0;
}

template <typename T>
StageArgs<T> stage_args(sbp_ctx* h) {
  StageArgs<T> a{};
  const Geometry& g = h->g;
  a.coef = (const T*)(h->ws + h->off_coef);
  a.face = (const T*)h->ws;
  for (int f = 0; f < 6; ++f) {
    a.face_off[f] = h->off_face[f] / sizeof(T);
    a.face_n[f] = h->face_n[f];
    a.gamma[f] = (T)h->gamma[f];
    a.traction[f] = (h->sat_variant == SBP_SAT_TRACTION && h->gamma[f] == 1.0) ? 1 : 0;
  }
  a.bounds = (const int*)(h->ws + h->off_bounds);
  a.nm = h->nm;
  a.ex = h->ex;
  a.ey = h->ey;
  a.sat = 1;
  a.plain = h->plain ? 1 : 0;
  a.plane = h->plane;
  a.field = h->field;
  a.px = h->px;
  a.nq = g.nq;
  a.nr = g.nr;
  a.ns = g.ns;
  a.nxt = h->nxt;
  a.nyt = h->nyt;
  a.nzc = h->nzc;
  a.ntiles = h->nxt * h->nyt * h->nzc;
  a.ncol = h->cl.ncol;
  a.inv_h[0] = (T)(g.nq - 1);
  a.inv_h[1] = (T)(g.nr - 1);
  a.inv_h[2] = (T)(g.ns - 1);
  a.tab = (const T*)(h->ws + h->off_tab);
  a.scl = (T*)(h->ws + h->off_scl);
  a.eqc = sizeof(T) == 4 ? (T*)(h->ws + h->off_eqc) : nullptr;
  a.nsrc = 0;
  return a;
}

// point sources of stage k at time tstage (g(t) evaluated on the host in double)
template <typename T>
SourceArgs<T> source_args(sbp_ctx* h, int k, double dt, double tstage, bool rhs_only, T* qout) {
  SourceArgs<T> s{};
  s.dq = (T*)(h->ws + h->off_dq);
  s.qout = rhs_only ? nullptr : qout;
  s.wm = (const T*)(h->ws + h->off_src);
  s.nm = h->nm;
  s.plane = h->plane;
  s.field = h->field;
  s.px = h->px;
  s.width = h->width;
  s.Bk = rhs_only ? T(0) : (T)kRkB[k];
  for (std::size_t i = 0; i < h->src.size(); ++i) {
    s.i0[i] = h->src[i].i0;
    s.j0[i] = h->src[i].j0;
    s.k0[i] = h->src[i].k0;
    s.gdt[i] = (T)((rhs_only ? 1.0 : dt) * stf_value(h->src[i], tstage));
  }
  s.clock = nullptr;
  s.stage = k;
  return s;
}

// single precision: the point sources of stage k go into the stage and edge
// kernels' update (StageArgs::nsrc and src_*), in place of a source_kernel
// launch; returns whether they did
template <typename T>
bool fuse_sources(sbp_ctx* h, StageArgs<T>& a, int k, double dt, double tstage, bool rhs_only,
                  const StepClock* clock) {
  a.nsrc = 0;
  if (sizeof(T) != 4 || h->src.empty()) return false;
  const SourceArgs<T> s = source_args<T>(h, k, dt, tstage, rhs_only, nullptr);
  a.nsrc = (int)h->src.size();
  a.src_w = s.width;
  a.src_stage = k;
  for (int i = 0; i < kMaxSources; ++i) {
    a.src_i0[i] = s.i0[i];
    a.src_j0[i] = s.j0[i];
    a.src_k0[i] = s.k0[i];
    a.src_gdt[i] = s.gdt[i];
  }
  a.src_wm = s.wm;
  a.src_clock = clock;
  return true;
}

// arguments of Runge-Kutta stage k (or of the right-hand side alone) with the
// input state in Q_b (c = 1) or Q_a (c = 0)
template <typename T>
StageArgs<T> stage_entry(sbp_ctx* h, const StageArgs<T>& a, int k, int c, double dt, bool rhs_only) {
  StageArgs<T> b = a;
  T* qa = (T*)(h->ws + h->off_qa);
  T* qb = (T*)(h->ws + h->off_qb);
  b.qin = c ? qb : qa;
  b.qout = c ? qa : qb;
  b.dq = (T*)(h->ws + h->off_dq);
  b.read_dq = (!rhs_only && k > 0) ? 1 : 0;
  b.Ak = rhs_only ? T(0) : (T)kRkA[k];
  b.Bk = rhs_only ? T(0) : (T)kRkB[k];
  b.dt = rhs_only ? T(1) : (T)dt;
  return b;
}

// The launches that follow the stage kernel of one grid: the edge kernel
// (when the tiles leave a last column or row) and the boundary penalties (when
// a.sat).  In single precision both go in one launch.
template <typename T>
hipError_t edge_and_penalties(const sbp_ctx* h, const StageArgs<T>& a, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (sizeof(T) == 4 && a.sat && (h->ex || h->ey)) return launch_edge_penalty<T>(h->order, a, st);
  if (h->ex || h->ey) e = launch_edge<T>(h->order, a, st);
  if (e == hipSuccess && a.sat) e = launch_penalty<T>(a, st);
  return e;
}

// One Runge-Kutta stage (or the right-hand side alone) on stream st: the
// stage kernel, the edge kernel, the boundary penalties, the point sources
// (dt * g from the clock's table when clock is not null, else evaluated here
// at tstage).  With profiling on (only on the handle's own stream) the stage
// kernel, and the edge and penalty kernels together, are bracketed by events
// and the host waits for them.
template <typename T>
int run_stage(sbp_ctx* h, StageArgs<T>& a, int k, double dt, double tstage, bool rhs_only, T* qin, T* qout,
              hipStream_t st, const StepClock* clock) {
  const int c = qin == (T*)(h->ws + h->off_qb) ? 1 : 0;
  a = stage_entry<T>(h, a, k, c, dt, rhs_only);
  const bool fused = fuse_sources<T>(h, a, k, dt, tstage, rhs_only, clock);
  const bool prof = h->prof && st == h->stream;
  if (prof) HIPCHK(hipEventRecord(h->ev[0], st));
  HIPCHK(launch_stage<T>(h->order, h->ty, a, st));
  if (prof) HIPCHK(hipEventRecord(h->ev[1], st));
  HIPCHK(edge_and_penalties<T>(h, a, st));
  if (prof) {
    HIPCHK(hipEventRecord(h->ev[2], st));
    HIPCHK(hipEventSynchronize(h->ev[2]));
    float t01 = 0.f, t12 = 0.f;
    HIPCHK(hipEventElapsedTime(&t01, h->ev[0], h->ev[1]));
    HIPCHK(hipEventElapsedTime(&t12, h->ev[1], h->ev[2]));
    h->prof_stage_ms += t01;
    h->prof_edge_ms += t12;
    ++h->prof_n;
  }
  if (!h->src.empty() && !fused) {
    SourceArgs<T> s = source_args<T>(h, k, dt, tstage, rhs_only, qout);
    s.clock = clock;
    HIPCHK(launch_source<T>(s, (int)h->src.size(), st));
  }
  return SBP_OK;
}

// The launches of one step on stream st, the state starting in buffer
// parity c (0: Q_a): five stages, the receivers, the clock tick.  Every step
// issues the same launches; the step-dependent values (source-time factors,
// receiver slot) come from the clock.
template <typename T>
int step_launches(sbp_ctx* h, StageArgs<T>& a, int c, double dt, hipStream_t st) {
  T* qa = (T*)(h->ws + h->off_qa);
  T* qb = (T*)(h->ws + h->off_qb);
  StepClock* clk = (StepClock*)(h->ws + h->off_clock);
  for (int k = 0; k < 5; ++k) {
    int rc = run_stage<T>(h, a, k, dt, 0.0, false, c ? qb : qa, c ? qa : qb, st, clk);
    if (rc) return rc;
    c ^= 1;
  }
  if (h->nrec > 0)
    HIPCHK(launch_record<T>(c ? qb : qa, h->field, (const long long*)(h->ws + h->off_rec), h->nrec, (T*)h->rec_out,
                            clk, st));
  HIPCHK(launch_clock_tick(clk, st));
  return SBP_OK;
}

// Captures step_launches for starting parity c into an executable graph
// (on the handle's private capture stream).
template <typename T>
int capture_step(sbp_ctx* h, StageArgs<T>& a, int c, double dt) {
  if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  if (h->gx[c]) {
    (void)hipGraphExecDestroy(h->gx[c]);
    h->gx[c] = nullptr;
  }
  HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  const int rc = step_launches<T>(h, a, c, dt, h->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(SBP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&h->gx[c], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) {
    h->gx[c] = nullptr;
    return fail(SBP_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  }
  h->gx_gen[c] = h->gen;
  h->gx_dt[c] = dt;
  return SBP_OK;
}

// nsteps steps from the current state.  Per chunk of at most kTabSteps
// steps: the source-time factors dt * g(t_n + C_k dt) of every step, stage
// and source are evaluated on the host (double) and uploaded, the device
// clock is set, and the steps are issued: the call's first step as direct
// launches, every later one as a replay of the step graph captured from
// those launches (all direct with graphs off or profiling on; either way the
// same kernels with the same arguments).
template <typename T>
int do_steps(sbp_ctx* h, int nsteps, double dt) {
  int rc = prepare_bounds(h);
  if (rc) return rc;
  StageArgs<T> a = stage_args<T>(h);
  StepClock* clk = (StepClock*)(h->ws + h->off_clock);
  const double t0 = h->t;
  // graphs replay only steps whose kernels use no scratch memory (a
  // graph-launched double-precision kernel with a large private segment
  // once ended in a memory fault whose cause was not found; kernels that
  // spill launch eagerly)
  const bool use_graph = h->graphs && !h->prof && step_scratch<T>(h->order, h->ty) == 0;
  for (int n0 = 0; n0 < nsteps; n0 += kTabSteps) {
    const int nc = std::min(kTabSteps, nsteps - n0);
    const int part = h->tab_next;
    h->tab_next = (part + 1) % kTabParts;
    char* dtab = h->ws + h->off_gtab + (std::size_t)part * h->tab_part_bytes;
    if (!h->src.empty()) {
      // the staging part is reused once its previous upload has completed
      if (h->tab_used[part]) HIPCHK(hipEventSynchronize(h->tab_ev[part]));
      T* ht = (T*)(h->tab_host + (std::size_t)part * h->tab_part_bytes);
      for (int nn = 0; nn < nc; ++nn) {
        const double tn = t0 + (n0 + nn) * dt;
        for (int k = 0; k < 5; ++k)
          for (std::size_t q = 0; q < h->src.size(); ++q)
            ht[((std::size_t)nn * 5 + k) * kMaxSources + q] = (T)(dt * stf_value(h->src[q], tn + kRkC[k] * dt));
      }
      HIPCHK(hipMemcpyAsync(dtab, ht, (std::size_t)nc * 5 * kMaxSources * sizeof(T), hipMemcpyHostToDevice,
                            h->stream));
      HIPCHK(hipEventRecord(h->tab_ev[part], h->stream));
      h->tab_used[part] = true;
    }
    HIPCHK(launch_clock_set(clk, dtab, h->rec_step, h->stream));
    for (int nn = 0; nn < nc; ++nn) {
      const int c = h->cur;
      // the first step of a call is issued directly, later ones replay the
      // graph captured from the same launches
      if (use_graph && n0 + nn > 0) {
        if (!h->gx[c] || h->gx_gen[c] != h->gen || h->gx_dt[c] != dt)
          if ((rc = capture_step<T>(h, a, c, dt))) return rc;
        HIPCHK(hipGraphLaunch(h->gx[c], h->stream));
      } else {
        if ((rc = step_launches<T>(h, a, c, dt, h->stream))) return rc;
      }
      h->cur ^= 1;  // five stages: the state ends in the other buffer
      if (h->nrec > 0) ++h->rec_step;
      ++h->steps;
    }
  }
  h->t = t0 + nsteps * dt;
  return SBP_OK;
}

// ---- batched stepping (sbp_step_batch) -------------------------------------
// Launch settings of a batch: every grid gets 8-row tiles and one s-chunk
// length L, chosen for the batch as a whole (each grid's own automatic
// choice assumes it has the whole GPU and cuts small grids into short
// chunks, each paying r + q + 1 warm-up planes); the handles' own settings
// are restored by BatchSettings' destructor.
struct BatchSettings {
  sbp_ctx** hs = nullptr;
  int n = 0;
  std::vector<int> ty, zc;
  BatchSettings(sbp_ctx** h, int nn) : hs(h), n(nn) {
    for (int g = 0; g < n; ++g) {
      ty.push_back(hs[g]->ty);
      zc.push_back(hs[g]->zchunk);
    }
  }
  ~BatchSettings() {
    for (int g = 0; g < n; ++g) {
      hs[g]->ty = ty[g];
      hs[g]->zchunk = zc[g];
      hs[g]->bounds_dirty = true;
    }
  }
};

int device_cus() {
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  return cus;
}

// the cost model's chunk length: waves of one block per compute unit times
// the planes a block marches (its chunk plus the warm-up planes)
int batch_cost_model_L(sbp_ctx** hs, int n) {
  const int cus = device_cus();
  int nsmax = 0;
  for (int g = 0; g < n; ++g) nsmax = std::max(nsmax, hs[g]->g.ns);
  long long best = -1;
  int bestL = nsmax;
  for (int L = nsmax; L >= 8; L = L * 3 / 4) {
    long long tiles = 0, planes = 0;
    for (int g = 0; g < n; ++g) {
      const sbp_ctx* h = hs[g];
      const int Lg = std::min(L, h->g.ns);
      const int nz = (h->g.ns + Lg - 1) / Lg;
      tiles += (long long)h->nxt * h->nyt * nz;
      planes = std::max<long long>(planes, (h->g.ns + nz - 1) / nz + h->cl.r + h->cl.q + 1);
    }
    const long long cost = (tiles + cus - 1) / cus * planes;
    if (best < 0 || cost < best) {
      best = cost;
      bestL = L;
    }
  }
  return bestL;
}

// applies chunk length L (0: the cost model's) and 8-row tiles to every grid
int batch_apply_L(sbp_ctx** hs, int n, int L) {
  for (int g = 0; g < n; ++g) {
    hs[g]->ty = 8;
    hs[g]->zchunk = 0;
    hs[g]->bounds_dirty = true;
    int rc = prepare_bounds(hs[g]);  // tiles across s (nxt, nyt)
    if (rc) return rc;
  }
  if (L <= 0) L = batch_cost_model_L(hs, n);
  for (int g = 0; g < n; ++g) {
    hs[g]->zchunk = std::min(L, hs[g]->g.ns);
    hs[g]->bounds_dirty = true;
    int rc = prepare_bounds(hs[g]);
    if (rc) return rc;
  }
  return SBP_OK;
}

// The work list: every grid's stage tiles and edge blocks, cut into 8
// contiguous segments of equal estimated cost (grids largest first, tiles
// in tile order, so that neighbouring tiles share a segment and hence an
// XCD's L2), each segment sorted longest first.
template <typename T>
int batch_items(sbp_ctx** hs, int n, std::vector<BatchItem>& items, std::vector<int>& seg) {
  struct W {
    BatchItem it;
    long long cost;
  };
  std::vector<int> byn(n);
  for (int g = 0; g < n; ++g) byn[g] = g;
  std::stable_sort(byn.begin(), byn.end(), [&](int a, int b) { return hs[a]->g.n > hs[b]->g.n; });
  std::vector<W> all;
  long long total = 0;
  for (int g : byn) {
    sbp_ctx* h = hs[g];
    const StageArgs<T> a = stage_args<T>(h);
    const long long planes = (h->g.ns + h->nzc - 1) / h->nzc + h->cl.r + h->cl.q + 1;
    for (int t = 0; t < a.ntiles; ++t) all.push_back({{g, 0, t, h->order}, planes * 64 * 8});
    const int eb = edge_blocks(a);
    // an edge block computes 64 x 8 points with gathers along its normal axis
    for (int b = 0; b < eb; ++b) all.push_back({{g, 1, b, h->order}, 4 * 64 * 8});
  }
  if ((long long)all.size() > kMaxItems)
    return fail(SBP_EINVAL, "batch has %zu blocks of work, more than %d", all.size(), kMaxItems);
  for (const W& w : all) total += w.cost;
  seg.assign(9, 0);
  items.clear();
  std::size_t p = 0;
  long long acc = 0;
  for (int x = 0; x < 8; ++x) {
    seg[x] = (int)items.size();
    const long long goal = total * (x + 1) / 8;
    std::vector<W> part;
    while (p < all.size() && (acc < goal || x == 7)) {
      acc += all[p].cost;
      part.push_back(all[p++]);
    }
    std::stable_sort(part.begin(), part.end(), [](const W& a, const W& b) { return a.cost > b.cost; });
    for (const W& w : part) items.push_back(w.it);
  }
  seg[8] = (int)items.size();
  return SBP_OK;
}

// Static tables of a batched run from the current state of each handle:
// stage arguments (5 stages x 2 parities of the stage input), the work list
// (one launch over it) or group prefixes (one launch per order), source arguments (clock-driven,
// 5 stages x 2 parities), receiver arguments (2 step parities).
template <typename T>
struct BatchPlan {
  bool worklist = true;  // one launch over the work list (else one per order)
  unsigned orders = 0;   // bit o: interior order o present
  int maxseg = 0;        // longest work-list segment
  int npen = 0;          // surface nodes of all grids (penalty launch)
  int n = 0;             // grids
  int ngroups = 0;
  std::vector<int> gstart, ord, sblocks, eblocks;
  std::vector<int> withsrc, withrec;
  int nsrc = 0, nrec = 0;
};

template <typename T>
int batch_upload(sbp_ctx** hs, int n, const double* dt, bool rhs_only, BatchPlan<T>& P) {
  sbp_ctx* h0 = hs[0];
  hipStream_t st = h0->stream;
  const BatchRegion R = batch_region();
  char* base = h0->ws + h0->off_batch;
  bool buf_ok = true;
  for (int g = 0; g < n; ++g) {
    const StageArgs<T> a = stage_args<T>(hs[g]);
    buf_ok = buf_ok && !a.plain && 12.0 * (double)a.field * sizeof(T) < 4294967296.0;
    buf_ok = buf_ok && worklist_order_ok<T>(hs[g]->order);
  }
  P.worklist = buf_ok;
  P.n = n;
  P.orders = 0;
  for (int g = 0; g < n; ++g) P.orders |= 1u << hs[g]->order;
  // stage argument tables: entry (k, P) of handle g, P the parity of the stage
  // input relative to the handle's current buffer
  std::vector<StageArgs<T>> sa((std::size_t)10 * kMaxBatch);
  for (int g = 0; g < n; ++g) {
    sbp_ctx* h = hs[g];
    StageArgs<T> a = stage_args<T>(h);
    // the work list runs stage tiles and edge blocks in one launch: the edge
    // blocks gather the last column's closure inputs themselves; the sources
    // follow in source_kernel_batch
    a.eqc = nullptr;
    a.nsrc = 0;
    for (int k = 0; k < 5; ++k)
      for (int p = 0; p < 2; ++p)
        sa[(std::size_t)(k * 2 + p) * kMaxBatch + g] = stage_entry<T>(h, a, k, h->cur ^ p, dt[g], rhs_only);
  }
  // wait for work of an earlier call that may still read the tables
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpyAsync(base + R.stage, sa.data(), sa.size() * sizeof(StageArgs<T>), hipMemcpyHostToDevice, st));
  if (P.worklist) {
    std::vector<BatchItem> items;
    std::vector<int> seg;
    int rc = batch_items<T>(hs, n, items, seg);
    if (rc) return rc;
    P.maxseg = 0;
    for (int x = 0; x < 8; ++x) P.maxseg = std::max(P.maxseg, seg[x + 1] - seg[x]);
    HIPCHK(hipMemcpyAsync(base + R.items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + R.seg, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice, st));
  } else {
    // grouped launches: the stage and edge blocks of all grids of one order
    // per launch (block -> grid through prefix sums)
    P.ord.resize(n);
    for (int g = 0; g < n; ++g) P.ord[g] = g;
    std::stable_sort(P.ord.begin(), P.ord.end(), [&](int a, int b) { return hs[a]->order < hs[b]->order; });
    P.gstart.assign(1, 0);
    for (int q = 1; q < n; ++q)
      if (hs[P.ord[q]]->order != hs[P.ord[q - 1]]->order) P.gstart.push_back(q);
    P.ngroups = (int)P.gstart.size();
    P.gstart.push_back(n);
    if (P.ngroups > kMaxGroups) return fail(SBP_EINVAL, "too many interior orders in a batch");
    // the grouped kernels index the argument table in group order
    std::vector<StageArgs<T>> sg((std::size_t)10 * kMaxBatch);
    for (int e = 0; e < 10; ++e)
      for (int q = 0; q < n; ++q) sg[(std::size_t)e * kMaxBatch + q] = sa[(std::size_t)e * kMaxBatch + P.ord[q]];
    HIPCHK(hipMemcpyAsync(base + R.stage, sg.data(), sg.size() * sizeof(StageArgs<T>), hipMemcpyHostToDevice, st));
    std::vector<int> firsts((std::size_t)2 * kMaxGroups * (kMaxBatch + 1), 0);
    P.sblocks.assign(P.ngroups, 0);
    P.eblocks.assign(P.ngroups, 0);
    for (int G = 0; G < P.ngroups; ++G) {
      int* fs = firsts.data() + (std::size_t)(2 * G) * (kMaxBatch + 1);
      int* fe = firsts.data() + (std::size_t)(2 * G + 1) * (kMaxBatch + 1);
      int ts = 0, te = 0;
      for (int q = P.gstart[G]; q < P.gstart[G + 1]; ++q) {
        const StageArgs<T> a = stage_args<T>(hs[P.ord[q]]);
        fs[q - P.gstart[G]] = ts;
        fe[q - P.gstart[G]] = te;
        ts += a.ntiles;
        te += edge_blocks(a);
      }
      fs[P.gstart[G + 1] - P.gstart[G]] = ts;
      fe[P.gstart[G + 1] - P.gstart[G]] = te;
      P.sblocks[G] = ts;
      P.eblocks[G] = te;
    }
    HIPCHK(hipMemcpyAsync(base + R.first, firsts.data(), firsts.size() * sizeof(int), hipMemcpyHostToDevice, st));
  }
  // boundary penalties: surface nodes of every grid, in the order of the
  // stage argument table
  {
    std::vector<int> pfirst(n + 1, 0);
    for (int q = 0; q < n; ++q) {
      const sbp_ctx* h = hs[P.worklist ? q : P.ord[q]];
      pfirst[q + 1] = pfirst[q] + (int)surface_nodes(h->g.nq, h->g.nr, h->g.ns, q0_in_stage<T>());
    }
    P.npen = pfirst[n];
    HIPCHK(hipMemcpyAsync(base + R.pen_first, pfirst.data(), pfirst.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // the host tables are released on return
  }
  if (rhs_only) return SBP_OK;
  // sources: handles with sources, compacted; entry (k, P) of each; the
  // source-time factor from the clock's table, row (step, k) of n x
  // kMaxSources entries, this handle's at g * kMaxSources
  P.withsrc.clear();
  P.withrec.clear();
  for (int g = 0; g < n; ++g) {
    if (!hs[g]->src.empty()) P.withsrc.push_back(g);
    if (hs[g]->nrec > 0) P.withrec.push_back(g);
  }
  const StepClock* clk = (const StepClock*)(base + R.clock);
  std::vector<int> sfirst(P.withsrc.size() + 1, 0), rfirst(P.withrec.size() + 1, 0);
  for (std::size_t q = 0; q < P.withsrc.size(); ++q) sfirst[q + 1] = sfirst[q] + (int)hs[P.withsrc[q]]->src.size();
  for (std::size_t q = 0; q < P.withrec.size(); ++q) rfirst[q + 1] = rfirst[q] + hs[P.withrec[q]]->nrec;
  P.nsrc = sfirst.back();
  P.nrec = rfirst.back();
  std::vector<SourceArgs<T>> stab((std::size_t)10 * kMaxBatch);
  for (std::size_t q = 0; q < P.withsrc.size(); ++q) {
    const int g = P.withsrc[q];
    sbp_ctx* h = hs[g];
    for (int k = 0; k < 5; ++k)
      for (int p = 0; p < 2; ++p) {
        const int c = h->cur ^ p;  // parity of the stage input
        T* qout = (T*)(h->ws + (c ? h->off_qa : h->off_qb));
        SourceArgs<T> sarg = source_args<T>(h, k, dt[g], 0.0, false, qout);
        sarg.clock = clk;
        sarg.tab_stride = n * kMaxSources;
        sarg.tab_off = g * kMaxSources;
        stab[(std::size_t)(k * 2 + p) * kMaxBatch + q] = sarg;
      }
  }
  std::vector<RecordArgs<T>> rtab((std::size_t)2 * kMaxBatch);
  for (std::size_t q = 0; q < P.withrec.size(); ++q) {
    sbp_ctx* h = hs[P.withrec[q]];
    for (int par = 0; par < 2; ++par) {
      // state after a step of parity par: five stages flip the buffer
      const int c = h->cur ^ (par ^ 1);
      RecordArgs<T> r{};
      r.q = (const T*)(h->ws + (c ? h->off_qb : h->off_qa));
      r.field = h->field;
      r.off = (const long long*)(h->ws + h->off_rec);
      r.out = (T*)h->rec_out;
      r.base = h->rec_step;
      rtab[(std::size_t)par * kMaxBatch + q] = r;
    }
  }
  HIPCHK(hipMemcpyAsync(base + R.src, stab.data(), stab.size() * sizeof(SourceArgs<T>), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(base + R.src_first, sfirst.data(), sfirst.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(base + R.rec, rtab.data(), rtab.size() * sizeof(RecordArgs<T>), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(base + R.rec_first, rfirst.data(), rfirst.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // the host tables are released on return
  return SBP_OK;
}

// The boundary penalties of every grid of a batch (one launch), after the
// stage launches.
template <typename T>
int batch_penalty_launch(sbp_ctx** hs, const BatchPlan<T>& P, const StageArgs<T>* dsa, hipStream_t st) {
  const BatchRegion R = batch_region();
  BatchArgs<T> b{};
  b.args = dsa;
  b.first = (const int*)(hs[0]->ws + hs[0]->off_batch + R.pen_first);
  b.n = P.n;
  b.total = P.npen;
  HIPCHK(launch_penalty_batch<T>(b, st));
  return SBP_OK;
}

// One batched stage launch (all grids) for argument entry e = k * 2 + P.
template <typename T>
int batch_stage_launch(sbp_ctx** hs, const BatchPlan<T>& P, int k, int e, hipStream_t st) {
  sbp_ctx* h0 = hs[0];
  const BatchRegion R = batch_region();
  char* base = h0->ws + h0->off_batch;
  const StageArgs<T>* dsa = (const StageArgs<T>*)(base + R.stage) + (std::size_t)e * kMaxBatch;
  if (P.worklist) {
    PersistArgs<T> pa{};
    pa.args = dsa;
    pa.items = (const BatchItem*)(base + R.items);
    pa.seg = (const int*)(base + R.seg);
    HIPCHK(launch_stage_worklist<T>(pa, P.orders, 8 * P.maxseg, st));
    return batch_penalty_launch<T>(hs, P, dsa, st);
  }
  const int* dfirst = (const int*)(base + R.first);
  for (int G = 0; G < P.ngroups; ++G) {
    BatchArgs<T> b{};
    b.args = dsa + P.gstart[G];
    b.n = P.gstart[G + 1] - P.gstart[G];
    b.first = dfirst + (std::size_t)(2 * G) * (kMaxBatch + 1);
    b.total = P.sblocks[G];
    const int order = hs[P.ord[P.gstart[G]]]->order;
    HIPCHK(launch_stage_batch<T>(order, 8, b, false, st));
    b.first = dfirst + (std::size_t)(2 * G + 1) * (kMaxBatch + 1);
    b.total = P.eblocks[G];
    HIPCHK(launch_edge_batch<T>(order, b, st));
  }
  return batch_penalty_launch<T>(hs, P, dsa, st);
}

// The launches of one batched step of parity par (0: even step of the call)
// on stream st: per stage the batched stage launch and the sources, then the
// receivers and the clock tick.
template <typename T>
int batch_step_launches(sbp_ctx** hs, const BatchPlan<T>& P, int par, hipStream_t st) {
  sbp_ctx* h0 = hs[0];
  const BatchRegion R = batch_region();
  char* base = h0->ws + h0->off_batch;
  StepClock* clk = (StepClock*)(base + R.clock);
  for (int k = 0; k < 5; ++k) {
    const int e = k * 2 + ((par + k) & 1);
    int rc = batch_stage_launch<T>(hs, P, k, e, st);
    if (rc) return rc;
    if (P.nsrc > 0) {
      SourceBatch<T> sb{};
      sb.args = (const SourceArgs<T>*)(base + R.src) + (std::size_t)e * kMaxBatch;
      sb.first = (const int*)(base + R.src_first);
      sb.n = (int)P.withsrc.size();
      sb.total = P.nsrc;
      HIPCHK(launch_source_batch<T>(sb, st));
    }
  }
  if (P.nrec > 0) {
    RecordBatch<T> rb{};
    rb.args = (const RecordArgs<T>*)(base + R.rec) + (std::size_t)par * kMaxBatch;
    rb.first = (const int*)(base + R.rec_first);
    rb.n = (int)P.withrec.size();
    rb.total = P.nrec;
    rb.clock = clk;
    HIPCHK(launch_record_batch<T>(rb, st));
  }
  HIPCHK(launch_clock_tick(clk, st));
  return SBP_OK;
}

// Several handles advanced together.  Per Runge-Kutta stage one launch
// covers the stage tiles and edge blocks of every grid (a work list cut into
// one segment per XCD, longest items first; with plain addressing, one stage
// and one edge launch per interior order), then one launch injects every
// source; per step one launch records every receiver.  In FP32 each step is
// a replay of one of two graphs captured for the call (even and odd steps;
// the argument tables hold both ping-pong parities); the per-step values
// come from a device clock and a source-time table uploaded every
// kBatchTabSteps steps.  Results agree with do_steps to rounding (the bodies
// are the same, instantiated in another kernel).
template <typename T>
int do_steps_batch(sbp_ctx** hs, int n, int nsteps, const double* dt) {
  sbp_ctx* h0 = hs[0];
  hipStream_t st = h0->stream;
  const BatchRegion R = batch_region();
  char* base = h0->ws + h0->off_batch;
  BatchSettings keep(hs, n);
  int rc = batch_apply_L(hs, n, h0->batch_L);
  if (rc) return rc;
  BatchPlan<T> P;
  if ((rc = batch_upload<T>(hs, n, dt, false, P))) return rc;
  if (!h0->btab_host) {
    HIPCHK(hipHostMalloc((void**)&h0->btab_host, 2 * R.gtab_part, hipHostMallocDefault));
    for (int p = 0; p < 2; ++p) HIPCHK(hipEventCreateWithFlags(&h0->btab_ev[p], hipEventDisableTiming));
  }
  StepClock* clk = (StepClock*)(base + R.clock);
  std::vector<double> t0(n);
  for (int g = 0; g < n; ++g) t0[g] = hs[g]->t;
  // step graphs (even, odd), captured for this call
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  struct Drop {
    hipGraphExec_t* g;
    ~Drop() {
      for (int i = 0; i < 2; ++i)
        if (g[i]) (void)hipGraphExecDestroy(g[i]);
    }
  } drop{gx};
  // graphs replay only batched steps whose kernels use no scratch memory
  // (the FP32 kernels), as in do_steps
  const bool use_graph = h0->graphs && P.worklist && batch_step_scratch<T>(P.orders) == 0;
  if (use_graph) {
    if (!h0->cap) HIPCHK(hipStreamCreateWithFlags(&h0->cap, hipStreamNonBlocking));
    for (int par = 0; par < 2 && par < nsteps; ++par) {
      HIPCHK(hipStreamBeginCapture(h0->cap, hipStreamCaptureModeThreadLocal));
      rc = batch_step_launches<T>(hs, P, par, h0->cap);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(h0->cap, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail(SBP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
      const hipError_t e2 = hipGraphInstantiate(&gx[par], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) return fail(SBP_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    }
  }
  const std::size_t row = (std::size_t)n * kMaxSources;
  for (int n0 = 0; n0 < nsteps; n0 += kBatchTabSteps) {
    const int nc = std::min(kBatchTabSteps, nsteps - n0);
    const int part = h0->btab_next;
    h0->btab_next ^= 1;
    char* dtab = base + R.gtab + (std::size_t)part * R.gtab_part;
    if (P.nsrc > 0) {
      if (h0->btab_used[part]) HIPCHK(hipEventSynchronize(h0->btab_ev[part]));
      T* ht = (T*)(h0->btab_host + (std::size_t)part * R.gtab_part);
      for (int nn = 0; nn < nc; ++nn)
        for (int k = 0; k < 5; ++k)
          for (int g : P.withsrc) {
            const double tn = t0[g] + (n0 + nn) * dt[g];
            for (std::size_t q = 0; q < hs[g]->src.size(); ++q)
              ht[((std::size_t)nn * 5 + k) * row + (std::size_t)g * kMaxSources + q] =
                  (T)(dt[g] * stf_value(hs[g]->src[q], tn + kRkC[k] * dt[g]));
          }
      HIPCHK(hipMemcpyAsync(dtab, ht, (std::size_t)nc * 5 * row * sizeof(T), hipMemcpyHostToDevice, st));
      HIPCHK(hipEventRecord(h0->btab_ev[part], st));
      h0->btab_used[part] = true;
    }
    HIPCHK(launch_clock_set(clk, dtab, n0, st));
    for (int nn = 0; nn < nc; ++nn) {
      const int par = (n0 + nn) & 1;
      if (use_graph) {
        HIPCHK(hipGraphLaunch(gx[par], st));
      } else if ((rc = batch_step_launches<T>(hs, P, par, st))) {
        return rc;
      }
    }
  }
  // host-side state of every handle, as after nsteps calls of do_steps
  for (int g = 0; g < n; ++g) {
    sbp_ctx* h = hs[g];
    h->cur ^= nsteps & 1;
    h->steps += nsteps;
    if (h->nrec > 0) h->rec_step += nsteps;
    h->t = t0[g] + nsteps * dt[g];
  }
  // the graphs are destroyed on return: the work must be done
  HIPCHK(hipStreamSynchronize(st));
  return SBP_OK;
}

// Batch launch-shape autotuner: times `reps` right-hand-side evaluations of
// every grid (one batched stage launch each; they write only the
// Runge-Kutta registers and the second state buffers) for the cost model's
// chunk length and a few others, and keeps the fastest in every handle.
template <typename T>
int do_autotune_batch(sbp_ctx** hs, int n, int reps, int* bestL, double* best_ms) {
  sbp_ctx* h0 = hs[0];
  hipStream_t st = h0->stream;
  const BatchRegion R = batch_region();
  char* base = h0->ws + h0->off_batch;
  int nsmax = 0;
  for (int g = 0; g < n; ++g) nsmax = std::max(nsmax, hs[g]->g.ns);
  std::vector<int> cands;
  {
    BatchSettings keep(hs, n);
    int rc = batch_apply_L(hs, n, 0);
    if (rc) return rc;
    const int L0 = batch_cost_model_L(hs, n);
    for (int L : {L0, L0 * 3 / 4, L0 * 3 / 2, L0 * 2, nsmax})
      if (L >= 8 && std::find(cands.begin(), cands.end(), std::min(L, nsmax)) == cands.end())
        cands.push_back(std::min(L, nsmax));
  }
  std::vector<double> dts(n, 1.0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = -1;
  int bL = 0, rc = SBP_OK;
  for (int L : cands) {
    BatchSettings keep(hs, n);
    if ((rc = batch_apply_L(hs, n, L))) break;
    BatchPlan<T> P;
    if ((rc = batch_upload<T>(hs, n, dts.data(), true, P))) break;
    auto launch = [&]() -> int { return batch_stage_launch<T>(hs, P, 0, 0, st); };
    if ((rc = launch())) break;  // warm-up
    if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SBP_EHIP, "hipEventRecord failed"); break; }
    for (int r = 0; r < reps && rc == SBP_OK; ++r) rc = launch();
    if (rc) break;
    float ms = 0.f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = fail(SBP_EHIP, "event timing failed");
      break;
    }
    if (best < 0 || ms / reps < best) {
      best = ms / reps;
      bL = L;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  for (int g = 0; g < n; ++g) hs[g]->batch_L = bL;
  if (bestL) *bestL = bL;
  if (best_ms) *best_ms = best;
  return SBP_OK;
}

template <typename T>
int do_rhs(sbp_ctx* h, void* out, double t) {
  int rc = prepare_bounds(h);
  if (rc) return rc;
  StageArgs<T> a = stage_args<T>(h);
  T* qa = (T*)(h->ws + h->off_qa);
  T* qb = (T*)(h->ws + h->off_qb);
  T* qin = h->cur ? qb : qa;
  T* qout = h->cur ? qa : qb;
  rc = run_stage<T>(h, a, 0, 1.0, t, true, qin, qout, h->stream, nullptr);
  if (rc) return rc;
  return copy_out(h, out, h->ws + h->off_dq, 9, hipMemcpyDeviceToDevice);
}

template <typename T>
int do_energy(sbp_ctx* h, double* E) {
  EnergyArgs<T> e{};
  const Geometry& g = h->g;
  e.q = (const T*)(h->ws + (h->cur ? h->off_qb : h->off_qa));
  e.coef = (const T*)(h->ws + h->off_coef);
  e.part = (double*)(h->ws + h->off_part);
  e.nm = h->nm;
  e.plane = h->plane;
  e.field = h->field;
  e.px = h->px;
  e.nq = g.nq;
  e.nr = g.nr;
  e.ns = g.ns;
  e.m = h->cl.m;
  e.h[0] = 1.0 / (g.nq - 1);
  e.h[1] = 1.0 / (g.nr - 1);
  e.h[2] = 1.0 / (g.ns - 1);
  for (int i = 0; i < kMaxM; ++i) e.w[i] = h->cl.w[i];
  const int nb = (int)std::min<std::size_t>(kMaxPart, (g.n + 255) / 256);
  HIPCHK(launch_energy<T>(e, nb, h->stream));
  std::vector<double> part(nb);
  HIPCHK(hipMemcpyAsync(part.data(), e.part, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double s = 0;
  for (double v : part) s += v;
  *E = s;
  if (!std::isfinite(s)) return fail(SBP_EUNSTABLE, "energy is not finite");
  return SBP_OK;
}

}  // namespace

// ============================================================================
namespace {

// Launch-shape autotuner: times `reps` right-hand-side evaluations (stage and
// edge kernel, sources off) for each candidate tile height and number of
// s-chunks and keeps the fastest.  A right-hand-side evaluation writes only
// the Runge-Kutta register and the second state buffer, which hold nothing
// between steps, so the state is untouched.
template <typename T>
int do_autotune(sbp_ctx* h, int reps, int* best_ty, int* best_zchunk, double* best_ms) {
  std::vector<int> tys{8};
  if (sizeof(T) == 4 && h->order <= 7) tys.push_back(16);  // 16-row order-8 tiles exceed the LDS
  const std::vector<Src> saved = h->src;
  h->src.clear();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = -1.0;
  int bty = h->ty, bzc = h->zchunk;
  int rc = SBP_OK;
  for (int ty : tys) {
    if (ty < h->cl.m) continue;
    // the cost model's chunk count, and one fewer / more chunks
    h->ty = ty;
    h->zchunk = 0;
    h->bounds_dirty = true;
    if ((rc = prepare_bounds(h))) break;
    const int nz0 = h->nzc;
    for (int nz = std::max(1, nz0 - 1); nz <= nz0 + 1 && rc == SBP_OK; ++nz) {
      h->ty = ty;
      h->zchunk = (h->g.ns + nz - 1) / nz;
      h->bounds_dirty = true;
      if ((rc = prepare_bounds(h))) break;
      StageArgs<T> a = stage_args<T>(h);
      T* qa = (T*)(h->ws + h->off_qa);
      T* qb = (T*)(h->ws + h->off_qb);
      T* qin = h->cur ? qb : qa;
      T* qout = h->cur ? qa : qb;
      if ((rc = run_stage<T>(h, a, 0, 1.0, h->t, true, qin, qout, h->stream, nullptr))) break;  // warm-up
      if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = fail(SBP_EHIP, "hipEventRecord failed"); break; }
      for (int r = 0; r < reps && rc == SBP_OK; ++r)
        rc = run_stage<T>(h, a, 0, 1.0, h->t, true, qin, qout, h->stream, nullptr);
      if (rc) break;
      float ms = 0.f;
      if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = fail(SBP_EHIP, "event timing failed");
        break;
      }
      const double per = ms / reps;
      if (best < 0 || per < best) {
        best = per;
        bty = ty;
        bzc = h->zchunk;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->src = saved;
  h->ty = bty;
  h->zchunk = bzc;
  h->bounds_dirty = true;
  if (rc) return rc;
  if (best_ty) *best_ty = bty;
  if (best_zchunk) *best_zchunk = bzc;
  if (best_ms) *best_ms = best;
  return SBP_OK;
}

// ---- discrete adjoint ---------------------------------------------------------
// Layout of the caller's adjoint workspace (byte offsets): checkpoints of the
// state every `every` steps, the state and the inputs of stages 2-5 of every
// step of one block of steps, the stage outputs of one step, the forward
// Runge-Kutta register, the adjoint state and register, W^{-1} dQb, a
// right-hand-side buffer, the unit-material coefficients, J and the three
// gradient fields.
struct AdjLayout {
  std::size_t ck = 0, blk = 0, st = 0, dqs = 0, qb = 0, dqb = 0, y = 0, r = 0, cu = 0, jac = 0, grad = 0, total = 0;
  int nck = 0, every = 0;
};

AdjLayout adj_layout(const sbp_ctx* h, int nsteps, int every) {
  AdjLayout L;
  const std::size_t F = h->field * h->esize;
  L.every = nsteps > 0 ? std::max(1, std::min(every, nsteps)) : 0;
  L.nck = nsteps > 0 ? (nsteps + L.every - 1) / L.every : 0;
  std::size_t o = 0;
  auto take = [&](std::size_t bytes) {
    std::size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.ck = take((std::size_t)L.nck * 9 * F);
  L.blk = take((std::size_t)L.every * 5 * 9 * F);
  L.st = take(5 * 9 * F);
  L.dqs = take(9 * F);
  L.qb = take(9 * F);
  L.dqb = take(9 * F);
  L.y = take(9 * F);
  L.r = take(9 * F);
  L.cu = take(kNumCoef * F);
  L.jac = take(F);
  L.grad = take(3 * F);
  L.total = o;
  return L;
}

// One Runge-Kutta stage (or right-hand side) with explicit buffers and
// coefficient array; sat = false leaves the boundary penalties out.
template <typename T>
int stage_explicit(sbp_ctx* h, const StageArgs<T>& base, int k, double dt, double tstage, const T* qin, T* qout,
                   T* dq, bool rhs_only, const T* coef, bool sat, bool sources) {
  StageArgs<T> b = base;
  b.qin = qin;
  b.qout = qout;
  b.dq = dq;
  b.read_dq = (!rhs_only && k > 0) ? 1 : 0;
  b.Ak = rhs_only ? T(0) : (T)kRkA[k];
  b.Bk = rhs_only ? T(0) : (T)kRkB[k];
  b.dt = rhs_only ? T(1) : (T)dt;
  b.coef = coef;
  b.sat = sat ? 1 : 0;
  const bool fused = sources && fuse_sources<T>(h, b, k, dt, tstage, rhs_only, nullptr);
  if (!sources) b.nsrc = 0;
  HIPCHK(launch_stage<T>(h->order, h->ty, b, h->stream));
  HIPCHK(edge_and_penalties<T>(h, b, h->stream));
  if (sources && !fused && !h->src.empty()) {
    SourceArgs<T> s = source_args<T>(h, k, dt, tstage, rhs_only, qout);
    s.dq = dq;
    HIPCHK(launch_source<T>(s, (int)h->src.size(), h->stream));
  }
  return SBP_OK;
}

// One step q0 -> q1 at time tn; the inputs of stages 1..4 land in S[0..3].
template <typename T>
int step_explicit(sbp_ctx* h, const StageArgs<T>& base, double tn, double dt, const T* q0, T* const S[4], T* q1,
                  T* dq) {
  const T* in = q0;
  for (int k = 0; k < 5; ++k) {
    T* out = k < 4 ? S[k] : q1;
    int rc = stage_explicit<T>(h, base, k, dt, tn + kRkC[k] * dt, in, out, dq, false, base.coef, true, true);
    if (rc) return rc;
    in = out;
  }
  return SBP_OK;
}

template <typename T>
AdjArgs<T> adj_args(sbp_ctx* h, char* adj, const AdjLayout& L) {
  AdjArgs<T> a{};
  const Geometry& g = h->g;
  a.nm = h->nm;
  a.field = h->field;
  a.nq = g.nq;
  a.nr = g.nr;
  a.ns = g.ns;
  a.m = h->cl.m;
  for (int i = 0; i < kMaxM; ++i) a.w[i] = (T)h->cl.w[i];
  a.h[0] = (T)(1.0 / (g.nq - 1));
  a.h[1] = (T)(1.0 / (g.nr - 1));
  a.h[2] = (T)(1.0 / (g.ns - 1));
  a.coef = (const T*)(h->ws + h->off_coef);
  a.face = (const T*)h->ws;
  for (int f = 0; f < 6; ++f) {
    a.face_off[f] = h->off_face[f] / sizeof(T);
    a.face_n[f] = h->face_n[f];
    a.gamma[f] = (T)h->gamma[f];
    a.traction[f] = (h->sat_variant == SBP_SAT_TRACTION && h->gamma[f] == 1.0) ? 1 : 0;
  }
  a.qb = (T*)(adj + L.qb);
  a.dqb = (T*)(adj + L.dqb);
  a.y = (T*)(adj + L.y);
  a.r = (const T*)(adj + L.r);
  a.jac = (const T*)(adj + L.jac);
  a.grad = (T*)(adj + L.grad);
  return a;
}

int check_adj_ws(const void* adj, std::size_t bytes, std::size_t need) {
  if (!adj) return fail(SBP_EINVAL, "NULL adjoint workspace");
  if ((std::uintptr_t)adj % 256) return fail(SBP_EINVAL, "adjoint workspace must be 256-byte aligned");
  if (bytes < need) return fail(SBP_ENOMEM, "adjoint workspace too small: %zu < %zu bytes", bytes, need);
  return SBP_OK;
}

// out = L^T lam (dense 9 fields in, dense 9 fields out)
template <typename T>
int do_adjoint_rhs(sbp_ctx* h, const void* lam, void* out, char* adj) {
  int rc = prepare_bounds(h);
  if (rc) return rc;
  const AdjLayout L = adj_layout(h, 0, 1);
  const StageArgs<T> base = stage_args<T>(h);
  AdjArgs<T> a = adj_args<T>(h, adj, L);
  if ((rc = copy_in(h, adj + L.dqb, lam, 9, hipMemcpyDeviceToDevice))) return rc;
  HIPCHK(launch_fill<T>(a.qb, 9 * h->field, T(0), h->stream));
  a.a = T(1);
  a.b = T(0);
  a.dt = T(1);
  HIPCHK(launch_adj_pre<T>(a, h->stream));
  if ((rc = stage_explicit<T>(h, base, 0, 1.0, 0.0, a.y, (T*)(adj + L.st), (T*)(adj + L.r), true, base.coef, false,
                              false)))
    return rc;
  HIPCHK(launch_adj_post<T>(a, h->stream));
  return copy_out(h, out, adj + L.qb, 9, hipMemcpyDeviceToDevice);
}

// Reverse sweep of the misfit gradient over nsteps steps of size dt that
// started at time t0, from the checkpoints in the adjoint workspace: block by
// block from the end, each block recomputed from its checkpoint (keeping every
// stage input of the block), then the reverse stages.
template <typename T>
int adj_reverse(sbp_ctx* h, int nsteps, double dt, double t0, const T* res, const AdjLayout& L, char* adj,
                void* grad_out, void* qbar_out) {
  int rc = prepare_bounds(h);
  if (rc) return rc;
  const StageArgs<T> base = stage_args<T>(h);
  AdjArgs<T> a = adj_args<T>(h, adj, L);
  const std::size_t F9 = 9 * h->field;
  const T* ck = (const T*)(adj + L.ck);
  T* blk = (T*)(adj + L.blk);
  T* spare = (T*)(adj + L.st) + 4 * F9;
  T* dqs = (T*)(adj + L.dqs);
  T* rbuf = (T*)(adj + L.r);
  T* cu = (T*)(adj + L.cu);
  const std::size_t bytes9 = F9 * sizeof(T);

  // unit material (lambda/J = 0, mu/J = 1, 1/(rho J) = 1), J, zeroed accumulators
  HIPCHK(hipMemcpyAsync(cu, h->ws + h->off_coef, 9 * h->field * sizeof(T), hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(launch_fill<T>(cu + 9 * h->field, h->field, T(0), h->stream));
  HIPCHK(launch_fill<T>(cu + 10 * h->field, 2 * h->field, T(1), h->stream));
  {
    std::vector<T> jt(h->g.n);
    for (std::size_t o = 0; o < h->g.n; ++o) jt[o] = (T)h->J[o];
    if ((rc = copy_in(h, adj + L.jac, jt.data(), 1, hipMemcpyHostToDevice))) return rc;
  }
  HIPCHK(launch_fill<T>(a.qb, F9, T(0), h->stream));
  HIPCHK(launch_fill<T>(a.grad, 3 * h->field, T(0), h->stream));
  const long long* roff = (const long long*)(h->ws + h->off_rec);

  for (int c = L.nck - 1; c >= 0; --c) {
    const int n0 = c * L.every, n1 = std::min(nsteps, n0 + L.every);
    // slot n - n0 of the block: the state of step n, then its stage inputs 2-5
    auto slot = [&](int n) { return blk + (std::size_t)(n - n0) * 5 * F9; };
    HIPCHK(hipMemcpyAsync(blk, ck + (std::size_t)c * F9, bytes9, hipMemcpyDeviceToDevice, h->stream));
    for (int n = n0; n < n1; ++n) {
      T* const Sn[4] = {slot(n) + F9, slot(n) + 2 * F9, slot(n) + 3 * F9, slot(n) + 4 * F9};
      if ((rc = step_explicit<T>(h, base, t0 + n * dt, dt, slot(n), Sn, n + 1 < n1 ? slot(n + 1) : spare, dqs)))
        return rc;
    }
    for (int n = n1 - 1; n >= n0; --n) {
      HIPCHK(launch_adj_inject<T>(a.qb, h->field, roff, h->nrec, res + (std::size_t)n * h->nrec * 3, h->stream));
      for (int k = 4; k >= 0; --k) {
        a.a = k == 4 ? T(0) : (T)kRkA[k + 1];
        a.b = (T)kRkB[k];
        a.dt = (T)dt;
        HIPCHK(launch_adj_pre<T>(a, h->stream));
        if ((rc = stage_explicit<T>(h, base, 0, 1.0, 0.0, a.y, spare, rbuf, true, base.coef, false, false))) return rc;
        HIPCHK(launch_adj_post<T>(a, h->stream));
        const T* qs = slot(n) + (std::size_t)k * F9;
        if ((rc = stage_explicit<T>(h, base, 0, 1.0, 0.0, qs, spare, rbuf, true, cu, false, false))) return rc;
        a.qs = qs;
        HIPCHK(launch_adj_grad<T>(a, h->stream));
      }
    }
  }
  if ((rc = copy_out(h, grad_out, adj + L.grad, 3, hipMemcpyDeviceToDevice))) return rc;
  if (qbar_out && (rc = copy_out(h, qbar_out, adj + L.qb, 9, hipMemcpyDeviceToDevice))) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  return SBP_OK;
}

// Misfit gradient: a forward run of nsteps from the current state that keeps
// checkpoints (receivers not recorded), then the reverse sweep.
template <typename T>
int do_gradient(sbp_ctx* h, int nsteps, double dt, const T* res, int every, char* adj, void* grad_out,
                void* qbar_out) {
  int rc = prepare_bounds(h);
  if (rc) return rc;
  const AdjLayout L = adj_layout(h, nsteps, every);
  const StageArgs<T> base = stage_args<T>(h);
  const std::size_t F9 = 9 * h->field;
  T* ck = (T*)(adj + L.ck);
  T* st = (T*)(adj + L.st);
  T* const S[4] = {st, st + F9, st + 2 * F9, st + 3 * F9};
  T* dqs = (T*)(adj + L.dqs);
  T* state = (T*)(h->ws + (h->cur ? h->off_qb : h->off_qa));
  const double t0 = h->t;
  const std::size_t bytes9 = F9 * sizeof(T);
  h->ck_valid = false;
  // forward pass with checkpoints (ping-pong through the y and r buffers)
  T* X = (T*)(adj + L.y);
  T* Y = (T*)(adj + L.r);
  HIPCHK(hipMemcpyAsync(X, state, bytes9, hipMemcpyDeviceToDevice, h->stream));
  for (int n = 0; n < nsteps; ++n) {
    if (n % L.every == 0)
      HIPCHK(hipMemcpyAsync(ck + (std::size_t)(n / L.every) * F9, X, bytes9, hipMemcpyDeviceToDevice, h->stream));
    if ((rc = step_explicit<T>(h, base, t0 + n * dt, dt, X, S, Y, dqs))) return rc;
    std::swap(X, Y);
  }
  HIPCHK(hipMemcpyAsync(state, X, bytes9, hipMemcpyDeviceToDevice, h->stream));
  if ((rc = adj_reverse<T>(h, nsteps, dt, t0, res, L, adj, grad_out, qbar_out))) return rc;
  h->t = t0 + nsteps * dt;
  h->steps += nsteps;
  return SBP_OK;
}

// sbp_step with checkpoints kept for a later sbp_gradient_from_checkpoints
template <typename T>
int do_step_checkpointed(sbp_ctx* h, int nsteps, double dt, int every, char* adj) {
  const AdjLayout L = adj_layout(h, nsteps, every);
  const std::size_t F9 = 9 * h->field;
  const std::size_t bytes9 = F9 * sizeof(T);
  h->ck_valid = false;
  const double t0 = h->t;
  const long long s0 = h->steps;
  for (int n = 0; n < nsteps; ++n) {
    if (n % L.every == 0) {
      const T* state = (const T*)(h->ws + (h->cur ? h->off_qb : h->off_qa));
      HIPCHK(hipMemcpyAsync(adj + L.ck + (std::size_t)(n / L.every) * bytes9, state, bytes9, hipMemcpyDeviceToDevice,
                            h->stream));
    }
    h->t = t0 + n * dt;  // the stage times of sbp_step(h, nsteps, dt)
    int rc = do_steps<T>(h, 1, dt);
    if (rc) return rc;
  }
  h->t = t0 + nsteps * dt;
  h->ck_valid = true;
  h->ck_id = ++h->ck_next;
  h->ck_ws = adj;
  h->ck_nsteps = nsteps;
  h->ck_every = every;
  h->ck_dt = dt;
  h->ck_t0 = t0;
  h->ck_steps = s0 + nsteps;
  return SBP_OK;
}

}  // namespace

extern "C" {

const char* sbp_last_error(void) { return g_err.c_str(); }

int sbp_workspace_bytes(int nq, int nr, int ns, int order, int dtype, size_t* bytes) {
  if (!bytes) return fail(SBP_EINVAL, "bytes is NULL");
  int rc = check_dims(nq, nr, ns, order, dtype);
  if (rc) return rc;
  sbp_ctx tmp;
  tmp.esize = dtype == SBP_F32 ? 4 : 8;
  tmp.g = Geometry{nq, nr, ns, (std::size_t)nq * nr * ns};
  layout(&tmp);
  *bytes = tmp.total;
  return SBP_OK;
}

int sbp_init_grid(sbp_handle* out, int nq, int nr, int ns, const double* xyz, int order, int dtype,
                  const double* gamma, int sat_variant, void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return fail(SBP_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_dims(nq, nr, ns, order, dtype);
  if (rc) return rc;
  if (!gamma) return fail(SBP_EINVAL, "gamma is NULL");
  for (int f = 0; f < 6; ++f)
    if (!(gamma[f] >= -1.0 && gamma[f] <= 1.0)) return fail(SBP_EINVAL, "gamma[%d] = %g outside [-1, 1]", f, gamma[f]);
  if (sat_variant != SBP_SAT_CHARACTERISTIC && sat_variant != SBP_SAT_TRACTION)
    return fail(SBP_EINVAL, "unknown sat_variant %d", sat_variant);
  if (!workspace) return fail(SBP_EINVAL, "workspace is NULL");
  if ((reinterpret_cast<std::uintptr_t>(workspace) & 255) != 0) return fail(SBP_EINVAL, "workspace not 256-byte aligned");
  sbp_ctx* h = new sbp_ctx();
  h->order = order;
  h->dtype = dtype;
  h->esize = dtype == SBP_F32 ? 4 : 8;
  h->g = Geometry{nq, nr, ns, (std::size_t)nq * nr * ns};
  for (int f = 0; f < 6; ++f) h->gamma[f] = gamma[f];
  h->sat_variant = sat_variant;
  h->stream = (hipStream_t)stream;
  h->ws = (char*)workspace;
  h->ws_bytes = workspace_bytes;
  h->width = 2 * (order / 2 + 1);
  layout(h);
  if (workspace_bytes < h->total) {
    std::size_t need = h->total;
    delete h;
    return fail(SBP_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  }
  const char* err = "";
  if (!build_closure(order, &h->cl, &err)) {
    delete h;
    return fail(SBP_EINVAL, "closure construction failed: %s", err);
  }
  {
    // closure rows: h D+ and h D- at the left end, then their negatives,
    // which are the right-end rows of h D+ and h D- against reversed columns
    std::vector<double> tab((std::size_t)kClosureTab * kMaxM * kMaxCols, 0.0);
    for (int r = 0; r < kMaxM; ++r)
      for (int c = 0; c < kMaxCols; ++c) {
        const std::size_t o = (std::size_t)r * kMaxCols + c;
        tab[0 * kMaxM * kMaxCols + o] = h->cl.dp[r][c];
        tab[1 * kMaxM * kMaxCols + o] = h->cl.dm[r][c];
        tab[2 * kMaxM * kMaxCols + o] = -h->cl.dm[r][c];
        tab[3 * kMaxM * kMaxCols + o] = -h->cl.dp[r][c];
      }
    rc = upload_vec(h, h->off_tab, tab);
    if (rc) {
      std::string keep = g_err;
      delete h;
      g_err = keep;
      return rc;
    }
  }
  // zero the state buffers and the Runge-Kutta register; pinned staging of
  // the source-time tables and one event per part
  hipError_t e = hipMemsetAsync(h->ws, 0, h->off_coef, h->stream);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->tab_host, kTabParts * h->tab_part_bytes, hipHostMallocDefault);
  for (int p = 0; p < kTabParts && e == hipSuccess; ++p)
    e = hipEventCreateWithFlags(&h->tab_ev[p], hipEventDisableTiming);
  if (e != hipSuccess) {
    sbp_destroy(h);
    return fail(SBP_EHIP, "set-up: %s", hipGetErrorString(e));
  }
  rc = compute_metrics(h, xyz);
  if (rc) {
    std::string keep = g_err;
    sbp_destroy(h);
    g_err = keep;
    return rc;
  }
  *out = h;
  return SBP_OK;
}

int sbp_set_material(sbp_handle h, const double* rho, const double* cp, const double* cs) {
  if (!h || !rho || !cp || !cs) return fail(SBP_EINVAL, "NULL argument");
  h->ck_valid = false;
  const Geometry& g = h->g;
  const std::size_t n = g.n;
  std::vector<double> lamJ(n), muJ(n), rJ(n);
  for (std::size_t o = 0; o < n; ++o) {
    const double mu = rho[o] * cs[o] * cs[o];
    const double lam = rho[o] * cp[o] * cp[o] - 2.0 * mu;
    if (!(rho[o] > 0) || !(mu > 0) || !(3 * lam + 2 * mu > 0))
      return fail(SBP_EINVAL, "material not positive definite at node %zu", o);
    lamJ[o] = lam / h->J[o];
    muJ[o] = mu / h->J[o];
    rJ[o] = 1.0 / (rho[o] * h->J[o]);
  }
  int rc;
  if ((rc = upload(h, h->off_coef + 9 * h->field * h->esize, lamJ.data()))) return rc;
  if ((rc = upload(h, h->off_coef + 10 * h->field * h->esize, muJ.data()))) return rc;
  if ((rc = upload(h, h->off_coef + 11 * h->field * h->esize, rJ.data()))) return rc;
  // face penalty coefficients
  for (int f = 0; f < 6; ++f) {
    const int xi = f / 2, side = f % 2;
    const std::size_t fn = h->face_n[f];
    const int N = xi == 0 ? g.nq : (xi == 1 ? g.nr : g.ns);
    const double hw0 = h->cl.w[0] / (N - 1);
    std::vector<double> fc(kNumFaceCoef * fn);
    std::size_t a = 0;
    auto node = [&](std::size_t idx) {
      const double M0 = h->Mface[f][idx], M1 = h->Mface[f][fn + idx], M2 = h->Mface[f][2 * fn + idx];
      std::size_t o;
      if (xi == 0) o = g.idx(side ? g.nq - 1 : 0, (int)(idx % g.nr), (int)(idx / g.nr));
      else if (xi == 1) o = g.idx((int)(idx % g.nq), side ? g.nr - 1 : 0, (int)(idx / g.nq));
      else o = g.idx((int)(idx % g.nq), (int)(idx / g.nq), side ? g.ns - 1 : 0);
      const double nrm = std::sqrt(M0 * M0 + M1 * M1 + M2 * M2);
      const double kappa = nrm / (h->J[o] * hw0);
      const double mu = rho[o] * cs[o] * cs[o];
      const double lam = rho[o] * cp[o] * cp[o] - 2.0 * mu;
      const double zp = rho[o] * cp[o], zs = rho[o] * cs[o];
      fc[FN_X * fn + idx] = M0 / nrm;
      fc[FN_Y * fn + idx] = M1 / nrm;
      fc[FN_Z * fn + idx] = M2 / nrm;
      fc[F_ZP * fn + idx] = zp;
      fc[F_ZS * fn + idx] = zs;
      fc[F_IZP * fn + idx] = 1.0 / zp;
      fc[F_IZS * fn + idx] = 1.0 / zs;
      fc[F_KR * fn + idx] = kappa / rho[o];
      fc[F_KL * fn + idx] = kappa * lam;
      fc[F_KM * fn + idx] = kappa * mu;
    };
    for (a = 0; a < fn; ++a) node(a);
    if ((rc = upload_vec(h, h->off_face[f], fc))) return rc;
  }
  h->have_material = true;
  return SBP_OK;
}

int sbp_add_source(sbp_handle h, const double* xi, const double* M, int stf, double param, double t0) {
  if (!h || !xi || !M) return fail(SBP_EINVAL, "NULL argument");
  h->ck_valid = false;
  if ((int)h->src.size() >= kMaxSources) return fail(SBP_EINVAL, "at most %d sources", kMaxSources);
  if (stf != SBP_STF_RICKER && stf != SBP_STF_EXPT) return fail(SBP_EINVAL, "unknown source-time function");
  if (!(param > 0)) return fail(SBP_EINVAL, "source parameter must be positive");
  for (int a = 0; a < 3; ++a)
    if (!(xi[a] >= 0.0 && xi[a] <= 1.0)) return fail(SBP_EINVAL, "source outside the block");
  const Geometry& g = h->g;
  const int w = h->width;
  int start[3];
  double d[3][kMaxSrcWidth];
  for (int ax = 0; ax < 3; ++ax) {
    const int N = g.len(ax);
    const double u = xi[ax] * (N - 1);
    start[ax] = delta_window(N, w, u);
    lagrange_basis(w, start[ax], u, d[ax], nullptr);
    for (int a = 0; a < w; ++a) {
      const int node = start[ax] + a;
      double Hw = 1.0;
      if (node < h->cl.m) Hw = h->cl.w[node];
      else if (node >= N - h->cl.m) Hw = h->cl.w[N - 1 - node];
      d[ax][a] /= Hw / (N - 1);
    }
  }
  const std::size_t per = (std::size_t)kMaxSrcWidth * kMaxSrcWidth * kMaxSrcWidth * 6;
  std::vector<double> wm(per, 0.0);
  for (int c = 0; c < w; ++c)
    for (int b = 0; b < w; ++b)
      for (int a = 0; a < w; ++a) {
        const int t = (c * w + b) * w + a;
        const double wt = d[0][a] * d[1][b] * d[2][c] / h->J[g.idx(start[0] + a, start[1] + b, start[2] + c)];
        for (int f = 0; f < 6; ++f) wm[(std::size_t)t * 6 + f] = wt * M[f];
      }
  const std::size_t off = h->off_src + h->src.size() * per * h->esize;
  int rc = upload_vec(h, off, wm);
  if (rc) return rc;
  Src s;
  s.i0 = start[0];
  s.j0 = start[1];
  s.k0 = start[2];
  for (int f = 0; f < 6; ++f) s.M[f] = M[f];
  s.stf = stf;
  s.param = param;
  s.t0 = t0;
  h->src.push_back(s);
  ++h->gen;
  return SBP_OK;
}

int sbp_locate(sbp_handle h, const double* x, double* xi) {
  if (!h || !x || !xi) return fail(SBP_EINVAL, "NULL argument");
  double res = 0.0;
  const int r = locate_point(h->g, h->X.data(), h->width, x, xi, &res);
  if (r == 1) return fail(SBP_EINVAL, "point (%g, %g, %g) lies outside the block", x[0], x[1], x[2]);
  if (r != 0) return fail(SBP_EINVAL, "the map could not be inverted at (%g, %g, %g)", x[0], x[1], x[2]);
  return SBP_OK;
}

int sbp_add_source_at(sbp_handle h, const double* x, const double* M, int stf, double param, double t0) {
  if (!h || !x || !M) return fail(SBP_EINVAL, "NULL argument");
  double xi[3];
  const int rc = sbp_locate(h, x, xi);
  if (rc) return rc;
  return sbp_add_source(h, xi, M, stf, param, t0);
}

int sbp_clear_sources(sbp_handle h) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  h->ck_valid = false;
  h->src.clear();
  ++h->gen;
  return SBP_OK;
}

int sbp_set_state(sbp_handle h, const void* q, int q_is_device, double t) {
  if (!h || !q) return fail(SBP_EINVAL, "NULL argument");
  h->ck_valid = false;
  char* dst = h->ws + (h->cur ? h->off_qb : h->off_qa);
  int rc = copy_in(h, dst, q, 9, q_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
  if (rc) return rc;
  if (!q_is_device) HIPCHK(hipStreamSynchronize(h->stream));
  h->t = t;
  return SBP_OK;
}

int sbp_get_state(sbp_handle h, void* q, int q_is_device, double* t_out) {
  if (!h || !q) return fail(SBP_EINVAL, "NULL argument");
  const char* src = h->ws + (h->cur ? h->off_qb : h->off_qa);
  int rc = copy_out(h, q, src, 9, q_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
  if (rc) return rc;
  if (!q_is_device) HIPCHK(hipStreamSynchronize(h->stream));
  if (t_out) *t_out = h->t;
  return SBP_OK;
}

int sbp_record(sbp_handle h, int nrec, const int* ijk, void* out_device, int max_steps) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (nrec < 0 || nrec > kMaxRec) return fail(SBP_EINVAL, "nrec must be in [0, %d]", kMaxRec);
  // checkpoints belong to the receivers they were taken with
  h->ck_valid = false;
  ++h->gen;
  if (nrec == 0) {
    h->nrec = 0;
    return SBP_OK;
  }
  if (!ijk || !out_device || max_steps <= 0) return fail(SBP_EINVAL, "invalid receiver arguments");
  const Geometry& g = h->g;
  std::vector<long long> off(nrec);
  for (int r = 0; r < nrec; ++r) {
    const int i = ijk[3 * r], j = ijk[3 * r + 1], k = ijk[3 * r + 2];
    if (i < 0 || i >= g.nq || j < 0 || j >= g.nr || k < 0 || k >= g.ns)
      return fail(SBP_EINVAL, "receiver %d outside the grid", r);
    off[r] = h->nm(i, j, k);
  }
  HIPCHK(hipMemcpyAsync(h->ws + h->off_rec, off.data(), nrec * sizeof(long long), hipMemcpyHostToDevice,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->nrec = nrec;
  h->rec_out = out_device;
  h->rec_max = max_steps;
  h->rec_step = 0;
  return SBP_OK;
}

int sbp_step(sbp_handle h, int nsteps, double dt) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called");
  if (nsteps < 0 || !(dt > 0) || !std::isfinite(dt)) return fail(SBP_EINVAL, "need nsteps >= 0 and dt > 0");
  if (h->nrec > 0 && h->rec_step + nsteps > h->rec_max)
    return fail(SBP_EINVAL, "receiver buffer holds %d steps; %lld recorded, %d requested", h->rec_max,
                h->rec_step, nsteps);
  return h->dtype == SBP_F32 ? do_steps<float>(h, nsteps, dt) : do_steps<double>(h, nsteps, dt);
}

// validation shared by the batch entry points (dt may be NULL)
static int check_batch(sbp_handle* hs, int n, const double* dt) {
  if (!hs) return fail(SBP_EINVAL, "NULL argument");
  if (n < 1 || n > kMaxBatch) return fail(SBP_EINVAL, "n must be in [1, %d]", kMaxBatch);
  for (int g = 0; g < n; ++g) {
    sbp_ctx* h = hs[g];
    if (!h) return fail(SBP_EINVAL, "NULL handle in batch (%d)", g);
    for (int e = 0; e < g; ++e)
      if (hs[e] == h) return fail(SBP_EINVAL, "handle %d appears twice in the batch", g);
    if (h->dtype != hs[0]->dtype) return fail(SBP_EINVAL, "all handles of a batch need the same dtype");
    if (h->stream != hs[0]->stream) return fail(SBP_EINVAL, "all handles of a batch need the same stream");
    if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called (handle %d)", g);
    if (dt && (!(dt[g] > 0) || !std::isfinite(dt[g]))) return fail(SBP_EINVAL, "need dt > 0 (handle %d)", g);
  }
  return SBP_OK;
}

int sbp_autotune_batch(sbp_handle* hs, int n, int reps, int* zchunk, double* ms) {
  int rc = check_batch(hs, n, nullptr);
  if (rc) return rc;
  if (reps < 1) return fail(SBP_EINVAL, "reps must be >= 1");
  return hs[0]->dtype == SBP_F32 ? do_autotune_batch<float>(hs, n, reps, zchunk, ms)
                                 : do_autotune_batch<double>(hs, n, reps, zchunk, ms);
}

int sbp_step_batch(sbp_handle* hs, int n, int nsteps, const double* dt) {
  if (!hs || !dt) return fail(SBP_EINVAL, "NULL argument");
  if (n < 1 || n > kMaxBatch) return fail(SBP_EINVAL, "n must be in [1, %d]", kMaxBatch);
  if (nsteps < 0) return fail(SBP_EINVAL, "need nsteps >= 0");
  for (int g = 0; g < n; ++g) {
    sbp_ctx* h = hs[g];
    if (!h) return fail(SBP_EINVAL, "NULL handle in batch (%d)", g);
    for (int e = 0; e < g; ++e)
      if (hs[e] == h) return fail(SBP_EINVAL, "handle %d appears twice in the batch", g);
    if (h->dtype != hs[0]->dtype) return fail(SBP_EINVAL, "all handles of a batch need the same dtype");
    if (h->stream != hs[0]->stream) return fail(SBP_EINVAL, "all handles of a batch need the same stream");
    if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called (handle %d)", g);
    if (!(dt[g] > 0) || !std::isfinite(dt[g])) return fail(SBP_EINVAL, "need dt > 0 (handle %d)", g);
    if (h->nrec > 0 && h->rec_step + nsteps > h->rec_max)
      return fail(SBP_EINVAL, "receiver buffer of handle %d holds %d steps; %lld recorded, %d requested", g,
                  h->rec_max, h->rec_step, nsteps);
  }
  if (nsteps == 0) return SBP_OK;
  return hs[0]->dtype == SBP_F32 ? do_steps_batch<float>(hs, n, nsteps, dt)
                                 : do_steps_batch<double>(hs, n, nsteps, dt);
}

int sbp_rhs(sbp_handle h, void* out_device, double t) {
  if (!h || !out_device) return fail(SBP_EINVAL, "NULL argument");
  if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called");
  return h->dtype == SBP_F32 ? do_rhs<float>(h, out_device, t) : do_rhs<double>(h, out_device, t);
}

int sbp_adjoint_bytes(sbp_handle h, int nsteps, int every, size_t* bytes) {
  if (!h || !bytes) return fail(SBP_EINVAL, "NULL argument");
  if (nsteps < 0 || (nsteps > 0 && every < 1)) return fail(SBP_EINVAL, "need nsteps >= 0 and every >= 1");
  *bytes = adj_layout(h, nsteps, every).total;
  return SBP_OK;
}

int sbp_adjoint_rhs(sbp_handle h, const void* lam_device, void* out_device, void* adj_ws, size_t adj_bytes) {
  if (!h || !lam_device || !out_device) return fail(SBP_EINVAL, "NULL argument");
  if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called");
  int rc = check_adj_ws(adj_ws, adj_bytes, adj_layout(h, 0, 1).total);
  if (rc) return rc;
  return h->dtype == SBP_F32 ? do_adjoint_rhs<float>(h, lam_device, out_device, (char*)adj_ws)
                             : do_adjoint_rhs<double>(h, lam_device, out_device, (char*)adj_ws);
}

int sbp_gradient(sbp_handle h, int nsteps, double dt, const void* residual_device, int every, void* adj_ws,
                 size_t adj_bytes, void* grad_device, void* qbar_device) {
  if (!h || !residual_device || !grad_device) return fail(SBP_EINVAL, "NULL argument");
  if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called");
  if (h->nrec <= 0) return fail(SBP_ESTATE, "no receivers: call sbp_record first");
  if (nsteps < 1 || every < 1 || !(dt > 0) || !std::isfinite(dt))
    return fail(SBP_EINVAL, "need nsteps >= 1, every >= 1 and dt > 0");
  int rc = check_adj_ws(adj_ws, adj_bytes, adj_layout(h, nsteps, every).total);
  if (rc) return rc;
  return h->dtype == SBP_F32
             ? do_gradient<float>(h, nsteps, dt, (const float*)residual_device, every, (char*)adj_ws, grad_device,
                                  qbar_device)
             : do_gradient<double>(h, nsteps, dt, (const double*)residual_device, every, (char*)adj_ws,
                                   grad_device, qbar_device);
}

int sbp_step_checkpointed(sbp_handle h, int nsteps, double dt, int every, void* adj_ws, size_t adj_bytes) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called");
  if (nsteps < 1 || every < 1 || !(dt > 0) || !std::isfinite(dt))
    return fail(SBP_EINVAL, "need nsteps >= 1, every >= 1 and dt > 0");
  if (h->nrec > 0 && h->rec_step + nsteps > h->rec_max)
    return fail(SBP_EINVAL, "receiver buffer holds %d steps; %lld recorded, %d requested", h->rec_max,
                h->rec_step, nsteps);
  int rc = check_adj_ws(adj_ws, adj_bytes, adj_layout(h, nsteps, every).total);
  if (rc) return rc;
  return h->dtype == SBP_F32 ? do_step_checkpointed<float>(h, nsteps, dt, every, (char*)adj_ws)
                             : do_step_checkpointed<double>(h, nsteps, dt, every, (char*)adj_ws);
}

int sbp_gradient_from_checkpoints(sbp_handle h, const void* residual_device, void* adj_ws, size_t adj_bytes,
                                  void* grad_device, void* qbar_device) {
  if (!h || !residual_device || !grad_device || !adj_ws) return fail(SBP_EINVAL, "NULL argument");
  if (!h->ck_valid || h->ck_ws != (const char*)adj_ws || h->ck_steps != h->steps)
    return fail(SBP_ESTATE, "no checkpoints of the current state in this workspace: call sbp_step_checkpointed");
  if (h->nrec <= 0) return fail(SBP_ESTATE, "no receivers: call sbp_record first");
  const AdjLayout L = adj_layout(h, h->ck_nsteps, h->ck_every);
  int rc = check_adj_ws(adj_ws, adj_bytes, L.total);
  if (rc) return rc;
  return h->dtype == SBP_F32
             ? adj_reverse<float>(h, h->ck_nsteps, h->ck_dt, h->ck_t0, (const float*)residual_device, L,
                                  (char*)adj_ws, grad_device, qbar_device)
             : adj_reverse<double>(h, h->ck_nsteps, h->ck_dt, h->ck_t0, (const double*)residual_device, L,
                                   (char*)adj_ws, grad_device, qbar_device);
}

int sbp_energy(sbp_handle h, double* E) {
  if (!h || !E) return fail(SBP_EINVAL, "NULL argument");
  if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called");
  return h->dtype == SBP_F32 ? do_energy<float>(h, E) : do_energy<double>(h, E);
}

int sbp_set_launch(sbp_handle h, int ty, int zchunk) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (ty != 8 && ty != 16) return fail(SBP_EINVAL, "ty must be 8 or 16");
  if (ty < h->cl.m) return fail(SBP_EINVAL, "ty must be >= %d for order %d", h->cl.m, h->order);
  if (ty == 16 && (h->dtype == SBP_F64 || h->order == 8))
    return fail(SBP_EINVAL, "16-row tiles exist for SBP_F32 orders 2 to 7 only (their LDS)");
  if (zchunk < 0) return fail(SBP_EINVAL, "zchunk must be >= 0");
  h->ty = ty;
  h->zchunk = zchunk;
  h->bounds_dirty = true;
  ++h->gen;
  return SBP_OK;
}

int sbp_set_addressing(sbp_handle h, int plain) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (plain != 0 && plain != 1) return fail(SBP_EINVAL, "plain must be 0 or 1");
  h->plain = plain == 1;
  ++h->gen;
  return SBP_OK;
}

int sbp_set_graphs(sbp_handle h, int on) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (on != 0 && on != 1) return fail(SBP_EINVAL, "on must be 0 or 1");
  h->graphs = on == 1;
  return SBP_OK;
}

int sbp_fill_scratch(sbp_handle h, double value) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  char* other = h->ws + (h->cur ? h->off_qa : h->off_qb);
  char* dq = h->ws + h->off_dq;
  char* scl = h->ws + h->off_scl;
  const std::size_t nscl = (std::size_t)2 * kMaxM * 6 * h->plane;
  if (h->dtype == SBP_F32) {
    HIPCHK(launch_fill<float>((float*)other, 9 * h->field, (float)value, h->stream));
    HIPCHK(launch_fill<float>((float*)dq, 9 * h->field, (float)value, h->stream));
    HIPCHK(launch_fill<float>((float*)scl, nscl, (float)value, h->stream));
    HIPCHK(launch_fill<float>((float*)(h->ws + h->off_eqc), eqc_elems(h->g.nr, h->g.ns), (float)value, h->stream));
  } else {
    HIPCHK(launch_fill<double>((double*)other, 9 * h->field, value, h->stream));
    HIPCHK(launch_fill<double>((double*)dq, 9 * h->field, value, h->stream));
    HIPCHK(launch_fill<double>((double*)scl, nscl, value, h->stream));
  }
  return SBP_OK;
}

int sbp_checkpoint_id(sbp_handle h, long long* id) {
  if (!h || !id) return fail(SBP_EINVAL, "NULL argument");
  *id = (h->ck_valid && h->ck_steps == h->steps) ? h->ck_id : 0;
  return SBP_OK;
}

int sbp_autotune(sbp_handle h, int reps, int* ty, int* zchunk, double* ms) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (!h->have_material) return fail(SBP_ESTATE, "sbp_set_material has not been called");
  if (reps < 1) return fail(SBP_EINVAL, "reps must be >= 1");
  return h->dtype == SBP_F32 ? do_autotune<float>(h, reps, ty, zchunk, ms)
                             : do_autotune<double>(h, reps, ty, zchunk, ms);
}

int sbp_time(sbp_handle h, double* t, long long* steps) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (t) *t = h->t;
  if (steps) *steps = h->steps;
  return SBP_OK;
}

int sbp_set_profiling(sbp_handle h, int on) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  if (on) {
    for (int e = 0; e < 3; ++e)
      if (!h->ev[e]) HIPCHK(hipEventCreate(&h->ev[e]));
  }
  h->prof = on != 0;
  h->prof_stage_ms = h->prof_edge_ms = 0.0;
  h->prof_n = 0;
  return SBP_OK;
}

int sbp_profile(sbp_handle h, double* stage_ms, double* edge_ms, long long* nstages, long long* stage_nodes) {
  if (!h) return fail(SBP_EINVAL, "NULL handle");
  int rc = prepare_bounds(h);
  if (rc) return rc;
  const double n = h->prof_n > 0 ? (double)h->prof_n : 1.0;
  if (stage_ms) *stage_ms = h->prof_stage_ms / n;
  if (edge_ms) *edge_ms = h->prof_edge_ms / n;
  if (nstages) *nstages = h->prof_n;
  if (stage_nodes) *stage_nodes = (long long)(h->g.nq - h->ex) * (h->g.nr - h->ey) * h->g.ns;
  return SBP_OK;
}

int sbp_destroy(sbp_handle h) {
  if (!h) return SBP_OK;
  // work still queued may read the staging buffer and the graphs
  if (h->tab_host || h->gx[0] || h->gx[1]) (void)hipStreamSynchronize(h->stream);
  for (int e = 0; e < 3; ++e)
    if (h->ev[e]) (void)hipEventDestroy(h->ev[e]);
  for (int p = 0; p < kTabParts; ++p)
    if (h->tab_ev[p]) (void)hipEventDestroy(h->tab_ev[p]);
  for (int c = 0; c < 2; ++c)
    if (h->gx[c]) (void)hipGraphExecDestroy(h->gx[c]);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->tab_host) (void)hipHostFree(h->tab_host);
  delete h;
  return SBP_OK;
}

}  // extern "C"
