// Kernel argument blocks and launchers (host <-> device interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "internal.hpp"

namespace sbp {

struct StepClock;

template <typename T>
struct StageArgs {
  const T* qin;       // 9 fields, current stage input
  T* qout;            // 9 fields, stage output
  T* dq;              // 9 fields, Runge-Kutta register (read if read_dq)
  const T* coef;      // 12 fields: M[xi][c] (3 xi + c), lambda/J, mu/J, 1/(rho J)
  const T* face;      // workspace base for the face coefficient arrays
  const int* bounds;  // tile bounds: q (nxt+1), r (nyt+1), s (nzc+1)
  // s closure terms of the closure planes, written and read by the stage
  // kernel: value (side, row, c) of node col at ((side * kMaxM + row) * 6 +
  // c) * plane + col; c = 0..2: h D+_s v_c, 3..5: h D-_s F_s,c
  T* scl;
  // v and the q flux F_q of the columns nq-NC .. nq-2 (the ones the q
  // closure row of the last column reads), written by the stage kernel for
  // the edge kernel of the same stage (single precision): 8 values per node
  // (v 0..2, F_q 3..5, 2 unused), node (i, j, k) at 8 * ((k * nr + j) *
  // (NC - 1) + i - (nq - NC)).  NULL: the edge kernel gathers those columns
  // itself (double precision; stage and edge blocks in one launch)
  T* eqc;
  // point sources that the single-grid stage and edge kernels add at the
  // stage update (single precision; nsrc = 0: none here, a source_kernel
  // launch follows instead): stencil width, corners, weights (as
  // SourceArgs::wm), dt g(t) from the clock's table when src_clock is not
  // null, else src_gdt
  int nsrc, src_w, src_stage;
  int src_i0[kMaxSources], src_j0[kMaxSources], src_k0[kMaxSources];
  T src_gdt[kMaxSources];
  const T* src_wm;
  const StepClock* src_clock;
  NodeMap nm;         // node -> element offset in a field
  std::size_t face_off[6];
  std::size_t face_n[6];
  std::size_t plane, field;
  int px, nq, nr, ns;
  int nxt, nyt, nzc, ntiles;
  int ncol;
  int read_dq;
  int ex, ey;         // edge kernel: last q column / last r row
  int sat;            // 1: boundary penalties follow (launch_penalty); 0: volume terms only
  int plain;          // 1: plain pointers even where buffer addressing fits
  int traction[6];
  T Ak, Bk, dt;
  T inv_h[3];
  T gamma[6];
  // closure rows, kClosureTab blocks of kMaxM x kMaxCols values: h D+ and
  // h D- at the left end, then -h D- and -h D+ (the right-end rows of h D+
  // and h D- read against reversed columns)
  const T* tab;
};

constexpr int kClosureTab = 4;

// Device-side clock of a run of steps: the steps of one sbp_step call are
// issued chunk by chunk; per chunk a table of dt * g(t_stage) values
// ([step][stage][source], handle dtype) is uploaded and the clock is set to
// (table, first receiver slot, step 0); every step ends with a kernel that
// advances `step`.  Kernels that depend on the step read it here, so the
// launches of one step are the same for every step (and can be replayed
// from a captured graph).
struct StepClock {
  const void* gtab;
  long long rec0;
  int step;
  int pad;
};

// batched stepping: receiver slot of a step = base (the handle's recorded
// steps before the call) + the clock's rec0 (steps before the chunk) + step
template <typename T>
struct RecordArgs;

template <typename T>
struct SourceArgs {
  T* dq;
  T* qout;       // may be null (RHS evaluation only)
  const T* wm;   // per source: width^3 nodes x 6 weights (w * M_c), padded to kMaxSrcWidth^3
  NodeMap nm;
  std::size_t plane, field;
  int px, width;
  int i0[kMaxSources], j0[kMaxSources], k0[kMaxSources];
  T gdt[kMaxSources];  // dt * g(t_stage) per source (used when clock is null)
  T Bk;
  const StepClock* clock;  // non-null: dt * g from the clock's table
  int stage;               // Runge-Kutta stage (index into the clock's table)
  int tab_stride;          // table entries per (step, stage) (0 means kMaxSources)
  int tab_off;             // this grid's first entry in a (step, stage) row
};

template <typename T>
struct EnergyArgs {
  const T* q;
  const T* coef;
  double* part;
  NodeMap nm;
  std::size_t plane, field;
  int px, nq, nr, ns, m;
  double h[3];
  double w[kMaxM];
};

// Work list of the batched stage kernel: one entry per block of work (a
// stage-kernel tile or an edge-kernel strip block of one grid), split into 8
// segments (one per XCD: block b of the launch takes entry b / 8 of segment
// b % 8); within a segment, longest first.
struct BatchItem {
  int grid;   // index into the argument table
  int kind;   // 0 stage tile, 1 edge block
  int local;  // tile / block index within the grid
  int order;  // interior order of the grid
};

template <typename T>
struct PersistArgs {
  const StageArgs<T>* args;  // per grid, this stage and ping-pong parity
  const BatchItem* items;
  const int* seg;            // segment starts, 9 entries (seg[8] = number of items)
};

// several grids in one launch: args[g] for grid g, whose blocks are
// first[g] .. first[g+1]-1 of the launch (first[0] = 0, total blocks)
template <typename T>
struct BatchArgs {
  const StageArgs<T>* args;
  const int* first;
  int n, total;
};

template <typename T>
struct RecordArgs {
  const T* q;
  std::size_t field;
  const long long* off;
  T* out;          // this step's slot, or the first slot with a clock
  long long base;  // with a clock: slot of the call's first step
};

template <typename T>
struct SourceBatch {
  const SourceArgs<T>* args;
  const int* first;
  int n, total;
};

template <typename T>
struct RecordBatch {
  const RecordArgs<T>* args;
  const int* first;
  int n, total;
  const StepClock* clock;  // non-null: slot from the clock
};

template <typename T>
hipError_t launch_stage(int order, int ty, const StageArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_edge(int order, const StageArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_stage_batch(int order, int ty, const BatchArgs<T>& b, bool buf, hipStream_t st);
template <typename T>
int edge_blocks(const StageArgs<T>& a);
// largest scratch (private segment) size, bytes per lane, of the kernels one
// step launches; (size_t)-1 if it cannot be queried
template <typename T>
std::size_t step_scratch(int order, int ty);
template <typename T>
std::size_t batch_step_scratch(unsigned orders);
template <typename T>
hipError_t launch_edge_batch(int order, const BatchArgs<T>& b, hipStream_t st);
template <typename T>
hipError_t launch_source_batch(const SourceBatch<T>& b, hipStream_t st);
// batched stage over a work list: `blocks` (8 x the longest segment) blocks
// of 64 x 8 threads (every stage tile has 8 rows); `orders` has bit o set
// for every interior order o in the list
template <typename T>
hipError_t launch_stage_worklist(const PersistArgs<T>& p, unsigned orders, int blocks, hipStream_t st);
template <typename T>
bool worklist_order_ok(int order);
template <typename T>
hipError_t launch_record_batch(const RecordBatch<T>& b, hipStream_t st);
// boundary penalties of the block's surface nodes, added to dQ and Q_out
// after the stage and edge kernels
template <typename T>
hipError_t launch_penalty(const StageArgs<T>& a, hipStream_t st);
// single precision: the edge kernel and every boundary penalty in one
// launch (edge blocks with their own nodes' penalties, then blocks for the
// penalties of the nodes the stage tiles computed), in place of launch_edge
// and launch_penalty
template <typename T>
hipError_t launch_edge_penalty(int order, const StageArgs<T>& a, hipStream_t st);
// the same for several grids: b.first holds the prefix sums of their
// surface node counts (surface_nodes)
template <typename T>
hipError_t launch_penalty_batch(const BatchArgs<T>& b, hipStream_t st);
// Single precision adds the penalty of the q = 0 face inside the stage
// kernel, at the nodes its tiles compute (lanes i = 0 of the first tiles
// along q hold the node's values there, while a separate pass would fetch a
// whole line of every field per node); in double precision the penalty's
// arithmetic does not fit beside the derivatives in 256 VGPRs, and the
// penalty kernel keeps that face.
template <typename T>
constexpr bool q0_in_stage() {
  return sizeof(T) == 4;
}
// nodes the penalty kernel visits (each once): the whole surface, or, with
// the q = 0 face in the stage kernel, the surface without the inside of that
// face (the q = nq-1 face, the r faces for i < nq-1, the s faces for i <
// nq-1 and 0 < j < nr-1)
__host__ __device__ inline long long surface_nodes(int nq, int nr, int ns, bool q0_stage) {
  if (q0_stage) return 1LL * nr * ns + 2LL * (nq - 1) * ns + 2LL * (nq - 1) * (nr - 2);
  return 2LL * nr * ns + 2LL * (nq - 2) * ns + 2LL * (nq - 2) * (nr - 2);
}
template <typename T>
hipError_t launch_source(const SourceArgs<T>& s, int nsrc, hipStream_t st);
template <typename T>
hipError_t launch_record(const T* q, std::size_t field, const long long* off, int nrec, T* out,
                         const StepClock* clock, hipStream_t st);
hipError_t launch_clock_set(StepClock* c, const void* gtab, long long rec0, hipStream_t st);
hipError_t launch_clock_tick(StepClock* c, hipStream_t st);
template <typename T>
hipError_t launch_energy(const EnergyArgs<T>& e, int nblocks, hipStream_t st);

}  // namespace sbp
