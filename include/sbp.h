/*
 * sbp.h -- C ABI of the MI355X (gfx950) upwind-SBP elastic wave solver.
 *
 * The library advances the semi-discrete 3D velocity-stress elastic wave
 * equation on one boundary-conforming curvilinear block (Duru, Fung &
 * Williams, arXiv:2011.02600):
 *
 *   P~^{-1} dQ/dt = grad_{D-} . F(Q) + sum_xi B_xi(grad_{D+} Q) + sum SAT   (eq. gen_hyp_transformed_discrete_SAT)
 *
 * with the upwind dual-pair SBP operators D+/D- (Sec. 4.1, Table tab:upwind)
 * applied along the reference axes q, r, s, the metric terms J and
 * J d(xi)/dx (Sec. 2.2), an isotropic medium rho, lambda, mu (eq. S matrix),
 * boundary penalties on the six faces (eq. SAT_free_surface, eq. SAT_General
 * with the hat variables of App. A), point moment-tensor sources
 * (eq. momententor_pointsource) and the five-stage fourth-order low-storage
 * Runge-Kutta scheme of Carpenter & Kennedy (Sec. 7).
 *
 * Conventions shared by every entry point
 *  - Every call returns an int: SBP_OK (0) or a negative SBP_E* code.  The
 *    text of the last failure on the calling thread is sbp_last_error().
 *    No C++ exception crosses the ABI.
 *  - Grid functions are dense arrays in (ns, nr, nq) order, q fastest
 *    ("row-wise" storage of Sec. 4.1 with q innermost).  A state holds the
 *    nine fields (vx, vy, vz, sxx, syy, szz, sxy, sxz, syz) one after another:
 *    9 * nq * nr * ns values of the handle's dtype.
 *  - Host inputs are copied; the caller keeps ownership of every pointer it
 *    passes.  Device memory is the caller's: all device state lives in the
 *    workspace given to sbp_init_grid, which must stay allocated until
 *    sbp_destroy; the library never allocates or frees device memory.
 *  - Work is queued asynchronously on the HIP stream given at init (NULL: the
 *    null stream).  Outputs written to device memory are valid once the
 *    caller has synchronised that stream.  Calls that return host data
 *    (sbp_get_state to host, sbp_energy) synchronise the stream themselves.
 *  - A handle is not thread-safe: use one handle per thread/stream.
 */
#ifndef SBP_H
#define SBP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbp_ctx* sbp_handle;

/* return codes */
enum {
    SBP_OK = 0,
    SBP_EINVAL = -1,    /* invalid argument (sizes, order, gamma, material, ...) */
    SBP_ENOMEM = -2,    /* workspace too small */
    SBP_EHIP = -3,      /* a HIP runtime call failed; see sbp_last_error() */
    SBP_ESTATE = -4,    /* call out of order (e.g. sbp_step before sbp_set_material) */
    SBP_EUNSTABLE = -5  /* non-finite energy detected */
};

/* arithmetic type of the device path */
enum { SBP_F32 = 32, SBP_F64 = 64 };

/* boundary-penalty variant */
enum {
    SBP_SAT_CHARACTERISTIC = 0, /* eq. SAT_General with hat variables, all faces */
    SBP_SAT_TRACTION = 1        /* eq. SAT_free_surface on faces with gamma == 1,
                                   characteristic penalty on the others */
};

/* source-time functions */
enum {
    SBP_STF_RICKER = 0, /* (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2 */
    SBP_STF_EXPT = 1    /* (t - t0) / T^2 exp(-(t - t0) / T) for t >= t0, else 0
                           (eq. momententor_pointsource, T = 0.1 s in Sec. 7.1) */
};

/*
 * Bytes of device workspace a handle needs for an nq x nr x ns grid (points
 * per axis, the reference axes q, r, s of Sec. 2.2) of interior order
 * `order` in `dtype`.  Writes the size to *bytes.  Same validation as
 * sbp_init_grid.
 */
int sbp_workspace_bytes(int nq, int nr, int ns, int order, int dtype, size_t* bytes);

/*
 * Create a solver for one curvilinear block.
 *  nq, nr, ns   points along q, r, s (uniform reference grid xi_i = i / (n-1),
 *               Sec. 4.1); each must be >= 2 * order so that the two
 *               boundary closures of the SBP operators do not overlap.
 *               One field of the device layout must stay below 4 GiB (the
 *               kernels address a field with 32-bit byte offsets): rows of
 *               nq - 1 points padded to 128 bytes, nr * ns of them, plus
 *               the last column, i.e. about 1.07e9 points for SBP_F32
 *               (1025 x 1024 x 1023 passes, 1025 x 1024 x 1024 does not)
 *               and 5.4e8 for SBP_F64.  Larger grids are SBP_EINVAL.
 *  xyz          host, 3 * nq * nr * ns doubles: x, then y, then z, each a
 *               grid function.  NULL selects the identity map of the unit
 *               cube.  Metric terms are computed on the host in double
 *               precision (x_xi = D0 x with D0 = (D+ + D-)/2, J = det, and the
 *               conservative cofactor form of J dxi/dx); a non-positive
 *               Jacobian anywhere is SBP_EINVAL.
 *  order        interior order of accuracy of the upwind pair, 2 to 8
 *               (Table tab:upwind; 9 is SBP_EINVAL).  The boundary closures are accurate to
 *               order order / 2 (rounded down); the paper does not print
 *               them: the library constructs them from the SBP and upwind
 *               properties of Sec. 4.1, the entries those leave free fixed
 *               where the spectral radius is smallest.
 *  dtype        SBP_F32 or SBP_F64 (every device array and kernel uses it).
 *  gamma        host, 6 doubles, reflection coefficient of eq. BC_General2
 *               per face in the order (q=0, q=1, r=0, r=1, s=0, s=1); each
 *               in [-1, 1]: 1 free surface, 0 absorbing, -1 clamped.
 *  sat_variant  SBP_SAT_CHARACTERISTIC or SBP_SAT_TRACTION.
 *  workspace    device pointer to >= sbp_workspace_bytes() bytes, 256-byte
 *               aligned, owned by the caller.
 *  stream       hipStream_t cast to void* (NULL = null stream).
 * On success *out holds the handle and the state is zero at t = 0.
 */
int sbp_init_grid(sbp_handle* out, int nq, int nr, int ns, const double* xyz, int order,
                  int dtype, const double* gamma, int sat_variant, void* workspace,
                  size_t workspace_bytes, void* stream);

/*
 * Set the medium: host grid functions rho, cp, cs (nq*nr*ns doubles each).
 * mu = rho cs^2, lambda = rho cp^2 - 2 mu (eq. S matrix); requires rho > 0,
 * mu > 0 and 3 lambda + 2 mu > 0, else SBP_EINVAL.  Impedances for the
 * penalties are Z_p = rho cp, Z_s = rho cs (Sec. 3).
 */
int sbp_set_material(sbp_handle h, const double* rho, const double* cp, const double* cs);

/*
 * Add a point moment-tensor source (eq. momententor_pointsource):
 *   d sigma / dt += M g(t) delta_h,
 *  xi       host, 3 doubles: source position in reference coordinates
 *           (q, r, s) in [0, 1]^3 (outside: SBP_EINVAL).
 *  M        host, 6 doubles (Mxx, Myy, Mzz, Mxy, Mxz, Myz).
 *  stf      SBP_STF_RICKER (param = peak frequency f0) or SBP_STF_EXPT
 *           (param = T); t0 = time shift.
 * delta_h is the tensor product of one-dimensional discrete deltas over the
 * 2(p+1) nodes nearest to xi per axis (Lagrange weights divided by the SBP
 * norm weights) divided by J; it reproduces the point value of tensor
 * polynomials of degree < 2(p+1).  At most 4 sources per handle.
 */
int sbp_add_source(sbp_handle h, const double* xi, const double* M, int stf, double param,
                   double t0);

/*
 * Reference coordinates of a physical point (the source position x_p of
 * eq. momententor_pointsource is a physical point): xi (host, 3 doubles,
 * (q, r, s) in [0, 1]^3) with X(xi) = x (host, 3 doubles), X the
 * tensor-product Lagrange interpolant of the node coordinates over the
 * 2(p+1) nearest nodes per axis (the window of the discrete delta).
 * Newton iteration started at the nearest node; the node coordinates are
 * those given to sbp_init_grid.  SBP_EINVAL if the point lies outside the
 * block (beyond a face by more than 1e-9 of the block's diagonal, in
 * reference or physical distance) or the iteration does not converge.
 */
int sbp_locate(sbp_handle h, const double* x, double* xi);

/*
 * sbp_add_source with the source given at a physical position x (host, 3
 * doubles): its reference coordinates come from sbp_locate.  Same arguments
 * otherwise; SBP_EINVAL outside the block.
 */
int sbp_add_source_at(sbp_handle h, const double* x, const double* M, int stf, double param, double t0);

/* Remove all sources. */
int sbp_clear_sources(sbp_handle h);

/*
 * Overwrite the state with 9 dense grid functions of the handle's dtype
 * (q_is_device != 0: device pointer, else host), set the time to t.
 */
int sbp_set_state(sbp_handle h, const void* q, int q_is_device, double t);

/*
 * Copy the state out (same layout as sbp_set_state); *t_out (may be NULL)
 * receives the current time.  A host destination synchronises the stream.
 */
int sbp_get_state(sbp_handle h, void* q, int q_is_device, double* t_out);

/*
 * Register receivers: nrec node indices (host, 3*nrec ints (i, j, k) along
 * q, r, s).  After every step the velocity (vx, vy, vz) at each receiver is
 * written to out_device[(step * nrec + r) * 3 + c] (dtype of the handle),
 * step counting from 0 at this call, for at most max_steps steps; an
 * sbp_step call that would exceed max_steps is SBP_EINVAL.  nrec = 0
 * disables recording.  out_device is owned by the caller.
 */
int sbp_record(sbp_handle h, int nrec, const int* ijk, void* out_device, int max_steps);

/*
 * Advance nsteps steps of size dt (> 0) with the five-stage 2N-storage
 * Runge-Kutta scheme; every stage evaluates the full right-hand side
 * (volume terms, penalties, sources) and is fused with the stage update
 * dQ <- A_k dQ + dt RHS, Q <- Q + B_k dQ.  Asynchronous on the stream.
 * SBP_ESTATE before sbp_set_material.
 * The call's first step is issued as direct launches (five stages of
 * stage, edge, penalty and source kernels, the receivers, a clock tick);
 * every later step is one replay of a HIP graph holding the same launches,
 * captured on first use and again whenever dt, the sources, the receivers or
 * the launch shape change -- when none of the step's kernels uses scratch
 * memory (register spills; the SBP_F32 kernels); otherwise every step is
 * issued directly.  The per-step values (the source-time factor
 * dt g(t_n + C_k dt) of every stage, evaluated on the host in double, and
 * the receiver slot) are read from a device table and a device step
 * counter, uploaded / set once per 512 steps.
 */
int sbp_step(sbp_handle h, int nsteps, double dt);

/*
 * on = 1 (default): sbp_step and sbp_step_batch replay captured step graphs
 * where their kernels use no scratch memory; on = 0: they issue the same
 * launches one by one.  Results are bitwise identical.  Profiling
 * (sbp_set_profiling) uses the one-by-one launches.
 */
int sbp_set_graphs(sbp_handle h, int on);

/*
 * Advance n handles (1 <= n <= 64) by nsteps steps each, handle i with step
 * dt[i] (host array of n doubles): batched stepping of many independent
 * sources or media ("shots") on grids of uneven size and mixed interior
 * orders.  Per Runge-Kutta stage one launch covers a list of the
 * stage-kernel tiles and edge-kernel blocks of every handle, split into one
 * segment per XCD of equal estimated cost, longest items first (block b of
 * the launch runs item b / 8 of segment b % 8); then one launch injects
 * every point source; per step one launch records every receiver.  Where
 * the kernels use no scratch memory (SBP_F32) each step is a replay of a
 * graph captured for the call (even and odd steps); otherwise the same
 * launches are issued directly.  The
 * source-time factors come from a device table uploaded every 64 steps.
 * Every grid uses
 * 8-row tiles and one s-chunk length for the batch (from
 * sbp_autotune_batch, else a cost model); the handles' own launch settings
 * are restored on return.  With plain addressing on any handle
 * (sbp_set_addressing), or with a handle of an order the work-list kernel
 * does not serve (order 8; orders 7 and 8 in SBP_F64), one stage and one
 * edge launch per interior order replace the work-list launch.  Each handle's state, time, step count and
 * receiver traces end up as after sbp_step(hs[i], nsteps, dt[i]), to
 * rounding (the batched kernels are separate instantiations of the same
 * kernel bodies).  All handles need the same dtype and the same stream,
 * distinct handles and a medium; the argument tables and the work list
 * (at most 65536 items) live in hs[0]'s workspace.  Synchronises the
 * stream before returning.
 */
int sbp_step_batch(sbp_handle* hs, int n, int nsteps, const double* dt);

/*
 * Launch-shape autotuner of sbp_step_batch: times `reps` batched
 * right-hand-side launches (the work-list launch over every handle's tiles;
 * they write only the Runge-Kutta registers and the second state buffers,
 * so the states are untouched) for the cost model's s-chunk length and a few
 * others, and keeps the fastest for later sbp_step_batch calls of these
 * handles.  Writes the chosen length and its time per launch (ms) to the
 * outputs (each may be NULL).  Same requirements on hs as sbp_step_batch.
 * Synchronises the stream.
 */
int sbp_autotune_batch(sbp_handle* hs, int n, int reps, int* zchunk, double* ms);

/*
 * Evaluate the semi-discrete right-hand side dQ/dt of the current state at
 * time t (sources evaluated at t) into out_device (9 dense grid functions,
 * handle dtype).  The state and the time are not changed.  Asynchronous.
 */
int sbp_rhs(sbp_handle h, void* out_device, double t);

/*
 * Discrete adjoint and misfit gradient (an extension built on the scheme; the
 * paper has no adjoint).  The differentiated map is the fully discrete
 * scheme as sbp_step runs it (the semi-discrete operator L of eq.
 * gen_hyp_transformed_discrete_SAT, point sources, the five-stage Runge-Kutta
 * scheme of Sec. 7) followed by the receivers (v after every step).
 *
 * sbp_adjoint_bytes: bytes of the caller-owned adjoint workspace that
 * sbp_gradient needs for nsteps steps with a checkpoint every `every` steps:
 * ceil(nsteps / every) + 5 every saved states plus about 100 grid functions
 * (nsteps = 0: the size sbp_adjoint_rhs needs).  every is clamped to
 * [1, nsteps].
 */
int sbp_adjoint_bytes(sbp_handle h, int nsteps, int every, size_t* bytes);

/*
 * out_device = L^T lam_device: the transpose of the semi-discrete operator
 * (volume terms and boundary penalties; sources do not enter), both 9 dense
 * grid functions in the handle dtype on the device.  adj_ws: device,
 * 256-byte aligned, >= sbp_adjoint_bytes(h, 0, 1, .) bytes, caller-owned,
 * its contents scratch.  Computed as -W L_v(W^{-1} lam) + Bd W^{-1} lam +
 * P^T lam (W the energy weights, Bd the boundary terms of the summation by
 * parts identity, P the face penalty blocks).  Asynchronous.
 */
int sbp_adjoint_rhs(sbp_handle h, const void* lam_device, void* out_device, void* adj_ws, size_t adj_bytes);

/*
 * Gradient of chi = sum_n sum_r m(trace(n, r)) for a caller-chosen misfit m
 * whose derivative dm/dtrace the caller supplies as residual_device
 * ([nsteps][nrec][3], handle dtype, device; the receivers are those of the
 * last sbp_record call, which must have nrec >= 1; for chi = 1/2 |traces -
 * data|^2 the residual is traces - data).  Starting from the current state
 * at the current time, runs nsteps steps of size dt (sources included,
 * receiver traces not recorded), keeping a checkpoint every `every` steps in
 * adj_ws, then the reverse sweep: each block of steps is recomputed from
 * its checkpoint, keeping the inputs of every stage of the block.  Writes d chi /
 * d (rho, lambda, mu) at every node to grad_device (3 dense grid functions:
 * rho, then lambda, then mu, with the other two held fixed) and, if
 * qbar_device is not NULL, d chi / d Q0 (9 dense grid functions).  The
 * handle ends as after sbp_step(h, nsteps, dt).  Synchronises the stream.
 * About five forward step costs per step.
 */
int sbp_gradient(sbp_handle h, int nsteps, double dt, const void* residual_device, int every, void* adj_ws,
                 size_t adj_bytes, void* grad_device, void* qbar_device);

/*
 * sbp_step (sources, receivers recorded) that also keeps the checkpoints a
 * later sbp_gradient_from_checkpoints needs, in adj_ws (the layout and size of
 * sbp_adjoint_bytes(h, nsteps, every, .)); for a forward pass whose gradient
 * may be wanted afterwards (the backward pass then skips the forward run).
 * Synchronises nothing; the checkpoints stay valid until the handle is
 * stepped again or its state, medium or sources change.
 */
int sbp_step_checkpointed(sbp_handle h, int nsteps, double dt, int every, void* adj_ws, size_t adj_bytes);

/*
 * Identifier of the checkpoints sbp_gradient_from_checkpoints would use
 * (> 0, a new value for every sbp_step_checkpointed call), or 0 if there
 * are none (the handle was stepped, or its state, medium, sources or
 * receivers changed since).  Lets a caller check that the checkpoints are
 * still those of its own forward run.
 */
int sbp_checkpoint_id(sbp_handle h, long long* id);

/*
 * The gradient of sbp_gradient for the run of the last sbp_step_checkpointed
 * on this handle (its nsteps, dt and every; adj_ws the same workspace), the
 * handle standing at the end of that run: only the reverse sweep.  Results
 * are those of sbp_gradient from the run's initial state.  SBP_ESTATE if
 * there are no such checkpoints.  Leaves the state and the checkpoints as
 * they are (so several residuals can be differentiated).  Synchronises the
 * stream.
 */
int sbp_gradient_from_checkpoints(sbp_handle h, const void* residual_device, void* adj_ws, size_t adj_bytes,
                                  void* grad_device, void* qbar_device);

/*
 * Discrete energy 1/2 <Q, P~^{-1} Q>_H = 1/2 sum H_ijk J (rho |v|^2 +
 * sigma^T C^{-1} sigma) of the current state (eq. physical_energy_discrete
 * with the curvilinear weight J), accumulated in double.  Synchronises the
 * stream.  SBP_EUNSTABLE if the result is not finite.
 */
int sbp_energy(sbp_handle h, double* E);

/*
 * Launch shape of the stage kernel: ty rows of 64 points per thread block
 * (8 or 16; 16 only for SBP_F32 at orders 2 to 7, else SBP_EINVAL) and
 * zchunk planes per block along s (>= 1; 0 = automatic).
 * Does not change results beyond floating-point summation order (it does
 * not change it at all: every node is computed by the same instructions).
 */
int sbp_set_launch(sbp_handle h, int ty, int zchunk);

/*
 * Addressing of the stage kernel's field arrays.  plain = 0 (default):
 * buffer resources (32-bit offsets from one descriptor per array) whenever
 * every array of up to 12 fields is below 4 GiB, plain 64-bit pointers
 * otherwise; plain = 1: plain pointers always, the path large grids take,
 * on any grid.  Results agree to rounding (two instantiations of the same
 * kernel body; the compiler may contract differently).  SBP_EINVAL for
 * other values.
 */
int sbp_set_addressing(sbp_handle h, int plain);

/*
 * Launch timing.  sbp_set_profiling(h, 1) resets the counters and from then
 * on brackets every stage-kernel launch (one Runge-Kutta stage of the nodes
 * covered by the tiles) and the launches that follow it (the remaining last
 * q column and last r row, and the boundary penalties: one launch in
 * SBP_F32) with HIP events on the handle's stream; the host
 * waits for each stage to finish, so stepping is slower while it is on.
 * sbp_set_profiling(h, 0) switches it off.  sbp_profile returns the average
 * durations in milliseconds (*stage_ms, *edge_ms), the number of timed stages
 * and the number of nodes one stage-kernel launch computes; any output
 * pointer may be NULL.  Results are not changed by profiling.
 */
int sbp_set_profiling(sbp_handle h, int on);
int sbp_profile(sbp_handle h, double* stage_ms, double* edge_ms, long long* nstages,
                long long* stage_nodes);

/*
 * Launch-shape autotuner.  Times `reps` right-hand-side evaluations of the
 * handle's own grid for each candidate launch shape (tile height 8, and 16
 * for SBP_F32 at orders up to 7; the cost model's number of s-chunks and one
 * fewer / one more) and keeps the fastest, as sbp_set_launch would.  Writes
 * the chosen tile height, s-chunk length and its time per evaluation (ms) to
 * the outputs (each may be NULL).  The state and time are not changed; call
 * it between steps.  Synchronises the stream.
 */
int sbp_autotune(sbp_handle h, int reps, int* ty, int* zchunk, double* ms);

/*
 * Fill the handle's scratch buffers -- the state buffer that does not hold
 * the current state (the next stage's output), the Runge-Kutta register and
 * the stage kernel's s closure terms -- with `value` (for instance a NaN),
 * asynchronously.  A check of the ping-pong design: every stage writes every
 * node of its output before the next stage reads it, the first stage does
 * not read the register, and every stage forms the closure terms it reads,
 * so sbp_step and sbp_rhs results do not depend on these contents.
 */
int sbp_fill_scratch(sbp_handle h, double value);

/* Current time and number of completed steps. */
int sbp_time(sbp_handle h, double* t, long long* steps);

/* Release the handle (not the workspace). */
int sbp_destroy(sbp_handle h);

/* Text of the last failure on the calling thread ("" if none). */
const char* sbp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SBP_H */
