/*
 * molt.h -- C-ABI of the MI355X (gfx950) MOL^T Cahn-Hilliard library (libmolt.so).
 *
 * Method: Causley, Cho, Christlieb, "Method of lines transpose: energy gradient
 * flows using direct operator inversion for phase field models",
 * arXiv:1611.04214.  The library applies the line-by-line O(N) inverse of the
 * modified Helmholtz operator L = I - d_xx/alpha^2 (Sec. 3.1-3.2, eqs. L_Inverse,
 * Iu, IL, IR, homogeneous) and takes Backward Euler / BDF2 time steps of the
 * Cahn-Hilliard equation with the factored fourth-order operator and the
 * splitting-absorbing fixed-point iteration (Sec. 3.1, 4.1, 5.1).
 *
 * Conventions shared by every entry point
 *  - Fields are row-major, f[iy*nx + ix]: rows are x-lines, columns y-lines.
 *    ny == 1 is a one-dimensional problem.
 *  - All field pointers are DEVICE pointers owned by the caller; the library
 *    never allocates or frees device memory.  Scratch memory is the caller's
 *    workspace (d_work, work_bytes), sized by the *_workspace_bytes queries.
 *  - Element type: double for MOLT_F64, float for MOLT_F32.  Device pointers
 *    must be aligned to the element size; 16-byte alignment is faster.
 *  - stream is a hipStream_t (NULL: the default stream).  Work is enqueued on
 *    it; mol_t_helmholtz_sweep returns without waiting, ch_step / ch_solve
 *    synchronize the stream before they return (they report per-step data).
 *  - Return value: MOLT_OK (0), MOLT_NOT_CONVERGED (+1: a step reached max_iter;
 *    the state is still advanced) or a negative error code.  No exception
 *    crosses the ABI.  molt_strerror() names a code, molt_last_error() gives
 *    the calling thread's last detailed message.
 *  - Calls that share a workspace must not overlap.
 */
#ifndef MOLT_H
#define MOLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MOLT_OK 0
#define MOLT_NOT_CONVERGED 1
#define MOLT_EINVAL (-1)       /* bad argument: sizes, alpha, eps, dt, enum, NULL pointer */
#define MOLT_EUNSUPPORTED (-2) /* valid but not implemented (e.g. line longer than 8192) */
#define MOLT_EHIP (-3)         /* a HIP runtime call failed; see molt_last_error() */
#define MOLT_EWORKSPACE (-4)   /* work_bytes smaller than the query returned */

/* boundary conditions of every line (Sec. 3.2: periodic eq. homogeneous;
 * Neumann and Dirichlet: the analogous 2x2 solve) */
#define MOLT_BC_PERIODIC 0
#define MOLT_BC_NEUMANN 1
#define MOLT_BC_DIRICHLET 2

/* time steppers (Sec. 3.1 eq. CH_BE; Sec. 4.1 eqs. BDF2, BDF3).  BDF3 starts
 * with two SDIRK2 steps (Sec. 4.2, 4.4), each solved as two BE stages of size
 * (1 - sqrt(2)/2) dt. */
#define MOLT_BE 0
#define MOLT_BDF2 1
#define MOLT_BDF3 2

/* models: the Cahn-Hilliard equation (eq. CahnHilliard) or the vector model of
 * three phases (eqs. CH_vector, CH_vector_reaction; Sec. 5.2) */
#define MOLT_MODEL_CH 0
#define MOLT_MODEL_VCH 1

/* initial iterate of the fixed point: previous step, or R = A1^{-1} A2^{-1} rhs */
#define MOLT_INIT_PREV 0
#define MOLT_INIT_LINEAR 1

/* arithmetic of the sweeps and fixed-point updates (weights, boundary solves,
 * residual, mass and energy are FP64 in both) */
#define MOLT_F64 0
#define MOLT_F32 1

/*
 * Grid (Sec. 3.2: nodes a = x_0 < ... < x_N = b, uniform spacing).
 *  periodic: nx (ny) UNIQUE nodes per line, h = (x1-x0)/nx, x_N = x_0;
 *  Neumann / Dirichlet: nx (ny) nodes including both ends, h = (x1-x0)/(nx-1).
 * order_M: local quadrature order M (2, 4 or 6; Sec. 3.2).  Every line needs
 * at least M+1 nodes.  Lines are limited to 8192 nodes along x.
 */
typedef struct {
  int32_t nx, ny;
  double x0, x1, y0, y1;
  int32_t bc;
  int32_t order_M;
} molt_grid;

/*
 * Cahn-Hilliard step parameters (Sec. 3.1, 4.1, 4.4).
 *  eps, dt      > 0
 *  tol          stop when max|v^{k+1} - v^k| < tol (ignored if fixed_iters > 0)
 *  sigma0       f'(0) of the shifted reaction; 2 for Cahn-Hilliard
 *  stepper      MOLT_BE, MOLT_BDF2 or MOLT_BDF3 (ch_step, ch_solve, Cahn-Hilliard
 *               model; the vector model and batched and served instances take
 *               MOLT_BE or MOLT_BDF2: MOLT_EUNSUPPORTED otherwise)
 *  max_iter     iteration cap (the step reports MOLT_NOT_CONVERGED if reached)
 *  init         MOLT_INIT_PREV or MOLT_INIT_LINEAR
 *  precision    MOLT_F64 or MOLT_F32
 *  fixed_iters  > 0: run exactly this many iterations (parity mode)
 *  have_prev    ch_step only: history fields held by d_u_prev.  BDF2: 1 if
 *               d_u_prev holds u^{n-1} (a BDF2 step), 0 for the start-up step
 *               (taken as BE).  BDF3: d_u_prev holds two fields,
 *               [u^{n-1} | u^{n-2}]; 2 gives a BDF3 step, less an SDIRK2 step.
 *  model        MOLT_MODEL_CH, or MOLT_MODEL_VCH: u = (u1, u2) with
 *               W(u) = prod_i |u - z_i|^2 over the cube roots of unity z_i; the
 *               scheme shifts by z_3 and the paper's sigma0 is 18 (Sec. 5.2).
 *               Every field of a VCH problem holds two components,
 *               component-major: u1 at [0, nx*ny), u2 at [nx*ny, 2*nx*ny).
 */
typedef struct {
  double eps, dt, tol;
  double sigma0;
  int32_t stepper;
  int32_t max_iter;
  int32_t init;
  int32_t precision;
  int32_t fixed_iters;
  int32_t have_prev;
  int32_t model;
  int32_t reserved;  /* 0 */
} molt_ch_params;

/* Per-step report.  residual: last max-norm increment (FP64); mass and energy
 * of u^{n+1} (FP64 reductions; periodic: h-weighted sum / forward-difference
 * energy, non-periodic: trapezoid weights; VCH: the energy of
 * eq. EnergyFunctional_vector, mass of u1, mass2 of u2); s1 >= s2: the factors
 * of (I - s1 Lap)(I - s2 Lap); sigma: the linear part moved to the left side. */
typedef struct {
  int32_t iters;
  int32_t converged;
  double residual;
  double mass, energy;
  double s1, s2, sigma;
  double mass2;
} molt_step_info;

/*
 * mol_t_helmholtz_sweep -- apply L^{-1} = (I - d^2/alpha^2)^{-1} along one axis
 * of `batch` stacked fields (Sec. 3.2: eqs. IL/IR recursions with the order-M
 * local quadrature, I = (IL + IR)/2, plus the boundary terms B_a e^{-alpha(x-a)}
 * + B_b e^{-alpha(b-x)}).
 *  axis: 0 = x (every row), 1 = y (every column; the identity when ny == 1).
 *  d_in, d_out: batch*ny*nx elements each; d_in == d_out is allowed.
 *  d_work: at least molt_sweep_workspace_bytes() bytes (may be 0 for axis x).
 * Asynchronous on `stream`.
 */
int32_t mol_t_helmholtz_sweep(const molt_grid* grid, int32_t axis, double alpha, int32_t precision,
                              const void* d_in, void* d_out, int64_t batch, void* d_work,
                              size_t work_bytes, void* stream);
size_t molt_sweep_workspace_bytes(const molt_grid* grid, int32_t axis, int32_t precision, int64_t batch);

/*
 * mol_t_helmholtz_sweep_noalloc -- mol_t_helmholtz_sweep without a workspace,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, same kernels and the same results (bit for bit) as
 * mol_t_helmholtz_sweep, except:
 *  - The y sweep's scratch (segment totals and seeds, closing-cell
 *    quadratures) is a static device array of MOLT_NOALLOC_SCRATCH_BYTES
 *    (molt_noalloc_scratch_bytes()) that each device the library runs on holds
 *    until the process ends.  A y sweep that needs more returns
 *    MOLT_EUNSUPPORTED (it needs about 2*nx*ny*batch*esz/(4*ky) bytes, ky the
 *    shape table's nodes per thread: a 4096 x 4096 FP32 field in one call).
 *  - In-place y sweeps (d_in == d_out) return MOLT_EINVAL: they need a copy of
 *    the field, which only the workspace variant has room for.
 *  - Every call on one device shares that device's array: calls that overlap on
 *    one device (several streams or threads) race and must be serialized by
 *    the caller.  Nothing needs clearing between calls.
 * No hipMalloc, hipFree or allocating library call is made.  The first call on a
 * device looks up the array's address on that device (it must be current).
 * Asynchronous on `stream`.
 */
#define MOLT_NOALLOC_SCRATCH_BYTES (16u * 1024u * 1024u)
int32_t mol_t_helmholtz_sweep_noalloc(const molt_grid* grid, int32_t axis, double alpha, int32_t precision,
                                      const void* d_in, void* d_out, int64_t batch, void* stream);
size_t molt_noalloc_scratch_bytes(void);

/*
 * ch_workspace_bytes -- bytes of device workspace ch_step / ch_solve need for
 * this grid and these parameters (0 on invalid arguments).
 */
size_t ch_workspace_bytes(const molt_grid* grid, const molt_ch_params* params);

/*
 * ch_step -- one time step of the Cahn-Hilliard equation (Sec. 3.1 eq. CH_BE,
 * Sec. 4.1 eq. BDF2) by the factored fixed point of Sec. 5.1.
 *  d_u:      in u^n, out u^{n+1} (the paper's u; the shift v = u+1 is internal).
 *            Dirichlet grids: the walls hold the homogeneous condition of the
 *            shifted variable (eq. CahnHilliard_v), u = -1 (vector model:
 *            u = z3 = (-1/2, -sqrt(3)/2)); u^n (and the histories) must hold
 *            that value on the walls, and u^{n+1} keeps it.  The step shifts
 *            d_u and the histories in place while it runs and back after it
 *            (so they may differ from their inputs by one rounding).
 *  d_u_prev: BDF2 history.  If params->have_prev and stepper == BDF2 it holds
 *            u^{n-1} and a BDF2 step is taken; otherwise a BE step.  If not
 *            NULL it receives u^n on return (history rotated in place).  BDF3:
 *            two fields [u^{n-1} | u^{n-2}] (see have_prev), rotated likewise.
 *  info:     filled when not NULL.
 * Synchronizes `stream` before returning.  The library remembers the
 * iteration count of the last step run in each workspace and uses it to size
 * its batches of queued iterations on the next call with that workspace
 * (results do not depend on it).
 */
int32_t ch_step(const molt_grid* grid, const molt_ch_params* params, void* d_u, void* d_u_prev,
                void* d_work, size_t work_bytes, molt_step_info* info, void* stream);

/*
 * ch_solve -- nsteps steps from d_u (BDF2: BE start-up step, then BDF2; BDF3:
 * two SDIRK2 start-up steps, then BDF3; the history kept in the workspace).
 * per_step: nsteps entries or NULL (an SDIRK2 step reports both stages'
 * iterations).
 * Returns MOLT_NOT_CONVERGED if any step reached max_iter.
 */
int32_t ch_solve(const molt_grid* grid, const molt_ch_params* params, void* d_u, int64_t nsteps,
                 void* d_work, size_t work_bytes, molt_step_info* per_step, void* stream);

/*
 * Adaptive time steps (Sec. 6, Algorithm 1) with the BE-BDF2 estimator.  Each
 * attempt solves a BE step and a variable-step BDF2 step (step ratio
 * w = dt_n/dt_{n-1}: v^{n+1} - beta dt F = rc0 v^n + rc1 v^{n-1} with
 * beta = (1+w)/(1+2w), rc0 = (1+w)^2/(1+2w), rc1 = -w^2/(1+2w)) from the same
 * state; eta = max|u_BE - u_BDF2| and the BDF2 solution is kept.  The first
 * step has no history and uses Algorithm 1's Richardson estimate of BE
 * (eta = max|u_dt - u_dt/2|/2, keeping the two half steps).  Then, with
 * N_it the largest iteration count of the attempt:
 *   eta <= lte_tol, N_it/nmaxit < 0.7:  accept, dt *= min(theta sqrt(lte_tol/eta), gamma)
 *   eta <= lte_tol, N_it/nmaxit < 1:    accept, dt *= min(theta sqrt(lte_tol/eta), 1)
 *   eta <= lte_tol, N_it >= nmaxit:     reject, dt /= gamma
 *   eta > lte_tol:                      reject, dt /= gamma if eta/lte_tol > 2,
 *                                       else dt *= theta sqrt(lte_tol/eta)
 * params: as for ch_step (stepper, dt, have_prev and fixed_iters are ignored;
 * max_iter is nmaxit).  The last step is shortened to end at t_end.
 * rec: one record per attempt (up to max_rec; *nrec = attempts made).
 * Returns MOLT_NOT_CONVERGED if max_attempts ended the run early or the step
 * fell below dt_min.  Synchronizes `stream`.
 */
typedef struct {
  double t_end;        /* integrate from t = 0 to t_end */
  double dt0;          /* first trial step */
  double lte_tol;      /* the error tolerance of Algorithm 1 */
  double theta, gamma; /* safety factors (0.8, 1.3 in the paper) */
  double dt_min, dt_max;
  int32_t nmaxit;      /* N_maxit: iteration cap of every solve */
  int32_t max_attempts;
} molt_adapt_params;

typedef struct {
  double t, dt, eta;   /* start time, trial step, error estimate */
  int32_t iters;       /* largest fixed-point iteration count of the attempt */
  int32_t accepted;
  double energy;       /* energy of the accepted state (0 if rejected) */
} molt_adapt_record;

size_t ch_adaptive_workspace_bytes(const molt_grid* grid, const molt_ch_params* params);
int32_t ch_solve_adaptive(const molt_grid* grid, const molt_ch_params* params, const molt_adapt_params* adapt,
                          void* d_u, void* d_work, size_t work_bytes, molt_adapt_record* rec, int32_t max_rec,
                          int32_t* nrec, double* t_final, void* stream);

/*
 * Batched instances (independent problems advanced together on one device).
 *  grid, params: as for ch_solve; params.have_prev is ignored (a BDF2
 *                instance starts with a BE step, as in ch_solve).
 *  d_u:          the instance's device field, u^0 in, u^nsteps out.
 *  nsteps:       time steps of this instance (0: left unchanged).
 * Every instance must use the same precision and be two-dimensional (ny > 1)
 * with periodic or Neumann boundaries; sizes, eps, dt, stepper, tolerance,
 * order M and boundary kind may differ.  Instances must not share fields.
 */
typedef struct {
  molt_grid grid;
  molt_ch_params params;
  void* d_u;
  int64_t nsteps;
} molt_instance;

/* Bytes of device workspace ch_solve_batch needs (0 on invalid arguments). */
size_t ch_batch_workspace_bytes(const molt_instance* inst, int32_t count);

/*
 * ch_solve_batch -- ch_solve of `count` instances at once (1..65535).  Each
 * instance advances through its own steps: every device tick runs one
 * fixed-point iteration (Sec. 5.1) for every instance that is iterating, and
 * the rhs sweeps R = A1^{-1} A2^{-1} rhs (Sec. 3.1, 4.1) for every instance
 * that starts a step, so instances with few iterations per step do not wait
 * for the others.  An instance's results are bitwise independent of the other
 * instances in the batch.
 *  per_step: sum(nsteps) records, instance-major (instance 0's steps first),
 *            or NULL.
 * Returns MOLT_NOT_CONVERGED if any step of any instance reached max_iter.
 * Synchronizes `stream` before returning.  With a non-NULL stream the ticks
 * are replayed as a captured HIP graph (see MOLT_OPT_BATCH_GRAPH).
 */
int32_t ch_solve_batch(const molt_instance* inst, int32_t count, void* d_work, size_t work_bytes,
                       molt_step_info* per_step, void* stream);

/*
 * Serving (continuous batching).  A server is a resident batched engine on
 * one stream: requests are queued in submission order and admitted as soon as
 * a slot and enough of the server's workspace pool are free (the footprint of
 * a request is molt_server_footprint: its ch_solve workspace plus its step
 * records); admitted requests advance together (the ticks of ch_solve_batch)
 * and leave as soon as their last step ends, freeing their slot and memory
 * for the next request.  A request's fields stay where the caller put them
 * (device memory the caller owns and must not touch until the result is
 * polled); its result is bitwise the same as alone or in any mix.
 *  molt_server_bytes:  workspace for max_slots slots and a pool of pool_bytes.
 *  molt_server_create: a server on a non-NULL stream over the caller's
 *                      workspace (descriptors, control words, block maps, then
 *                      the pool); allocates two small pinned host buffers.
 *  molt_server_submit: queue a request (checked like a ch_solve_batch
 *                      instance; its precision must be the server's;
 *                      MOLT_EUNSUPPORTED if it can never fit the pool).
 *  molt_server_run:    admit what fits, then queue `rounds` rounds of ticks
 *                      (MOLT_OPT_BATCH_TICKS each); the rounds before the last
 *                      one are retired, their finished requests become
 *                      results.  Reports the admitted and queued counts.  With
 *                      nothing admitted or queued it drains and returns.
 *  molt_server_poll:   move up to max_results finished results out (in the
 *                      order they finished); returns how many.
 *  molt_server_destroy: synchronize the stream and release the server.
 * One thread drives a server; servers on different streams are independent.
 */
typedef struct molt_server molt_server;
typedef struct {
  int64_t id;            /* the submit id */
  int32_t status;        /* MOLT_OK or MOLT_NOT_CONVERGED (some step reached max_iter) */
  int32_t steps;
  int64_t iters;         /* fixed-point iterations over all steps */
  molt_step_info last;   /* the last step's report */
} molt_result;
size_t molt_server_footprint(const molt_instance* inst);
size_t molt_server_bytes(int32_t precision, int32_t max_slots, size_t pool_bytes);
int32_t molt_server_create(int32_t precision, int32_t max_slots, void* d_work, size_t work_bytes, void* stream,
                           molt_server** out);
int32_t molt_server_submit(molt_server* server, const molt_instance* inst, int64_t id);
int32_t molt_server_run(molt_server* server, int32_t rounds, int32_t* active, int32_t* queued);
int32_t molt_server_poll(molt_server* server, molt_result* out, int32_t max_results);
int32_t molt_server_destroy(molt_server* server);

/*
 * Line-block shapes (not part of the method; they change only the rounding
 * order of the scans).  Per precision and line-length class (class c holds
 * lines of n <= 128 * 2^c nodes, c = 0..MOLT_TUNE_CLASSES-1, the last class
 * up to the longest supported line) the table holds kx, the nodes per thread
 * of an x-line (4, 8, 16, 32 FP32 only; a line is owned by at most 256
 * threads, n <= 256*kx, or for lines longer than 2048 nodes by 512 threads,
 * n <= 512*kx), and ky, the nodes per thread of a y-line (4, 8, 16 FP32 only).
 * Every path reads the table at call time, so ch_step, ch_solve and
 * ch_solve_batch agree bit for bit under one table (the batched kernels give
 * a row at most 256 threads: for a class whose kx needs 512 they take the
 * smallest kx that fits 256, and agree with the others to rounding only).
 * Process-wide; change it only while no solve is running.
 *  molt_tune_get / molt_tune_set: read / write one class (MOLT_EINVAL if the
 *    shape is not valid for the class).
 *  molt_autotune: for every class up to max_n (128..8192 FP32, ..4096 FP64),
 *    times an iteration y-pass for each ky, then an iteration x-pass for each
 *    kx, on an n x n periodic field in the caller's workspace (at least
 *    molt_autotune_workspace_bytes), and stores the fastest shapes; the
 *    current entry is timed first and a shape replaces it only when at least
 *    3 % faster (8 timed launches each), so that repeated tunings agree.
 *    Synchronizes `stream`.
 */
#define MOLT_TUNE_CLASSES 7
int32_t molt_tune_get(int32_t precision, int32_t size_class, int32_t* kx, int32_t* ky);
int32_t molt_tune_set(int32_t precision, int32_t size_class, int32_t kx, int32_t ky);
size_t molt_autotune_workspace_bytes(int32_t precision, int32_t max_n);
int32_t molt_autotune(int32_t precision, int32_t max_n, void* d_work, size_t work_bytes, void* stream);

/*
 * Kernel timing (not part of the method): HIP events recorded around every
 * kernel the library launches, on the launch stream, accumulated per kind.
 * kind = family*8 + program, plus 48 for FP64 launches (an FP32 step runs its
 * R sweeps and first iteration in FP64); family 0 x-pass, 1 y-pass totals,
 * 2 y-pass combine, 3 y-pass final, 4 pointwise, 5 other; program 0 sweep,
 * 1 rhs sweep, 2-5 the four fixed-point passes P1-P4.  molt_profile(1) enables and resets,
 * molt_profile(0) disables; molt_profile_read fills up to max_entries kinds
 * that ran and returns how many.  molt_profile_only(kind) restricts the timing
 * to one kind (two events per launch of it, none elsewhere: the events cost
 * the stream a few microseconds each), molt_profile_only(-1) times every kind
 * again; MOLT_EINVAL for a kind outside -1..95.  Process-wide; use from one
 * thread.
 */
typedef struct {
  int32_t kind;
  int64_t launches;
  double total_ms;
} molt_prof_entry;
int32_t molt_profile(int32_t enable);
int32_t molt_profile_only(int32_t kind);
int32_t molt_profile_read(molt_prof_entry* out, int32_t max_entries);

/*
 * Tuning options (process-wide; not part of the method).
 * Returns MOLT_OK or MOLT_EINVAL for an unknown option or a value out of range.
 */
/*  MOLT_OPT_BATCH_TICKS (1..1024, default 8): device ticks of ch_solve_batch
 *    between two host checks of whether every instance has finished.
 *  MOLT_OPT_BATCH_GRAPH (0 or 1, default 1): replay those ticks as one
 *    captured HIP graph (used when the stream is not NULL and kernel timing is
 *    off); 0 launches the kernels one by one. */
/*  MOLT_OPT_BATCH_LEAN (0..1024, default 16): in ch_solve_batch (not the
 *    server), with at most this many instances still running, every tick of a
 *    round but its last runs the iteration
 *    only (no step finish): fewer launches per iteration for the last long
 *    instances, while an instance that converged waits for the round's end
 *    to start its next step.  Results are unchanged. */
/*  MOLT_OPT_STEP_GRAPH (0 or 1, default 1): in ch_step, ch_solve and the
 *    drivers built on them, launch runs of 4 increment-form iterations as one
 *    executable HIP graph, captured on a private stream of the library the
 *    first time a run with those arguments is needed and kept (at most 8 per
 *    process, least recently used replaced); off while kernel timing is on.
 *    0 launches every kernel on the caller's stream.  Results are unchanged. */
#define MOLT_OPT_BATCH_TICKS 2
#define MOLT_OPT_BATCH_GRAPH 3
#define MOLT_OPT_BATCH_LEAN 5
#define MOLT_OPT_STEP_GRAPH 6
int32_t molt_set_option(int32_t option, int64_t value);

/* Static name of a status code. */
const char* molt_strerror(int32_t status);

/* Last detailed error message of the calling thread ("" if none). */
const char* molt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MOLT_H */
