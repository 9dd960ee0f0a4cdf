/*
 * fvm.h -- C ABI of the MI355X (gfx950) first-order finite-volume library.
 *
 * The library advances a two-dimensional system of conservation laws
 *     dW/dt + div F(W) = S(W)                       (Sec. 2.1)
 * on an Nx x Ny Cartesian grid with the explicit first-order scheme
 *     W* = W^n - dt/dx (F~_{i+1/2} - F~_{i-1/2}) - dt/dy (G~_{j+1/2} - G~_{j-1/2})
 *                                                   (Sec. 2.2.1, eq. VF_scheme)
 * followed by the split source step W^{n+1} = W* + dt S(W*)
 *                                                   (Sec. 2.2.2, eq. SourceTerm)
 * and a time-step reduction over the characteristic speeds
 *                                                   (Sec. 2.2.1, eq. CFL_cond).
 *
 * Models: linear advection (upwind flux), the Euler equations of a perfect
 * gas with the Lax-Friedrichs (Rusanov) flux (Sec. 5, eq. Euler), and the
 * six-moment evaporating-spray system with a kinetic upwind flux and an
 * evaporation + drag source (Sec. 6.1, eq. Essadki).
 *
 * Conventions common to every call
 * --------------------------------
 *  - States are FP64 in device memory, one contiguous row of nx values (row
 *    pitch ld >= nx elements) per variable and grid row, 0 <= i < nx,
 *    0 <= j < ny, in one of two layouts (fvm_params.layout):
 *      FVM_LAYOUT_PLANES: variable v of cell (i, j) at w[(v * ny + j) * ld + i]
 *                         (one plane per variable);
 *      FVM_LAYOUT_ROWS:   at w[(j * nVar + v) * ld + i] (the nVar rows of a
 *                         grid row are adjacent in memory).
 *    Both hold nVar * ny * ld doubles and give bitwise the same results; the
 *    row layout streams faster on HBM3E (fewer far-apart streams per strip).
 *    Cell centres are ((i+1/2)dx, (j+1/2)dy),
 *    dx = lx/nx, dy = ly/ny. nVar is 1 (advection), 4 (Euler: rho, rho u,
 *    rho v, rho E) or 6 (spray: m_0, m_{1/2}, m_{2/2}, m_{3/2}, q_x, q_y).
 *  - The caller owns all device memory (state buffers, the spray gas
 *    velocity, scratch, checkpoints, adjoint buffers). The library never
 *    allocates or frees device memory. Host-side plans (fvm_grid, fvm_batch)
 *    are allocated by the library and released by the matching destroy call.
 *  - Every call that launches work enqueues it asynchronously on the stream
 *    given at bind time (a hipStream_t passed as void*; NULL = the null
 *    stream) and returns without waiting. Errors detected on the device (a
 *    non-finite or non-physical state, a failed CFL check) are recorded in a
 *    sticky status word in the scratch buffer and returned by the next
 *    synchronising call (fvm_sync, fvm_cfl_dt_host, fvm_get_status).
 *  - Every function returns an int status; no exception or abort crosses the
 *    ABI. Invalid arguments are rejected before anything is enqueued.
 *  - Calls on one grid must not overlap from several host threads.
 */
#ifndef FVM_H
#define FVM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FVM_OK 0
#define FVM_EINVAL (-1)       /* bad shape, pitch, pointer, dt or parameter  */
#define FVM_EDEVICE (-2)      /* a HIP runtime call failed                   */
#define FVM_ECFL (-3)         /* fixed-dt step failed the CFL check          */
#define FVM_ENONFINITE (-4)   /* NaN/inf speed, rho <= 0, p < 0, m_k < 0     */
#define FVM_EUNSUPPORTED (-5) /* operation not available for this model      */
#define FVM_EIO (-6)          /* a snapshot file could not be written        */

/* ---- models and boundary conditions ------------------------------------ */
#define FVM_ADV 0    /* u_t + a.grad u = 0, flux a+ u_L + a- u_R             */
#define FVM_EULER 1  /* Sec. 5 eq. (Euler), Lax-Friedrichs flux (Sec. 2.2.1) */
#define FVM_SPRAY 2  /* Sec. 6.1 eq. (Essadki), kinetic upwind flux          */

#define FVM_PERIODIC 0     /* the domain wraps around (Sec. 5)                */
#define FVM_TRANSMISSIVE 1 /* ghost cell = boundary cell (zero gradient)      */
#define FVM_DIRICHLET 2    /* ghost cell = a prescribed state per side         */

#define FVM_CLOSURE_LOGNORMAL 0 /* spray n(S=0), m_{-1/2}: lognormal fit       */
#define FVM_CLOSURE_MAXENT 1    /* the entropy maximiser (Sec. 6.2)             */

#define FVM_LAYOUT_PLANES 0 /* w[(v * ny + j) * ld + i]                       */
#define FVM_LAYOUT_ROWS 1   /* w[(j * nVar + v) * ld + i]; nVar * ld <= 2^31-1 */

typedef struct fvm_params {
  int model;     /* FVM_ADV, FVM_EULER or FVM_SPRAY                          */
  int bc;        /* FVM_PERIODIC, FVM_TRANSMISSIVE or FVM_DIRICHLET          */
  int nx, ny;    /* cells, >= 1 each                                         */
  int npart_x;   /* NPartX: balanced subdomains along x, nx % npart_x == 0   */
  int npart_y;   /* NPartY (Sec. 3.2); the result does not depend on them    */
  int ld;        /* row pitch in elements, >= nx                             */
  int layout;    /* FVM_LAYOUT_PLANES or FVM_LAYOUT_ROWS                     */
  double lx, ly; /* domain lengths (> 0); dx = lx/nx, dy = ly/ny             */
  double gamma;  /* Euler: ratio of specific heats (> 1)                     */
  double ax, ay; /* advection velocity                                       */
  double K;      /* spray: evaporation rate (>= 0)                           */
  double theta;  /* spray: drag relaxation time (> 0; +inf = no drag)        */
  double s_eps;  /* spray: size at which n(S=0) is evaluated (0 < s_eps < 1) */
  double cfl;    /* Courant number C of the adaptive step (> 0)              */
  double dt_max; /* time step when every speed is zero (0 = error)           */
  int closure;   /* spray: FVM_CLOSURE_LOGNORMAL (fused into the step) or
                    FVM_CLOSURE_MAXENT (a transport step, then a source pass
                    that reconstructs n(S) per cell; periodic or transmissive
                    boundaries, no halo rows); 0 for the other models       */
} fvm_params;

typedef struct fvm_grid fvm_grid;
typedef struct fvm_batch fvm_batch;

/* Human-readable text of a status code. Never NULL. */
const char* fvm_strerror(int status);

/* nVar of a model, or 0 for an unknown model. */
int fvm_nvar(int model);

/* Checks a parameter set: FVM_OK or FVM_EINVAL (including nx % npart_x or
 * ny % npart_y != 0, the balanced-subdomain rule of Sec. 3.2). */
int fvm_validate(const fvm_params* p);

/* Bytes of device scratch a grid needs (speed maxima, arrival counter, time
 * step, status word); a multiple of 256. */
size_t fvm_scratch_bytes(const fvm_params* p);

/* ---- single grid ------------------------------------------------------- */

/* Creates a host-side plan for one grid. No device work, no allocation of
 * device memory. *out receives the plan (NULL on error). */
int fvm_create(const fvm_params* p, fvm_grid** out);

/* Releases the plan and any cached HIP graphs. NULL is accepted. */
int fvm_destroy(fvm_grid* g);

/* Binds caller-owned device memory and a stream to the plan:
 *   w_a, w_b : two state buffers of nVar * ny * ld doubles each (ping-pong);
 *              w_a holds the current state after binding;
 *   ug       : spray only, the gas velocity (u_gx, u_gy) as a 2-variable
 *              field with the state's ld and layout (2 * ny * ld doubles),
 *              read-only; NULL for other models;
 *   scratch  : fvm_scratch_bytes(p) bytes, 256-byte aligned;
 *   stream   : hipStream_t (void*), NULL = null stream.
 * Enqueues a kernel that clears the scratch (speeds unknown, status 0). */
int fvm_bind(fvm_grid* g, double* w_a, double* w_b, const double* ug,
             void* scratch, void* stream);

/* Dirichlet boundaries (bc == FVM_DIRICHLET): the state of the ghost cells
 * beyond each side of the domain, the overlap a subdomain at the domain's
 * edge receives (Sec. 4.2). ghost is a host array of 4 * nVar doubles, the
 * conservative states of the west (i = -1), east (i = nx), south (j = -1)
 * and north (j = ny) sides in that order; the plan keeps a copy, used by the
 * steps enqueued after the call. FVM_EINVAL for another boundary condition
 * or a non-finite value. Until the first call the ghost states are zero. */
int fvm_set_boundary_states(fvm_grid* g, const double* ghost);

/* Halo rows (the one-GPU share of the multi-GPU decomposition into slabs):
 * south and north are caller-owned device buffers, each one row of the
 * state in the layout [v * ld + i] (nVar * ld doubles), that the steps read
 * as rows j = -1 and j = ny instead of applying the boundary condition
 * there -- the rows a slab receives from its neighbours, as the overlap
 * strips of Sec. 3.2 / 4.1 carry them between subdomains. NULL leaves that
 * side to the boundary condition. The buffers are read when each step runs,
 * so the caller may refresh them between steps on the same stream. The
 * adjoint calls return FVM_EUNSUPPORTED while a halo row is set, and so does
 * this call for a grid with Dirichlet boundaries. */
int fvm_set_halo_rows(fvm_grid* g, const double* south, const double* north);

/* Entropy-maximising spray closure (FVM_CLOSURE_MAXENT): a caller-owned
 * device buffer of 4 * ny * nx doubles (contents need not be initialised)
 * in which the source pass keeps every cell's converged multipliers, so
 * that the next step's Newton iteration starts from them (it falls back to
 * the cold start where that fails). Results agree with the cold start within
 * the convergence tolerance, not bit for bit. NULL (the default) turns it
 * off; setting a state forgets the kept multipliers. FVM_EUNSUPPORTED for a
 * non-NULL buffer on any other closure. The buffer must stay valid while
 * set. */
int fvm_set_closure_buffer(fvm_grid* g, double* lam);

/* Changes the stream later calls enqueue on. */
int fvm_set_stream(fvm_grid* g, void* stream);

/* Device pointer of the buffer that holds the current state. */
int fvm_current(const fvm_grid* g, double** w);

/* Copies a state (the grid's ld and layout) into the current buffer; src
 * is a host pointer if src_on_device == 0 (the call then waits for the
 * copy), else a device pointer (asynchronous). Marks the speed maxima as
 * unknown. */
int fvm_set_state(fvm_grid* g, const double* src, int src_on_device);

/* Copies the current state (ld and layout kept) to dst; a host destination
 * makes the call wait. */
int fvm_get_state(fvm_grid* g, double* dst, int dst_on_device);

/* Speed maxima of the current state (checkTimeStep, Sec. 4.2) and the
 * adaptive time step dt = C / (Sx/dx + Sy/dy), where Sx (Sy) is the largest
 * |eigenvalue| along x (y) over all cells. Asynchronous; the dt is kept on the
 * device for the next adaptive step and also written to *dt_dev if non-NULL
 * (device pointer). */
int fvm_cfl_dt(fvm_grid* g, double* dt_dev);

/* As fvm_cfl_dt, then waits and returns dt (and the maxima if non-NULL) on
 * the host; returns the sticky device status. */
int fvm_cfl_dt_host(fvm_grid* g, double* dt, double* sx, double* sy);

/* One step with a caller-given dt > 0. The step first checks the paper's
 * condition dt * max_cells max_p |lambda_p| <= min(dx, dy) (eq. CFL_cond) on
 * the device; if it fails the state is left unchanged and FVM_ECFL is
 * recorded in the sticky status. */
int fvm_step(fvm_grid* g, double dt);

/* nsteps adaptive steps: step n uses dt_n = C / (Sx^n/dx + Sy^n/dy) computed
 * on the device from the maxima of W^n, which the previous step produced in
 * its epilogue. If dts_dev is non-NULL (device, >= nsteps doubles) it
 * receives dt_0 .. dt_{nsteps-1}. Replays a cached HIP graph. */
int fvm_run(fvm_grid* g, int nsteps, double* dts_dev);

/* nsteps steps with the given time steps (device array, no CFL logic): the
 * frozen-dt replay used by the adjoint and by finite-difference checks. */
int fvm_run_dts(fvm_grid* g, int nsteps, const double* dts_dev);

/* nsteps steps with one fixed time step dt (> 0, finite), the policy of
 * Sec. 2.2.1: before each step the state's largest speed is checked against
 * eq. CFL_cond, dt * max(Sx, Sy) <= min(dx, dy), as the checkTimeStep task
 * does (Sec. 4.2). A step that fails the check leaves the state unchanged and
 * sets the sticky FVM_ECFL status (so does every later step of the run); the
 * next synchronising call reports it. Replays a cached HIP graph. */
int fvm_run_fixed(fvm_grid* g, int nsteps, double dt);

/* As fvm_run, and stores checkpoints: ckpts[s] (host array of device
 * pointers, ceil(nsteps / ckpt_every) of them, each a full state in the grid's
 * ld and layout) receives W^{s * ckpt_every}. The step that produces a checkpointed
 * state writes it straight into the checkpoint buffer. */
int fvm_run_ckpt(fvm_grid* g, int nsteps, int ckpt_every,
                 double* const* ckpts, double* dts_dev);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): fvm_run without a plan
 * and without a scratch buffer. It allocates nothing, host or device, and
 * builds no graph: it enqueues plain kernel launches on `stream` (hipStream_t
 * as void*, NULL = null stream) and returns.
 *   p         : parameters as for fvm_create; periodic or transmissive
 *               boundaries and the lognormal closure (FVM_EUNSUPPORTED for
 *               Dirichlet boundaries and the entropy closure);
 *   w_a, w_b  : two state buffers as for fvm_bind; w_a holds W^0 on entry.
 *               Step k reads one and writes the other, so W^nsteps ends in
 *               w_a if nsteps is even and in w_b if it is odd;
 *   ug        : the spray's gas velocity (as for fvm_bind), NULL otherwise;
 *   dts_dev   : nullable device array of >= nsteps doubles, receives
 *               dt_0 .. dt_{nsteps-1};
 *   status_dev: nullable device int, receives at the end FVM_OK,
 *               FVM_ENONFINITE (a non-finite or non-physical state) or
 *               FVM_EINVAL (every speed zero and dt_max == 0).
 * The steps, tile shape and results are those of fvm_run with the default
 * tiling (bitwise: the result does not depend on the tiling). The scratch
 * block (fvm_scratch_bytes(p) bytes, at most 256) lives in a static device
 * array of 256 bytes per device, kept until the process ends; parameters
 * needing more are rejected with FVM_EINVAL. Each call clears it with a
 * kernel before its steps. Calls that overlap on one device (several host
 * threads, or several streams in flight) share that array and race.
 * Invalid arguments are rejected before anything is enqueued. */
int fvm_run_noalloc(const fvm_params* p, double* w_a, double* w_b,
                    const double* ug, int nsteps, double* dts_dev,
                    int* status_dev, void* stream);

/* Waits for the stream and returns the sticky device status. */
int fvm_sync(fvm_grid* g);

/* Waits, then returns the sticky device status (and clears it if clear != 0). */
int fvm_get_status(fvm_grid* g, int clear);

/* Gradient of a loss of the final state with respect to the initial state,
 * through nsteps steps with frozen time steps (every model, closure and
 * boundary condition; FVM_EUNSUPPORTED with halo rows). A transmissive ghost is
 * a copy of its boundary cell, so its sensitivity goes to that cell; a
 * Dirichlet ghost is a constant state and takes none. The adjoint of one
 * transport step is
 *   lam^n = lam^{n+1} + dt/dx [J_L(i+1/2)^T (lam_{i+1} - lam_i)
 *                             + J_R(i-1/2)^T (lam_i - lam_{i-1})] + (same in y)
 * with J_L, J_R the Jacobians of the numerical flux with respect to its left
 * and right states (derived from Sec. 2.2.1; max() follows its left argument
 * on ties). For the spray the split source of Sec. 2.2.2 comes first:
 * lam^{n+1} is replaced by lam^{n+1} + dt J_S(W*)^T lam^{n+1}, with J_S the
 * Jacobian of the source of Sec. 6.1 at the transported state W* (a clipped
 * lognormal width counts as a constant), before the transport's adjoint.
 * With the entropy-maximising closure (Sec. 6.2) the closure rows of J_S
 * come from the dual's optimality conditions at the converged multipliers:
 * d lambda / d m = H^{-1}, H the moment Hessian; each such step runs the
 * transport step, the source's adjoint and the transport's adjoint in the
 * grid's free ping-pong buffer (the one not holding the current state), so
 * none of the buffers below may be that one (FVM_EINVAL), and it holds no
 * state afterwards; Newton starts cold in every cell.
 * Inputs (all device memory, the grid's ld and layout):
 *   ckpts[s]   : host array of device pointers, W^{s * ckpt_every}, as
 *                written by fvm_run_ckpt;
 *   dts_dev    : the nsteps forward time steps;
 *   lam        : in: dL/dW^N; out: dL/dW^0;
 *   lam_tmp    : one state of workspace;
 *   seg_buf    : (ckpt_every - 1) states of workspace for the recomputed
 *                forward states of one segment (may be NULL if ckpt_every
 *                is 1).
 * Each segment recomputes its forward states from its checkpoint with the
 * forward kernel, then runs its adjoint steps in reverse. Asynchronous. */
int fvm_adjoint_run(fvm_grid* g, double* const* ckpts, int ckpt_every,
                    const double* dts_dev, int nsteps, double* lam,
                    double* lam_tmp, double* seg_buf);

/* One adjoint step at state w with time step dt: lam_out = (dW^{n+1}/dW^n)^T
 * lam_in (device pointers, the grid's ld and layout; lam_out must not alias
 * w or lam_in). The spray's step reads the bound gas velocity. Same
 * restrictions as fvm_adjoint_run (with the entropy closure none of w,
 * lam_in, lam_out may be the grid's free ping-pong buffer). Asynchronous. */
int fvm_adjoint_step(fvm_grid* g, const double* w, double dt,
                     const double* lam_in, double* lam_out);

/* Kernel tiling of the fused step: rows marched per wave strip and wave
 * strips per workgroup. 0 keeps the current value. Returns FVM_EINVAL for
 * values the kernels do not support. */
int fvm_set_tiling(fvm_grid* g, int rows_per_strip, int waves_per_block);
int fvm_get_tiling(const fvm_grid* g, int* rows_per_strip, int* waves_per_block);

/* Tile shape and lane layout of the adjoint kernel: rows per strip, waves
 * per block, and cells per lane (1, the default: 62-column strips; 2:
 * 128-column strips with 16-byte accesses, taken only where the pitch is even
 * and the state and multiplier buffers of a launch are 16-byte aligned, else
 * 1); 0 keeps the current value. fvm_autotune chooses among all of them.
 * Results do not depend on any of them. The spray's adjoint kernel ignores
 * them (it has one fixed tile shape). */
int fvm_set_adjoint_tiling(fvm_grid* g, int rows_per_strip, int waves_per_block,
                           int cells_per_lane);

/* Lanes of the fused step: 1 = one cell per lane (any pitch), 2 = two
 * adjacent cells per lane with 16-byte accesses (needs an even ld and 16-byte
 * aligned buffers; otherwise the call falls back to 1), 0 = the model's
 * default. Results are bitwise identical either way.
 * fvm_get_cells_per_lane returns the value in use. */
int fvm_set_cells_per_lane(fvm_grid* g, int cells_per_lane);
int fvm_get_cells_per_lane(const fvm_grid* g);

/* Resident runs: fvm_run on a grid whose two states fit in one workgroup's
 * LDS (2 x nVar x nx x ny <= 18432 doubles, e.g. advection up to 96 x 96,
 * Euler up to 48 x 48; no halo rows; the spray with the lognormal closure
 * only) executes all its adaptive steps (Sec. 2.2.1 eq. VF_scheme and
 * eq. CFL_cond, one dt per step) in one launch of one workgroup, which keeps
 * the state in LDS between steps, instead of one launch per step. States,
 * dts, the dt log, the maxima and the status are bitwise those of the step
 * launches; the other ping-pong buffer ends up holding the state before the
 * last step, as with step launches. enable != 0 (the default) allows it,
 * 0 forces step launches. FVM_EINVAL for a NULL grid. */
int fvm_set_resident_runs(fvm_grid* g, int enable);

/* Autotuner: picks the tiling and lane layout of the fused step by timing
 * dry-run steps of every candidate (dt = 0, which leaves the bound state bit
 * for bit unchanged) on the bound buffers and stream, re-times the six
 * fastest three more times over longer windows and applies the lowest
 * median, and, if cache_path is non-NULL, appends it to that text file; a
 * later call
 * with the same device, model, grid shape and layout reuses the stored
 * choice without timing (the spray's closure is part of the key). For
 * advection and Euler grids it then picks the adjoint kernel's tile shape
 * the same way (dry adjoint launches with dt = 0 that write the ping-pong
 * buffer not holding the current state). This is the analogue of the
 * paper's per-codelet performance models (Sec. 5.3.2): the task size that runs
 * fastest is chosen by measurement. Synchronises the stream. */
int fvm_autotune(fvm_grid* g, const char* cache_path);

/* Adjoint tuner on the caller's buffers: times adjoint steps with dt = 0
 * (lam_out receives lam_in bit for bit) of every tile shape and lane layout
 * on w and lam_in -> lam_out (distinct buffers of one state each, as
 * fvm_adjoint_step takes them), applies the fastest and caches it like
 * fvm_autotune (its own key). Separate multiplier buffers move the traffic
 * of real adjoint steps, which the in-place dry launches of fvm_autotune
 * only approximate. FVM_EUNSUPPORTED for the spray (its adjoint kernel has
 * one fixed tile shape) and where fvm_adjoint_step is.
 * Synchronises the stream. */
int fvm_autotune_adjoint(fvm_grid* g, const double* w, const double* lam_in, double* lam_out,
                         const char* cache_path);

/* ---- batches of independent grids -------------------------------------- */

/* Creates a plan for n independent grids solved together, one persistent
 * launch per time step for all of them (each grid keeps its own adaptive
 * dt). p[k] are the grids' parameters (all the same model and boundary
 * condition, not spray, not Dirichlet);
 * offsets[k] is the element offset of grid k's state inside the packed
 * buffers, a multiple of 32 elements (256 bytes). */
int fvm_batch_create(int n, const fvm_params* p, const size_t* offsets,
                     fvm_batch** out);
int fvm_batch_destroy(fvm_batch* b);

/* Scratch bytes of a batch (per-grid maxima, counters, dt, status, and the
 * per-grid records of the work list of (grid, group of strips) items). */
size_t fvm_batch_scratch_bytes(const fvm_batch* b);

/* Binds the packed state buffers (each holding every grid at its offset),
 * the scratch and a stream; w_a holds the current states. */
int fvm_batch_bind(fvm_batch* b, double* w_a, double* w_b, void* scratch,
                   void* stream);

/* Computes every grid's speed maxima and adaptive dt (asynchronous). */
int fvm_batch_cfl(fvm_batch* b);

/* nsteps adaptive steps of every grid, one persistent launch per step
 * replayed from a cached HIP graph. dts_dev (nullable) receives
 * dts_dev[s * n + k] = dt of grid k at step s. */
int fvm_batch_run(fvm_batch* b, int nsteps, double* dts_dev);

/* The same steps with one launch per grid per step (the reference schedule
 * the persistent launch is compared against). */
int fvm_batch_run_per_grid(fvm_batch* b, int nsteps, double* dts_dev);

/* Device pointer of the packed buffer holding the current states. */
int fvm_batch_current(const fvm_batch* b, double** w);

/* Waits and returns the sticky status of the batch. */
int fvm_batch_sync(fvm_batch* b);

/* Tile shape of the batched step: the tallest row block a strip marches
 * (each grid's blocks are of near-equal height, at most this) and the waves
 * per workgroup (1, 2, 4 or 8; a work item is that many strips of one grid);
 * 0 keeps the current value. Results do not depend on it. */
int fvm_batch_set_tiling(fvm_batch* b, int rows_per_strip, int waves_per_block);

/* Launch schedule of the batched step: persistent != 0 (the default) runs a
 * resident set of workgroups that take work items from an atomic queue;
 * 0 launches one workgroup per item and lets the hardware dispatcher
 * balance them. fit_blocks != 0 cuts each grid into row blocks (at most the
 * tiling's rows high) whose strip count fills whole workgroups where that
 * costs fewer wave-rows than idle waves would; 0 (the default) keeps blocks
 * of the tiling's height. Results are bitwise the same either way. */
int fvm_batch_set_schedule(fvm_batch* b, int persistent, int fit_blocks);

/* Lane layout of the batched step: cells_per_lane 2 (the default) runs two
 * adjacent cells per lane (16-byte accesses) on every grid whose pitch is
 * even and one elsewhere; 1 runs one cell per lane on every grid (a kernel
 * with fewer registers per lane, so more waves per SIMD, and fewer idle lanes
 * in each grid's last strip). Other values give FVM_EINVAL. Results are
 * bitwise the same either way. */
int fvm_batch_set_layout(fvm_batch* b, int cells_per_lane);

/* Autotuner of the batched step's tile shape and schedule (dry runs with
 * every dt scaled to 0, states unchanged); cache as for fvm_autotune, keyed
 * by the device, model and the list of grid shapes. Synchronises the
 * stream. */
int fvm_batch_autotune(fvm_batch* b, const char* cache_path);

/* ---- asynchronous solution output (Sec. 4.3) ----------------------------
 * The solution is dumped without holding up the time steps: a gather kernel
 * copies the current state, in stream order on the grid's stream, into one
 * contiguous output buffer (one dense plane per variable, pitch nx: the
 * global buffer whose NPartX x NPartY subdomain blocks are the per-part views
 * of that pitch, filled by all parts at once); the device-to-host copy of that
 * buffer runs on a second stream and the file is written by a host thread of
 * the output stage, while the grid's stream goes on with the next steps.
 *
 * Snapshot file: a 64-byte little-endian header
 *   char magic[8] = "FVMSNAP1"; int32 model, nvar, nx, ny;
 *   int64 step; double time, lx, ly; int32 npart_x, npart_y;
 * followed by nvar * ny * nx doubles, variable v of cell (i, j) at
 * (v * ny + j) * nx + i. */
typedef struct fvm_output fvm_output;

/* Output stage for a bound grid. staging: device buffer of
 * nVar * ny * nx doubles; host: pinned host buffer (hipHostMalloc or a pinned
 * tensor) of the same size; copy_stream: the hipStream_t (as void*) the
 * device-to-host copies run on, not the grid's stream. The caller owns the
 * three and keeps them alive until fvm_output_destroy returns; the grid must
 * outlive the stage and keep its shape. Starts the writer thread. */
int fvm_output_create(fvm_grid* g, double* staging, double* host, void* copy_stream,
                      fvm_output** out);

/* Enqueues one snapshot of the grid's current state, to be written to `path`
 * (copied) with the given step number and time in the header. Returns once
 * the gather and the copy are enqueued; it waits on the host only while the
 * previous snapshot's file is still being written from the host buffer.
 * Returns the first error of an earlier snapshot (FVM_EIO, FVM_EDEVICE) if
 * there was one. */
int fvm_output_snapshot(fvm_output* o, const char* path, long long step, double time);

/* Waits until every snapshot enqueued so far is on disk; returns FVM_OK or
 * the first error. */
int fvm_output_wait(fvm_output* o);

/* Waits for the pending snapshots, stops the writer thread and frees the
 * stage; returns what fvm_output_wait would. */
int fvm_output_destroy(fvm_output* o);

#ifdef __cplusplus
}
#endif

#endif /* FVM_H */
