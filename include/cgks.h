/*
 * cgks.h -- C ABI of libcgks.so: the ASE-DFF compact gas-kinetic scheme
 * (Mu, Zhang, Ji, Zhang, Chen, Xu, "Very high-order compact gas-kinetic
 * scheme with discontinuity feedback factor", arXiv 2508.13705) on one AMD
 * MI355X (gfx950).
 *
 * The library advances the compressible Euler / Navier-Stokes equations
 * W_t = -div F(W) (Sec. 2.2) on a uniform 1-D or 2-D Cartesian grid.  Its
 * state is the set of cell averages plus, per cell, the cell-averaged slope
 * (1-D) or the line-averaged slopes on the Gauss lines (2-D, Sec. 3.3); one
 * call of cgks_step is one two-stage fourth-order step (Eq. 2.13-2.23, 2.25,
 * 2.29, 2.30) with ASE-DFF reconstruction (Sec. 3, Algorithm 1) and the
 * gas-kinetic interface flux (Eq. 2.6-2.8).
 *
 * Conventions (all functions):
 *  - C99, no exceptions cross the boundary; every function returns a
 *    cgks_status.  CGKS_EINVAL is returned before anything is enqueued.
 *    Detail of the last failure on the calling thread: cgks_last_error().
 *  - Device buffers (d_state, d_work) are allocated and freed by the caller,
 *    sized by cgks_plan_sizes; the library never allocates or frees them.
 *    Host arrays are caller-owned and only read/written during the call.
 *  - `stream` is a hipStream_t passed as void* (NULL: the default stream).
 *    cgks_init_state and cgks_step only enqueue work (no host sync, no
 *    allocation); cgks_read_state and cgks_query_health synchronise `stream`.
 *  - A plan is immutable after creation: steps of different states on
 *    different streams may share it.  Calls on the same state must be ordered
 *    on one stream.
 *  - Units are those of the problem (the paper's tests are dimensionless).
 */
#ifndef CGKS_H
#define CGKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CGKS_OK = 0,
  CGKS_EINVAL = 1,          /* bad argument or shape; nothing was enqueued */
  CGKS_ENOMEM = 2,          /* host allocation failed */
  CGKS_EHIP = 3,            /* a HIP runtime call failed (see cgks_last_error) */
  CGKS_ENONPHYSICAL = 4,    /* a cell average reached rho <= 0 or p <= 0 (sticky, per state) */
  CGKS_ESTATE = 5,          /* the work buffer does not hold an initialised state */
  CGKS_EBUDGET = 6          /* batch: the job does not fit the memory budget or the slot table */
} cgks_status;

/* Boundary kinds of a side.  Transmissive, reflective and no-slip ghosts
 * mirror the interior cells: reflective (slip) walls negate the normal
 * momentum, no-slip adiabatic walls both momentum components (the wall sees
 * zero velocity and, the temperature being mirrored, no heat flux; the
 * walls of the viscous shock tube, Sec. 4.9).  A prescribed state (inflow)
 * fills the ghosts with that state and zero slopes (the jets' nozzle and
 * the post-shock inflow of the double Mach reflection, Sec. 4.8, 4.10).  A
 * segmented side applies different kinds along the side, with breakpoints
 * that may move at constant speed (the double Mach reflection's bottom and
 * its top boundary, which follows the exact shock). */
enum {
  CGKS_BC_PERIODIC = 0,
  CGKS_BC_TRANSMISSIVE = 1,
  CGKS_BC_REFLECTIVE = 2,
  CGKS_BC_NOSLIP = 3,
  CGKS_BC_INFLOW = 4,       /* prescribed state: side[k].prim[0] */
  CGKS_BC_SEGMENTED = 5     /* side[k] */
};
enum { CGKS_TAU_ZERO = 0, CGKS_TAU_INVISCID = 1, CGKS_TAU_VISCOUS = 2 };
enum { CGKS_FP64 = 0, CGKS_FP32_FLUX = 1 };

#define CGKS_MAX_SEGMENTS 3

/* One side split along its coordinate (y on the x-sides, x on the y-sides;
 * absolute coordinates).  Segment k < nseg - 1 holds the ghost cells whose
 * centre lies below end0[k] + speed[k] t (the first such k, t the time the
 * ghosts are filled for: the start of the step, or of its second stage);
 * the last segment holds the rest.  Strengths of ghost faces beyond a
 * prescribed state are zero (its ghosts are uniform). */
typedef struct {
  int nseg;                                   /* 1..CGKS_MAX_SEGMENTS */
  int type[CGKS_MAX_SEGMENTS];                /* TRANSMISSIVE, REFLECTIVE, NOSLIP or INFLOW */
  double prim[CGKS_MAX_SEGMENTS][4];          /* INFLOW: rho, u, v, p (1-D: rho, u, p); rho, p > 0 */
  double end0[CGKS_MAX_SEGMENTS - 1];
  double speed[CGKS_MAX_SEGMENTS - 1];
} cgks_bc_side;

/* Uniform grid.  dim = 1: ny must be 1 and bc[2], bc[3] are ignored.
 * nx, ny >= 5 (the widest stencil); a periodic direction must be periodic on
 * both ends (periodic sides cannot be segmented).  side[k] is read only when
 * bc[k] is CGKS_BC_INFLOW (segment 0's state) or CGKS_BC_SEGMENTED. */
typedef struct {
  int dim;                  /* 1 or 2 */
  int nx, ny;               /* cells per direction */
  double x0, x1, y0, y1;    /* domain [x0, x1] x [y0, y1] */
  int bc[4];                /* x-lo, x-hi, y-lo, y-hi: CGKS_BC_* */
  cgks_bc_side side[4];
} cgks_grid_desc;

/* Scheme parameters (Sec. 3.1, 3.2 and 4).  order 5, 7, 9 uses m = 2, 3, 4
 * Gauss points per face.  Collision time: CGKS_TAU_ZERO (tau = 0),
 * CGKS_TAU_INVISCID (tau = c1 dt + c2 |pl-pr|/(pl+pr) dt) or
 * CGKS_TAU_VISCOUS (tau = mu/p + c2 |pl-pr|/(pl+pr) dt).  prandtl != 1 adds
 * the standard gas-kinetic Prandtl-number fix to the energy flux: (1/Pr - 1)
 * times the time-integrated heat flux in the frame of the interface
 * equilibrium velocity (not part of the paper).
 * sigma_thres: the DFF threshold (1 for compact stencils); gamma_hi, gamma_lo:
 * linear weights of the AO(5,3) reconstruction; weno_eps: its epsilon.
 * precision: CGKS_FP64, or CGKS_FP32_FLUX (reconstruction and flux moments in
 * FP32; cell-average accumulation, conservation sums and the exponential
 * time coefficients in FP64; the device copies of the slopes, of the stage
 * state's and accumulator's slopes and of the Step 1 line values are stored
 * in FP32, the cell averages and interface strengths in FP64). */
typedef struct {
  int order;
  double gamma;
  int tau_model;
  double c1, c2, mu, prandtl;
  double sigma_thres, gamma_hi, gamma_lo, weno_eps;
  int precision;
  int reading_flags;        /* 0, or a set of CGKS_READ_* below */
} cgks_scheme_desc;

/* Alternative readings of points the paper leaves open (reading_flags; 0
 * gives the defaults):
 *  - CGKS_READ_A3_GAMMA1_LO: the linear weights of Eq. 3.12, whose printed
 *    form does not sum to one, read with gamma_1 = (1 - gamma_Hi) gamma_Lo and
 *    gamma_0 = gamma_2 = (1 - gamma_Hi)(1 - gamma_Lo)/2 (default: the central
 *    S2 takes the gamma_Lo share and gamma_0 = gamma_1, the mirror-symmetric
 *    choice);
 *  - CGKS_READ_A5_UNSCALED_BETA: the smoothness indicators of Eq. 3.13 from the
 *    members before their DFF scaling of Eq. 3.19 (default: after it);
 *  - CGKS_READ_A10_SIGMA0_ZERO: the strengths of the step before the first
 *    set to zero (default: those of the piecewise-constant states, Eq. 3.2). */
enum { CGKS_READ_A3_GAMMA1_LO = 1, CGKS_READ_A5_UNSCALED_BETA = 2, CGKS_READ_A10_SIGMA0_ZERO = 4 };

typedef struct cgks_plan cgks_plan;

/* Counters accumulated on the device since cgks_init_state.
 * Reconstructions are counted once per (cell, Gauss line or node) and stage,
 * as Algorithm 1 takes them: in 1-D the cells 0..nx-1 and the two ghost cells
 * beside the boundary faces; in 2-D, per direction, the interior cells of
 * Step 1 (line values, Sec. 3.3) and of Step 2 on each of the m Gauss lines.
 * recon_total = steps * 2 * (nx + 2) in 1-D, steps * 2 * 2 nx ny (1 + m) in
 * 2-D, is split by branch: ao_branch + linear[0] + linear[1] + linear[2]. */
typedef struct {
  long long nonphysical;        /* cell averages found with rho <= 0 or p <= 0 */
  long long fallbacks;          /* Gauss-point states replaced by the cell average (rho or p <= 0) */
  long long steps;              /* completed steps */
  long long recon_total;        /* reconstructions taken (see above) */
  long long dff_lt1;            /* reconstructions in which the DFF of the scheme's full stencil was
                                   below 1, so the cascade stepped down (Eq. 3.3, Algorithm 1) */
  long long ao_branch;          /* reconstructions by the AO(5,3) branch (DFF of the 5th-order stencil < 1) */
  long long linear[3];          /* reconstructions by the linear 5th-, 7th- and 9th-order stencils */
  long long near_ties;          /* cascade decisions taken with the stencil sum A (Eq. 3.4) within
                                   1e-12 sigma_thres (FP64) or 1e-5 sigma_thres (FP32-flux) of the
                                   threshold, where rounding can change the branch */
} cgks_health;

/* Validate the descriptors and build a plan (host metadata only).
 * Errors: CGKS_EINVAL (order not 5/7/9, gamma <= 1, nx/ny < 5, dim not 1/2,
 * inconsistent periodic ends, prandtl <= 0, NULL pointers). */
cgks_status cgks_plan_create(const cgks_grid_desc* grid, const cgks_scheme_desc* scheme, cgks_plan** out);

/* Bytes of the caller-owned device buffers.  d_state holds the conserved
 * cell averages (FP64) and slopes (FP64, or FP32 under CGKS_FP32_FLUX) with a
 * ghost halo, in a layout private to the library: cgks_init_state and
 * cgks_read_state convert from and to the FP64 host layouts; d_work holds the stage state,
 * the stage accumulator, the interface strengths (Eq. 3.1), reconstruction
 * intermediates, and a 256-byte header (time, step, dt, counters). */
cgks_status cgks_plan_sizes(const cgks_plan* plan, size_t* state_bytes, size_t* work_bytes);

/* Copy an initial state to the device (enqueued on `stream`, host arrays are
 * staged synchronously, so they may be freed on return).  Layouts, FP64,
 * C order:
 *   h_avg      [nv][ny][nx]      conservative cell averages (nv = 3 in 1-D: rho,
 *                                 rho u, rho E; nv = 4 in 2-D: rho, rho u, rho v, rho E)
 *   h_slope_x  1-D: [3][nx] cell-averaged d/dx;  2-D: [4][m][ny][nx] d/dx averaged
 *              along the horizontal Gauss line y_j + x_l dy of each cell
 *   h_slope_y  2-D: [4][m][ny][nx] d/dy averaged along the vertical Gauss line
 *              x_i + x_l dx (ignored in 1-D; may be NULL there)
 *   h_sigma_x, h_sigma_y: interface strengths of a previous step ([ny][nx+1]
 *              and [ny+1][nx]; 1-D: [nx+1]) to resume a run, or NULL to start
 *              from the strengths of the piecewise-constant states (Eq. 3.2).
 *   t0: the time of the state.  Resets the step count and health counters. */
cgks_status cgks_init_state(const cgks_plan* plan, void* d_state, void* d_work, const double* h_avg,
                            const double* h_slope_x, const double* h_slope_y, const double* h_sigma_x,
                            const double* h_sigma_y, double t0, void* stream);

/* Enqueue one two-stage step.  dt > 0: fixed step; dt <= 0: dt = cfl *
 * min(h / max(|U| + c), h^2 min(rho) / (4 mu)) from the cell averages at the
 * start of the step, computed on the device.  t_end > 0: the step is clipped
 * so the time does not pass t_end (a step at t >= t_end does nothing).  No
 * host synchronisation and no allocation: the call can be captured in a
 * hipGraph.  Errors: CGKS_EINVAL (cfl not in (0, 1] when dt <= 0). */
cgks_status cgks_step(const cgks_plan* plan, void* d_state, void* d_work, double dt, double cfl, double t_end,
                      void* stream);

/* Profiling variant of cgks_step: the same launches, with a HIP event
 * recorded on `stream` around every kernel launch.  Synchronises `stream`,
 * then writes the duration (ms) of each launch in launch order to
 * kernel_ms[0..*count-1] (*count <= 16; kernel_ms must hold 16 entries).
 * Names of the launches: cgks_kernel_name. */
cgks_status cgks_step_timed(const cgks_plan* plan, void* d_state, void* d_work, double dt, double cfl,
                            double t_end, void* stream, double* kernel_ms, int* count);

/* Name of launch `index` of a step of this plan ("" when out of range). */
const char* cgks_kernel_name(const cgks_plan* plan, int index);

/* Copy the state back (synchronises `stream`).  Any pointer may be NULL.
 * Layouts as in cgks_init_state; h_time, h_steps: scalars.
 *   h_grad_x, h_grad_y  [nv][ny][nx] cell-averaged gradients: in 2-D the
 *              Gauss-weighted means of the line-averaged slopes,
 *              sum_l w_l h_slope_x[v][l] (Sec. 3.3); in 1-D h_grad_x is the
 *              cell-averaged slope and h_grad_y is not written.
 * Returns CGKS_ENONPHYSICAL (after copying) if a nonphysical cell average
 * was seen. */
cgks_status cgks_read_state(const cgks_plan* plan, const void* d_state, const void* d_work, double* h_avg,
                            double* h_grad_x, double* h_grad_y, double* h_slope_x, double* h_slope_y,
                            double* h_sigma_x, double* h_sigma_y, double* h_time, long long* h_steps,
                            void* stream);

/* Totals of the conserved variables over the interior cells, sum_i W_i (so
 * h^d times the totals of Sec. 2.2), in FP64: d_sums[0..nv-1] in device
 * memory (caller-owned), written on `stream` (no host synchronisation, no
 * allocation; capturable in a hipGraph).  Deterministic: a fixed-order
 * tree of compensated (double-double) partial sums that depends only on the
 * grid size, so the same state gives the same bits on every call; the
 * result is within an ulp or two of the exactly rounded sum.  Uses the
 * reduction area of d_work, so it must not overlap a step of the same state
 * on another stream.  Errors: CGKS_EINVAL (NULL pointers), CGKS_EHIP. */
cgks_status cgks_conservation_sums(const cgks_plan* plan, const void* d_state, void* d_work, double* d_sums,
                                   void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * totals as cgks_conservation_sums, bit for bit, without d_work.  The block
 * partials go to a fixed scratch array in the library's device memory
 * (256 KiB per device, held until the process ends), so grids are limited to
 * 2^26 interior cells (8192 x 8192).  No allocation of any kind; the first
 * call on a device resolves the array's address there.  Every call on one
 * device shares that array: calls that overlap on one device (different
 * streams, or different host threads) race and must be ordered by the
 * caller.  Errors: CGKS_EINVAL (NULL pointers, or a grid beyond the limit;
 * nothing enqueued), CGKS_EHIP. */
cgks_status cgks_conservation_sums_static(const cgks_plan* plan, const void* d_state, double* d_sums, void* stream);

/* Device counters (synchronises `stream`); returns CGKS_ENONPHYSICAL when
 * nonphysical > 0. */
cgks_status cgks_query_health(const cgks_plan* plan, const void* d_work, cgks_health* out, void* stream);

/* Free the plan's host memory. */
cgks_status cgks_plan_destroy(cgks_plan* plan);

/* Static strings; cgks_last_error is per thread. */
const char* cgks_status_string(cgks_status s);
const char* cgks_last_error(void);

/* ------------------------------------------------------------------------
 * Batches: many independent states of one dimension and precision advanced
 * together.  Each phase of the step (dt, ghosts, Step 1 line values, x-face
 * and y-face reconstruction + flux + update, per stage; Sec. 2.2, 3.3) is one
 * persistent launch over the tiles of every job, computed by the same device
 * code and with the same tiles as cgks_step: a job's result in a batch equals
 * its result stepped alone.  Jobs may differ in grid size, order, boundary
 * conditions, scheme parameters, dt/CFL, t_end and step limit; batched
 * kernels take prandtl = 1 only.
 *
 * Life cycle: create -> add/remove jobs -> commit (uploads the job table,
 * synchronises the stream) -> step or capture + launch -> poll -> read each
 * job's state with cgks_read_state on its own plan and buffers -> remove ->
 * commit ...  The job buffers stay caller-owned and must outlive the job's
 * membership.  A batch is not thread-safe; its launches must be ordered on
 * one stream at a time.
 * ------------------------------------------------------------------------ */
typedef struct cgks_batch cgks_batch;

/* Progress of one job slot (cgks_batch_poll). */
typedef struct {
  double t;                 /* time reached */
  double dt;                /* last step size (0 once stopped) */
  long long steps;          /* completed steps */
  int status;               /* 0 running, 1 finished (t_end or max_steps), 2 nonphysical */
  int in_use;               /* 1 if the slot holds a job */
} cgks_job_status;

/* Launch shape of the persistent kernels: grid = (resident blocks per CU) x
 * CUs x grid_mult; xcd_remap != 0 gives consecutive tiles to blocks of one
 * XCD.  Tile shapes of the 2-D kernels: face_tile 0 = 16 faces along the
 * normal x 8/5/4 lines (orders 5/7/9; the single-grid shape), 1 = 32 x
 * 4/2/2, 2 = 8 x 16/10/8; line_tile (Step 1) 0 = 32 x 8 cells, 1 = 16 x 16.
 * Every shape computes the same results.  ms_per_step: the time measured by
 * cgks_batch_tune (else 0). */
typedef struct {
  int grid_mult;
  int xcd_remap;
  int face_tile;
  int line_tile;
  float ms_per_step;
} cgks_batch_tuning;

/* Create an empty batch of up to max_jobs jobs (1..2^20).  hbm_budget_bytes
 * bounds the sum of the jobs' state + work bytes (0: no bound).  Allocates
 * the device job table (about 400 bytes per slot) on the current device.
 * Errors: CGKS_EINVAL, CGKS_ENOMEM, CGKS_EHIP. */
cgks_status cgks_batch_create(int dim, int precision, int max_jobs, size_t hbm_budget_bytes, cgks_batch** out);

/* Release the table and any captured graph (not the jobs' buffers). */
cgks_status cgks_batch_destroy(cgks_batch* batch);

/* Admit a state initialised by cgks_init_state (reads its header
 * synchronously).  The job runs until it has taken max_steps steps (> 0) or
 * reached t_end (> 0), whichever comes first; dt > 0 fixes the step, else dt
 * comes from cfl as in cgks_step.  Takes effect at the next commit; *slot
 * receives the job's slot.  Errors: CGKS_EINVAL (dimension or precision
 * differs from the batch, prandtl != 1, no stopping rule, bad cfl),
 * CGKS_ESTATE (uninitialised work buffer), CGKS_EBUDGET (the budget or the
 * slot table is full; nothing changed). */
cgks_status cgks_batch_add(cgks_batch* batch, const cgks_plan* plan, void* d_state, void* d_work,
                           long long max_steps, double dt, double cfl, double t_end, int* slot);

/* Retire the job in `slot` (takes effect at the next commit; its buffers are
 * the caller's again after that commit).  Errors: CGKS_EINVAL (empty slot). */
cgks_status cgks_batch_remove(cgks_batch* batch, int slot);

/* Upload the job table on `stream` and synchronise it.  Must follow any
 * add/remove before the next step, launch or tune (else CGKS_ESTATE). */
cgks_status cgks_batch_commit(cgks_batch* batch, void* stream);

/* Enqueue nsteps steps of every committed job (no host synchronisation, no
 * allocation, no copies).  Jobs that have stopped are skipped. */
cgks_status cgks_batch_step(cgks_batch* batch, int nsteps, void* stream);

/* Capture nsteps batch steps into a hipGraph held by the batch (replacing the
 * previous one).  The graph reads the job table from device memory, so it
 * stays valid across commits; cgks_batch_set_tuning / cgks_batch_tune drop
 * it.  Errors: CGKS_EHIP. */
cgks_status cgks_batch_capture(cgks_batch* batch, int nsteps);

/* Launch the captured graph on `stream`.  Errors: CGKS_ESTATE (no graph, or
 * the batch changed since the last commit). */
cgks_status cgks_batch_launch(cgks_batch* batch, void* stream);

/* Progress of every slot: out[0..max_jobs-1] (synchronises `stream`). */
cgks_status cgks_batch_poll(cgks_batch* batch, cgks_job_status* out, void* stream);

/* Jobs held, their state + work bytes, the device table bytes, and the grid
 * of the persistent face (2-D) or stage (1-D) launch.  For the face launch
 * this is the grid sized by the fewest resident blocks of the current tile
 * shape's face kernels; the FP32-flux face kernels each run a grid sized by
 * their own (at least this one).  Any pointer may be NULL. */
cgks_status cgks_batch_info(const cgks_batch* batch, int* njobs, size_t* bytes_used, size_t* table_bytes,
                            int* grid_face);

/* Set / read the launch shape (set drops a captured graph; a change of tile
 * shape also changes the jobs' tile counts, so the batch must be committed
 * again before the next step).  Errors: CGKS_EINVAL (grid_mult outside
 * 1..16, face_tile outside 0..2, line_tile outside 0..1). */
cgks_status cgks_batch_set_tuning(cgks_batch* batch, const cgks_batch_tuning* tuning);
cgks_status cgks_batch_get_tuning(const cgks_batch* batch, cgks_batch_tuning* tuning);

/* Autotune the launch shape on the committed jobs: each candidate runs
 * steps_per_trial real steps, timed with HIP events on `stream`.  2-D
 * batches first try every face_tile x line_tile pair (re-committing the table
 * for each), then grid_mult 1, 2, 4 x xcd_remap 0, 1 with the fastest
 * shapes; 1-D batches the latter only.  The fastest is kept (the batch stays
 * committed) and written to *chosen (may be NULL).  All candidates compute
 * the same result, so the trial steps advance the jobs like ordinary steps.
 * Synchronises `stream`; drops a captured graph. */
cgks_status cgks_batch_tune(cgks_batch* batch, int steps_per_trial, void* stream, cgks_batch_tuning* chosen);

#ifdef __cplusplus
}
#endif
#endif /* CGKS_H */
