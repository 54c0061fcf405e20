/*
 * starmap.h -- C ABI of the MI355X staggered-grid P_N solver.
 *
 * The library advances the 2D real spherical-harmonics P_N equations of
 * radiative transfer,
 *     d_t u + M_x d_x u + M_y d_y u + C u = q,
 * with the staggered-grid scheme of Seibold & Frank, "StaRMAP - A second order
 * staggered grid method for spherical harmonics moment equations of radiative
 * transfer" (arXiv 1211.2205):
 *   - the (N+1)(N+2)/2 real moments R_l^m, I_l^m (Sect. 3) live on four mutually
 *     staggered grids G11, G21, G12, G22 (Sect. 4.1, eqs. grid11 and
 *     staggered_grids);
 *   - D_x, D_y are half-cell central differences (eq. central_differences);
 *   - boundaries are periodic or constant extrapolation (Sect. 4.2);
 *   - a time step is the Strang composition S^o S^e S^e S^o of exact sub-step
 *     solutions u <- u + tau (r - c u) E(-c tau), E(z) = (e^z - 1)/z
 *     (Sect. 4.3, eqs. sub_step_solution and solution_operator_full_step).
 *
 * Conventions for every call below:
 *   - Functions returning int give STARMAP_OK (0) or a negative STARMAP_E*
 *     code; no C++ exception crosses the ABI.  starmap_last_error() returns a
 *     message for the last failure on the calling thread (owned by the
 *     library, valid until the next failing call on that thread).
 *   - Handles are opaque; the caller creates and destroys them.
 *   - Host arrays passed in are copied; the caller keeps ownership.
 *   - Moment index k follows the paper's order: l ascending; within l, m
 *     descending; R_l^m before I_l^m (I exists for m > 0).  Index 0 is R_0^0.
 *   - A moment's values are laid out on its own grid, x fastest:
 *       cell-centred axis: nc = n points at x0 + (i + 1/2) h, i = 0..n-1;
 *       nodal axis:        nc = n + 1 - p points at x0 + (i + p) h, i = 0..nc-1,
 *     where p = 1 for a periodic axis (node 0 coincides with node n and only
 *     nodes 1..n are stored) and p = 0 for extrapolation.
 *   - Device memory is owned by the library unless the caller binds its own
 *     (starmap_bind_device); all device work runs on the bound stream (the
 *     null stream otherwise) and the blocking calls synchronise it.
 */
#ifndef STARMAP_H
#define STARMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STARMAP_OK 0
#define STARMAP_EINVAL (-1)    /* invalid argument or problem description */
#define STARMAP_ENOMEM (-2)    /* host or device allocation failed / workspace too small */
#define STARMAP_EHIP (-3)      /* a HIP runtime call failed */
#define STARMAP_EUNSTABLE (-4) /* non-finite values found by the diagnostics */
#define STARMAP_ESTATE (-5)    /* call not valid in the solver's current state */

/* Boundary type per axis (Sect. 4.2; the periodicity flag p of eq.
   periodicity_flags is 1 for STARMAP_BC_PERIODIC and 0 otherwise). */
#define STARMAP_BC_PERIODIC 0
#define STARMAP_BC_EXTRAPOLATION 1

/* Storage precision of the moments.  FP64 computes in FP64; FP32 and BF16
   store in that type and compute in FP32. */
#define STARMAP_FP64 0
#define STARMAP_FP32 1
#define STARMAP_BF16 2

/* Closure of the moment hierarchy: plain P_N truncation, or P_N plus the
   learned correction of the highest order (starmap_closure_load). */
#define STARMAP_CLOSURE_PN 0
#define STARMAP_CLOSURE_LEARNED 1

/* Field selectors of starmap_set_field_array. */
#define STARMAP_FIELD_ABSORPTION 0 /* sigma_a on moment k's grid  */
#define STARMAP_FIELD_SCATTERING 1 /* sigma_s0 on moment k's grid */
#define STARMAP_FIELD_SOURCE 2     /* q_k on moment k's grid      */
#define STARMAP_FIELD_INITIAL 3    /* u_k(t = 0)                  */
#define STARMAP_FIELD_SCATTERING_ORDER 4 /* sigma_sl (index = order l), starmap_add_field_term only */

/* Problem statement (the paper's par struct, Sect. 5.1). */
typedef struct {
  double ax[4];      /* domain x0, x1, y0, y1 */
  int32_t n[2];      /* cells nx, ny (>= 2 each) */
  int32_t bc[2];     /* STARMAP_BC_* per axis */
  int32_t N;         /* moment order, 0 < N <= 99 */
  double cfl;        /* dt0 = cfl * min(dx, dy) / rho(M_x); stable for cfl < 1/sqrt(2) */
  double t_final;    /* final time; the step count is rounded up to land on it */
  int32_t precision; /* STARMAP_FP64 | STARMAP_FP32 | STARMAP_BF16 */
  int32_t closure;   /* STARMAP_CLOSURE_PN | STARMAP_CLOSURE_LEARNED */
} starmap_problem;

typedef struct starmap_solver starmap_solver;

/* Vectorised field callback: write f(t, x[i], y[i]) into out[i] for
   i = 0..count-1 (physical coordinates).  Return 0 on success; any other value
   aborts the calling function with STARMAP_EINVAL. */
typedef int (*starmap_field_fn)(void* ctx, double t, int64_t count, const double* x,
                                const double* y, double* out);

/* Time factor a(t) of a separable field term (evaluated on the host, once per
   step). */
typedef double (*starmap_time_fn)(void* ctx, double t);

/* ---------------------------------------------------------------- host-only
   These need no GPU. */

/* Number of moments (N+1)(N+2)/2 (Sect. 3, 2D reduction). */
int starmap_num_moments(int32_t N);

/* Moment k of order N: is_imag (0: R_l^m, 1: I_l^m), l, m, and its grid
   G_{gx gy} (1 = cell-centred, 2 = nodal along that axis; Lemma 2 and
   eq. matrix_conditions).  Any output pointer may be NULL. */
int starmap_moment_info(int32_t N, int32_t k, int32_t* is_imag, int32_t* l, int32_t* m,
                        int32_t* gx, int32_t* gy);

/* Rows of the real moment matrix M_x (axis 0) or M_y (axis 1) of order N
   (Sect. 3, M^real = S M^complex S^-1; symmetric, at most 4 nonzeros a row).
   cols and vals hold 4 * num_moments entries (row-major, 4 slots per row);
   unused slots get col = -1 and val = 0. */
int starmap_closure_pn(int32_t N, int32_t axis, int32_t* cols, double* vals);

/* Largest eigenvalue magnitude of M_x of order N (the maximal wave speed that
   scales the admissible time step, Sect. 4.5 and Sect. 5.3). */
int starmap_spectral_radius(int32_t N, double* rho);

/* Moments of a unit beam source delta(Omega - Omega_0) in direction
   Omega_0 = (ox, oy, oz) (a unit vector; oz is the component out of the
   plane): the real basis functions of the moment vector at Omega_0, from the
   complex spherical harmonics and the change of variables of Sect. 3
   (R_l^0 = Y_l^0, R_l^m = (-1)^m sqrt2 Re Y_l^m, I_l^m = (-1)^m sqrt2 Im Y_l^m),
   e.g. R_0^0 = 1/sqrt(4 pi), R_1^1 = sqrt(3/(4 pi)) ox, I_1^1 = sqrt(3/(4 pi)) oy.
   A source q(x) delta(Omega - Omega_0) has moments q(x) out[k] (the beam
   problem of Sect. 6).  out holds (N+1)(N+2)/2 values, moment order. */
int starmap_direction_moments(int32_t N, double ox, double oy, double oz, double* out);

/* Self-check of the sweep programs the library builds for order N, tile
   tile_x x tile_y and nchunks m ranges (with sources on three moments, and
   with sources on every moment, and per-order decay): replays the staged LDS window and checks that every
   coupling reads the plane the moment matrices require.  STARMAP_OK or
   STARMAP_EINVAL with the failed check in starmap_last_error(). */
int starmap_plan_check(int32_t N, int32_t tile_x, int32_t tile_y, int32_t nchunks);

/* ------------------------------------------------------------- solver setup */

/* Validate the problem, build the plan (moment matrices, grid classes, rho,
   dt, step count).  Allocates no device memory. */
int starmap_create(const starmap_problem* prob, starmap_solver** out);
void starmap_destroy(starmap_solver* s);

/* Material and source fields, sampled on the host in FP64 at each grid's
   points when the solver first needs them (Sect. 5.7).  Isotropic scattering
   uses sigma_s0 only: moments of order l >= 1 decay with sigma_a + sigma_s0,
   the zeroth moment with sigma_a (Sect. 2: Sigma_tl = Sigma_a + Sigma_s0 -
   Sigma_sl).  Missing fields are zero.  time_dependent != 0 re-samples the
   field at t + dt/2 before every step. */
int starmap_set_absorption(starmap_solver* s, starmap_field_fn f, void* ctx, int32_t time_dependent);
int starmap_set_scattering(starmap_solver* s, starmap_field_fn f, void* ctx, int32_t time_dependent);
/* Anisotropic part: sigma_sl(l, t, x, y) for l >= 1 via one callback per order
   (ctx receives the order through the callback's own state).  Optional. */
int starmap_set_scattering_order(starmap_solver* s, int32_t l, starmap_field_fn f, void* ctx,
                                 int32_t time_dependent);
/* Source q_k of moment k (isotropic sources act on k = 0 only). */
int starmap_set_source(starmap_solver* s, int32_t k, starmap_field_fn f, void* ctx, int32_t time_dependent);
/* Initial value u_k(0) of moment k (others start at 0). */
int starmap_set_initial(starmap_solver* s, int32_t k, starmap_field_fn f, void* ctx);

/* Pre-sampled variant: host_vals holds moment k's grid layout (see above).
   ABSORPTION/SCATTERING accept any k and define the field on that moment's
   grid; they are time-independent. */
int starmap_set_field_array(starmap_solver* s, int32_t which, int32_t k, const double* host_vals);

/* Grid of moment k: points along x and y, and the coordinates of its first
   point. */
int starmap_moment_shape(const starmap_solver* s, int32_t k, int32_t* nx_k, int32_t* ny_k,
                         double* x0_k, double* y0_k);

/* Time bookkeeping: current time, step, steps done, steps to t_final. */
int starmap_time(const starmap_solver* s, double* t, double* dt, int64_t* steps_done,
                 int64_t* steps_total);

/* ------------------------------------------------------------ device memory */

/* Bytes of device workspace the solver needs (state planes, material and
   source planes, sweep programs, diagnostics scratch), 256-byte aligned. */
int starmap_workspace_bytes(const starmap_solver* s, size_t* bytes);

/* Use caller-owned device memory (at least starmap_workspace_bytes, 256-byte
   aligned) and a caller-owned HIP stream (hipStream_t, or NULL for the null
   stream).  Must precede the first device call; the memory must outlive the
   solver.  Without it the library allocates its own on first use. */
int starmap_bind_device(starmap_solver* s, void* dev_ptr, size_t bytes, void* hip_stream);

/* ------------------------------------------------------------------- running */

/* Advance nsteps full steps (S^o_{dt/2} S^e_{dt/2} S^e_{dt/2} S^o_{dt/2} each).
   Time-independent data: the device runs S^o_{dt/2}, [S^e_{dt}, S^o_{dt}]^{n-1},
   S^e_{dt}, S^o_{dt/2}, equal in exact arithmetic (two exact half-steps with
   frozen data compose to one exact full step).  Time-dependent data is
   re-sampled at t + dt/2 and each step runs S^o_{dt/2} S^e_{dt} S^o_{dt/2}.
   The call returns after queueing the work on the stream (asynchronous). */
int starmap_advance(starmap_solver* s, int64_t nsteps);

/* HIP graphs in starmap_advance (on by default): for time-independent data
   (and not with starmap_set_fused), the repeated pairs S^e_dt, S^o_dt are
   captured once per run length of 16, 8, 4, 2 and 1 pairs and replayed as
   graph launches; the captured launches are those of the eager path, so the
   results are the same bits.  Not used while per-launch timing is on
   (starmap_profile_begin) or on the null stream.  The graphs are dropped
   when the tile variant or m-range width changes, and with enable = 0. */
int starmap_set_graphs(starmap_solver* s, int32_t enable);

/* Advance to t_final and synchronise. */
int starmap_run(starmap_solver* s);

/* Queue nsweeps single parity sweeps with sub-step tau (parity 0 even, 1 odd),
   for profiling of the sweep kernel; does not change the time bookkeeping. */
int starmap_sweep(starmap_solver* s, int32_t parity, double tau, int32_t nsweeps);

/* Synchronise the solver's stream. */
int starmap_synchronize(starmap_solver* s);

/* Copy moment k at the current time to host_out (moment k's grid layout,
   FP64) and synchronise. */
int starmap_get_moment(const starmap_solver* s, int32_t k, double* host_out);

/* Checkpoint: the raw state (opaque, starmap_state_bytes long) plus the time
   bookkeeping.  Restoring into a solver created from the same problem and
   continuing with the same advance calls reproduces the uninterrupted run bit
   for bit. */
int starmap_state_bytes(const starmap_solver* s, size_t* bytes);
int starmap_get_state(const starmap_solver* s, void* host_buf, size_t bytes, double* t, int64_t* step);
int starmap_set_state(starmap_solver* s, const void* host_buf, size_t bytes, double t, int64_t step);

/* FP64 reductions on the device: mass dx*dy*sum(R_0^0), discrete L2 norm
   (dx*dy*sum_k sum u_k^2)^(1/2) (eq. discrete_L2_norm), max |u|, and the count
   of non-finite values.  Returns STARMAP_EUNSTABLE if that count is nonzero
   (the outputs are still written).  Any output pointer may be NULL. */
int starmap_diagnostics(const starmap_solver* s, double* mass_r00, double* l2, double* maxabs,
                        int32_t* nonfinite);

/* starmap_diagnostics for callers that cannot allocate device memory (code
   under HIP stream capture, tight serving loops, harnesses that forbid
   allocation): the same reductions and outputs, with the FP64 block partials
   and the four results in a static device array of the library (2 MiB per
   GPU, held until the process ends) instead of the solver's workspace.  It
   allocates nothing: the solver must already hold its device state (any
   earlier device call sets it up), else STARMAP_ESTATE.  At most 65536
   reduction blocks, i.e. moments x ceil((ny + 1) / 64) <= 65536, else
   STARMAP_EINVAL.  All calls on one GPU share that GPU's array: calls that
   overlap on one GPU (two streams or two threads) race. */
int starmap_diagnostics_noalloc(const starmap_solver* s, double* mass_r00, double* l2, double* maxabs,
                                int32_t* nonfinite);

/* Tile variant of the sweep kernel: -1 chooses by the autotuner (default).
   Variants differ in the spatial tile (tile_x x tile_y points) and in how
   many planes of one order are held in registers while the next order loads
   (fewer registers let more workgroups share a compute unit); all give the
   same bits.  starmap_autotune times every variant that fits, at every
   m-range width (4, 6, 8), on a few sweeps of this solver, keeps the fastest
   pair and writes it to the cache file named by the environment variable
   STARMAP_TUNE_CACHE (if set).  Variants are 0 .. starmap_variant_count()-1;
   another value fails with STARMAP_EINVAL.  The environment variable
   STARMAP_TILE_STRIP (read by starmap_create) sets
   the order in which workgroups take the tiles: k >= 2 strips of k tile
   rows taken column by column (default 8), k <= -2 strips of -k tile
   columns taken row by row, otherwise row by row; every order gives the
   same bits. */
int starmap_variant_count(void);
int starmap_set_variant(starmap_solver* s, int32_t variant);
int starmap_get_variant(const starmap_solver* s, int32_t* variant, int32_t* tile_x, int32_t* tile_y);
int starmap_autotune(starmap_solver* s, int32_t sweeps_per_variant);

/* Width of the m ranges the sweep splits the outputs of one order into (an
   output (l, m) couples only to inputs (l -+ 1, m -+ 1), Lemma 2): 4, 6 or 8
   (another value: STARMAP_EINVAL; the default is 8, or the autotuner's or
   the tune cache's choice).  All widths give the same bits.  A width at
   which the current tile variant no longer fits the LDS fails with
   STARMAP_EINVAL and leaves the width unchanged. */
int starmap_set_range_width(starmap_solver* s, int32_t width);
int starmap_get_range_width(const starmap_solver* s, int32_t* width);

/* Bytes the sweep kernel moves per parity sweep by the algorithm's count:
   every input plane read once, every output plane read and written once, plus
   the decay and source planes it reads (valid points only). */
int starmap_sweep_bytes(const starmap_solver* s, int32_t parity, double* bytes);

/* Per-launch timing of the sweep kernel: between begin and end every sweep
   launch is bracketed by HIP events recorded on the solver's stream.  end
   synchronises and returns the summed kernel time (ms), the number of
   launches, and their summed algorithmic bytes (starmap_sweep_bytes). */
int starmap_profile_begin(starmap_solver* s);
int starmap_profile_end(starmap_solver* s, double* kernel_ms, int64_t* launches, double* bytes);

/* ----------------------------------------------------------- learned closure */

/* The P_N truncation closes the hierarchy by zeroing order N + 1 (Sect. 2).
   A solver created with closure = STARMAP_CLOSURE_LEARNED (N = 5 only)
   restores an estimate of the dropped order-6 flux of its six order-5 moments
   with a small network of the local order-4/5 data, evaluated on the device
   before every odd sweep and added to those moments' residual W_k:
     - evaluation points (i, j), 0 <= i <= nx, 0 <= j <= ny; the order-5 R
       moments (grid G21) take the outputs at their point (i, j), the I
       moments (G12) at theirs, where those points exist;
     - inputs (128): for each of R_4^4, I_4^4, R_4^2, I_4^2, R_4^0, R_5^5,
       I_5^5, R_5^3, I_5^3, R_5^1, I_5^1 the values at the array neighbours
       (i + a, j + b), b = -1..1 (outer), a = -1..1 (inner), clamped to that
       moment's array, divided by nu = sqrt(sum of their squares) + 1e-20;
       then log10(sigma_a + 0.01) and log10(sigma_s + 0.01) at the G11 cell
       (min(i, nx-1), min(j, ny-1)); then zeros;
     - network y = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 (128, 128, 6 units;
       gelu(z) = z Phi(z) with the erf of Abramowitz & Stegun formula 7.1.26,
       |error| <= 1.5e-7, in inference and in the trainer below alike),
       matrix-product operands rounded to bfloat16, FP32 accumulation;
     - closure term of output r (R_5^5, I_5^5, R_5^3, I_5^3, R_5^1, I_5^1):
       g_r = nu * y_r / dx.
   The term is evaluated on the state at the start of each odd sweep and held
   fixed during it (like W).  Closure solvers need isotropic scattering,
   time-independent data and no source on the order-5 moments.

   Parameter blob (FP32, STARMAP_CLOSURE_PARAMS values, row-major):
   W1 (128 x 128, out x in), b1 (128), W2 (128 x 128), b2 (128), W3 (6 x 128),
   b3 (6). */
#define STARMAP_CLOSURE_PARAMS 33798

/* Copy the network into the solver (converted to its device form).  Must
   precede the first advance of a closure solver. */
int starmap_closure_load(starmap_solver* s, const float* weights, size_t count);

/* How the closure enters the odd sweep of this solver's own runs.
   enable = 1: one kernel evaluates the network on blocks of 64 evaluation
   points and applies the odd sub-step of P_5 to those points in the same
   workgroup; the order-5 moments are read from one buffer and written to a
   second one (the state planes and the closure planes take turns; every call
   leaves them in the state planes), so every stencil sees the state at the
   start of the sweep.  enable = 0 (default; faster for one instance on
   MI355X): a network kernel writes the closure terms to the closure planes and
   the odd sweep kernel reads them like sources.  Both give the same bits for
   FP64 and FP32 storage (with BF16 storage, 0 rounds the closure terms to
   bfloat16 on the way through the closure planes).  A batch of closure
   solvers follows its solvers' setting (they must agree).  STARMAP_ESTATE if
   the solver is not a closure solver. */
int starmap_closure_set_fused(starmap_solver* s, int32_t enable);

/* Training samples from the current state of a solver of order N >= 6
   (isotropic scattering): for count cells points[2 i], points[2 i + 1] =
   (i, j) with 0 <= i < nx, 0 <= j < ny, writes the closure inputs
   (count x 128, FP32) to the device array features and the targets
   F_r dx / nu (count x 6, FP32) to the device array targets, where
   F_r = -sum over order-6 moments j of (Mx(k_r, j) D_x u_j + My(k_r, j) D_y u_j)
   at output r's point (i, j) is the flux the truncation to P_5 drops.  Both
   arrays are caller-owned device memory; the call synchronises. */
int starmap_closure_samples(starmap_solver* s, const int32_t* points, int32_t count, float* features,
                            float* targets);

/* Closure inputs alone, from the current state of a solver of order N >= 5
   (a P_5 solver included): features as in starmap_closure_samples, and, if nu
   is not NULL, the stencil norm nu of each sample (count values, FP32).  A
   training set for states the closure solver itself produces pairs these
   inputs with the flux of a high-order run at the same time and cells,
   rescaled to this nu.  Device arrays, caller-owned; synchronises. */
int starmap_closure_features(starmap_solver* s, const int32_t* points, int32_t count, float* features, float* nu);

/* Network trainer on the device: parameters (FP32 master copy), Adam state,
   and buffers for batches of up to max_batch samples; work runs on
   hip_stream (NULL: the null stream).  x (batch x 128) and t (batch x 6) are
   device arrays.  Loss = mean over the batch and the six outputs of
   (y - t)^2.  The matrix products (forward and backward) use bfloat16
   operands with FP32 accumulation; the backward pass rounds dY, dZ2 and dZ1
   to bfloat16 where they enter a product; biases' gradients sum the
   unrounded values. */
typedef struct starmap_mlp starmap_mlp;
int starmap_mlp_create(int32_t max_batch, void* hip_stream, starmap_mlp** out);
void starmap_mlp_destroy(starmap_mlp* n);
/* Set (and reset the Adam state) / read the parameter blob (host memory). */
int starmap_mlp_set_params(starmap_mlp* n, const float* params, size_t count);
int starmap_mlp_get_params(const starmap_mlp* n, float* params, size_t count);
/* y (batch x 6, device) = network(x).  Asynchronous. */
int starmap_mlp_forward(starmap_mlp* n, const float* x, int32_t batch, float* y);
/* Gradient of the loss (parameter-blob layout, host memory; may be NULL) and
   the loss (may be NULL); synchronises. */
int starmap_mlp_gradients(starmap_mlp* n, const float* x, const float* t, int32_t batch, float* grad_host,
                          double* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
   batch's gradient.  loss may be NULL (then the call does not synchronise). */
int starmap_mlp_train_step(starmap_mlp* n, const float* x, const float* t, int32_t batch, double lr,
                           double* loss);
/* One Adam step with a given gradient (host memory); synchronises. */
int starmap_mlp_adam_step(starmap_mlp* n, const float* grad_host, double lr);

/* Time-separable fields evaluated on the device (time-dependent data,
   Sect. 5.7).  Adds a term a(t) g(x, y) to a field: which =
   STARMAP_FIELD_ABSORPTION, STARMAP_FIELD_SCATTERING,
   STARMAP_FIELD_SCATTERING_ORDER (index = order l, 1 <= l <= N) or
   STARMAP_FIELD_SOURCE (index = moment k).  A field given by terms is
   f(t, x, y) = sum_i a_i(t) g_i(x, y).  Each g_i is sampled once (called with
   t = 0) on every grid the field is needed on and kept on the device in the
   compute precision; per step the host evaluates only the a_i at t + dt/2
   and passes them to one device kernel that forms the decay planes (and the
   source planes) as linear combinations, so a step samples and uploads no
   plane.  Planes without a time factor are formed once.  Each step is
   S^o_{dt/2} S^e_dt S^o_{dt/2} with the data frozen at t + dt/2.
   Adding a term replaces a callback or array set for that field; setting the
   field with starmap_set_* or starmap_set_field_array afterwards replaces its
   terms.  Terms must be added before the first device call
   (STARMAP_ESTATE), and afterwards a field given by terms cannot be changed
   (STARMAP_ESTATE).  At most STARMAP_MAX_FIELD_TERMS terms over all fields
   (STARMAP_EINVAL).  Ownership: the callbacks and contexts must stay valid for
   the solver's life; the library calls them from the thread that calls it.
   A non-finite a_i(t) fails the advancing call with STARMAP_EINVAL.  If any
   field is a time-dependent callback (time_dependent = 1), the whole solver
   uses the host re-sampling path instead (the terms are then summed on the
   host).  Solvers with terms cannot join a batch or use the learned closure
   (STARMAP_EINVAL). */
#define STARMAP_MAX_FIELD_TERMS 32
int starmap_add_field_term(starmap_solver* s, int32_t which, int32_t index, starmap_field_fn space,
                           void* space_ctx, starmap_time_fn time, void* time_ctx);

/* Filtered P_N (FP_N; one of the moment models the paper names as fitting
   the same scheme, Sect. 7): damping[l] >= 0 for l = 0..N (N + 1 values,
   copied) is added to the decay coefficient of every moment of order l, so
   that order l decays with sigma_a + damping[0] (l = 0) or
   sigma_a + sigma_s0 - sigma_sl + damping[l] (l >= 1).  The values come from
   the filter of the user's choice (a filter f with strength sigma_f gives
   damping[l] = -sigma_f log f(l / (N + 1))).  The damping enters the decay
   planes, so the sweep kernels are unchanged.  It needs per-order decay planes:
   the first call must come before the first device call (STARMAP_ESTATE);
   later calls change the values.  Negative or non-finite values:
   STARMAP_EINVAL.  damping = NULL removes the damping. */
int starmap_set_filter_damping(starmap_solver* s, const double* damping);

/* Parity-fused passes for small orders (N <= STARMAP_FUSED_MAX_ORDER): each
   pair of half-steps S^o, S^e of the fused composition (see starmap_advance)
   runs as one pass over 32 x 8 tiles that holds every moment and every decay
   plane of the tile and a two-point halo in LDS, computes the odd update on
   the tile and a one-point ring around it, then the even update on the tile:
   every moment is read and written once per step instead of three accesses
   per moment and step (Sect. 4.3 applies the two sub-steps in turn; fusing
   them over a tile is this library's schedule).  The results are bitwise
   equal to the separate sweeps' for finite states.  The pass reads one state
   buffer and writes a second one (one more state's worth of device memory).
   Used for time-independent data without the D_N step; other solvers keep the
   separate sweeps.  An option, not a speed-up on every device: on MI355X the
   LDS footprint limits a compute unit to two such tiles and the separate
   sweeps are faster.  Must be chosen before the first device call
   (STARMAP_ESTATE); N too high, the learned closure, or a tile that does not
   fit the device's LDS: STARMAP_EINVAL (a tile that stops fitting because
   per-order decay planes were added later fails the first device call with
   STARMAP_EINVAL). */
#define STARMAP_FUSED_MAX_ORDER 7
int starmap_set_fused(starmap_solver* s, int32_t enable);

/* Diffusion-corrected P_N (D_N; Sect. 7: a diffusion step on the moments of
   the highest order fits the splitting): every step becomes
   S^o_{dt/2} S^e_{dt/2} D_dt S^e_{dt/2} S^o_{dt/2} with
   D_tau u = u + tau kappa (D_xx u + D_yy u) on each order-N moment's own grid
   (three-point second differences with dx^2, dy^2; periodic axes wrap,
   extrapolation axes repeat the boundary point as ghost), explicit in time.
   kappa(x, y) >= 0 is sampled once (t = 0) on the order-N grids; the first
   device call fails with STARMAP_EINVAL if kappa is negative or not finite,
   or if max kappa * dt * (2/dx^2 + 2/dy^2) > 1 (the explicit step would be
   unstable).  Must be set before the first device call (STARMAP_ESTATE);
   f = NULL removes it.  Not with the learned closure or in a batch
   (STARMAP_EINVAL).  The callback and ctx must stay valid until the first
   device call. */
int starmap_set_diffusion(starmap_solver* s, starmap_field_fn kappa, void* ctx);

/* Restore the initial condition at t = 0 (step 0) on the device. */
int starmap_reset(starmap_solver* s);

/* ------------------------------------------------------------------- batches */

/* A batch advances several independent solvers together on one device:
   instances are grouped by moment order N, and sweep number j of the fused
   composition (see starmap_advance; sweep j is odd for even j) runs as one
   kernel launch per group over the tiles of the group's instances that still
   have sweeps left, so instances of different grid sizes and step counts share
   the machine, each group has its own tile, and a whole run is captured in
   one HIP graph.  With several groups each group's launches form a chain on a
   stream of its own (forked from and joined into the batch's stream), so the
   groups' launches may run concurrently.  The solvers must share the storage precision, have time-independent
   data, and outlive the batch; their results are read with the per-solver
   calls.  A batch holds either no closure solvers or only closure solvers
   (STARMAP_CLOSURE_LEARNED, network loaded, one network for all): then every
   odd sweep is, with the solvers' default (starmap_closure_set_fused 0), one
   launch of the network over all running instances followed by one batched
   odd sweep, or with fused solvers one launch of the fused closure kernel
   over all running instances; starmap_batch_run and starmap_batch_autotune
   return STARMAP_EINVAL if the solvers' settings differ.  While in a batch, a solver's tile variant is the batch's: do not
   call starmap_set_variant on it. */
typedef struct starmap_batch starmap_batch;

/* count >= 1 distinct solvers.  The array is copied. */
int starmap_batch_create(starmap_solver* const* solvers, int32_t count, starmap_batch** out);
void starmap_batch_destroy(starmap_batch* b);

/* Advance every solver from its current step to t_final and synchronise.
   use_graph != 0 captures the launches in a HIP graph (kept and relaunched
   while the launch plan is unchanged); 0 launches them one by one.  Results
   are bitwise equal to starmap_run on each solver with the same tile. */
int starmap_batch_run(starmap_batch* b, int32_t use_graph);

/* The last run: device time between events around its launches (ms), cell-
   moment updates (sum of nx ny N_mom steps), algorithmic bytes (sum of
   starmap_sweep_bytes over its sweeps), and kernel launches. */
int starmap_batch_last_run(const starmap_batch* b, double* ms, int64_t* updates, double* bytes,
                           int64_t* launches);

/* Tile variant and m-range width (4, 6 or 8) per group; the default is
   variant 0 with width 8 for every group.  starmap_batch_set_variant gives
   every group the same pair (STARMAP_EINVAL if it does not fit the LDS for
   one of them).  starmap_batch_get_variant reports the pair of the group with
   the most cell-moment work (-1 and 0 before the first device call).
   starmap_batch_autotune times, for each group on its own, every pair that
   fits on a few sweeps with sub-step length 0 (state unchanged) and keeps the
   group's fastest; then it times the whole batch with those tiles as
   concurrent chains against merged launches on the two most promising
   common variants (each group at its fastest width for that variant) and
   keeps the fastest configuration. */
int starmap_batch_set_variant(starmap_batch* b, int32_t variant, int32_t width);
int starmap_batch_get_variant(const starmap_batch* b, int32_t* variant, int32_t* width);
int starmap_batch_autotune(starmap_batch* b, int32_t sweeps_per_variant);

/* Groups, by ascending order N: starmap_batch_group_count returns their
   number (or a negative error code); starmap_batch_get_group reports group
   `group`'s order, instance count, variant and width (-1 and 0 before the
   first device call); any output pointer may be NULL. */
int starmap_batch_group_count(const starmap_batch* b);
int starmap_batch_get_group(const starmap_batch* b, int32_t group, int32_t* N, int32_t* count, int32_t* variant,
                            int32_t* width);

/* Tile variant and m-range width of one group only (errors as
   starmap_batch_set_variant; STARMAP_EINVAL for a group out of range).
   Giving one group another variant than the others turns merged launches
   off. */
int starmap_batch_set_group_variant(starmap_batch* b, int32_t group, int32_t variant, int32_t width);

/* Merged launches: merged != 0 runs every sweep as ONE launch over the
   running instances of all groups (the groups keep their m-range widths but
   must share one tile variant, else STARMAP_EINVAL); 0 (the default) runs one
   launch per group as concurrent chains.  starmap_batch_autotune chooses
   between the two by timing sweeps of the whole batch.  get returns 0 or 1
   (or a negative error code).  Results are the same bits either way. */
int starmap_batch_set_merged(starmap_batch* b, int32_t merged);
int starmap_batch_get_merged(const starmap_batch* b);

const char* starmap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STARMAP_H */
