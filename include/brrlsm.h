/*
 * brrlsm — block-row recursive least-squares migration on MI355X (gfx950).
 *
 * C ABI of the library. It follows the method of Kazemi & Sacchi, "Block row
 * recursive least squares migration" (CSEG 2015, arXiv 1801.00819):
 *
 *   - eq. 1 (d = A m + n) and eq. 2 (migration = A^T d): A is wave-equation
 *     Born modelling on a regular grid and A^T its exact discrete adjoint;
 *   - eq. 3 / eq. 10: each window of shots solves
 *       min ||A_w m - d_w||^2 + lambda ||m||^2
 *     by conjugate gradients on the least-squares form (normal equations
 *     eq. 4, never formed);
 *   - eq. 10-11 and Fig. 1: the window slides by adding shots (update) and
 *     removing the oldest ones (downdate); each solve starts from the image of
 *     the previous window (warm start).
 *
 * The operator is the two-way acoustic Born operator: 8th-order (radius 4)
 * central differences in space, second order in time, absorbing sponge of nb
 * cells on every face, Ricker source (delay 1.5/f0), sources and receivers on
 * grid points, m = relative perturbation of squared slowness.
 *
 * Conventions
 *   - Model-space arrays (velocity, image, m): [nz][ny][nx] row-major, x
 *     fastest, ny = 1 in 2-D. float32 unless stated.
 *   - Shot data: [nt][nrec] per shot, float32. Window data are the shots'
 *     arrays concatenated in window order (the order shots were added).
 *   - Every function returns BRLS_OK (0) or a negative BRLS_E* code; the
 *     message of the last error is available from brls_last_error. Nothing
 *     throws across the ABI.
 *   - Pointers to shot data, images and window data are host pointers unless
 *     the context was opened with BRLS_DEVICE_PTRS, in which case they are
 *     device pointers valid on the context's stream. Geometry and velocity
 *     are always host pointers. The library copies every input at call time;
 *     the caller keeps ownership of all buffers it passes.
 *   - A context is bound to the device current at brls_open and to the
 *     stream given there; it is not thread-safe. All work is ordered on that
 *     stream. Functions that return host results synchronise the stream.
 */
#ifndef BRRLSM_H
#define BRRLSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BRLS_OK 0
#define BRLS_EINVAL (-1)     /* bad argument, shape, position or CFL */
#define BRLS_ENOMEM (-2)     /* device allocation failed */
#define BRLS_EFULL (-3)      /* window already holds q_max shots */
#define BRLS_ENOSHOT (-4)    /* no shot with that id in the window */
#define BRLS_EBREAKDOWN (-5) /* CG breakdown: <p, (A^T A + lambda I) p> <= 0 */
#define BRLS_ENONFINITE (-6) /* NaN or Inf in inputs or CG scalars */
#define BRLS_EDEVICE (-7)    /* HIP runtime error or library not built for gfx950 */
#define BRLS_EDUP (-8)       /* a shot with that id is already in the window */

/* brls_grid.flags */
#define BRLS_DEVICE_PTRS 1u

/* execution modes (brls_set_exec) */
#define BRLS_EXEC_PLAIN 0   /* one kernel launch per shot and per time step */
#define BRLS_EXEC_BATCHED 1 /* one launch per time step for all window shots */
#define BRLS_EXEC_GRAPH 2   /* batched; the time loop is replayed as a hipGraph */
#define BRLS_EXEC_PERSISTENT 3 /* one launch per operator application: a
                                  resident grid runs every time step, with
                                  a grid barrier between two-step levels
                                  (replayed as a hipGraph) */

typedef struct brls_ctx brls_ctx;

typedef struct {
  int32_t ndim;       /* 2 or 3 */
  int32_t nz, ny, nx; /* model grid (ny ignored in 2-D) */
  int32_t nb;         /* absorbing cells on every face, >= 1 */
  int32_t nt_max;     /* largest number of time samples of any shot */
  int32_t nrec_max;   /* largest number of receivers of any shot */
  int32_t q_max;      /* largest number of shots held at once */
  double h;           /* grid spacing (m) */
  double dt;          /* time step (s) */
  double lambda;      /* damping of eq. 3, absolute */
  int32_t ckpt_interval; /* background wavefield strategy:
                            0  store its Born source for every step (fast;
                               (nt_max-1)*nz*nx floats per shot);
                            k > 0  keep the background state every k steps
                               and recompute it (2 fields per checkpoint);
                            -1 checkpoints every ceil(sqrt(nt_max)) steps */
  uint32_t flags;     /* BRLS_DEVICE_PTRS */
} brls_grid;

typedef struct {
  int64_t id;           /* caller's key, unique within the window */
  int32_t sz, sy, sx;   /* source grid point, model grid (sy ignored in 2-D) */
  int32_t nt, nrec;     /* 2 <= nt <= nt_max, 1 <= nrec <= nrec_max */
  double f0;            /* Ricker peak frequency (Hz) */
  const int32_t* rec;   /* host [nrec][3]: (z, y, x) model grid points */
  const float* data;    /* observed data [nt][nrec] or NULL for zeros */
} brls_shot;

typedef struct {
  int32_t iters;   /* CG iterations run */
  double s0_norm;  /* ||A^T (d - A m0) - lambda m0|| at the start */
  double s_norm;   /* same quantity at the end */
  double r_norm;   /* ||d - A m|| at the end */
  double seconds;  /* wall time of the call */
  double ref_norm; /* ||A^T d|| when rtol > 0 (the stop test's scale), else 0 */
} brls_stats;

typedef struct {
  char name[48];   /* kernel family, e.g. "born_step", "adjoint_step" */
  int64_t launches;
  double total_ms; /* summed durations between events bracketing each launch */
} brls_kstat;

/* Create a context for one velocity model: the background medium in which
 * eq. 1's de-migration operator A and eq. 2's migration operator A^T are
 * linearised (Least squares migration section), the damping lambda of
 * eq. 3, and an empty window of at most q_max shots for the block-row
 * recursion (eqs. 10-11), whose image starts at zero.
 * g: grid (copied). vel: host [nz][ny][nx] velocity in m/s, all > 0.
 * stream: hipStream_t to order all work on; NULL gives the context a private
 * stream that synchronises with the null stream (graphs cannot capture the
 * null stream itself).
 * Checks CFL stability of the scheme (v_max dt / h below 0.5546 in 2-D and
 * 0.4529 in 3-D for the 8th-order stencil) and returns BRLS_EINVAL
 * otherwise. Also BRLS_EINVAL: a padded grid (or its wavefield storage) of
 * 2^29 points or more in 2-D, 2^30 in 3-D (the kernels' 32-bit byte
 * offsets), or nt_max * nrec_max above 2^30.
 * Allocates the device state for q_max shots (see brls_memory_bytes). */
int brls_open(const brls_grid* g, const float* vel, void* stream,
              brls_ctx** out);

/* End the recursion of eqs. 10-11 on this context: release every device
 * and host resource (the window's data, background caches and image). NULL
 * is a no-op. */
void brls_close(brls_ctx* ctx);

/* Message of the last failing call on ctx (or of the last failing brls_open
 * when ctx is NULL). Valid until the next call on the same context. The
 * failures it explains are those of the calls above: invalid windows or
 * shots (the update and downdate after eq. 10), breakdown or non-finite
 * scalars of the window CG (eq. 10), device errors. */
const char* brls_last_error(const brls_ctx* ctx);

/* Rank-one part of the paper's rank-K update (after eq. 10, Fig. 1): add one
 * shot at the end of the window. Copies geometry and data; the background
 * wavefield it needs is computed lazily by the next operator call.
 * Errors: BRLS_EFULL, BRLS_EDUP, BRLS_EINVAL (positions, sizes),
 * BRLS_ENONFINITE (data holds NaN/Inf). */
int brls_update(brls_ctx* ctx, const brls_shot* shot);

/* Rank-one part of the rank-K downdate: drop the shot with this id.
 * Errors: BRLS_ENOSHOT. */
int brls_downdate(brls_ctx* ctx, int64_t id);

/* Replace the observed data of a shot already in the window ([nt][nrec]). */
int brls_set_data(brls_ctx* ctx, int64_t id, const float* data);

/* Ids of the window's shots in window order. ids may be NULL to only query
 * the count; otherwise it has room for cap entries. */
int brls_window(const brls_ctx* ctx, int64_t* ids, int32_t cap, int32_t* n);

/* Total float count of the window's concatenated data (sum of nt * nrec). */
int brls_window_data_size(const brls_ctx* ctx, int64_t* n);

/* Solve eq. 10 on the current window by CG on the least-squares form,
 * starting from the current image (eq. 11's warm start) and leaving the
 * result as the current image. Stops after max_iter iterations or once
 * ||A^T r - lambda m|| <= rtol * ||A^T d|| (rtol <= 0 disables this test;
 * with brls_set_regularization mode 1 the damping term is
 * lambda (m - m_start); with brls_set_precond mode 1 the CG is
 * preconditioned).
 * Vectors are float64 (float32 with brls_set_precision); the CG scalars
 * (alpha, beta, norms) are float64.
 * An empty window or a zero gradient returns at once with iters = 0.
 * stats may be NULL. Errors: BRLS_EBREAKDOWN, BRLS_ENONFINITE. */
int brls_solve_window(brls_ctx* ctx, int32_t max_iter, double rtol,
                      brls_stats* stats);

/* The CG recurrences of the last brls_solve_window (eq. 10's solve): per
 * iteration k = 1 .. n, alpha_k, beta_k and ||A^T r_k - lambda m_k||
 * (the damping term as in brls_solve_window). *n receives the iteration
 * count; each non-NULL array (host memory) receives min(n, cap) values.
 * Errors: BRLS_EINVAL (n NULL, cap < 0). */
int brls_solve_history(brls_ctx* ctx, int32_t cap, double* alpha,
                       double* beta, double* s_norm, int32_t* n);

/* Copy the current image [nz][ny][nx] out (synchronises the stream): the
 * window's solution of eq. 10, m after the last window being the chain's
 * result (Fig. 2d). */
int brls_image(brls_ctx* ctx, float* out);

/* Set the current image: the start of the next solve (eq. 11's warm start
 * from a given image, or m = 0 to start afresh). */
int brls_set_image(brls_ctx* ctx, const float* m);

/* The same in float64. With float64 CG vectors (brls_set_precision) the
 * image is kept in float64 between solves, so the chain's state is this
 * image and the window: a chain interrupted after a window and resumed
 * with brls_set_image64 of brls_image64's output continues bitwise as if
 * uninterrupted (brls_set_image rounds it to float32 first). out / m:
 * host or device [nz][ny][nx] doubles per flags. */
int brls_image64(brls_ctx* ctx, double* out);
int brls_set_image64(brls_ctx* ctx, const double* m);

/* Preconditioner of brls_solve_window. The paper asks for one in each
 * window's CG (to cluster the normal operator's eigenvalues near 1) and
 * names none; mode 1 is this library's diagonal one: M = I + 0.01 mean(I),
 * I the window's source-side illumination (brls_illumination), and the CG
 * runs preconditioned (directions follow M^-1 s, gamma = <s, M^-1 s>; the
 * stop test keeps ||s||). Mode 0 (default): none. Mode 1 needs stored Born
 * sources (ckpt_interval 0); otherwise BRLS_EINVAL. */
int brls_set_precond(brls_ctx* ctx, int32_t mode);
int brls_get_precond(const brls_ctx* ctx, int32_t* mode);

/* What the damping term of brls_solve_window pulls towards. Mode 0
 * (default): zero, i.e. each window solves eq. 10 as posed, whole image
 * regularised, warm-started from the current image (eq. 11 read with
 * eq. 10's lambda). Mode 1: the image the solve starts from (the previous
 * window's): min ||A_w m - d_w||^2 + lambda ||m - m_prev||^2, the
 * correction-regularised recursion, which keeps memory of earlier windows.
 * Other modes: BRLS_EINVAL. */
int brls_set_regularization(brls_ctx* ctx, int32_t mode);
int brls_get_regularization(const brls_ctx* ctx, int32_t* mode);

/* Arithmetic precision of two parts of the path (bits, 32 or 64 each).
 * background: the background wavefield u0 of each shot entering the window
 *   (the reference field of eq. 1's linearisation, computed once per shot),
 *   advanced in float64 and its Born-source frames D2u0^n stored in float32
 *   (64, the default with stored Born sources), or advanced in float32 by
 *   the stencil kernels (32; the only choice with checkpoints). Changing it
 *   rebuilds the window's stored sources at the next operator call.
 * vectors: the CG vectors of brls_solve_window (eq. 10's m, the search
 *   direction, the gradient and the residual) in float64 (64, the default)
 *   or float32 (32). The operators always take float32 inputs and
 *   propagate float32 wavefields; the CG scalars are float64 either way.
 * Both guard the final image of a truncated window solve, which amplifies
 * rounding of its inputs (eqs. 10-11). Errors: BRLS_EINVAL (other values;
 * background 64 with checkpoints). */
int brls_set_precision(brls_ctx* ctx, int32_t background, int32_t vectors);
int brls_get_precision(const brls_ctx* ctx, int32_t* background,
                       int32_t* vectors);

/* Misfit weight of one window shot (default 1, reset by brls_update): the
 * window solve minimises sum_j w_j ||A_j m - d_j||^2 + the damping term,
 * CG with A^T W r in place of A^T r and <q, W q> in place of ||q||^2 (the
 * stop test then reads ||A^T W r - ...|| <= rtol ||A^T W d||). Setting
 * w_j = beta^age at each slide, age the windows a shot has already been
 * in, gives the exponentially weighted window of forgetting-factor RLS,
 * the form of memory the paper's prior work uses (cited with eq. 11). The
 * illumination preconditioner stays unweighted. Weight 0 leaves the shot
 * in the window without effect. Errors: BRLS_ENOSHOT; BRLS_EINVAL for a
 * negative or non-finite weight. */
int brls_set_shot_weight(brls_ctx* ctx, int64_t id, double w);
int brls_get_shot_weight(const brls_ctx* ctx, int64_t id, double* w);

/* The window's illumination [nz][ny][nx]: at each model point the sum over
 * the window's shots and time levels n = 0 .. nt-2 of (D2 u0^n)^2, the
 * squared Born source of eq. 1's linearisation (F2). Needs stored Born
 * sources (BRLS_EINVAL otherwise). out: host or device per flags. */
int brls_illumination(brls_ctx* ctx, float* out);

/* Eq. 1 without noise on the current window: d_out = A_w m (window data
 * layout, brls_window_data_size floats). */
int brls_apply_born(brls_ctx* ctx, const float* m, float* d_out);

/* Eq. 2 on the current window: m_out = A_w^T d (sum over the window's shots,
 * in window order). */
int brls_apply_adjoint(brls_ctx* ctx, const float* d, float* m_out);

/* brls_apply_adjoint for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result, with the adjoint's float64 image
 * accumulators held in a static device array of 16 MiB per device instead
 * of the context's; it calls no hipMalloc, hipFree or other allocating
 * routine (the context's buffers were allocated by brls_open). Runs the
 * batched launches whatever brls_set_exec chose. The accumulators need
 * ceil(window shots / adjoint shots per work item) * nz * ny * nx doubles;
 * a window needing more than 16 MiB gets BRLS_EINVAL. Every call on a GPU
 * shares that GPU's array (zeroed at the start of each call): calls that
 * overlap on one GPU, from any context or stream, race. */
int brls_apply_adjoint_static(brls_ctx* ctx, const float* d, float* m_out);

/* Finite-difference modelling in the context's own velocity (the kind of
 * data the paper's examples migrate: finite-difference shot gathers of a
 * Ricker source, Examples section): every window shot's background
 * wavefield u0 at its receivers, u0^n for n = 0 .. nt-1 (u0^0 = 0), in the
 * window data layout. Nonlinear data of a model are the difference of this
 * output for its true velocity and for a background velocity. Runs one
 * background pass from rest; stored Born sources and checkpoints are left
 * as they are. out: host or device per flags. */
int brls_background_window(brls_ctx* ctx, float* out);

/* Execution mode for the operator pair (BRLS_EXEC_*). Results agree across
 * modes to rounding of the image reduction order. BRLS_EXEC_PERSISTENT
 * needs a 2-D context with stored Born sources and a tile variant of kind
 * 4 (BRLS_EINVAL otherwise): each Born or adjoint application is one
 * launch of at most as many blocks as the device holds at once, which
 * runs all time steps, every block waiting at a grid barrier between
 * consecutive two-step levels (all the window's shots and time steps in
 * one launch, as a batching form of the method's operators, eqs. 1-2 per
 * window, eq. 10). */
int brls_set_exec(brls_ctx* ctx, int32_t mode);

/* Concurrent launch chains of the batched and graph modes (1 or 2; default
 * 2 for 2-D contexts with stored Born sources, 1 otherwise): with 2 and at
 * least two shot groups in the window, each operator
 * application (eqs. 1-2 over the window's shots, eq. 10) runs its time
 * loop as two independent chains of launches, over the first half of the
 * shot groups and the rest, on two streams that run concurrently (the
 * second forked from and joined back to the context's stream, inside a
 * captured graph too). Results are bitwise those of one chain. Not used
 * with per-launch kernel timing or persistent launches. Errors:
 * BRLS_EINVAL for other counts. */
int brls_set_chains(brls_ctx* ctx, int32_t n);
int brls_get_chains(const brls_ctx* ctx, int32_t* n);

/* Bound of the persistent kernel's barrier waits, in polls (default 2^20,
 * about a second). A wait that reaches it gives up: the launch ends, the
 * operator call returns BRLS_EDEVICE and its result is invalid; no launch
 * can hang. Tests set 0 to force that path. */
int brls_set_spin_limit(brls_ctx* ctx, int32_t polls);

/* Tile shape of the stencil kernels: index into the compiled variants
 * (brls_tile_count); -1 restores the default. brls_tile_info reports a
 * variant's tile width tx, height tz, thread rows, and its kind in
 * `pipelined`: 0 = a block stages the tile (with its 4-cell halo) in LDS and
 * runs its shots in turn; 1 = the same, the next shot's loads issued before
 * the current shot is computed; 2 = z-marching wavefronts: each wavefront
 * walks a tx-column strip down a tz-row chunk with the z-stencil in
 * registers and the x-stencil from neighbouring lanes (thread rows 1);
 * 3 = the same taking two time steps per launch; 4 = two steps per launch,
 * each wavefront marching a segment of tz rows for one shot with the rows
 * shared by consecutive chunks kept in registers, a block holding the
 * wavefronts of one shot group (needed by BRLS_EXEC_PERSISTENT). */
int brls_set_tile(brls_ctx* ctx, int32_t variant);
int brls_tile_count(int32_t* n);
/* 3-D variants: XY tile tx x ty and the shots a block advances together
 * (a 3-D context's shots per block follow its variant). */
int brls_tile3_count(int32_t* n);
int brls_tile3_info(int32_t variant, int32_t* tx, int32_t* ty,
                    int32_t* shots);
int brls_tile_info(int32_t variant, int32_t* tx, int32_t* tz,
                   int32_t* thread_rows, int32_t* pipelined);

/* Shots one block handles in turn in batched modes (default 4), for both
 * operators. */
int brls_set_shots_per_block(brls_ctx* ctx, int32_t per_block);
int brls_get_tile(const brls_ctx* ctx, int32_t* variant, int32_t* per_block);

/* Grid shape of the stencil kernels: 0 (default) launches one block per
 * (tile, shot group) work item; 1 launches only as many blocks as fit on the
 * device at once, each looping over work items. */
int brls_set_resident_grid(brls_ctx* ctx, int32_t enable);
int brls_get_resident_grid(const brls_ctx* ctx, int32_t* enable);

/* Set / read the launch choice: tile variant, and shots per block and grid
 * shape of the Born (and background) launches and of the adjoint launches.
 * Grid shape bits: bit 0 = resident grid (as brls_set_resident_grid);
 * bit 1 (2-D only) = work items dealt to blocks in launch order instead of
 * in 8 contiguous ranges, one per XCD; bit 2 (2-D two-step variants) =
 * strips vary fastest along the work items (wavefronts that run together
 * cover whole grid rows) instead of chunks of one strip. 3-D variants fix
 * the shots per block. */
int brls_set_tuning(brls_ctx* ctx, int32_t variant, int32_t born_pb,
                    int32_t born_grid, int32_t adj_pb, int32_t adj_grid);
int brls_get_tuning(const brls_ctx* ctx, int32_t* variant, int32_t* born_pb,
                    int32_t* born_grid, int32_t* adj_pb, int32_t* adj_grid);

/* 3-D only: z planes per work item of the 3-D kernels (default 32; 1 ..
 * 4096). Errors: BRLS_EINVAL (2-D context or out of range). */
int brls_set_zchunk(brls_ctx* ctx, int32_t planes);
int brls_get_zchunk(const brls_ctx* ctx, int32_t* planes);

/* Time every tile variant, shots-per-block choice and grid shape (3-D:
 * also z planes per work item 8, 16, 32, 64) on the current window
 * (Born and adjoint applications of 400 time steps, results discarded)
 * and keep the fastest, shots per block and grid shape chosen per operator.
 * Returns the chosen variant in *best. In persistent execution only the
 * variants that support it are tried. */
int brls_autotune(brls_ctx* ctx, int32_t* best);

/* Per-kernel timing with HIP events around every launch (adds small gaps
 * between launches; off by default). brls_kernel_stats fills up to cap
 * entries and resets the counters. */
int brls_kernel_timing(brls_ctx* ctx, int32_t enable);
int brls_kernel_stats(brls_ctx* ctx, brls_kstat* out, int32_t cap, int32_t* n);

/* Device bytes held by the context. */
int brls_memory_bytes(const brls_ctx* ctx, int64_t* bytes);

/* Wait for all work queued on the context's stream. */
int brls_sync(brls_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* BRRLSM_H */
