/*
 * mrtlb.h -- C ABI of the MI355X (gfx950) D2V16 MRT finite-difference lattice
 * Boltzmann library.
 *
 * The scheme is the one of Chen, Xu, Zhang, Li and Succi, "Multiple-relaxation-
 * time lattice Boltzmann approach to compressible flows with flexible specific-
 * heat ratio and Prandtl number" (EPL letter):
 *   df_i/dt + v_ia df_i/dx_a = -Minv_il S_lk (fhat_k - fhat^eq_k)        (Eq. 3)
 * on the 16-velocity Kataoka-Tsutahara set with the extra-dof parameter eta
 * (section "Construction of energy-conserving MRT LB model"), the
 * transformation matrix M and the equilibrium moments fhat^eq of the Appendix,
 * forward-Euler time stepping and Lax-Wendroff space differencing (same
 * section, last paragraph before Fig. 1), with R = 1.
 *
 * Conventions shared by every entry point
 *  - Every function returns MRT_OK (0) or a negative MRT_E* code; no C++
 *    exception crosses the ABI.  mrt_last_error() gives a message for the last
 *    failure on a context (a pointer into the context, valid until the next
 *    call on it).
 *  - A context owns one grid and runs on one HIP stream (the caller's, or the
 *    null stream).  Work is enqueued asynchronously on that stream unless a
 *    function says it synchronises.  A context is not thread-safe.
 *  - Grid fields are row-major ny x nx arrays (x fastest), cell-centred:
 *    cell (i, j) sits at ((i + 1/2) dx, (j + 1/2) dy).
 *  - Populations are stored as rows of 16 population sub-rows: f_i at cell
 *    (x, j) is element f[i * plane + origin + j * pitch + x] (x fastest, then
 *    the population, then the row: the 16 populations of one grid row are
 *    contiguous), with one ghost cell on each side (-1 <= x <= nx,
 *    -1 <= j <= ny) that the library fills from the boundary conditions as the
 *    step needs it; plane (the sub-row length, a multiple of 256, >= nx + 3),
 *    pitch (16 plane + 256: a padded row) and origin come from mrt_get_layout.  Only these
 *    three numbers describe the layout: code that indexes with them does not
 *    depend on it.  Velocity order: shell 1 (speed 1) and shell 2
 *    (speed 6) as (+x, +y, -x, -y); shell 3 (sqrt(2)(+-1,+-1)) and shell 4
 *    ((3/sqrt 2)(+-1,+-1)) as (++, -+, --, +-).
 *  - Device pointers are plain HIP device addresses; host pointers are
 *    ordinary host memory.  Buffers passed in stay owned by the caller.
 */
#ifndef MRTLB_H
#define MRTLB_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MRT_OK          0
#define MRT_EINVAL     -1   /* bad argument or parameter                          */
#define MRT_EDEVICE    -2   /* a HIP call failed                                  */
#define MRT_ESTATE     -3   /* call out of order (params or fields not set yet)   */
#define MRT_EUNSTABLE  -4   /* a kernel saw NaN/Inf, rho <= 0 or T <= 0           */
#define MRT_ENOMEM     -5   /* device allocation failed                           */

/* precision of a context */
#define MRT_FP64        0   /* FP64 storage and arithmetic                        */
#define MRT_FP32        1   /* FP32 storage and arithmetic; conserved sums
                               compensated                                        */
#define MRT_FP32_EQ64   2   /* FP32 storage and Lax-Wendroff stencil; moments,
                               equilibrium, relaxation and Minv in FP64           */

/* boundary kinds, one per side in the order x-lo, x-hi, y-lo, y-hi */
#define MRT_BC_PERIODIC 0   /* both sides of an axis must be periodic             */
#define MRT_BC_EQ       1   /* ghost = f^eq of a fixed state: the paper's
                               f_i = f_i^eq on boundary nodes (section (b)), also
                               used for inflow (section (d))                      */
#define MRT_BC_OUTFLOW  2   /* ghost = copy of the adjacent interior cell         */
#define MRT_BC_REFLECT  3   /* ghost = f^eq of the mirror-image interior cell with
                               its normal velocity reversed (section (d))         */

typedef struct mrt_ctx mrt_ctx;
typedef struct mrt_batch mrt_batch;

/* Scheme parameters (copied by mrt_set_params). */
typedef struct mrt_params {
    double gamma;          /* specific-heat ratio; b = 2/(gamma-1) dof, the
                              extra (b-2) carried by eta; 1 < gamma <= 2           */
    double Pr;             /* if > 0: s[7] = s[8] = Pr * s[5] (Pr = s_8/s_6 from
                              Eqs. 12b-12d) and s[6] must equal s[5]              */
    double s[16];          /* relaxation rates s_1..s_16 (s[k-1] = s_k).  s_1..4
                              multiply collision invariants and are ignored;
                              s_5..16 must lie in [0, 1/dt] (text after Eq. 12d;
                              s dt up to 1 + 1e-6 is accepted)                  */
    double dt, dx, dy;     /* time step and cell sizes, all > 0                   */
    double eta0;           /* eta on shell 1; the paper fixes 5/2 and so does this
                              library: 5/2 or 0 (which selects 5/2); any other
                              value: MRT_EINVAL                                  */
    double side_state[4][4]; /* (rho, ux, uy, T) of each MRT_BC_EQ side           */
} mrt_params;

/* ---------------------------------------------------------------- grid */

/* Create a context for an nx x ny grid.
 * precision: MRT_FP64 / MRT_FP32 / MRT_FP32_EQ64.
 * bc[4]:     boundary kinds (x-lo, x-hi, y-lo, y-hi); periodic sides must pair.
 * f_dev:     NULL: the library allocates two population buffers;
 *            else two caller-owned device buffers f_dev[0], f_dev[1], each of
 *            mrt_population_bytes(nx, ny, precision) bytes, which must outlive
 *            the context.
 * stream:    hipStream_t to run on (NULL = null stream).
 * Errors: MRT_EINVAL (nx, ny < 1, a grid of 2^32 or more padded elements
 * per state (FP32: beyond ~16000 x 16000 cells; the kernels use 32-bit
 * offsets), bad precision or bc), MRT_ENOMEM, MRT_EDEVICE.  On error *out
 * is NULL. */
int mrt_init_grid(mrt_ctx** out, int nx, int ny, int precision, const int bc[4],
                  void* const f_dev[2], void* stream);

/* Bytes of one population buffer for a grid (ny + 2 rows of 16 padded
 * population sub-rows); 0 for a grid that mrt_init_grid rejects by size. */
long long mrt_population_bytes(int nx, int ny, int precision);

/* Row stride (pitch), population stride (plane) and offset of cell (0, 0)
 * of population 0 (origin), in elements, of the population layout.  Any
 * output may be NULL. */
int mrt_get_layout(const mrt_ctx* ctx, long long* pitch, long long* plane, long long* origin);

/* Validate and copy parameters (see mrt_params).  Computes the ghost
 * equilibria of MRT_BC_EQ sides.  Errors: MRT_EINVAL. */
int mrt_set_params(mrt_ctx* ctx, const mrt_params* p);

/* Initialise the populations to the local equilibrium of the given fields,
 * f = Minv fhat^eq(rho, u, T) (the equilibrium of section (b), used at t = 0).
 * rho, ux, uy, T: ny*nx doubles, host memory (on_device = 0) or device memory
 * (on_device = 1).  Host input is staged and the call synchronises the stream.
 * Errors: MRT_ESTATE (params unset), MRT_EINVAL (rho <= 0 or T <= 0 seen;
 * host input only). */
int mrt_set_fields(mrt_ctx* ctx, const double* rho, const double* ux, const double* uy,
                   const double* T, int on_device);

/* Advance n time steps (Eq. 3, forward Euler, Lax-Wendroff).  Asynchronous.
 * One kernel pass per step, or per two steps (mrt_set_steps_per_pass; the
 * default from about 1024 x 1024 cells on), an odd
 * last step then taking a one-step pass.  Health (NaN, rho <= 0, T <= 0) is
 * recorded on the device and reported by the next synchronising call.
 * Errors: MRT_ESTATE, MRT_EINVAL (n < 0). */
int mrt_step(mrt_ctx* ctx, int n);

/* Capture, instantiate and upload (without running any kernel) the HIP
 * graphs that a following mrt_step(ctx, n) will replay, so that their
 * one-time capture, instantiation and upload cost (about a millisecond for
 * 64 passes) falls outside a timed region or a latency-critical loop.  The
 * kernel passes of mrt_step(n) (n, or n / 2 with two steps per pass) are
 * replayed as replays of one 64-pass graph and one graph of the remaining
 * passes, per start buffer (an odd step of the two-step mode is launched
 * directly); the graphs are kept until the tile, steps per pass, scheme or
 * context changes.  Launches no kernel (the uploads are enqueued on the
 * context's stream); errors as mrt_step. */
int mrt_prepare_steps(mrt_ctx* ctx, int n);

/* Macroscopic fields of the current populations: the conserved moments
 * rho = fhat_1, j = (fhat_2, fhat_3), e = fhat_4 (Appendix rows m1..m4), then
 * u = j/rho and T = (e - rho u^2)/(b rho) from e = b rho R T + j^2/rho
 * (definitions under Eqs. 12a-12d) with R = 1 (section "Numerical
 * simulation").  Outputs ny*nx doubles on the host
 * (on_device = 0; the call synchronises) or on the device (on_device = 1;
 * asynchronous).  Any output pointer may be NULL.
 * Errors: MRT_ESTATE, MRT_EUNSTABLE (health flag set since the last check;
 * the outputs are still written). */
int mrt_read_moments(mrt_ctx* ctx, double* rho, double* ux, double* uy, double* T,
                     int on_device);

/* Copy the current populations out / in, converted to FP64, in the unpadded
 * layout f[(i * ny + j) * nx + x] (16*ny*nx doubles).  Host memory
 * (on_device = 0, synchronises) or device memory (on_device = 1). */
int mrt_get_populations(mrt_ctx* ctx, double* f, int on_device);
int mrt_set_populations(mrt_ctx* ctx, const double* f, int on_device);

/* Raw device pointer of the current population buffer (storage precision,
 * padded layout) and of the other (scratch) buffer. */
int mrt_current_buffer(mrt_ctx* ctx, void** cur, void** other);

/* Synchronise the stream and test the health flag (MRT_EUNSTABLE if set;
 * the flag is cleared). */
int mrt_sync(mrt_ctx* ctx);

/* Tile shape of the one-step kernel: rows per work item (>= 1; each work item
 * is 256 columns, one 4-wave workgroup) and workgroups launched (0 = one per
 * work item).  mrt_init_grid picks rows from the grid size (about 8192 work
 * items, at most 6 rows); mrt_autotune replaces them with measured ones. */
int mrt_set_tile(mrt_ctx* ctx, int rows_per_item, int grid_blocks);
int mrt_get_tile(const mrt_ctx* ctx, int* rows_per_item, int* grid_blocks);

/* Time steps per pass over the populations: 1, 2 or 4 (default: 4 for the
 * grids the tube march below covers; 2 for grids whose population buffer
 * exceeds the 256 MB last-level cache or that give at least 512 two-step
 * work items of 8-row bands, about 1024 x 1024 cells and up; else 1.
 * mrt_autotune times all that apply and keeps the fastest).  With 2, one kernel launch
 * advances the state two steps of Eq. 3 (the same per-site arithmetic as two
 * single steps, f^{n+1} rounded to the storage precision as a stored state
 * would be, so the same result up to rounding order: measured bit-identical
 * in the FP32 storage forms, within a few roundings in FP64):
 * each work item reads f^n once, keeps f^{n+1} in registers and writes
 * f^{n+2}, recomputing f^{n+1} on the two rows above and below its band of
 * `rows` rows (1..MRT_MAX_BAND_ROWS_2; 0 = by grid size: 8, 16 or 32 rows in
 * FP32 storage, up to 64 in FP64, which runs one block per CU, chosen for
 * the fewest rounds of resident blocks x (rows + 5)) and on its
 * two edge columns, which halves the memory traffic per step.  An odd last
 * step of mrt_step runs the single-step kernel.  Every precision; the
 * default scheme only (variants set by mrt_set_scheme run one step per
 * pass).
 * steps = 4, the tube march: for grids of 1, 2 or 4 rows, periodic in y,
 * with fixed-equilibrium x sides (the shock tubes of section (b)): one
 * launch advances four steps of Eq. 3, each block holding all rows of 256
 * columns in registers and storing the 248 that are exact after four steps
 * (the overlap is recomputed); rows is ignored; steps beyond a multiple of
 * four run one by one.  Results equal single steps to rounding order
 * (measured bit-identical in the FP32 storage forms).  mrt_autotune times it
 * too on such grids.  Synchronises.
 * Errors: MRT_EINVAL (steps not 1, 2 or 4; rows out of range; 4 on another
 * grid). */
#define MRT_MAX_BAND_ROWS_2 64
int mrt_set_steps_per_pass(mrt_ctx* ctx, int steps, int rows);
int mrt_get_steps_per_pass(const mrt_ctx* ctx, int* steps, int* rows);

/* Scheme variants (the paper's discretisation passage admits three
 * readings; section "Construction", last paragraph before Fig. 1):
 *   0                      unsplit forward Euler, per-axis Lax-Wendroff
 *                          (five points): f + LW(f) - dt C(f)   [default]
 *   MRT_SCHEME_SPLIT       collide, then convect the post-collision state:
 *                          h = f - dt C(f), f^{n+1} = h + LW(h)
 *   MRT_SCHEME_LW_CROSS    full 2D Lax-Wendroff: adds the mixed-derivative
 *                          term (c_x c_y / 4)(f_NE - f_NW - f_SE + f_SW)
 * (flags combine).  Corner ghosts, which only the nine-point stencil reads,
 * follow the y side's rule applied to the x-side ghost next to them.  The
 * variants run one thread per cell (the split form in two passes through a
 * library-owned third state buffer, allocated here on first use); they are
 * for comparing readings, the default is the tuned path.  mrt_step_buffers,
 * the checkpointed calls and the adjoint support the default only
 * (MRT_EINVAL otherwise).  Errors: MRT_EINVAL (unknown flags), MRT_ENOMEM. */
#define MRT_SCHEME_SPLIT 1
#define MRT_SCHEME_LW_CROSS 2
int mrt_set_scheme(mrt_ctx* ctx, int flags);

/* Time candidate launches on the current state (the populations are saved
 * and restored): one-step tiles (rows 1..128, grid sizes) and two steps per
 * pass with bands of 8, 16 and 32 rows; keep the fastest per step.
 * Synchronises. */
int mrt_autotune(mrt_ctx* ctx, int steps_per_trial);

void mrt_destroy(mrt_ctx* ctx);
const char* mrt_last_error(const mrt_ctx* ctx);

/* ------------------------------------------------------------- adjoint
 * Discrete adjoint of one step on a fully periodic grid (other boundary kinds:
 * MRT_EINVAL).  With F the one-step map f^{n+1} = F(f^n; s):
 *   lam_n = (dF/df^n)^T lam_next
 *   ds[k] += sum over cells and populations of lam_next * dF/ds_k,
 *            dF/ds_k = -dt Minv[:,k] (fhat_k - fhat^eq_k)      (derived from Eq. 3)
 * lam_next, f_n, lam_n: device buffers in the context's storage precision and
 * padded layout (as mrt_current_buffer).  ds: 16 device doubles, accumulated
 * (the caller zeroes it).  Asynchronous.  lam_n must not alias lam_next;
 * neighbours across the grid edges are read from the wrapped cells (the ghost
 * ring is neither read nor written). */
int mrt_adjoint_step(mrt_ctx* ctx, const void* lam_next, const void* f_n, void* lam_n,
                     double* ds);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * adjoint step as mrt_adjoint_step (same kernels, same arguments, bitwise the
 * same lam_n and ds), with the rate-gradient partial sums in a fixed 1 MiB
 * device array of the library instead of the context's own buffer.  The call
 * allocates and frees nothing.  Grids of up to 8128 adjoint work items
 * (256-column chunks of row bands; e.g. 4096 x 4096 uses 4096): larger ones
 * get MRT_EINVAL with a message.  Every call on one GPU shares that array:
 * calls that overlap on one GPU (from several contexts or streams at once)
 * race; calls ordered on one stream do not (each overwrites the rows it
 * reads).  Errors as mrt_adjoint_step. */
int mrt_adjoint_step_noalloc(mrt_ctx* ctx, const void* lam_next, const void* f_n, void* lam_n,
                             double* ds);

/* Forward pass that keeps sqrt(N)-style checkpoints for a later
 * mrt_adjoint_sweep: checkpoints[k] receives f^(k * segment) for
 * k * segment < nsteps (f^0 by a copy, the others written there by their
 * step directly), stepping as mrt_step_buffers.  segment = 1 keeps every
 * state (no recomputation in the sweep).  f: on entry f^0, on return f^nsteps.  f_tmp: one more
 * state buffer (overwritten).  checkpoints: ceil(nsteps / segment) buffers.
 * All device buffers in the storage precision and padded layout, owned by the
 * caller and distinct.  MRT_EINVAL on NULL or aliased buffers, segment < 1 or
 * nsteps < 0.  Asynchronous. */
int mrt_step_checkpointed(mrt_ctx* ctx, void* f, void* f_tmp, int segment, int nsteps,
                          void* const* checkpoints);

/* Backward pass over nsteps steps from the checkpoints written by
 * mrt_step_checkpointed (same segment): the discrete adjoint of nsteps
 * forward steps of Eq. 3 (forward Euler, Lax-Wendroff), lam^n =
 * (dF/df^n)^T lam^{n+1} per step as in mrt_adjoint_step, derived from Eq. 3
 * and the Appendix equilibrium.  Segment by segment, newest first, it
 * recomputes f^start+1 .. f^stop-1 from checkpoint f^start into `work`, then
 * runs mrt_adjoint_step for n = stop-1 down to start.  The checkpointing
 * keeps ceil(N / segment) + segment states for one extra forward step per
 * step (segment ~ sqrt(N) minimises the memory).
 *   lam      on entry lam^N, on return lam^0
 *   lam_tmp  one more buffer (overwritten)
 *   work     nwork state buffers (overwritten); nwork >= w = min(segment,
 *            nsteps) - 1.  With nwork >= 2 w (and two segments or more) the
 *            next segment's states are recomputed on a second stream of the
 *            context into the other w buffers while the adjoint steps of the
 *            current segment run on the context's stream (the two kernels
 *            share the GPU); the adjoint steps stay in order on one stream,
 *            so lam and ds are bitwise those of the one-set sweep.  The call
 *            returns with all of its work ordered before later work on the
 *            context's stream.
 *   ds       16 device doubles, accumulated (the per-cell contributions of
 *            all steps are summed per wave first and reduced once, so ds
 *            equals the sum of nsteps mrt_adjoint_step calls up to rounding
 *            order, and is bitwise reproducible)
 * Buffers as for mrt_step_checkpointed (the checkpoints are only read).
 * Periodic grids only (MRT_EINVAL otherwise; also for nwork < w or NULL,
 * lam-aliased work buffers).  Asynchronous. */
int mrt_adjoint_sweep(mrt_ctx* ctx, const void* const* checkpoints, int segment, int nsteps,
                      void* const* work, int nwork, void* lam, void* lam_tmp, double* ds);

/* One forward step between explicit device buffers (storage precision,
 * padded layout), without touching the context's own buffers: used to
 * recompute states from checkpoints.  The ghost ring of f_in is refilled
 * (its cells are not changed).  Asynchronous. */
int mrt_step_buffers(mrt_ctx* ctx, const void* f_in, void* f_out);

/* Density of an explicit population buffer: rho[j*nx+x] = sum_i f_i (device
 * doubles).  Asynchronous. */
int mrt_density(mrt_ctx* ctx, const void* f, double* rho);

/* Adjoint of mrt_density: lam_i = g_rho for all 16 populations (device
 * buffers).  Asynchronous. */
int mrt_density_adjoint(mrt_ctx* ctx, const double* g_rho, void* lam);

/* Adjoint of mrt_set_fields (f^0 = Minv fhat^eq(rho, u, T)): given lam0 and
 * the device fields, writes g_x[j*nx+x] = sum_i lam0_i df^0_i/dx for x in
 * (rho, ux, uy, T).  Any output may be NULL.  Asynchronous. */
int mrt_init_adjoint(mrt_ctx* ctx, const void* lam0, const double* rho, const double* ux,
                     const double* uy, const double* T, double* g_rho, double* g_ux,
                     double* g_uy, double* g_T);

/* Initialise an explicit population buffer from device fields (as
 * mrt_set_fields with on_device = 1, but into f).  Asynchronous. */
int mrt_init_buffer(mrt_ctx* ctx, const double* rho, const double* ux, const double* uy,
                    const double* T, void* f);

/* -------------------------------------------------------------- batch
 * Many independent grids (e.g. shock tubes of different length, gamma, Pr and
 * Mach) advanced together: each instance is the scheme of Eq. 3 with its own
 * specific-heat ratio (the extra degrees of freedom b, section "Construction"),
 * its own rates (Pr = s_8/s_6 from Eqs. 12b-12d), grid and boundaries (the
 * fixed-equilibrium ends of section (b)); every step of every instance runs
 * in one kernel launch over a table of (instance, tile) work items, and
 * mrt_batch_step(n) replays one captured HIP graph of n launches.  Storage precision is the
 * batch's; each instance has its own nx, ny, boundary kinds and parameters. */
typedef struct mrt_instance {
    int nx, ny;
    int bc[4];
    mrt_params params;
} mrt_instance;

/* Errors: MRT_EINVAL (count < 1, any instance invalid or too large, as in
 * mrt_init_grid), MRT_ENOMEM. */
int mrt_batch_create(mrt_batch** out, int count, const mrt_instance* desc, int precision,
                     void* stream);
/* Fields of instance i (host doubles, ny*nx each).  Synchronises. */
int mrt_batch_set_fields(mrt_batch* b, int i, const double* rho, const double* ux,
                         const double* uy, const double* T);
int mrt_batch_step(mrt_batch* b, int n);
/* As mrt_prepare_steps, for mrt_batch_step. */
int mrt_batch_prepare_steps(mrt_batch* b, int n);
/* Moments of instance i to host doubles (any may be NULL).  Synchronises;
 * MRT_EUNSTABLE if any instance went unhealthy. */
int mrt_batch_read_moments(mrt_batch* b, int i, double* rho, double* ux, double* uy, double* T);
/* Unpadded FP64 populations of instance i (16*ny*nx host doubles). */
int mrt_batch_get_populations(mrt_batch* b, int i, double* f);
/* Rows per work item of the one-step kernel (each work item is 256 columns
 * of one instance, one 4-wave workgroup) and workgroups launched (0 = one
 * per work item); autotune times candidates, one, two and (where allowed)
 * four steps per pass, on the current state (saved and restored) and keeps
 * the fastest.  Changing the tile drops the captured graphs. */
int mrt_batch_set_tile(mrt_batch* b, int rows_per_item, int grid_blocks);
int mrt_batch_get_tile(const mrt_batch* b, int* rows_per_item, int* grid_blocks);
/* As mrt_set_steps_per_pass, for every instance of the batch (default 4 on
 * a batch the tube march covers, else 1; rows 0 = 32, bands never exceed an
 * instance's height).  steps = 4: the
 * tube march, for batches whose instances all have the same height of 1, 2
 * or 4 periodic rows and fixed-equilibrium x sides (the shock tubes of
 * section (b)), any precision.  Synchronises.
 * Errors: MRT_EINVAL (steps not 1, 2 or 4; rows out of range; 4 on a batch
 * the tube march does not cover). */
int mrt_batch_set_steps_per_pass(mrt_batch* b, int steps, int rows);
int mrt_batch_get_steps_per_pass(const mrt_batch* b, int* steps, int* rows);
int mrt_batch_autotune(mrt_batch* b, int steps_per_trial);
long long mrt_batch_cells(const mrt_batch* b);
void mrt_batch_destroy(mrt_batch* b);
const char* mrt_batch_last_error(const mrt_batch* b);

/* ------------------------------------------------------ host utilities
 * The library's own transform code evaluated on the host in FP64 (the
 * kernels run the same templates).  They need no GPU.
 *  mrt_host_transform: which = 0: out = M in (populations -> moments, the
 *    Appendix rows); 1: out = Minv in; 2: out = M^T in; 3: out = Minv^T in.
 *  mrt_host_equilibrium: f = Minv fhat^eq(rho, u, T) (Appendix), R = 1.
 *  mrt_host_collision: out = dt Minv diag(s) (M f - fhat^eq)   (Eq. 3).
 *  mrt_host_cell_adjoint: coll = dt (dC/df)^T lam at one cell, and
 *    dsk[k] = dt (fhat_k - fhat^eq_k)(Minv^T lam)_k.
 * Arrays are 16 doubles; s holds s_1..s_16.  MRT_EINVAL on NULL or gamma<=1.
 *  mrt_host_conserved_fp32: the conserved moments (rho, jx, jy, e; rows
 *    m1..m4 of the Appendix matrix) of 16 FP32 populations f as the MRT_FP32
 *    form computes them, compensated FP32 sums within one unit in the last
 *    place of the exact sums; q receives 4 floats.  MRT_EINVAL on NULL. */
int mrt_host_transform(int which, const double* in, double* out);
int mrt_host_equilibrium(double gamma, double rho, double ux, double uy, double T, double* f);
int mrt_host_collision(double gamma, const double* s, double dt, const double* f, double* out);
int mrt_host_cell_adjoint(double gamma, const double* s, double dt, const double* f,
                          const double* lam, double* coll, double* dsk);
int mrt_host_conserved_fp32(const float* f, float* q);

#ifdef __cplusplus
}
#endif
#endif /* MRTLB_H */
