/*
 * lb.h -- C ABI of the MI355X (gfx950) library for the symmetric
 * free-energy multicomponent lattice Boltzmann method of Li & Wagner,
 * "A Symmetric Free Energy Based Multi-Component Lattice Boltzmann Method"
 * (arXiv:0704.3444).
 *
 * The library advances N component distributions f^sigma_i on a periodic
 * lattice (or a box closed by walls) by the per-component lattice Boltzmann
 * equation Eq. (ssLB) (BGK collision with relaxation time tau plus a forcing
 * term, then streaming),
 * with the equilibrium moments and forcing moments Eqs. (ff1)-(ff3) of
 * Sec. III, the force of Eq. (definef), and the chemical potentials of the
 * Flory-Huggins free energy Eq. (lgf) of Sec. IV (taken per mer, plus a
 * square-gradient term -kappa lap rho^sigma).
 *
 * Conventions shared by every entry point:
 *   - lattice units, dt = dx = 1, c_s^2 = 1/3;
 *   - site index s = x + nx*(y + ny*z); every axis is periodic unless
 *     lb_params.walls closes it;
 *   - host arrays are caller-owned FP64, component-major structure of
 *     arrays (e.g. rho[sigma][s]);
 *   - device state is owned by the context (in caller-provided device
 *     memory when a workspace is passed to lb_init);
 *   - all device work is issued on params.stream (a hipStream_t, NULL for
 *     the null stream) in issue order; only lb_moments, lb_get_f and
 *     lb_get_state/lb_set_state wait for the stream;
 *   - calls on one context are not thread-safe; distinct contexts are
 *     independent;
 *   - no C++ exception crosses this boundary; every int-returning call
 *     returns LB_OK or a negative lb_status.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_MAX_COMP 8
#define LB_ABI_VERSION 1

typedef enum lb_status {
  LB_OK = 0,
  LB_EINVAL = -1,    /* invalid argument or parameter (message: lb_last_error) */
  LB_ENOMEM = -2,    /* device or host allocation failed, or workspace too small */
  LB_ENOTSUP = -3,   /* valid but not supported by this library                 */
  LB_EDEVICE = -4,   /* a HIP runtime call failed                               */
  LB_ENUMERIC = -5   /* a non-finite or non-positive density was detected       */
} lb_status;

/* Velocity sets: D1Q3 is the paper's (Sec. IV); D2Q9 and D3Q19 are the
 * standard second-order sets with sum_i w_i v_i v_i = I/3. */
typedef enum lb_lattice { LB_D1Q3 = 1, LB_D2Q9 = 2, LB_D3Q19 = 3 } lb_lattice;

/* Storage and arithmetic precision of the populations.
 *   LB_F64:  stored and computed in FP64.
 *   LB_F32:  stored and computed in FP32.
 *   LB_F16S: computed in FP32; each site keeps, per component, an FP16
 *            reference h = rho^sigma / (36 s^sigma) of its own density, set
 *            by its collision, and stores each moving population (i > 0)
 *            that it sends as the FP16 deviation f_i / s^sigma - 36 w_i h
 *            from the equilibrium at that reference, with s^sigma twice the
 *            smallest power of two >= max rho0^sigma; the rest slot holds an
 *            FP32 ledger that absorbs the FP16 rounding, so that every
 *            collision keeps each component's mass exactly (all stored
 *            quantities are multiples of 2^-24 s^sigma and their sums are
 *            exact).  Populations and the reference take 2 bytes, the rest
 *            slot 4 (22 bytes per site and component on D2Q9, against 36 for
 *            LB_F32).  The rounding error of a stored value is at most
 *            2^-11 of its deviation from the equilibrium at the sending
 *            site's density, so it stays small in every phase, the scarce
 *            one included. */
typedef enum lb_storage { LB_F64 = 0, LB_F32 = 1, LB_F16S = 2 } lb_storage;

/* Which line of Eq. (definef) forms the force rho^sigma a^sigma, with
 * c = 1 - 1/(2 tau):
 *   LB_FORCE_LOG:      -c rho^s grad(mu^s - (1/3) ln rho^s)  (first line)
 *   LB_FORCE_EXPANDED: -c (rho^s grad mu^s - (1/3) grad rho^s) (second line)
 * The two agree in the continuum.  Gradients use the isotropic lattice
 * stencil grad g = 3 sum_i w_i v_i g(r + v_i); the Laplacian in mu is
 * lap g = 6 sum_i w_i (g(r + v_i) - g(r)). */
typedef enum lb_force_form { LB_FORCE_LOG = 0, LB_FORCE_EXPANDED = 1 } lb_force_form;

/* Kernel path.
 *   LB_PATH_AUTO:  the fastest path that supports the run (sweep, then tile,
 *                  then split).
 *   LB_PATH_TILE:  fused one-kernel D2Q9 step over 2-D tiles with a two-site
 *                  density halo (any nx, every storage, periodic box or
 *                  walls).
 *   LB_PATH_SPLIT: three kernels per step (density, potential, collide and
 *                  stream); every lattice, periodic box or walls.
 *   LB_PATH_SWEEP: fused one-kernel step that sweeps the box: on D2Q9
 *                  64-column strips row by row (LB_F32 or LB_F16S, N <= 4,
 *                  nx a multiple of 64), on D3Q19 pencils of 64 x 4 sites
 *                  plane by plane (LB_F32, N <= 3, nx a multiple of 64, ny
 *                  of 4); periodic boxes or walls on the swept axis (y
 *                  on D2Q9, z on D3Q19), population copies below 4 GiB.
 * Asking for a path that does not support the run gives LB_ENOTSUP. */
typedef enum lb_path { LB_PATH_AUTO = 0, LB_PATH_TILE = 1, LB_PATH_SPLIT = 2, LB_PATH_SWEEP = 3 } lb_path;

typedef struct lb_params {
  int32_t n_comp;        /* N, 1 .. LB_MAX_COMP                                   */
  int32_t lattice;       /* lb_lattice                                            */
  int32_t storage;       /* lb_storage                                            */
  int32_t force_form;    /* lb_force_form                                         */
  int64_t nx, ny, nz;    /* box; D1Q3 needs ny = nz = 1, D2Q9 nz = 1; each >= 1  */
  double tau[LB_MAX_COMP];  /* tau^sigma; all equal (the total-fluid equation,
                              Eq. (sgLB), needs one tau) and > 1/2             */
  double theta;          /* temperature of Eq. (lgf), > 0                         */
  double kappa;          /* square-gradient coefficient, >= 0                     */
  double m[LB_MAX_COMP]; /* polymerisation m^sigma > 0                            */
  double chi[LB_MAX_COMP * LB_MAX_COMP]; /* chi^{sigma sigma'}, row-major with
                              leading dimension LB_MAX_COMP; the N x N block must
                              be symmetric with zero diagonal (Sec. IV)          */
  int32_t path;          /* lb_path                                               */
  int32_t check_every;   /* every K steps lb_step also checks every density for
                            NaN or <= 0 (0: only in lb_moments); a failed check
                            makes the next synchronising call return LB_ENUMERIC */
  void* stream;          /* hipStream_t for all device work (NULL: null stream)   */
  int32_t walls;         /* 0: periodic box (the paper's).  Bit a set: axis a
                            (0 x, 1 y, 2 z) is closed by walls half a site
                            beyond its first and last layers -- not in the
                            paper, this library's own addition: populations that
                            would cross a wall bounce back to their site
                            reversed (no slip; every component's mass kept), and
                            the density and potential stencils mirror the layer
                            next to the wall (zero normal gradient, a wall that
                            favours no component).  LB_PATH_SPLIT; on D2Q9
                            also LB_PATH_TILE; LB_PATH_SWEEP for walls on y
                            only (D2Q9) or z only (D3Q19).  Every path gives
                            the same values bit for bit. */
  int32_t reserved;      /* 0                                                     */
} lb_params;

typedef struct lb_ctx lb_ctx;

/* Device bytes that lb_init needs for params p (two population copies plus
 * scratch), or 0 when p is invalid. */
size_t lb_workspace_bytes(const lb_params* p);

/* Create a context and set every site to rest equilibrium,
 * f^sigma_i = w_i rho0^sigma (the paper prescribes the initial volume
 * fractions of a fluid at rest).  Waits for the stream before returning.
 *   p          parameters, copied.
 *   rho0       host FP64 [N][S] initial component densities, each > 0; copied.
 *   workspace  device memory of at least lb_workspace_bytes(p) bytes, 256-byte
 *              aligned, owned by the caller and kept alive until lb_free; or
 *              NULL, in which case the library allocates (and frees) its own.
 *   out        receives the context.
 * On the strip-sweep path (lb_path_in_use) of a grid of at least 2^20
 * sites, lb_init also chooses the sweep's segment length on the new state:
 * it takes 48 steps, then times up to 8 segment lengths (twice each: one
 * step to switch, then 4 between events on the stream), times the two
 * fastest again (twice each, alternately, over 12 steps), keeps the faster
 * and returns the state to rest equilibrium before returning (a few tens of
 * milliseconds at 2048^2).  Every segment length gives the same results bit
 * for bit; lb_step itself never times or waits.
 * Errors: LB_EINVAL (parameters, rho0 <= 0 or non-finite, misaligned
 * workspace), LB_ENOMEM (workspace_bytes too small, allocation failure),
 * LB_EDEVICE. */
int lb_init(const lb_params* p, const double* rho0, void* workspace, size_t workspace_bytes,
            lb_ctx** out);

/* Advance nsteps >= 0 time steps of Eq. (ssLB): per site and component the
 * moments, chemical potentials, force, equilibrium, forcing term, BGK
 * collision and streaming.  Asynchronous on the context's stream: it only
 * enqueues kernels (it may be recorded under stream capture). */
int lb_step(lb_ctx* c, int64_t nsteps);

/* Observables at the current time, computed on the device in FP64 from the
 * stored populations and copied to caller-owned host buffers (any pointer
 * may be NULL).  Synchronises the stream.
 *   rho   [N][S]   component densities rho^sigma = sum_i f^sigma_i
 *   U     [D][S]   macroscopic velocity U = u + (1/2) sum_sigma A^sigma / rho
 *                  (Sec. III), u the barycentric velocity
 *   mu    [N][S]   per-mer chemical potentials mu^sigma
 *   P     [D(D+1)/2][S] pressure tensor xx, xy, (xz), yy, (yz), (zz) of the
 *                  free energy with the square-gradient term; bulk part
 *                  sum rho mu - psi, Eq. (ppp) (a diagnostic; the update does
 *                  not use it)
 *   mass  [N]      sum over sites of rho^sigma
 *   mom   [D]      sum over sites and components of the first moments
 *   step  [1]      number of steps taken
 * Returns LB_ENUMERIC if any density is non-finite or <= 0 (outputs are
 * still written). */
int lb_moments(lb_ctx* c, double* rho, double* U, double* mu, double* P, double* mass,
               double* mom, int64_t* step);

/* lb_moments for callers that cannot allocate device memory (loops that
 * must not call hipMalloc between steps, harnesses that forbid it): the
 * same outputs, bit for bit, from the same kernels, but the device buffers
 * in which the fields are formed (rho, mu, h, U and P in FP64:
 * (3 N + D + D (D + 1) / 2) * S * 8 bytes) are a static array of
 * LB_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends; it allocates nothing, on the device or
 * the host.  The mass and momentum sums use the context's own workspace.
 * The calling thread's current device must be the context's.  Every call on
 * one device shares that device's array: calls that overlap on one device
 * (from several threads, or on several streams) race.  Each call writes
 * every element it reads, so no state carries over between calls.
 * Errors: as lb_moments, and LB_ENOMEM (any field pointer non-NULL while the
 * fields need more than LB_NOALLOC_SCRATCH_BYTES; mass, mom and step alone
 * need no scratch), LB_EINVAL (another device current), LB_EDEVICE (the
 * array's address could not be obtained). */
#define LB_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int lb_moments_noalloc(lb_ctx* c, double* rho, double* U, double* mu, double* P, double* mass,
                       double* mom, int64_t* step);

/* Populations f^sigma_i(r, t) at the current time as host FP64 [N][Q][S],
 * velocity order of the lattice tables (lb_lattice_tables).  Synchronises. */
int lb_get_f(lb_ctx* c, double* f);

/* Checkpoint: the raw device state (storage precision), the reference of
 * LB_F16S storage (s^sigma; zero for the other storages) and
 * the step counter.  lb_state_bytes gives the size; lb_get_state copies it
 * to host memory, lb_set_state restores it into a context created with the
 * same parameters (any rho0).  Both synchronise. */
size_t lb_state_bytes(const lb_ctx* c);
int lb_get_state(lb_ctx* c, void* host, size_t bytes);
int lb_set_state(lb_ctx* c, const void* host, size_t bytes);

/* Lattice tables: Q, D, velocities v[Q][3] and weights w[Q] (host). */
int lb_lattice_tables(int32_t lattice, int32_t* Q, int32_t* D, int32_t* v, double* w);

/* Path that lb_step runs for this context (LB_PATH_TILE, LB_PATH_SPLIT or
 * LB_PATH_SWEEP). */
int lb_path_in_use(const lb_ctx* c);

/* Release the context and any memory the library allocated.  NULL is a
 * no-op.  Waits for the context's stream. */
void lb_free(lb_ctx* c);

/* ------------------------------------------------------------------------
 * Batches: many independent runs stepped together.
 *
 * A batch holds up to max_slots D2Q9 runs ("slots") of one storage
 * precision, each with its own box, N <= max_comp and parameters of
 * Eq. (ssLB) / Eq. (lgf), and steps all of them with one persistent kernel
 * launch per time step: the launch walks the tiles of every live slot (the
 * tile step is the one of LB_PATH_TILE, so a slot's result is bit for bit
 * the one of the same run alone).  Runs of graph_steps steps are replayed
 * from a captured hipGraph.  Each slot stops at its own target step; slots
 * join (lb_batch_add) and leave (lb_batch_remove) between calls without
 * re-capturing the graph, since the kernel reads the slot table and the
 * per-slot step counters from device memory.
 *
 * Memory: one device arena of arena_bytes, allocated at creation, holds the
 * slots; lb_batch_add admits a run only if its footprint
 * (lb_batch_footprint) fits in a free range (first fit), and returns
 * LB_ENOMEM otherwise, so a caller can queue the run and retry after a
 * removal.  Admission (lb_init's work) and observables run on a second,
 * library-owned stream, overlapping the stepping of the other slots.
 * Calls on one batch are not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct lb_batch lb_batch;

typedef struct lb_batch_params {
  int32_t storage;      /* LB_F64, LB_F32 or LB_F16S, for every slot             */
  int32_t max_comp;     /* bound on N of the slots, 1 .. 4                        */
  int32_t max_slots;    /* slot capacity, 1 .. 4096                               */
  int32_t config;       /* kernel configuration (tile shape and grid), index
                           below lb_batch_config_count; -1 for the default       */
  int32_t graph_steps;  /* steps per captured graph, >= 1 (0: 16)                 */
  int32_t reserved;
  size_t arena_bytes;   /* device memory for the slots                           */
  void* stream;         /* hipStream_t of the stepping (NULL: null stream)       */
} lb_batch_params;

/* Create a batch (allocates the arena, the slot table and a second stream).
 * Errors: LB_EINVAL, LB_ENOTSUP (storage / max_comp), LB_ENOMEM, LB_EDEVICE. */
int lb_batch_create(const lb_batch_params* bp, lb_batch** out);

/* Arena bytes that a run with params p takes in batch b (0 if p is invalid
 * or not admissible to b). */
size_t lb_batch_footprint(const lb_batch* b, const lb_params* p);

/* Admit a run: validate p (D2Q9, periodic, the batch's storage, N <= max_comp; path,
 * check_every and stream are ignored), carve its workspace from the arena,
 * set rest equilibrium from rho0 (host FP64 [N][S], as lb_init) and make it
 * a live slot that lb_batch_step advances until it has taken nsteps steps.
 * Writes the slot id to *slot.  Synchronises the library's second stream
 * only.  Errors: LB_EINVAL, LB_ENOTSUP, LB_ENOMEM (no free slot or no arena
 * range large enough: retry after lb_batch_remove), LB_EDEVICE. */
int lb_batch_add(lb_batch* b, const lb_params* p, const double* rho0, int64_t nsteps, int32_t* slot);

/* Advance every live slot by up to nsteps steps (a slot stops at its
 * target), asynchronously on the batch stream, and queue a snapshot of the
 * step counters. */
int lb_batch_step(lb_batch* b, int64_t nsteps);

/* Step counters of all max_slots slots (-1 for a free slot) into
 * steps_done, from the snapshot queued `lag` lb_batch_step calls before the
 * latest one (lag 0: the latest), waiting for it to complete; lag must be
 * below 4.  A slot whose counter equals its target is finished: its state
 * no longer changes. */
int lb_batch_poll(lb_batch* b, int32_t lag, int64_t* steps_done);

/* Observables of a finished slot (as lb_moments; finished in the last
 * snapshot lb_batch_poll returned).  Runs on the library's second stream and
 * waits for it; the batch stream keeps going.  Errors: LB_EINVAL (slot not
 * live or not finished), LB_ENUMERIC, LB_EDEVICE. */
int lb_batch_moments(lb_batch* b, int32_t slot, double* rho, double* U, double* mu, double* P, double* mass,
                     double* mom, int64_t* step);

/* Release a slot and its arena range (a slot still running is stopped). */
int lb_batch_remove(lb_batch* b, int32_t slot);

/* Kernel configurations of the batched kernel for (storage, max_comp):
 * their number, and the tile shape, threads per workgroup and workgroups
 * per compute unit of the persistent grid of configuration `config`. */
int lb_batch_config_count(int32_t storage, int32_t max_comp);
int lb_batch_config_info(int32_t storage, int32_t max_comp, int32_t config, int32_t* tile_x, int32_t* tile_y,
                         int32_t* threads, int32_t* groups_per_cu);

/* Switch the batch to configuration `config` (re-captures the graph). */
int lb_batch_set_config(lb_batch* b, int32_t config);

/* Autotuner: time every configuration on the batch's live slots for `steps`
 * steps each (after one warm-up step), with HIP events on the batch stream,
 * and switch to the fastest.  The slots advance by (steps + 1) times the
 * number of configurations (every configuration gives the same results bit
 * for bit, so this is ordinary progress).  ms_per_step receives the timings
 * (lb_batch_config_count entries, may be NULL); *best the chosen index.
 * Waits for the batch stream. */
int lb_batch_tune(lb_batch* b, int32_t steps, double* ms_per_step, int32_t* best);

/* Free the batch, its slots and its arena (waits for both streams). */
void lb_batch_free(lb_batch* b);

/* ------------------------------------------------------------------------
 * Groups of one-dimensional runs (the phase-equilibrium experiments of
 * Sec. IV: D1Q3 lines, one run per interaction strength, relaxation time or
 * starting composition).
 *
 * A group steps the runs of several contexts made by lb_init with one
 * kernel launch per call: one wavefront holds a whole line in registers and
 * takes all nsteps steps there, reading and writing the populations in
 * device memory once per call.  A run's populations after lb_lines_step are
 * bit for bit those lb_step gives it.  The contexts stay usable as before
 * (lb_moments, lb_get_f, checkpoints) and keep their step counters.
 *
 * Requirements on the contexts: lattice LB_D1Q3, storage LB_F64 or LB_F32,
 * nx = 64, 128, 192 or 256, N <= 4, periodic (no walls); within a group
 * the same N, storage, nx and stream; no context twice.  Parameters of
 * Eq. (ssLB) and Eq. (lgf) (tau, theta, m, chi, kappa, force form) may
 * differ between runs.
 * ------------------------------------------------------------------------ */
typedef struct lb_lines lb_lines;

/* Form a group of n contexts (ctxs[0..n-1], host array of handles; the
 * library keeps the handles, not the array).  Uploads a table of the runs'
 * parameters and population addresses to device memory and waits for it.
 * Every context holds two population copies; the current one must be the
 * same of the two in every context (as after numbers of lb_step steps of
 * the same parity, e.g. all freshly made).  The contexts must outlive the
 * group.  Errors: LB_EINVAL (NULL, duplicates, mixed N / storage / nx /
 * stream / current copy), LB_ENOTSUP (lattice, storage, nx or N outside the
 * requirements), LB_ENOMEM, LB_EDEVICE. */
int lb_lines_create(lb_ctx* const* ctxs, int32_t n, lb_lines** out);

/* Advance every run of the group by nsteps steps, asynchronously on the
 * group's stream; each context's step counter grows by nsteps.  A density
 * that is not finite and > 0 in any step sets the context's health flag
 * (lb_moments then returns LB_ENUMERIC); the periodic checks of
 * check_every are not run.  A call moves every context to its other copy.
 * Steps taken outside the group in between are allowed when they leave
 * each context on the copy the group left it on (an even number of lb_step
 * steps).  Errors: LB_EINVAL (nsteps < 0, or a context whose current copy
 * has changed since the group's last call), LB_EDEVICE. */
int lb_lines_step(lb_lines* g, int64_t nsteps);

/* Release the group (not its contexts); waits for the group's stream.  NULL
 * is a no-op. */
void lb_lines_free(lb_lines* g);

/* Static description of a status code. */
const char* lb_strerror(int code);

/* Message of the last failed call on this thread (empty if none). */
const char* lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LB_H */
