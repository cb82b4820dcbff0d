/*
 * psatd.h -- C ABI of the MI355X (gfx950) PSATD Maxwell step with guard cells.
 *
 * One call of psatd_step_g1 performs one time step of the ultra-high-order
 * pseudo-spectral analytical time-domain (PSATD) Maxwell solver on one box of
 * the global grid (a whole "group" of the hybrid solver, or one sub-domain of
 * the local solver), as described in Kallala, Vay & Vincenti, "A generalized
 * massively parallel ultra-high order FFT-based Maxwell solver",
 * arXiv:1812.07357:
 *   - guard fill: the box (interior + guard cells) is gathered from the
 *     global grid G1 (Sec. 2.5.2, coupling step 1; guards of G2 are filled
 *     from G1, periodic wrap);
 *   - forward 3D FFT of E, B, J, rho_old, rho_new (Sec. 1.1);
 *   - analytic k-space push of E and B with order-p modified wavenumbers
 *     (Sec. 1.1 and 1.3: order p = centred stencil of half width p/2,
 *     p -> infinity = spectral);
 *   - inverse 3D FFT of E, B;
 *   - guard merge: the interior of E, B is copied back to G1 (Sec. 2.5.2,
 *     coupling step 3).
 *
 * Conventions (all entry points):
 *   - Arrays are contiguous, x fastest: element (i, j, k) of an nx*ny*nz array
 *     is at offset (k * ny + j) * nx + i.  A torch tensor of shape (nz, ny, nx).
 *   - Every data pointer is a DEVICE pointer on the current HIP device, of type
 *     float (PSATD_FP32 plans) or double (PSATD_FP64 plans).  The caller owns
 *     all field buffers and keeps them alive until the stream has finished.
 *   - The eleven field slots are, in this order: Ex Ey Ez Bx By Bz Jx Jy Jz
 *     rho_old rho_new.  J is the current at the half step and is held constant
 *     over the step; rho_old / rho_new are the charge densities at the start and
 *     at the end of the step.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = default
 *     stream) and return without synchronising.  A plan (or batch) owns its
 *     workspace, so one plan must not run on two streams at once: a step
 *     called on a stream other than the previous step's, while that step is
 *     still running, returns PSATD_ESTATE (checked with an event query; steps
 *     enqueued on a stream under graph capture are not checked).
 *   - Return values: PSATD_OK or a negative PSATD_E* code; psatd_last_error()
 *     then returns a message for the calling thread.  Errors of kernels already
 *     in flight surface as PSATD_EHIP at a later call.
 *   - Units: c and eps0 are plan parameters (1 and 1 by default).
 */
#ifndef PSATD_H
#define PSATD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psatd_plan psatd_plan;

enum {
  PSATD_OK = 0,
  PSATD_EINVAL = -1,      /* bad argument (sizes, order, NULL pointer, ...) */
  PSATD_ENOMEM = -2,      /* device allocation failed; nothing leaked */
  PSATD_EHIP = -3,        /* HIP runtime error (launch, copy, earlier kernel) */
  PSATD_EUNSUPPORTED = -4,/* valid request this build cannot serve */
  PSATD_ESTATE = -5       /* object in the wrong state for the call */
};

enum { PSATD_FP32 = 0, PSATD_FP64 = 1 };

/* Plan descriptor.  Sizes are INTERIOR cells; the transformed box has
 * n + 2*ng cells per axis.  order: 0 = infinite order (exact k), otherwise an
 * even integer >= 2 used on all three axes.  dx, dy, dz > 0; dt != 0; c > 0;
 * eps0 > 0.  flags: a combination of the PSATD_FLAG_* bits below. */
enum {
  /* Staggered (Yee) grid instead of the collocated one: Ex, Ey, Ez sit half a
   * cell up along x, y, z; Bx, By, Bz half a cell up along (y, z), (x, z),
   * (x, y); J like E; rho on the nodes.  Array index i of a component holds its
   * value at (i + offset) d.  Derivatives are order-p staggered differences,
   * sum_l a_l (f(x + (l - 1/2) d) - f(x - (l - 1/2) d)) / d (exact k at infinite
   * order), the grid of the production PSATD codes the paper builds on (Sec.
   * 1.1, 1.3).  The coefficient tables then hold the staggered symbol k_s. */
  PSATD_FLAG_STAGGERED = 1,
  /* The plan allocates no spectral workspace: it can only step through
   * psatd_step_g1_noalloc (the other step calls and the autotuner return
   * PSATD_ESTATE), and its box must fit that call's static scratch.  Not
   * allowed for the boxes of a batch. */
  PSATD_FLAG_NO_WORKSPACE = 2
};
typedef struct {
  int nx, ny, nz;
  int ngx, ngy, ngz;
  int order;
  double dx, dy, dz;
  double dt;
  double c;
  double eps0;
  int precision; /* PSATD_FP32 or PSATD_FP64 */
  int flags;
} psatd_plan_desc;

/* Simple constructor of the common case: FP32, c = eps0 = 1, dx = dy = dz,
 * the same guard width on every side of every axis.  Builds the FFT schedule,
 * twiddles and PSATD coefficient tables (in FP64 on the device, stored at the
 * working precision) and allocates the workspace.  Synchronises the device.
 * Returns NULL on error (psatd_last_error() says why). */
psatd_plan* psatd_plan_create(int nx, int ny, int nz, int nguard, int order, double dx, double dt);

/* General constructor; *out receives the plan.  Same behaviour as above. */
int psatd_plan_create_ex(const psatd_plan_desc* desc, psatd_plan** out);

/* Releases a plan.  NULL-safe.  The caller synchronises the plan's stream first. */
void psatd_plan_destroy(psatd_plan* plan);

/* Box-level step (Sec. 1.1): E and B are advanced in place on box-shaped arrays
 * of (nx+2ngx) x (ny+2ngy) x (nz+2ngz) cells, the box being taken as periodic.
 * E[3], B[3]: read and overwritten; J[3], rho_old, rho_new: read only.
 * All eleven arrays must be distinct. */
int psatd_push(psatd_plan* plan, void* const E[3], void* const B[3], const void* const J[3],
               const void* rho_old, const void* rho_new, void* stream);

/* Guard fill (Sec. 2.5.2, step 1): for each of `nfields` arrays,
 *   box[k][j][i] = g1[(oz-ngz+k) mod GZ][(oy-ngy+j) mod GY][(ox-ngx+i) mod GX]
 * for the whole box.  g1[f] are global arrays of gdims = {GX, GY, GZ} cells;
 * box[f] are box-shaped arrays.  origin = {ox, oy, oz} is the global index of
 * the first interior cell (0 <= o < G).  Guards may be wider than G. */
int guard_fill(psatd_plan* plan, const void* const* g1, void* const* box, int nfields,
               const int origin[3], const int gdims[3], void* stream);

/* Guard merge (Sec. 2.5.2, step 3).  mode 0 (copy): the interior of each box
 * array is written to g1 at (o + i) mod G.  mode 1 (add): every box cell,
 * guards included, is added to g1 at its wrapped global index (for sources
 * deposited on boxes); with mode 1 cells that wrap onto the same global cell
 * are summed in a fixed order, so the result is deterministic. */
int guard_merge(psatd_plan* plan, const void* const* box, void* const* g1, int nfields,
                const int origin[3], const int gdims[3], int mode, void* stream);

/* The whole step on G1 with the guard fill fused into the first FFT pass and
 * the interior merge fused into the last one: g1[0..10] are the eleven global
 * arrays (gdims cells each); E and B (slots 0..5) are overwritten with the
 * interior of the advanced box.  Jacobi order: every read of g1 by this call
 * happens before its first write, so the box may wrap onto itself (a single
 * group covering the whole periodic grid). */
int psatd_step_g1(psatd_plan* plan, void* const* g1, const int origin[3], const int gdims[3],
                  void* stream);

/* psatd_step_g1 without any allocation, for callers that cannot allocate
 * device memory while stepping (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, same result, same
 * kernels as psatd_step_g1; the two spectral workspaces live in a fixed
 * device array of the library (256 MiB per GPU, held until the process ends)
 * instead of the plan.  The box must fit it: 2 * 11 * (box_x/2+1) * box_y *
 * box_z complex values of the plan's precision (e.g. 160^3 in FP32, 128^3 in
 * FP64); larger boxes return PSATD_EINVAL.  The call itself does no hipMalloc,
 * hipFree, event or stream creation.  All calls on one GPU share the array:
 * calls that overlap on one GPU race, and a call on a stream other than the
 * previous call's while that call still runs returns PSATD_ESTATE.  Nothing a
 * call reads from the array was left there by an earlier call.  Plans made
 * with PSATD_FLAG_NO_WORKSPACE hold only their tables. */
int psatd_step_g1_noalloc(psatd_plan* plan, void* const* g1, const int origin[3], const int gdims[3],
                          void* stream);

/* Read-only plan properties (for bindings and benchmarks). */
enum {
  PSATD_Q_BOX_X = 0, PSATD_Q_BOX_Y = 1, PSATD_Q_BOX_Z = 2,
  PSATD_Q_PRECISION = 3,
  PSATD_Q_WORKSPACE_BYTES = 4,  /* device bytes owned by the plan */
  PSATD_Q_SPECTRUM_POINTS = 5,  /* (box_x/2+1) * box_y * box_z */
  PSATD_Q_Z_COLUMNS = 6,        /* (kx, ky) columns per tile of the k-space pass */
  PSATD_Q_TWO_STAGE = 7         /* bit i set: pass i+1 of the step runs a kernel compiled for its
                                   two-stage line schedule (x forward, y forward, k-space, y inverse,
                                   x inverse); the autotuner keeps the faster kernel per pass */
};
int psatd_plan_query(const psatd_plan* plan, int what, long long* value);

/* Copies the plan's PSATD coefficient tables to `dst` (device, plan precision):
 * 5 consecutive arrays C, S1, X1, X2, X3, each of PSATD_Q_SPECTRUM_POINTS
 * values, already multiplied by 1/(box_x*box_y*box_z), in the order
 * [kx][ky][kz] (kz fastest) with kx in [0, box_x/2] and ky, kz over all DFT
 * indices.  Followed by the three modified-wavenumber tables kx (box_x/2+1
 * values), ky (box_y), kz (box_z) (the staggered symbol k_s on staggered plans).  dst must hold
 * 5*PSATD_Q_SPECTRUM_POINTS + box_x/2+1 + box_y + box_z values. */
int psatd_plan_tables(const psatd_plan* plan, void* dst, void* stream);

/* Schedule autotuner.  For each axis, times the passes that transform along
 * it (x: first and last pass, y: second and fourth, z: the k-space pass) for
 * several radix factorisations / orders of the line length and several tile
 * sizes on the plan's own workspace, and keeps the fastest.  Results are cached
 * per (precision, axis, length, other box lengths): in memory for the process,
 * and in the JSON file `cache_path` if it is not NULL (read first, rewritten
 * after).  Synchronises `stream`.  Results of later steps are unchanged up to
 * rounding (the same transform, another factorisation). */
int psatd_plan_autotune(psatd_plan* plan, const char* cache_path, void* stream);

/* Current schedule of `axis` (0 x, 1 y, 2 z): writes the radix sequence into
 * radices[0 .. max_radices-1], the tile parameter into *tile (real y-lines
 * per x tile, lines per y tile, threads of the z pass) and returns the number
 * of radices (or a negative error). */
int psatd_plan_schedule(const psatd_plan* plan, int axis, int* radices, int max_radices, int* tile);

/* Per-pass timing for benchmarks.  While enabled, every step records HIP
 * events on its stream before and after each of its five passes (x forward
 * with guard fill, y forward, z forward + push + z inverse, y inverse, x
 * inverse with guard merge).  psatd_plan_pass_times waits for the last
 * recorded step, returns the mean duration of each pass in milliseconds over
 * the steps recorded since timing was enabled (or since the previous call),
 * their number in *nsteps, and releases the events. */
int psatd_plan_set_timing(psatd_plan* plan, int enable);
int psatd_plan_pass_times(psatd_plan* plan, double ms[5], long long* nsteps);

/* ---------------------------------------------------------------- batches
 * Many sub-domains of one global grid G1, each a box with its own size, guard
 * width and stencil order (the local decomposition of Fig. 1(a) / Sec. 1.3,
 * possibly with guards wider than a neighbour, which then come from further
 * sub-domains).  One step advances every box: all guard fills read the fields
 * of the previous step before any interior is written back (Jacobi order,
 * Sec. 2.5.2).  Per pass, the boxes are grouped into classes of equal block
 * size and similar LDS size, and each class is one persistent launch over the
 * tiles of its boxes.
 *
 * subs[b] describes box b (interior sizes, guards, order); dx, dy, dz, dt, c,
 * eps0 and precision must agree across boxes.  origins[3*b .. 3*b+2] is the
 * global index of box b's first interior cell; gdims = {GX, GY, GZ}.  Every
 * box interior must fit in G1, and no two interiors may share a G1 cell
 * (periodic wrap included): PSATD_EINVAL otherwise, checked on the host before
 * anything is allocated.  G1 cells outside every interior keep their values.
 * The batch owns a plan per box (tables and workspace). */
typedef struct psatd_batch psatd_batch;
int psatd_batch_create(int nsub, const psatd_plan_desc* subs, const int* origins, const int gdims[3],
                       psatd_batch** out);

/* One step of every box on the eleven G1 arrays g1[0..10] (E, B updated in
 * place), launched eagerly on `stream`. */
int psatd_batch_step(psatd_batch* batch, void* const* g1, void* stream);

/* `nsteps` steps, replayed from a hipGraph that holds nsteps x 5 batched
 * launches.  The graph is captured on the first call (and again whenever
 * nsteps or the g1 pointers change), then launched on `stream`.  Results are
 * identical to nsteps calls of psatd_batch_step.  The sources (J, rho) are
 * held fixed over the steps. */
int psatd_batch_run(psatd_batch* batch, void* const* g1, int nsteps, void* stream);

/* Releases a batch (NULL-safe; synchronise its streams first). */
void psatd_batch_destroy(psatd_batch* batch);

/* Autotunes every box plan of the batch (see psatd_plan_autotune); the next
 * step rebuilds the batch's descriptors and graph. */
int psatd_batch_autotune(psatd_batch* batch, const char* cache_path, void* stream);

/* Batch properties: PSATD_QB_BOXES, PSATD_QB_TILES (tiles of the five passes
 * summed), PSATD_QB_BOX_CELLS, PSATD_QB_INTERIOR_CELLS, PSATD_QB_WORKSPACE_BYTES. */
enum {
  PSATD_QB_BOXES = 0, PSATD_QB_TILES = 1, PSATD_QB_BOX_CELLS = 2, PSATD_QB_INTERIOR_CELLS = 3,
  PSATD_QB_WORKSPACE_BYTES = 4
};
int psatd_batch_query(const psatd_batch* batch, int what, long long* value);

/* ---------------------------------------------------------------- guard-width surrogate
 * A 6 -> 64 -> 64 -> 1 network that predicts log10 of the truncation error of
 * a local-with-guards run against the global solve, so that the smallest safe
 * guard width can be chosen (the paper calls such a model of n_g versus order,
 * time step and cell size crucial, Sec. 1.4, and ties n_g to memory and cost,
 * Sec. 2.2).  Inputs per sample (six floats, in this order): 2/p (0 for
 * infinite order), log2 n_g, c dt/dx, laser wavelength / dx, spectral width
 * 1/(k0 L), log2 steps.  The network standardises them,
 * x = (features - in_mean) * in_scale, computes
 * h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2), u = W3 h2 + b3
 * (silu(z) = z / (1 + exp(-z))) and predicts out_mean + out_scale * u.
 *
 * Parameters: PSATD_MLP_NPARAM floats, W1 (64 x 6, row-major out x in), b1
 * (64), W2 (64 x 64), b2 (64), W3 (64), b3 (1).  The object keeps an FP32
 * master copy, which Adam updates, and a bfloat16 copy (round to nearest,
 * ties to even) that prediction and gradients use; activations and sums are
 * FP32.  Training minimises the mean over the batch of
 * (u - (target - out_mean) / out_scale)^2.
 *
 * All X, target, index, gradient and loss pointers are DEVICE pointers;
 * X is n x 6 row-major float, targets n floats, idx int32.  Calls are
 * asynchronous on `stream`, except create/set/get, which synchronise the
 * device.  One object must not be used on two streams at once. */
#define PSATD_MLP_NPARAM 4673
typedef struct psatd_mlp psatd_mlp;

/* Creates a network from `init` (host, PSATD_MLP_NPARAM floats), the
 * standardisation constants (host, 6 floats each) and the output affine map;
 * `max_batch` bounds the batch of psatd_mlp_grad / psatd_mlp_train.  Adam's
 * moments start at zero. */
int psatd_mlp_create(const float* init, const float* in_mean, const float* in_scale, float out_mean,
                     float out_scale, int max_batch, psatd_mlp** out);

/* Replaces the master weights (host array), re-rounds the bfloat16 copy and
 * resets Adam (moments and step count). */
int psatd_mlp_set(psatd_mlp* mlp, const float* master);

/* Copies the master weights and/or the bfloat16 copy (as raw 16-bit
 * patterns) to host arrays; either may be NULL. */
int psatd_mlp_get(const psatd_mlp* mlp, float* master, unsigned short* bf16);

/* y[i] = prediction for X[i], i < n (n = 0 is a no-op). */
int psatd_mlp_predict(const psatd_mlp* mlp, const float* X, int n, float* y, void* stream);

/* Gradient of the batch loss with respect to the (bfloat16) weights.  The
 * batch is samples idx[0 .. batch-1] of X / target (idx NULL: samples
 * 0 .. batch-1, which requires batch <= n); an index outside [0, n)
 * contributes nothing.  The gradient (PSATD_MLP_NPARAM floats) and the loss
 * (1 float) are kept in the object and also copied to `grad` / `loss` when
 * these are not NULL.  The sums run in a fixed order, so results are
 * reproducible. */
int psatd_mlp_grad(psatd_mlp* mlp, const float* X, const float* target, int n, const int* idx, int batch,
                   float* grad, float* loss, void* stream);

/* One Adam step (Kingma & Ba, 2015, with bias correction) from the gradient
 * of the last psatd_mlp_grad, on the master weights; the bfloat16 copy is
 * refreshed. */
int psatd_mlp_adam(psatd_mlp* mlp, float lr, float beta1, float beta2, float eps, void* stream);

/* `nsteps` steps of minibatch training: step k takes the batch
 * idx[k*batch .. k*batch + batch - 1] (idx NULL: the first `batch` samples
 * every step), computes the gradient and applies Adam.  The batch loss of
 * every step (before its update) goes to loss_hist[k] when not NULL. */
int psatd_mlp_train(psatd_mlp* mlp, const float* X, const float* target, int n, const int* idx, int nsteps,
                    int batch, float lr, float beta1, float beta2, float eps, float* loss_hist, void* stream);

/* Releases the network (NULL-safe; synchronise its stream first). */
void psatd_mlp_destroy(psatd_mlp* mlp);

/* Default line-transform schedule of this build for a box edge of n cells
 * (host only, no GPU needed): the radices of the Stockham stages, in order,
 * written to radices[0 .. max_radices-1], and in *transform_len the length
 * they transform: n itself when every prime factor of n has a compiled radix
 * (at most 17), otherwise the padded length m >= 2n - 1 of Bluestein's
 * chirp-z form.  The factorisation is the cheapest under the build's per-stage
 * cost model; plans start from it and the autotuner may reorder or replace it.
 * Returns the number of stages, or PSATD_EINVAL / PSATD_EUNSUPPORTED. */
int psatd_default_schedule(int n, int* radices, int max_radices, int* transform_len);

/* ---------------------------------------------------------------- resources
 * Device memory held by the library (plans, batches; not the surrogate
 * network) is counted.  psatd_set_device_budget(bytes) caps it: an allocation
 * that would pass the cap fails exactly like a failed hipMalloc, i.e. the
 * constructor returns PSATD_ENOMEM and releases everything it had allocated.
 * bytes < 0 removes the cap (the default).  Meant for callers that share the
 * device with other work, and for testing the out-of-memory paths.  The cap is
 * process-wide; it does not touch existing allocations. */
int psatd_set_device_budget(long long bytes);
/* Device bytes currently held by the library's plans and batches. */
long long psatd_device_bytes_in_use(void);

/* Reads an autotuner cache file (the format psatd_plan_autotune writes) into
 * the process cache without a GPU.  An entry is accepted only if the file's
 * schema version is the library's own and its radices are compiled and multiply to
 * the transform length named in its key; tiles are checked again against the
 * plan's limits when an entry is used.  Reading stops at malformed text.
 * *accepted / *rejected (either may be NULL) receive the counts.  A missing
 * file is not an error (both counts 0). */
int psatd_tune_cache_load(const char* path, int* accepted, int* rejected);

/* ---------------------------------------------------------------- absorbing layers
 * Two-step perfectly matched layers (the absorbing boundaries the paper's
 * solver uses, Sec. 2.6: the two-step PML of Shapoval, Vay and Vincenti, 2019).
 * The plan's box (interior + guards, box arrays as for psatd_push) becomes a
 * domain with absorbing layers at its ends instead of a periodic one.  Every
 * field component is split into two parts by the direction of the derivative
 * that drives it, twelve box arrays in this order:
 *   set A: E_xy, E_yz, E_zx, B_xy, B_yz, B_zx   (component a, axis a+1)
 *   set B: E_xz, E_yx, E_zy, B_xz, B_yx, B_zy   (component a, axis a+2)
 * The full field is the sum of its two parts (E_x = E_xy + E_xz, ...).
 * One step: (1) every part gains, without absorption, the integral over the
 * step of its own right-hand side along the exact (PSATD) evolution of the
 * full fields with the sources held constant, set A also taking the part of
 * the increment not driven by a derivative, so that the two parts always add
 * up to psatd_push's step; (2) each part is multiplied by exp(-sigma dt) of
 * its axis, sigma = sigma_max (depth / width)^power in a layer of `width`
 * cells at both ends of the axis (depth = width at the outer cell, 1 at the
 * innermost) and 0 inside.  Collocated plans only. */

/* Sets (or changes) the layers: width[3] cells per axis (0 = no layer; at
 * most half the box edge), sigma_max >= 0, power >= 0.  The first call
 * allocates the damping tables and twelve box arrays of scratch.
 * Synchronises the device. */
int psatd_pml_set(psatd_plan* plan, const int width[3], double sigma_max, double power);

/* One PML step: parts[0..11] the split fields (read and overwritten),
 * src[0..4] = Jx Jy Jz rho_old rho_new (read only), all box arrays of the plan
 * precision and distinct.  PSATD_ESTATE before psatd_pml_set. */
int psatd_pml_step(psatd_plan* plan, void* const* parts, const void* const* src, void* stream);

/* ---------------------------------------------------------------- particles
 * The particle side of the PIC cycle around the step (Sec. 2.5.1, Fig. 4:
 * push the particles with the fields at their positions, deposit their current
 * and charge with linear or higher-order interpolation, solve Maxwell's
 * equations, gather the new fields back at the same order).  Particle-mesh work runs on the global grid G1 cut into
 * sub-domains D1 whose guard cells are as wide as the stencil (Sec. 2.5.2):
 * here a D1 sub-domain is a tile of tile^3 cells handled by one workgroup,
 * whose guard contributions are added into the neighbouring tiles' cells.
 *
 * Grid quantities are the eleven G1 arrays of psatd_step_g1 (gdims cells, x
 * fastest, slot order Ex Ey Ez Bx By Bz Jx Jy Jz rho_old rho_new), with the
 * precision of the object.  A quantity with half-cell offsets o (all zero on
 * the collocated grid; PSATD_FLAG_STAGGERED: the Yee offsets of the plan flag,
 * J like E, rho on the nodes) has its array index i at (i + o/2) d; the grid is
 * periodic with lengths L = (gx dx, gy dy, gz dz).  A particle at x takes part
 * in the (k+1)^3 points around s = (x - o d/2) / d with the product of the 1D
 * centred B-spline weights of degree k = shape (Sec. 2.5.1):
 *   k = 1 (cloud in cell): points floor(s) + {0, 1}, weights 1 - t, t (t = s - floor(s));
 *   k = 2 (triangular-shaped cloud): points round(s) + {-1, 0, 1}, t = s - round(s),
 *         weights (1/2 - t)^2 / 2, 3/4 - t^2, (1/2 + t)^2 / 2;
 *   k = 3 (cubic): points floor(s) + {-1, 0, 1, 2}, t = s - floor(s), weights
 *         (1 - t)^3 / 6, (4 - 6t^2 + 3t^3) / 6, (1 + 3t + 3t^2 - 3t^3) / 6, t^3 / 6.
 * Gather and deposit use the same shape.  Particles are structure-of-arrays: x[0..2] the
 * positions (x, y, z), u[0..2] the momentum per mass u = gamma v, n values each
 * (device arrays of the object's precision).  Positions lie in [0, L). */
typedef struct {
  int gx, gy, gz;    /* G1 cells */
  double dx, dy, dz; /* cell sizes (> 0) */
  double dt, c;      /* time step and speed of light (> 0); c dt <= 0.999 min(dx, dy, dz) */
  double q;          /* macro-particle charge */
  double q_over_m;   /* charge per mass of the species */
  int max_particles; /* bound on n of every call (>= 0) */
  int tile;          /* D1 tile edge in cells, 1..12; 8 is a good default */
  int precision;     /* PSATD_FP32 or PSATD_FP64 */
  int flags;         /* 0 or PSATD_FLAG_STAGGERED */
  int shape;         /* degree of the particle shape: 1, 2 or 3 (0 means 1) */
} psatd_pic_desc;
typedef struct psatd_pic psatd_pic;

/* Checks the descriptor and allocates the per-tile lists (12 bytes per tile
 * + 4 bytes per particle); for shapes 2 and 3 on grids that the tiles divide
 * with at least two tiles per axis, also one block of 5 (tile + 5)^3 values
 * per tile (52 bytes per cell in FP32 at tile 8; without that memory the
 * deposit falls back to atomics).  A tile accumulates over itself and guard cells per
 * axis, one below and two above for shape 1, two below and three above for
 * shapes 2 and 3: the reach of the stencil of a particle that started in the
 * tile and moved less than a cell (tile 8: 11^3 or 13^3 cells, 53 or 88 KB of
 * LDS).  PSATD_EUNSUPPORTED if
 * c dt exceeds 0.999 of the smallest cell size (a particle could then leave
 * those guard cells within one step; the margin absorbs the rounding of
 * positions) or the tile's LDS block does not fit the device. */
int psatd_pic_create(const psatd_pic_desc* desc, psatd_pic** out);
void psatd_pic_destroy(psatd_pic* pic);

/* Gather and push of n particles: E and B (g1[0..5]) interpolated at x, then the
 * relativistic Boris step of u (half electric kick, rotation about B at the
 * mid-step gamma, half kick), then x += dt u / gamma, wrapped into [0, L).
 * x_old[0..2] receive the positions before the move (for the deposit).  g1
 * holds the eleven slot pointers; only 0..5 are read.  n = 0 is a no-op
 * (the particle pointers may then be NULL). */
int psatd_pic_push(psatd_pic* pic, void* const* g1, void* const* x, void* const* u, void* const* x_old, int n,
                   void* stream);

/* Deposit of n particles that moved from x_old to x with the half-step u:
 * g1[6..8] = J = sum q v S(mid-point) / (dx dy dz), v = u / gamma, mid-point
 * x_old + v dt / 2; g1[9] = rho_old at x_old, g1[10] = rho_new at x, both
 * sum q S / (dx dy dz).  Slots 6..10 are overwritten (zeroed first, also for
 * n = 0, when the particle pointers may be NULL); 0..5 are not touched.  The
 * particles are listed per D1 tile of their start position, each tile
 * accumulates in LDS over itself and its guard cells in 64-bit fixed point (a
 * power-of-two scale per tile: exact integer sums of the rounded
 * contributions), and the block is added into G1 with floating-point atomics,
 * whose order between neighbouring tiles varies from run to run; with the
 * per-tile blocks of shapes 2 and 3 (see psatd_pic_create) the blocks are
 * stored and each G1 cell sums the blocks that cover it in a fixed order.
 * A tile's particle list is built with atomics, so the rounding of the
 * per-thread sums may still vary in the last bits. */
int psatd_pic_deposit(psatd_pic* pic, void* const* g1, const void* const* x_old, const void* const* x,
                      const void* const* u, int n, void* stream);

/* Message for the last non-OK return on the calling thread ("" if none). */
const char* psatd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSATD_H */
