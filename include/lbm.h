/*
 * lbm.h -- C ABI of the MI355X (gfx950) D3Q27 colour-fluid lattice Boltzmann library.
 *
 * The library advances the two-fluid lattice Boltzmann model of Saito, Abe & Koyama,
 * "Lattice Boltzmann modeling and simulation of liquid jet breakup", Phys. Rev. E 96,
 * 013317 (2017), on one GPU.  One call of lbm_step performs, per cell and per step, the
 * operator split of Sec. II: colour-gradient stencil, MRT collision with the enhanced
 * equilibrium Eq. (EES) and the forcing term Eq. (ketF), the generalised perturbation
 * Eq. (perturb), the recolouring operator, and streaming Eq. (LBE) with the boundary rules
 * of Secs. III C and IV A.
 *
 * Conventions shared by every call:
 *  - Lattice index: cell = (z * ny + y) * nx + x, x fastest.  Fields passed in or out are
 *    arrays of ncells doubles in that order; vector fields are 3 consecutive such arrays.
 *  - Velocity index 0..26 is the paper's i = 1..27 (the order of Appendix A).
 *  - Host pointers are owned by the caller; the library copies from or into them and keeps
 *    no reference after the call returns.  Device memory is owned by the library.
 *  - No call throws.  Each returns an lbm_status; lbm_last_error() gives a message.
 *  - Work is enqueued on the stream given to lbm_create (NULL = the default stream);
 *    lbm_step returns without waiting.  Read-back calls synchronise that stream.
 *  - A context must not be used from two host threads at once.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = 1,    /* invalid argument or parameter combination */
  LBM_ENOMEM = 2,    /* device or host allocation failed */
  LBM_EDEVICE = 3,   /* a HIP call failed (no GPU, launch failure, fault) */
  LBM_EUNSTABLE = 4, /* the state holds a NaN or a non-positive density */
  LBM_ESTATE = 5     /* call out of order (e.g. lbm_step before lbm_init_fields) */
} lbm_status;

/* Storage of the populations in HBM.  Arithmetic is FP32 in every case; the FP16/BF16
 * forms store the deviation of each population from the local rest equilibrium. */
typedef enum { LBM_F32 = 0, LBM_F16 = 1, LBM_BF16 = 2 } lbm_storage;

/* Face rules (Secs. III C, IV A).  The two x faces must be both periodic or both free-slip
 * (the lateral walls of the jet, Sec. IV A), and likewise the two y faces; each z face takes
 * any rule (outflow on +z only), periodic only in pairs. */
typedef enum {
  LBM_PERIODIC = 0,   /* wrap-around streaming and stencil */
  LBM_BOUNCEBACK = 1, /* no-slip wall, half-way bounce-back, half a cell outside the plane */
  LBM_FREESLIP = 2,   /* specular reflection (Succi 2001), half a cell outside the plane */
  LBM_OUTFLOW = 3     /* convective outflow (Lou et al. 2013); +z face only */
} lbm_face;

typedef struct {
  int nx, ny, nz;        /* lattice size, each >= 1; nz >= 3 when a z face is not periodic;
                            nx*ny*108 < 2^31 (at most 19 884 107 cells per x-y plane) */
  double rho_r0, rho_b0; /* reference densities of the red and blue fluids; their ratio
                            gamma = rho_r0/rho_b0 sets alpha_r = 1 - (1 - 8/27)/gamma (Sec. II),
                            which must lie in [0, 1) */
  double nu_r, nu_b;     /* kinematic viscosities (> 0); the local value is interpolated
                            linearly in phi and sets s_nu = 1/(3 nu + 1/2), Eq. (shear) */
  double A;              /* surface-tension parameter of Eq. (perturb), >= 0 */
  double beta;           /* recolouring parameter, in [0, 1] */
  double s[27];          /* relaxation rate of each moment row of Eq. (momentSet); all zero
                            selects the set of Sec. II (s1 = 0, s5 = 1.5, s11 = 1.5, s14 = 1.83,
                            s17 = 1.4, s18 = 1.61, s19 = s21 = 1.98, s24 = s27 = 1.74).  Rows
                            6-10 always take the local s_nu; rows 1-4 must be 0 */
  int face[6];           /* lbm_face for -x, +x, -y, +y, -z, +z */
  int force;             /* 0: no body force; 1: F = (rho - rho_ref) g */
  double g[3];
  double rho_ref;
  int storage;           /* an lbm_storage value; others are rejected with LBM_EINVAL */
} lbm_params;

/* Interfacial tension of the perturbation operator, Eq. (sigma): sigma = (4/9) A tau in
 * lattice units, tau = 3 nu + 1/2 the relaxation time of the fluid whose viscosity nu is
 * given (at a jet's interface, the continuous phase's).  lbm_A_from_sigma inverts it.  Pure
 * host arithmetic; NaN for nu <= 0 or a negative A / sigma. */
double lbm_sigma_from_A(double A, double nu);
double lbm_A_from_sigma(double sigma, double nu);

/* Create a context: validates the parameters, allocates the device state (two copies of
 * 27 populations plus 5 per-cell scalars per cell) and uploads the constants.  No kernel
 * runs.  hip_stream is a hipStream_t or NULL.  On success *out owns the device memory. */
lbm_status lbm_create(const lbm_params *params, void *hip_stream, lbm_ctx **out);

/* Set the initial state (reading R1: each colour at its equilibrium Eq. (EES) with
 * Phi = 0 at the given densities and velocity).  rho_r, rho_b: ncells doubles each, >= 0
 * with rho_r + rho_b > 0; u: 3*ncells doubles (ux, uy, uz arrays) or NULL for rest.  Resets
 * the step counter to 0. */
lbm_status lbm_init_fields(lbm_ctx *ctx, const double *rho_r, const double *rho_b, const double *u);

/* Inflow disk on the -z face (Sec. IV A): sites on the plane z = 0 with
 * (x - xc)^2 + (y - yc)^2 < (diameter/2)^2 are not collided; at every step they emit the
 * red equilibrium at rho_r0 and velocity u_normal (1 + noise_rel xi) e_z with Phi = 0, and
 * no blue.  xi in [-1, 1) is drawn per site and step from SplitMix64 at counter
 * step * ncells + cell, offset by seed.  Call before lbm_init_fields. */
lbm_status lbm_set_inflow(lbm_ctx *ctx, double xc, double yc, double diameter, double u_normal, double noise_rel,
                          unsigned long long seed);

/* Tile shape of the step kernel: (tx, ty) in {(32, 4), (32, 8), (32, 16), (64, 4), (64, 8)}
 * cells per workgroup, zchunk >= 1 z planes per workgroup, or 0 to let the library choose
 * it from the number of workgroups the device holds at once.  Default: (64, 4, 0) for
 * nx >= 64, (32, 8, 0) otherwise.  With free-slip x or y faces a step is several launches:
 * the interior tiles (no cell or ring cell on a wall), the tiles along the x walls and along
 * the y walls (with FP16 storage: along each of the -x, +x, -y and +y walls), and the
 * corners; with zchunk = 0 each gets its own z chunk.
 * Results do not depend on the tiling; this is a tuning hook.  LBM_EINVAL for other shapes
 * or zchunk < 0. */
lbm_status lbm_set_tiling(lbm_ctx *ctx, int tx, int ty, int zchunk);

/* Time each supported tile shape (32x8, 64x4, 32x4) for trial_steps steps on a scratch
 * lattice with this context's parameters (blue fluid at rest; it needs the device memory of
 * a second lattice of this size while it runs) and keep the fastest for lbm_step.  The
 * context's state is not touched and results do not depend on the choice.  LBM_EINVAL for
 * trial_steps < 1; allocation or device errors as lbm_create / lbm_step. */
lbm_status lbm_autotune(lbm_ctx *ctx, int trial_steps);

/* The tile shape lbm_step uses: (tx, ty) and the z chunk.  A value not yet chosen (by
 * lbm_set_tiling, lbm_autotune or the first lbm_step) reads 0.  LBM_EINVAL for a NULL
 * argument. */
lbm_status lbm_get_tiling(const lbm_ctx *ctx, int *tx, int *ty, int *zchunk);

/* Enqueue nsteps time steps (nsteps >= 0) on the context's stream; returns at once. */
lbm_status lbm_step(lbm_ctx *ctx, int nsteps);

/* Wait for queued work.  LBM_EDEVICE if a kernel failed; LBM_EUNSTABLE if, since the state
 * was set, the step kernel met a cell whose pulled density was NaN, infinite or <= 0 (the
 * check runs on every cell at every step; the flag is cleared by lbm_init_fields and
 * restored by lbm_load_state). */
lbm_status lbm_sync(lbm_ctx *ctx);

/* Number of steps taken since lbm_init_fields. */
long long lbm_step_count(const lbm_ctx *ctx);

/* Macroscopic fields of the current time (post-streaming, pre-collision):
 * LBM_FIELD_RHO_R, _RHO_B: colour densities; _UX.._UZ: u = (sum_i f_i c_i + F/2)/rho
 * (Eq. (Momentum)); _PHI: Eq. (order); _P: sum_k rho_k 9 (1 - alpha_k)/19 (Eq. (press)).
 * Inflow sites report rho_r0, 0 and their set velocity.  dst: ncells doubles (host). */
enum { LBM_FIELD_RHO_R = 0, LBM_FIELD_RHO_B = 1, LBM_FIELD_UX = 2, LBM_FIELD_UY = 3, LBM_FIELD_UZ = 4,
       LBM_FIELD_PHI = 5, LBM_FIELD_P = 6 };
lbm_status lbm_read_field(lbm_ctx *ctx, int field, double *dst);

/* Same for the box [x0, x0+wx) x [y0, y0+wy) x [z0, z0+wz); dst: wx*wy*wz doubles.
 * The read-back calls fill dst and then return LBM_EUNSTABLE if the step kernel has flagged
 * the state (see lbm_sync). */
lbm_status lbm_read_field_box(lbm_ctx *ctx, int field, int x0, int y0, int z0, int wx, int wy, int wz, double *dst);

/* The same read-back for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): lbm_read_field_box without any
 * hipMalloc or hipFree.  The FP64 staging of the fields kernel is a fixed 8 MiB array per
 * device (2^20 doubles, held until the process ends; its address is taken in lbm_create)
 * instead of a buffer the context allocates on demand.  The box is read in z slices of at
 * most 2^20 / 7 cells; a box with wx*wy > 149796 is rejected with LBM_EINVAL.  All contexts
 * on one device share the array: calls that overlap on one device race.  Other arguments,
 * results and errors as lbm_read_field_box. */
lbm_status lbm_read_field_box_noalloc(lbm_ctx *ctx, int field, int x0, int y0, int z0, int wx, int wy, int wz,
                                      double *dst);

/* Coarse-grained state of the current time for the learned surrogate: over every block of
 * factor^3 cells, the means of phi and of u / u_scale (FP32), written to DEVICE memory dst as
 * [cz][cy][cx][4] inside a padded box of pd x ph x pw voxels (entries outside the coarse
 * lattice are not written; dst 16-byte aligned).  Enqueued on the context's stream (no
 * synchronisation).  LBM_EINVAL unless factor divides nx, ny and nz, the coarse lattice fits
 * the box and u_scale > 0. */
lbm_status lbm_coarse_state(lbm_ctx *ctx, int factor, double u_scale, float *dst, int pd, int ph, int pw);

/* Pre-collision populations of the current time, per colour: dst holds 2*27*ncells
 * doubles ordered [colour (0 red, 1 blue)][velocity][cell]. */
lbm_status lbm_read_populations(lbm_ctx *ctx, double *dst);

/* Checkpoint: the opaque device state (populations, scalars, outlet plane, step counter,
 * instability flag).  lbm_state_bytes gives the size; lbm_save_state copies it into host
 * memory dst (bytes >= lbm_state_bytes); lbm_load_state restores it into a context created
 * with the same parameters.  The first 64 bytes are a header: "LBMD3Q27", the step (int64),
 * nx, ny, nz, storage, the six face rules and the flag (int32 each); lbm_load_state returns
 * LBM_EINVAL, leaving the context unchanged, for a buffer that is too small, is not a saved
 * state, or comes from a lattice of another size, storage or face set. */
size_t lbm_state_bytes(const lbm_ctx *ctx);
lbm_status lbm_save_state(lbm_ctx *ctx, void *dst, size_t bytes);
lbm_status lbm_load_state(lbm_ctx *ctx, const void *src, size_t bytes);

/* Global diagnostics with FP64 accumulation on the GPU (deterministic order):
 * mass_r, mass_b: sum of the colour densities; umax: max |u|; p_in, p_out: mean pressure
 * over cells within r_in of (xc, yc, zc) and beyond r_out from it (the static-droplet
 * pressure jump of Sec. III A); nan_cells: cells with a NaN or rho <= 0.  Returns
 * LBM_EUNSTABLE (out filled) if nan_cells > 0 or the step kernel has flagged the state. */
typedef struct {
  double mass_r, mass_b, umax, p_in, p_out;
  long long n_in, n_out, nan_cells, step;
} lbm_diag;
lbm_status lbm_diagnostics(lbm_ctx *ctx, double xc, double yc, double zc, double r_in, double r_out, lbm_diag *out);

/* Average duration in milliseconds of one step's kernels over the last lbm_step call,
 * measured with HIP events on the context's stream around the whole call (0 if none): the
 * step kernel's launches and, where the lattice has them, the small outlet and inflow
 * kernels. */
double lbm_last_step_kernel_ms(const lbm_ctx *ctx);

/* Human-readable text of the last error on ctx (or of the last failed lbm_create when ctx
 * is NULL).  The pointer stays valid until the next call on ctx. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Free the device memory and the context.  NULL is ignored. */
void lbm_destroy(lbm_ctx *ctx);

/* ---------------------------------------------------------------- batches
 * Several independent lattices (e.g. the jet cases of a regime map, Sec. IV C) advanced
 * together: each step is one launch of the step kernel over all cases that share a storage
 * type and tile shape, instead of one launch per case.
 *
 * lbm_batch_create: params points to ncases parameter blocks (validated as lbm_create); the
 *   cases share hip_stream.  On success *out owns every case's device memory.
 * lbm_batch_case: the context of case k (0 <= k < ncases), owned by the batch.  Use it with
 *   lbm_set_inflow, lbm_init_fields, lbm_set_tiling, lbm_read_*, lbm_diagnostics and the
 *   checkpoint calls; lbm_step on it returns LBM_ESTATE.  NULL for a bad index.
 * lbm_batch_step: nsteps steps of every case (all cases must be initialised and at the same
 *   step, else LBM_ESTATE).  Waits for work queued by the previous call before enqueuing.
 *   A case the step kernel flags as unstable (see lbm_sync) is not stepped further: within
 *   the call its workgroups return at once, and later calls leave it out (its step count
 *   stops).  The batch does not fail for it; LBM_EUNSTABLE only when every case is flagged.
 * lbm_batch_unstable_cases: waits for the batch's stream, then writes 1 (unstable) or 0 per
 *   case into flags (ncases ints, or NULL) and returns the number of unstable cases; -1 on a
 *   device error.
 * lbm_batch_autotune: chooses each case's tile shape by timing every supported shape on a
 *   scratch lattice of the same size and physics for trial_steps steps; the cases' states
 *   are not touched.  Results do not depend on the tile shape.
 * lbm_batch_last_step_ms: mean wall time per step of the last lbm_batch_step call (HIP
 *   events on the stream).
 * Errors of batch calls: lbm_batch_last_error(batch). */
typedef struct lbm_batch lbm_batch;
lbm_status lbm_batch_create(const lbm_params *params, int ncases, void *hip_stream, lbm_batch **out);
lbm_ctx *lbm_batch_case(lbm_batch *batch, int k);
int lbm_batch_size(const lbm_batch *batch);
lbm_status lbm_batch_autotune(lbm_batch *batch, int trial_steps);
lbm_status lbm_batch_step(lbm_batch *batch, int nsteps);
lbm_status lbm_batch_sync(lbm_batch *batch);
int lbm_batch_unstable_cases(lbm_batch *batch, int *flags);
double lbm_batch_last_step_ms(const lbm_batch *batch);
const char *lbm_batch_last_error(const lbm_batch *batch);
void lbm_batch_destroy(lbm_batch *batch);

/* Diagnostic, not used by lbm_step: the step's per-cell collision arithmetic compiled for
 * the host, for checks without a GPU.  fr, fb: the cell's 27 pre-collision populations per
 * colour; grad_phi, grad_rho: 3 each; out_r, out_b: the 27 post-collision (recoloured)
 * populations per colour.  Uses the parameters of params (body force from the cell's rho). */
lbm_status lbm_selftest_collide_host(const lbm_params *params, const double *fr, const double *fb,
                                     const double *grad_phi, const double *grad_rho, double *out_r, double *out_b);

/* Diagnostic, not used by lbm_step: how a step with tile shape tx x ty (32x4, 32x8, 64x4,
 * 64x8 or 32x16) distributes the tiles of a lattice with these parameters over its launches.
 * counts (caller-owned, 3 * tiles_x * tiles_y ints, tiles_x = ceil(nx/tx), tiles_y =
 * ceil(ny/ty), tile (i, j) at j * tiles_x + i) receives for each tile how many times the launch
 * over all tiles (block 0), over the interior tiles (block 1) and over the frame tiles (block 2)
 * would process it.  Without lateral walls one launch covers all tiles; with free-slip x or y
 * faces the interior tiles (none of whose cells or ring cells lies on a wall) take the plain
 * pull, and the frame is up to three launches (x edges, y edges, corners), five with FP16
 * storage (one per wall along the edges, one for the corners), with the instances that
 * reflect at those walls.  LBM_EDEVICE if a tile falls
 * outside the lattice or touches a wall its launch does not reflect at (an internal error);
 * LBM_EINVAL for invalid parameters or shapes. */
lbm_status lbm_selftest_tile_sets_host(const lbm_params *params, int tx, int ty, int *counts);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H_ */
