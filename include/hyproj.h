/*
 * hyproj: hybrid CNN + Jacobi pressure projection on a 2D MAC grid, for
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The operation (arXiv 2109.09363, Sec. 2.2 and Sec. 3.3): given the
 * intermediate velocity u* on a MAC grid with obstacle flags, solve the
 * pressure Poisson equation (Eq. 3) and subtract the pressure gradient
 * (Eq. 2) so that the mean |div u| over fluid cells falls below a user
 * threshold (the hybrid criterion E_1 of Sec. 4.1).  The pressure is first
 * predicted by a multi-scale CNN (Sec. 3.1) and then refined by Jacobi
 * iterations (Sec. 2.2); plain Jacobi and Jacobi-preconditioned CG are the
 * baselines.
 *
 * Grid conventions (all arrays row-major, x fastest, no padding):
 *   cells      (ny, nx)      index j*nx + i, j = 0 is the bottom row
 *   u faces    (ny, nx+1)    u[j*(nx+1) + i] is the x-face left of cell (i,j)
 *   v faces    (ny+1, nx)    v[j*nx + i] is the y-face below cell (i,j)
 *   flags      (ny, nx) u8   bit0 = solid obstacle cell,
 *                            bit1 = the face below this row-0 cell is an inflow
 *                                   face with a prescribed velocity
 * The left, right and bottom domain edges are walls; the top edge is open
 * (a ghost row of cells with pressure 0 above row ny-1).  Enclosed fluid
 * pockets (no 4-connected path to the open top) are treated as solid.
 *
 * Ownership: the caller owns every device buffer, including the workspace
 * (size from hyp_workspace_size).  The library allocates no device memory
 * in any call; its only device memory of its own is the static array of
 * hyp_project_noalloc (HYP_NOALLOC_MAX_BYTES per GPU, held from the code
 * object's load until the process ends).  A context holds host state only.  Calls are asynchronous on
 * the given HIP stream; one context/workspace pair must not be used by two
 * streams at once.
 *
 * Errors: a negative return value means the call was rejected before
 * anything was enqueued (HYP_E*).  Conditions found on the device are
 * reported in hyp_result.status (HYP_STATUS_*).
 */
#ifndef HYPROJ_H
#define HYPROJ_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYP_VERSION 10000

/* return codes */
#define HYP_OK             0
#define HYP_EINVAL        -1  /* null pointer, bad size or option */
#define HYP_EUNSUPPORTED  -2  /* e.g. grid side not divisible by 2^(scales-1) */
#define HYP_EWORKSPACE    -3  /* workspace too small */
#define HYP_EHIP          -4  /* a HIP launch or API call failed */
#define HYP_EINTERNAL     -5  /* unexpected host-side failure */
#define HYP_ENOWEIGHTS    -6  /* CNN method requested without a network */

/* device-side statuses (hyp_result.status) */
#define HYP_STATUS_OK         0  /* threshold reached (or fixed_iters done) */
#define HYP_STATUS_MAXITER    1  /* max_iters reached; last iterate returned */
#define HYP_STATUS_NONFINITE  2  /* NaN/Inf in the residual; iterate returned */
#define HYP_STATUS_FLOOR      3  /* PCG: the true residual stayed above the
                                    threshold after 3 defect-correction folds
                                    (the threshold lies below what FP32
                                    reaches); the last iterate is returned */
#define HYP_STATUS_ABORTED    4  /* a persistent solver stopped waiting for
                                    data from another work-group (a 2 s limit
                                    per wait; an internal error): the outputs
                                    are not valid */

/* methods */
#define HYP_METHOD_HYBRID  0  /* CNN initial guess, then Jacobi (Sec. 3.3) */
#define HYP_METHOD_JACOBI  1  /* Jacobi from p_init or zero (Sec. 2.2) */
#define HYP_METHOD_PCG     2  /* Jacobi-preconditioned CG from p_init or zero */
#define HYP_METHOD_CNN     3  /* CNN prediction only, no iterations */

/* CNN precision */
#define HYP_PREC_FP32  0  /* FP32 activations/weights, FP32 MFMA */
#define HYP_PREC_BF16  1  /* BF16 3x3 layers on MFMA with FP32 accumulation;
                             1x1 output, pressure and solvers in FP32 */

typedef struct hyp_ctx hyp_ctx;

/* hyp_opts.criterion: the quantity compared with the threshold */
#define HYP_CRIT_E1    0  /* mean |div u| over fluid cells (E_1, Sec. 4.1) */
#define HYP_CRIT_EINF  1  /* max |div u| over fluid cells (E_inf) */

/* hyp_net_desc.flags */
#define HYP_NET_TRAIN  1  /* keep every layer's activations (and the backward
                             buffers) in the workspace for hyp_project_backward */

/* hyp_net_desc.arch: the network that predicts the initial pressure. */
#define HYP_ARCH_PARALLEL    0  /* S parallel branches (one per 2x2-mean pyramid
                                   level) of four 3x3 + ReLU layers and a 1x1
                                   output, summed coarse to fine after bilinear
                                   x2 upsampling (Sec. 3.1's multi-scale idea) */
#define HYP_ARCH_MULTISCALE  1  /* the paper's cascaded MultiScale (Sec. 3.1,
                                   Fig. 3): branches at n/4, n/2, n of 5, 7, 7
                                   layers; each coarser output is upsampled x2
                                   and concatenated to the next branch's input */
#define HYP_ARCH_SMALLSCALE  2  /* the same cascade with 32 channels (Sec. 3.1's
                                   SmallScale) */
#define HYP_ARCH_UNET        3  /* the paper's Unet (Sec. 3.1, Fig. 4): scales
                                   n .. n/16, max pooling down, bilinear x2 up,
                                   skip concatenation */

/* Network shape.  HYP_ARCH_PARALLEL: scales in 1..5; channels 16, 32 or 64
 * with FP32 (64: inference only, HYP_EUNSUPPORTED with HYP_NET_TRAIN), 32 or
 * 64 with BF16.  HYP_ARCH_MULTISCALE / SMALLSCALE: scales 3 (or 0), channels
 * 64 / 32 (or 0), FP32 or BF16; the grid sides must be multiples of 4.
 * HYP_ARCH_UNET: scales 5 (or 0), channels 64 (or 0), FP32 or BF16; grid
 * sides multiples of 16.  The paper's networks train in FP32 only
 * (HYP_NET_TRAIN with BF16 gives HYP_EUNSUPPORTED). */
typedef struct {
  int32_t scales;
  int32_t channels;
  int32_t precision;  /* HYP_PREC_* */
  int32_t flags;      /* HYP_NET_* */
  int32_t arch;       /* HYP_ARCH_* */
} hyp_net_desc;

typedef struct {
  int32_t nx, ny;  /* cells */
  double dx;       /* cell size */
  double dt;       /* time step: p = rho0 * phi / dt */
  double rho0;     /* reference density of Eq. (2) */
} hyp_grid;

typedef struct {
  float* u;              /* (ny, nx+1) in/out: corrected in place */
  float* v;              /* (ny+1, nx) in/out: corrected in place */
  const float* rho;      /* (ny, nx) density: read only with
                            hyp_opts.variable_density (then required, > 0 on
                            fluid cells); the constant-coefficient operator
                            of Eq. (3) uses rho0 */
  const uint8_t* flags;  /* (ny, nx) input flags (bit0 solid, bit1 inflow) */
  float* p;              /* (ny, nx) out: pressure p = rho0 * phi / dt */
  const float* p_init;   /* nullable: warm start (as p, same scaling) for
                            the JACOBI / PCG methods */
  float* phi_ckpt;       /* nullable: Jacobi checkpoints (see
                            hyp_opts.checkpoint_every): n_ckpt planes of
                            (ny, nx) phi = (dt / rho0) p after every
                            checkpoint_every sweeps, caller-owned */
} hyp_fields;

typedef struct {
  int32_t method;       /* HYP_METHOD_* */
  int32_t max_iters;    /* cap on sweeps / CG iterations (>= 0) */
  int32_t check_every;  /* test E_1 every k updates (>= 1) and at max_iters */
  int32_t fixed_iters;  /* > 0: ignore the threshold, do exactly this many */
  float omega;          /* Jacobi weight > 0, 1 = the paper's undamped form (else HYP_EINVAL) */
  int32_t fold_window;  /* defect correction (FP32 residual floor): Jacobi
                           folds its pressure into the faces and restarts on
                           the recomputed divergence when E_1 fell by less
                           than 1 % over this many sweeps (0: 1024 when a
                           threshold decides, no folds with fixed_iters);
                           PCG folds when its true residual does not confirm
                           a stop (at most 3 folds, then HYP_STATUS_FLOOR). */
  int32_t checkpoint_every;  /* HYBRID/JACOBI with fixed_iters > 0 and
                           fields.phi_ckpt set: after sweep c, 2c, ... <=
                           fixed_iters (c = checkpoint_every) the iterate phi
                           of the interior is written to plane k/c - 1 of
                           phi_ckpt (at most 64 planes); without folds it
                           restarts the iteration bit-exactly as a warm
                           start.  0: none.  EINVAL otherwise. */
  int32_t tile_rows;    /* Jacobi tile: rows per wave in registers (4, 8,
                           12, 16, 24 or 32); 0: the tuned table for this
                           grid (csrc/tile_table.h), else the smallest that
                           fits one work-group per CU.  EUNSUPPORTED when the
                           tiles do not fit. */
  int32_t variable_density; /* 1: keep the cell density inside Eq. (3)-(2)
                           (the paper writes them with rho0, Sec. 2.2):
                           div(beta grad phi) = div u*, u = u* - beta grad phi
                           with beta = rho0 / rho_face on open faces (mean of
                           the two cells' densities; the top cell's on an open
                           top face), phi = (dt / rho0) p as before.  Jacobi,
                           PCG, HYBRID (the network's guess is unchanged) and
                           CNN; needs rho; not with the batch or the adjoint
                           (EUNSUPPORTED).  0: rho0 everywhere. */
  int32_t criterion;    /* HYP_CRIT_E1 (the paper's hybrid criterion, mean
                           |div u| over fluid cells) or HYP_CRIT_EINF (max
                           |div u|, the earlier work's criterion compared in
                           Sec. 4.1) for the threshold test; the result's
                           e1_cnn then holds the chosen measure of the guess.
                           Not with the batch (EUNSUPPORTED). */
  int32_t block_sweeps; /* Jacobi sweeps between halo exchanges, 1..16 (a
                           halo of block_sweeps + 1 cells is recomputed by
                           each tile; the iterates do not depend on it); 0:
                           the tuned table for this grid (csrc/tile_table.h)
                           when its block fits check_every, else
                           min(check_every, 8).  Clipped to check_every when
                           a threshold decides.  EINVAL outside 0..16. */
} hyp_opts;

/* Written by the device when the projection's last kernel completes. */
typedef struct {
  int32_t iters;       /* sweeps or CG iterations performed */
  int32_t status;      /* HYP_STATUS_* */
  double e1_init;      /* mean |div u*| over fluid cells before projection */
  double e1_cnn;       /* mean |d - L phi0| of the initial guess (max with
                          HYP_CRIT_EINF) */
  double e1_final;     /* mean |div u| recomputed from the returned faces */
  double einf_final;   /* max  |div u| recomputed from the returned faces */
  double s;            /* CNN input scale sqrt(mean d^2) (0 without CNN) */
  int32_t n_fluid;     /* fluid cells after the pocket fill */
  int32_t reserved;
  double dt;           /* time step of hyp_step (CFL); unset by hyp_project */
} hyp_result;

int hyp_version(void);
const char* hyp_status_str(int code);

/* Create a context.  `net` may be NULL (no CNN: JACOBI and PCG only).
 * Host allocation only.  Returns HYP_EINVAL on a bad shape. */
int hyp_create(hyp_ctx** out, const hyp_net_desc* net);
int hyp_destroy(hyp_ctx* ctx);

/* Number of float32 parameters of the context's network (0 without one). */
int64_t hyp_param_count(const hyp_ctx* ctx);

/* Point the context at caller-owned FP32 parameters on the device, in the
 * packed layout of its architecture.  HYP_ARCH_PARALLEL: for each scale
 * k = 0 (finest) .. S-1, four 3x3 layers as W[Cout][3][3][Cin] then
 * bias[Cout] (Cin = 2 for the first layer: the normalised divergence and the
 * solid mask; C after), then the 1x1 output as w[C] then bias[1].
 * HYP_ARCH_MULTISCALE / SMALLSCALE (C = 64 / 32): branches from the coarsest
 * (n/4) to the finest (n), each layer as W[Cout][k][k][Cin] then b[Cout]:
 *   n/4:      5x5 2->C, 3x3 C->C, 3x3 C->C, 3x3 C->C (linear), 1x1 C->1
 *   n/2 and n: 5x5 3->C, 3x3 C->C, 3x3 C->32, 3x3 32->C, 3x3 C->C,
 *             3x3 C->C (linear), 1x1 C->1
 * with ReLU after every layer but the last two of a branch, and input
 * channels (normalised divergence, solid mask, upsampled coarser output)
 * (419,459 and 126,819 parameters).  HYP_ARCH_UNET (widths w = 16, 16, 64,
 * 64, 64 at scales 0..4), each layer as W[Cout][3][3][Cin] then b[Cout]:
 * encoder scales l = 0..4: 3x3 Cin->w[l], 3x3 w[l]->w[l] (Cin = 2, then
 * w[l-1]); decoder scales l = 3..0: 3x3 (w[l] + w[l+1])->w[l] on the skip
 * channels followed by the upsampled ones, 3x3 w[l]->w[l]; then the 1x1
 * output w[0]->1; ReLU on all but the output (443,441 parameters).  The buffer is read at every projection
 * and must stay valid; it is never copied.  n_params must equal
 * hyp_param_count. */
int hyp_set_weights(hyp_ctx* ctx, const float* dev_params, int64_t n_params);

/* Workspace bytes for a grid (and the context's network).  The workspace
 * holds the planned cell flags, the divergence, the solver state, the CNN
 * activations and the reduction scratch. */
int hyp_workspace_size(const hyp_ctx* ctx, const hyp_grid* g, size_t* bytes);

/* Planning (once per geometry): pocket fill and neighbour structure of the
 * flags into the workspace.  Must precede hyp_project on that workspace
 * whenever the flags change.  Asynchronous on `stream`. */
int hyp_plan(hyp_ctx* ctx, const hyp_grid* g, const uint8_t* flags,
             void* ws, size_t ws_bytes, hipStream_t stream);

/* One projection (Eq. 2-3): enforce the boundary faces, divergence, initial
 * guess, iterate until E_1 < threshold (strict; tested before the first
 * update, every check_every updates and at max_iters), subtract the
 * gradient, write p and the result.  `res` must be device memory or
 * host-pinned memory; it is valid once `stream` has completed the call.
 * The call may be recorded by stream capture (as may hyp_step): the
 * persistent solver is then a plain launch of the same grid, sized by the
 * occupancy query, so a replay must run with the GPU otherwise idle for its
 * work-groups to be resident; a grid barrier that is not reached within 2 s
 * ends the solve with HYP_STATUS_ABORTED instead of hanging.  A captured
 * call replays with the pointers and options it was recorded with. */
int hyp_project(hyp_ctx* ctx, const hyp_grid* g, const hyp_fields* f,
                double threshold, const hyp_opts* o, void* ws,
                size_t ws_bytes, hipStream_t stream, hyp_result* res);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hyp_plan
 * on f->flags followed by hyp_project, with the workspace taken from a
 * static device array of HYP_NOALLOC_MAX_BYTES that the library holds on
 * every GPU it runs on until the process ends.  Nothing is allocated; the
 * caller passes inputs and outputs only (device memory, as for
 * hyp_project; res device or host-pinned).  HYP_EWORKSPACE when the grid
 * and network need more than HYP_NOALLOC_MAX_BYTES (hyp_workspace_size),
 * any other rejection as hyp_project; nothing is enqueued then.  All calls
 * on one GPU share that GPU's array: calls that overlap on one GPU (two
 * streams or threads) race and must be serialised by the caller.  The
 * results equal hyp_plan + hyp_project on a caller workspace. */
#define HYP_NOALLOC_MAX_BYTES (128u << 20)
int hyp_project_noalloc(hyp_ctx* ctx, const hyp_grid* g, const hyp_fields* f, double threshold,
                        const hyp_opts* o, hipStream_t stream, hyp_result* res);

/* Adjoint of the projection (the gradient of the correction of Eq. 2 is
 * known, Sec. 3.2): gradient of  loss = scale * sum_F r^2,  r = d - L phi_K,
 * the divergence left after the CNN guess and exactly `sweeps` Jacobi sweeps
 * of weight `omega`.  Must follow, on the same stream and workspace, the
 * forward hyp_project of a context created with HYP_NET_TRAIN, run with
 * method HYP_METHOD_HYBRID and fixed_iters = sweeps (or HYP_METHOD_CNN when
 * sweeps = 0).  Writes (or adds to, when accumulate != 0) dL/du (ny, nx+1),
 * dL/dv (ny+1, nx) and dL/dparams (packed layout); each pointer may be NULL.
 * `loss` (device double, nullable) receives the loss.  Deterministic: every
 * reduction has a fixed order. */
int hyp_project_backward(hyp_ctx* ctx, const hyp_grid* g, int32_t sweeps, float omega,
                         double scale, int32_t accumulate, float* du, float* dv,
                         float* dparams, double* loss, void* ws, size_t ws_bytes,
                         hipStream_t stream);

/* One Adam update of n parameters (step >= 1 for the bias correction):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).  All device FP32. */
int hyp_adam(float* params, const float* grads, float* m, float* v, int64_t n, int32_t step,
             float lr, float beta1, float beta2, float eps, hipStream_t stream);

/* Phase timing (the t_ad / t_inf / t_p / t_it split of Sec. 5): when
 * enabled, HIP events are recorded on the call's stream around each phase of
 * hyp_project / hyp_step (a few microseconds of overhead per call). */
int hyp_set_timing(hyp_ctx* ctx, int enable);
/* Milliseconds of the last call, after waiting for it: ms[0] advection (0 for
 * hyp_project), ms[1] divergence + CNN inference, ms[2] the iterative solver
 * launch, ms[3] gradient correction + final check, ms[4] total. */
int hyp_get_timing(hyp_ctx* ctx, float* ms);

/* Physical parameters of the plume time step (Sec. 2.1-2.2). */
typedef struct {
  double g;      /* gravity (from the Richardson number, Eq. 1) */
  double rho0;   /* reference (heavy) density */
  double drho;   /* density contrast Delta rho / rho0 of the injected fluid */
  double u_in;   /* inflow velocity */
  double cfl;    /* dt = cfl dx / max(max|u|, max|v|, u_in) */
} hyp_physics;

typedef struct {
  float* rho;            /* (ny, nx) density, advected in place */
  float* u;              /* (ny, nx+1) velocity faces, advanced in place */
  float* v;              /* (ny+1, nx) */
  float* p;              /* (ny, nx) out: pressure of the projection */
  const uint8_t* flags;  /* (ny, nx) input flags, as for hyp_project */
  const float* xi;       /* (nx) inflow noise of this step: v_in = u_in (1 + xi) */
} hyp_state;

/* One full time step of the plume (Sec. 2.2): CFL time step, MacCormack
 * semi-Lagrangian advection of rho, u and v with the start-of-step velocity
 * (min/max limiter), buoyancy by forward Euler on interior and top v faces,
 * inflow reset, boundary faces, then the projection exactly as hyp_project
 * with p = rho0 phi / dt.  g->dt is ignored (the step computes its own dt,
 * returned in res->dt).  Requires hyp_plan on the workspace. */
int hyp_step(hyp_ctx* ctx, const hyp_grid* g, const hyp_physics* ph, const hyp_state* st,
             double threshold, const hyp_opts* o, void* ws, size_t ws_bytes,
             hipStream_t stream, hyp_result* res);

/* The advection + force half of hyp_step alone (produces u* in st->u,
 * st->v and the advected density; st->p is not used).  For generating the
 * intermediate velocities the projection receives, e.g. training data. */
int hyp_advect(hyp_ctx* ctx, const hyp_grid* g, const hyp_physics* ph, const hyp_state* st,
               void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- batched form: many plumes of uneven sizes ---------------------------
 * The batched workload of many independent plumes (the launch-bound regime
 * of small grids that Sec. 5.2 discusses): a batch fixes the instances
 * (grids, state pointers, thresholds, physics, options) once.  Every phase
 * of a step is one launch over all instances (advection passes, boundary
 * faces + divergence, the network's input, convolution layers and
 * upsample-sum, the gradient correction and the final check), and the
 * Jacobi sweeps of every instance run in ONE persistent launch over a
 * global tile list, with per-instance E_1 tests (finished instances drop
 * out).  The tiles sweep 8 times between halo exchanges; o->check_every
 * (>= 1) is rounded up to whole exchanges of 8 sweeps, and E_1 is tested
 * at that interval, on the network's output and at max_iters (an instance
 * that meets the threshold between tests sweeps on until the next one).
 * Methods HYBRID (HYP_ARCH_PARALLEL networks) and JACOBI; fold_window is
 * not used; criterion E_1 only.
 * o->variable_density applies the variable-density operator of
 * hyp_opts.variable_density to every instance (each with its own rho).
 * o->tile_rows: 0 (the tuned tile rows per grid side), or 8 or 16 for every
 * constant-density instance (variable-density tiles use 8).  The network
 * weights are the context's at creation (the buffer's contents may change
 * between calls, not its address).  The workspace holds the batch tables
 * followed by one projection workspace per instance. */
typedef struct hyp_batch hyp_batch;

int hyp_batch_workspace_size(hyp_ctx* ctx, int32_t n, const hyp_grid* grids, size_t* bytes);
/* Validates, uploads the tables and plans every instance (synchronous).
 * physics: NULL (projection only) or n entries, one per instance (gravity,
 * density contrast, inflow and CFL of that plume: Eq. 1 gives each its own
 * g); states[i].rho and .xi may be NULL when only hyp_batch_project is
 * used (rho is required with variable_density). */
int hyp_batch_create(hyp_ctx* ctx, int32_t n, const hyp_grid* grids, const hyp_state* states,
                     const double* thresholds, const hyp_physics* physics, const hyp_opts* o,
                     void* ws, size_t ws_bytes, hyp_batch** out);
/* Projection of the current faces of every instance; res: n results
 * (device or host-pinned), written at the end of the call's work. */
int hyp_batch_project(hyp_batch* b, hipStream_t stream, hyp_result* res);
/* One time step (advection, buoyancy, inflow, projection) of every instance
 * with its own physics (HYP_EINVAL when the batch was created without). */
int hyp_batch_step(hyp_batch* b, hipStream_t stream, hyp_result* res);
/* Record hyp_batch_step into a hipGraph (replayed by hyp_batch_launch on any
 * stream).  The inflow noise arrays are read at replay time.  Inside the
 * graph the persistent Jacobi launch is a plain launch of as many
 * work-groups as the GPU holds at once; its grid barriers give up after 2 s
 * (status ABORTED) if they are ever not all resident. */
int hyp_batch_capture(hyp_batch* b, hipStream_t stream, hyp_result* res);
int hyp_batch_launch(hyp_batch* b, hipStream_t stream);
int hyp_batch_destroy(hyp_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* HYPROJ_H */
