/*
 * swe_nh.h -- C ABI of the MI355X (gfx950) implementation of the per-time-step
 * hot path of the locally adaptive non-hydrostatic shallow water model of
 * Firdaus & Behrens ("Locally Adaptive Non-Hydrostatic Shallow Water
 * Extension for Moving Bottom-Generated Waves").
 *
 * One step (Sec. 3 and Sec. 5 of the paper):
 *   1. hydrostatic predictor: Heun (Eqs. 8-9) over a second-order
 *      finite-volume operator with the Rusanov flux (Sec. 3.1), giving
 *      Q~ = (h~, hu~, [hv~,] hw~);
 *   2. criterion on Q~ against k_nh and enlargement of the marked area
 *      (Sec. 5.1, 5.2), then compaction of the marked cells;
 *   3. assembly of the elliptic system of Eqs. 12-17 on the marked cells
 *      (zero Dirichlet data for the non-hydrostatic pressure outside them)
 *      and its solution;
 *   4. projection of hu (and hv) and hw with Eqs. 10-11; h = h~ (no mass
 *      correction, Sec. 3.2).
 *
 * Memory: every array argument is a DEVICE pointer to contiguous FP64 (or
 * uint8 for masks) memory owned by the caller, structure-of-arrays, x
 * fastest; 2D arrays are [ny][nx].  The library allocates no device memory:
 * all scratch lives in a caller-provided workspace of swe_nh_workspace_bytes(),
 * except for the fixed static scratch of swe_nh_cnn_forward_noalloc.
 * Host pointers are marked "host".
 *
 * Streams and asynchrony: every call is enqueued on the stream given to
 * swe_nh_init and returns without waiting, except the calls documented as
 * synchronising.  Argument errors are returned immediately.  Numerical
 * failures (dry cells, non-finite state, no convergence) are recorded on the
 * device and returned by swe_nh_sync_stats().
 *
 * Errors: no exception crosses this interface; every call returns a
 * swe_nh_status.  swe_nh_last_error() gives a message for the last failure of
 * a context.  A context is not re-entrant: concurrent calls on one context
 * are not allowed.
 */
#ifndef SWE_NH_H
#define SWE_NH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SWE_NH_OK = 0,
  SWE_NH_EINVAL = -1,   /* bad argument or configuration */
  SWE_NH_ENOCONV = -2,  /* elliptic solve did not reach tol within max_iter */
  SWE_NH_EDRY = -3,     /* a cell or reconstructed face depth <= 0 */
  SWE_NH_ENAN = -4,     /* non-finite state on entry to a step */
  SWE_NH_EHIP = -5,     /* HIP runtime error */
  SWE_NH_ENOMEM = -6    /* workspace too small */
} swe_nh_status;

/* Adaptivity criteria of Sec. 5.1 (indicator > k_nh marks a cell), plus the
 * global model (every cell) and the pure hydrostatic model (no cell).
 * In 2D the indicators are |grad eta|, |(u, v)|, the Frobenius norm of
 * grad(u, v) and |grad w|. */
typedef enum {
  SWE_NH_CRIT_ETA_D = 0,
  SWE_NH_CRIT_ETA_X = 1,
  SWE_NH_CRIT_U = 2,
  SWE_NH_CRIT_U_X = 3,
  SWE_NH_CRIT_W = 4,
  SWE_NH_CRIT_W_X = 5,
  SWE_NH_CRIT_GLOBAL = 6,
  SWE_NH_CRIT_NONE = 7
} swe_nh_criterion;

/* Moving rigid body carried by the bottom: d(x, y, t) = d_s - B(x - X(t), y - y0),
 * X(t) = x0 + dir * s(t).  Shapes: the quartic slide of Eq. 20 (amp = H_s,
 * len = L_s, on |x - X| < L_s / 2) or a Gaussian mound amp exp(-r^2 / len^2).
 * Laws s(t): fixed; constant velocity q[0]; sinusoidal ramp
 * (q[0] / 2)(1 - cos(pi t / q[1])) then q[0]; the accelerate / coast /
 * decelerate law of Eq. 21 with q = (a0, u_t, t1, t2, t3). */
enum { SWE_NH_BODY_NONE = 0, SWE_NH_BODY_QUARTIC = 1, SWE_NH_BODY_GAUSS = 2 };
enum { SWE_NH_LAW_FIXED = 0, SWE_NH_LAW_CONST_VEL = 1, SWE_NH_LAW_SIN_RAMP = 2,
       SWE_NH_LAW_PIECEWISE = 3 };

typedef struct {
  int32_t kind;
  int32_t law;
  double amp, len, x0, y0, dir;
  double q[5];
} swe_nh_body;

typedef struct {
  int32_t dim;              /* 1 or 2 */
  int32_t nx, ny;           /* 2D grid; ny ignored in 1D */
  int32_t batch;            /* 1D: number of independent channels (>= 1) */
  const int64_t* offsets;   /* host [batch + 1]: channel c owns packed cells
                               offsets[c] .. offsets[c+1]-1; NULL when batch == 1
                               (then the single channel has nx cells) */
  double dx, dy;            /* cell sizes (m) */
  double g, rho;            /* 9.81, 1000 */
  double cfl;               /* > 0: dt = cfl dx / max(|u| + sqrt(g h)) per channel
                               (2D: cfl / max(lx/dx + ly/dy)); <= 0: dt = dt_fixed */
  double dt_fixed;
  int32_t crit;             /* swe_nh_criterion */
  double k_nh;              /* threshold, paper value 1e-3 */
  int32_t enlarge;          /* cells added on each side of the marked area (paper: 1) */
  int32_t first_global;     /* |w| and |w_x|: global model on the first step (Sec. 5.1.2) */
  int32_t precision;        /* 0: FP64 solve; 1: FP32 inner solve + FP64 residual refinement
                               (1D fused step, enlarge <= 8: each tile's interior system
                               is reduced in FP32 and refined with FP64 residuals, the
                               tiles' coupling system is solved in FP64) */
  double tol;               /* 2D PCG and the 1D unfused refinement (enlarge > 8):
                               ||b - A p||_2 <= tol ||b||_2.  1D fused refinement: each
                               tile's componentwise backward error
                               max_j |r_j| / (|A| |x| + |b|)_j <= tol */
  int32_t max_iter;         /* PCG iterations (2D) or refinement sweeps (precision 1) */
  int32_t warm;             /* 2D initial guess: 0 zero, 1 previous p (the p array on
                               entry), 2 the warm-start network */
  int32_t tile1d;           /* 1D cells per block of the stencil kernels, 32..512, or 0
                               for the built-in choice.  The kernels' LDS windows come
                               in capacities of 128, 256 and 512 cells; the smallest
                               that holds the tile is used.  The fused step's
                               window adds 6 + enlarge cells on each side, so a tile of
                               capacity - 2 (6 + enlarge) cells fills whole wavefronts */
  int32_t step1d_form;      /* 1D fused step: 0 one kernel when the blocks of every tile
                               fit on the device at once (and the two-kernel form
                               otherwise), 1 always the two-kernel form (step kernel,
                               level-1 solve, projection kernel) */
  int32_t tensor2d;         /* 2D elliptic operator: 0 the diagonal of the face tensor
                               S12^{-1} (5-point stencil), 1 the exact tensor: its
                               off-diagonal d_x d_y / alpha coupling on pairs of faces
                               (the x-face east of a cell with the y-face north of it),
                               a 7-point stencil that adds the neighbours (i-1, j+1) and
                               (i+1, j-1) (Sec. 3.2 Eqs. 12-17 in the 2D vector form).
                               1 is solved by CG with the multigrid preconditioner on the
                               active cells' bounding box at every active-tile count, so
                               the grid must coarsen by 2 x 2 aggregation to at most 4096
                               cells (nx, ny multiples of 2^L with nx ny / 4^L <= 4096,
                               L >= 1), else init fails with SWE_NH_EINVAL; 1D: 0 */
  const double* depth_static;  /* device [cells]: static depth d_s */
  const swe_nh_body* bodies;   /* host [batch] (1D) or [1] (2D) */
} swe_nh_config;

typedef struct {
  int64_t n_active;         /* cells in the non-hydrostatic area of the last step */
  int32_t iters;            /* PCG iterations (2D) / refinement sweeps of the last step
                               (1D fused: the most sweeps any tile took) */
  int32_t status;           /* swe_nh_status of the last step(s) (first failure wins) */
  double rel_res;           /* ||b - A p|| / ||b|| of the last solve (when computed; 1D
                               fused refinement: the largest tile backward error) */
  double dt;                /* time step of the last step (channel 0) */
  double t;                 /* time after the last step (channel 0) */
  int64_t steps;            /* steps taken since init */
  int64_t iters_total;      /* PCG iterations summed over all solves since init (2D; 0 in 1D) */
} swe_nh_stats;

typedef struct swe_nh_ctx swe_nh_ctx;

/* Bytes of device workspace needed for cfg (0 on invalid cfg). */
size_t swe_nh_workspace_bytes(const swe_nh_config* cfg);

/* Validate cfg, carve the caller's device workspace (>= workspace_bytes,
 * 256-byte aligned), upload channel tables and set t = 0.  stream is a
 * hipStream_t (NULL = the default stream).  The workspace must outlive the
 * context.  Returns SWE_NH_EINVAL / SWE_NH_ENOMEM / SWE_NH_EHIP on failure.
 *
 * The 1D fused step of a grid of at most 512 tiles whose blocks all fit
 * on the device at once runs as one kernel whose blocks exchange tagged
 * words (the 2D solver's iterations do the same); such kernels assume that
 * no other long-running kernel holds the device's compute units while they
 * run.  Every wait is bounded: a step that cannot complete ends with
 * SWE_NH_EHIP after about 0.5 s.  cfg->step1d_form = 1 selects the two-kernel
 * form, which has no such waits. */
int swe_nh_init(const swe_nh_config* cfg, void* workspace, size_t workspace_bytes, void* stream,
                swe_nh_ctx** out);

void swe_nh_destroy(swe_nh_ctx* ctx);
const char* swe_nh_last_error(const swe_nh_ctx* ctx);

/* Set / read the model time of every channel (host arrays [batch]; 2D: [1]).
 * swe_nh_get_time synchronises the stream. */
int swe_nh_set_time(swe_nh_ctx* ctx, const double* t_host);
int swe_nh_get_time(swe_nh_ctx* ctx, double* t_host);

/* Advance nsteps full steps in place: h, hu, hw (and hv in 2D; must be NULL
 * in 1D) hold Q^n on entry and Q^{n+1} on return; p receives the NH
 * pressure of the last step (0 outside the NH area) and, in 2D with
 * warm = 1, is the initial guess.  mask (may be NULL) receives the NH area of
 * the last step.  The step sequence is captured once into a hipGraph per
 * distinct argument set and replayed. */
int swe_nh_step(swe_nh_ctx* ctx, double* h, double* hu, double* hv, double* hw, double* p,
                uint8_t* mask, int32_t nsteps);

/* Synchronise the stream and read the statistics of the last step. */
int swe_nh_sync_stats(swe_nh_ctx* ctx, swe_nh_stats* out);

/* One full step (Secs. 3.1, 3.2, 5.1, 5.2: predictor, criterion and
 * enlargement, elliptic solve, projection) with the model time in device
 * memory: t_dev (device FP64, [batch] in 1D, [1] in 2D) holds t^n on entry and
 * t^{n+1} on return; the context's own time is set from it first, so calls
 * may interleave with swe_nh_step.  h, hu, hv, hw and p as for swe_nh_step
 * (no mask output).  stats (host memory, may be NULL): when given, the call
 * synchronises the stream and fills it as swe_nh_sync_stats does; when NULL
 * the call returns without waiting.  Errors: SWE_NH_EINVAL for null
 * arguments, the status codes of the step through stats. */
int swe_nh_step_t(swe_nh_ctx* ctx, double* h, double* hu, double* hv, double* hw, double* p,
                  double* t_dev, swe_nh_stats* stats);

/* Stage entry points (same kernels as swe_nh_step), for callers that drive
 * the stages themselves and for parity tests. */

/* Hydrostatic predictor (Sec. 3.1): Q~ from Q^n over [t, t + dt] with the
 * context's bottom law.  Outputs may not alias inputs. */
int swe_nh_predict(swe_nh_ctx* ctx, const double* h, const double* hu, const double* hv,
                   const double* hw, const double* t_host, const double* dt_host, double* ht,
                   double* mt, double* nt, double* kt);

/* Criterion and enlargement (Sec. 5.1, 5.2) on a predictor state at time t1
 * (t_host[batch]); first_step selects the global first step of the |w|,
 * |w_x| criteria.  mask_out: uint8 [cells]; n_active_host: total marked
 * cells (synchronises when non-NULL). */
int swe_nh_mask(swe_nh_ctx* ctx, const double* ht, const double* mt, const double* nt,
                const double* kt, const double* t_host, int32_t first_step, uint8_t* mask_out,
                int64_t* n_active_host);

/* Elliptic system of Eqs. 12-17 on the cells with mask != 0 for the
 * predictor state at t1 = t_host with step dt_host, solved for the NH
 * pressure p (zero elsewhere).  In 2D p_inout is the initial guess when
 * warm = 1.  iters / rel_res (host, may be NULL) synchronise. */
int swe_nh_solve_pressure(swe_nh_ctx* ctx, const double* ht, const double* mt, const double* nt,
                          const double* kt, const uint8_t* mask, const double* t_host,
                          const double* dt_host, double* p_inout, int32_t* iters_host,
                          double* rel_res_host);

/* Projection (Eqs. 10-11): hu, hv, hw from the predictor state and p on the
 * marked cells; unmarked cells copy the predictor values. */
int swe_nh_correct(swe_nh_ctx* ctx, const double* ht, const double* mt, const double* nt,
                   const double* kt, const uint8_t* mask, const double* p, const double* t_host,
                   const double* dt_host, double* m_out, double* n_out, double* k_out);

/* ---- learned warm start of the 2D pressure solve ----
 * A fixed convolutional network (six 3x3 layers, channels 16 -> 32 -> 32 ->
 * 32 -> 32 -> 32 -> 1, ReLU between layers, zero padding; 5 input features,
 * the other 11 input channels zero) maps the predictor state to a guess of
 * the non-hydrostatic pressure.  It is not part of the paper's method: the
 * PCG still iterates to the same tolerance from the guess, so the guess only
 * changes the iteration count.  Parameters are one FP32 vector: per layer
 * the weights [Cout][3][3][Cin] then the Cout biases.  Activations are BF16
 * NHWC; products accumulate in FP32 on the matrix cores.  Images must have a
 * height and width that are multiples of 16. */
size_t swe_nh_cnn_param_count(void);

/* Device workspace for a batch of n images of h x w (0 if the shape is not supported). */
size_t swe_nh_cnn_workspace_bytes(int32_t n, int32_t h, int32_t w);

/* out[n][h][w] (FP32) = network(x), x: BF16 NHWC [n][h][w][16]; keeps the
 * activations in ws for a following swe_nh_cnn_backward. */
int swe_nh_cnn_forward(const float* params, const uint16_t* x, int32_t n, int32_t h, int32_t w,
                       float* out, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of swe_nh_cnn_forward for callers that cannot
 * allocate device memory: code under stream or graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same network, kernels and output
 * as swe_nh_cnn_forward, but the packed weights and the activations live in
 * the library's own static device scratch of SWE_NH_CNN_NOALLOC_SCRATCH_BYTES
 * (one copy per device, held from the library's load until the process ends)
 * instead of a caller workspace; the call allocates nothing.  params, x, out
 * as in swe_nh_cnn_forward (caller-owned device buffers).
 * Limits: n * h * w <= SWE_NH_CNN_NOALLOC_MAX_PIXELS (else SWE_NH_ENOMEM), h
 * and w multiples of 16 (else SWE_NH_EINVAL); stream must belong to the
 * current device (else SWE_NH_EINVAL; NULL = its default stream).  Inference
 * only: nothing is kept for swe_nh_cnn_backward.  Every call on a device
 * uses that device's one scratch, which keeps the last call's contents: calls
 * that overlap in time on one device (several streams or threads) race, and
 * the caller must serialise them. */
#define SWE_NH_CNN_NOALLOC_MAX_PIXELS 131072
#define SWE_NH_CNN_NOALLOC_SCRATCH_BYTES (17u << 20)
int swe_nh_cnn_forward_noalloc(const float* params, const uint16_t* x, int32_t n, int32_t h,
                               int32_t w, float* out, void* stream);

/* grad (parameter-shaped, FP32) = d(sum(out * dout)) / d(params) for the
 * batch of the last swe_nh_cnn_forward on the same workspace. */
int swe_nh_cnn_backward(const float* params, const uint16_t* x, const float* dout, int32_t n,
                        int32_t h, int32_t w, float* grad, void* ws, size_t ws_bytes,
                        void* stream);

/* Weighted mean squared error: *loss = sum wt (out - target)^2 / sum wt
 * (device scalar), dout = its gradient with respect to out. */
int swe_nh_cnn_mse(const float* out, const float* target, const float* weight, int32_t n,
                   int32_t h, int32_t w, float* dout, float* loss, void* ws, size_t ws_bytes,
                   void* stream);

/* The mask proposal's loss: weighted binary cross-entropy of the logits out
 * against targets in [0, 1], *loss = sum wt l / sum wt with
 * l = max(o, 0) - o t + log(1 + exp(-|o|)) (device scalar, accumulated in
 * FP64), dout = wt (1 / (1 + exp(-o)) - t) / sum wt.  Same buffers and
 * workspace as swe_nh_cnn_mse. */
int swe_nh_cnn_bce(const float* out, const float* target, const float* weight, int32_t n,
                   int32_t h, int32_t w, float* dout, float* loss, void* ws, size_t ws_bytes,
                   void* stream);

/* One Adam step (Kingma & Ba 2015) on FP32 parameters; step counts from 1. */
int swe_nh_cnn_adam(float* params, float* m, float* v, const float* grad, int64_t count,
                    int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* Network input of a 2D predictor state at time t1_host: BF16 NHWC
 * [ny][nx][16] with eta / s0, hu / s1, hv / s2, -d_t / s3 and the mask, the
 * other channels 0 (scales_host: the four s_k > 0). */
int swe_nh_features(swe_nh_ctx* ctx, const double* ht, const double* mt, const double* nt,
                    const uint8_t* mask, const double* t1_host, const double* scales_host,
                    uint16_t* out);

/* Use the network (device parameters, kept by reference: the biases are read
 * at each step, the weights are packed for the matrix cores by this call,
 * so call it again after changing them) as the initial guess of the 2D
 * pressure solve of swe_nh_step when the context was created with warm = 2:
 * inputs scaled as in swe_nh_features, guess = p_scale * network output on
 * the marked cells (Pa).  The network sees a window of at most 256 x 256
 * cells placed over the active tiles each step; marked cells outside it
 * start from 0. */
int swe_nh_set_warm_start_net(swe_nh_ctx* ctx, const float* params, const double* scales_host,
                              double p_scale);

/* Measurement: launch one stage kernel of the step nreps times back to back
 * on the context's stream, with the launch configuration swe_nh_step uses,
 * between two HIP events, and return the mean time per launch in
 * microseconds (synchronises).  The launches are captured into a graph of
 * up to 50 of them, replayed once untimed and then timed, so the host's
 * per-launch cost is not counted; nreps is rounded up to a multiple of the
 * graph's length.  The state arrays must hold a valid state of
 * the context (for instance after swe_nh_step).
 * 1D with enlarge <= 8 (the fused step, either precision): stage 0 the fused
 * step kernel (predictor, criterion, assembly, tile reduction; in the
 * one-kernel step of grids of at most 512 tiles also the level-1 solve and
 * the projection), 1 the separate level-1 solve, 2 the projection kernel
 * (both report 0 in the one-kernel step, which has neither), 3 the
 * stand-alone predictor; outputs go to workspace scratch, the caller's
 * arrays and the time are not modified.
 * Otherwise: stage 0 predictor, 1 criterion/mask, 2 elliptic solve (all
 * solver launches of one solve), 3 projection; stage 0 uses the time step of
 * the last step and writes only the workspace, stages 1-3 reuse the
 * workspace of the last step and may overwrite hu, hw (and hv) and p on the
 * marked cells with the same values. */
int swe_nh_time_stage(swe_nh_ctx* ctx, int32_t stage, int32_t nreps, double* h, double* hu,
                      double* hv, double* hw, double* p, double* avg_us_host);

/* ---- The paper's own 1D discretisation (one channel; global or adaptive) ----
 * Sec. 3.1 Eqs. 6-9: RKDG with nodal P1 elements (consistent mass, element
 * integrals of the flux and of the bed source g h d_x by three-point Gauss
 * quadrature, Rusanov flux at the faces, mirror states at the walls, Heun
 * with the bottom at t^{n+1} in stage 2); Sec. 3.2 Eqs. 14-17: LDG-P1 for
 * the elliptic system with the alternating flux p* = p+, (hu)* = (hu)-,
 * p* = 0 at both walls and at the left wall (hu)* = (hu)+ - p+ / (s12 dx);
 * Eqs. 10-11: hu = q and hw from the bottom pressure, node by node.  The
 * bottom is d = d_static - B(x - X(t)) (flat static depth, the body of
 * swe_nh_body with y ignored).  No slope limiter and no wetting and drying. */
#define SWE_NH_DG_MAX_ELEMS 1024

typedef struct {
  int32_t n;           /* elements, 1 .. SWE_NH_DG_MAX_ELEMS; element i spans [i dx, (i+1) dx] */
  double dx, dt;       /* element width (m) and fixed time step (s) */
  double g, rho;
  double d_static;     /* flat static depth (m), > 0 */
  swe_nh_body body;    /* moving bottom (kind SWE_NH_BODY_NONE: flat bottom) */
  /* The adaptive model (Sec. 5) on elements.  adaptive = 0 (a zeroed tail):
   * the global model, the fields below ignored.  adaptive = 1: an element is
   * non-hydrostatic when the criterion crit (SWE_NH_CRIT_*) on the
   * predictor's node values exceeds k_nh at one of its two nodes (strictly;
   * |eta/d|, |u| = |hu / h|, |w| = |hw / h|), the derivative criteria taking
   * the magnitude of the element's P1 slope; the set is widened by enlarge
   * elements on each side (Sec. 5.2, 0 .. SWE_NH_DG_MAX_ENLARGE).  With
   * first_global, |w| and |w_x| mark every element in the first step of the
   * call (Sec. 5.1.2, for water initially at rest).  The LDG system is solved
   * on the marked elements with the other elements' unknowns fixed at p = 0
   * and hu = hu~ (the zero Dirichlet condition of the non-hydrostatic part,
   * Sec. 5); the unmarked elements keep the predictor's state and p = 0.
   * marked: optional (NULL) device int32 [nsteps], the number of marked
   * elements of each step. */
  int32_t adaptive, crit, enlarge, first_global;
  double k_nh;
  int32_t* marked;
} swe_nh_dg1d_config;
#define SWE_NH_DG_MAX_ENLARGE 64

/* Advance nsteps steps of dt from time t0 in one launch on stream (one
 * workgroup holds the channel).  h, hu, hw: device [n][2] node values,
 * element-major (node j of element i at 2 i + j), Q^n on entry and Q^{n+1}
 * on return; p: device [n][2], receives the NH pressure of the last step;
 * status: a device int32 the call uses as scratch.  Synchronises the stream.
 * Returns SWE_NH_EINVAL (bad sizes, criterion or enlargement, or null
 * pointers), SWE_NH_EDRY (a node
 * depth <= 0 entered a predictor stage), SWE_NH_ENAN (non-finite result) or
 * SWE_NH_EHIP. */
int swe_nh_dg1d_run(const swe_nh_dg1d_config* cfg, double t0, int32_t nsteps, double* h,
                    double* hu, double* hw, double* p, int32_t* status, void* stream);

/* A batch of independent channels in one launch, one workgroup per channel
 * (the same discretisation and arithmetic as swe_nh_dg1d_run, each channel
 * with its own config, global or adaptive).  cfgs: host array [nch],
 * 1 <= nch <= SWE_NH_DG_MAX_BATCH.  h, hu, hw, p: device arrays of all
 * channels' node values packed in channel order, element-major: channel c's
 * element i node j at 2 (E_c + i) + j with E_c the elements of the channels
 * before c.  Every channel advances nsteps steps of its own dt from t0.
 * status: a device int32 scratch word, the OR of every channel's status.
 * Allocates and frees a small device argument table (nch entries of about
 * 200 bytes), synchronises the stream.  Returns SWE_NH_EINVAL (any config
 * invalid, bad nch, null pointers), SWE_NH_EDRY or SWE_NH_ENAN (for any
 * channel), or SWE_NH_EHIP. */
#define SWE_NH_DG_MAX_BATCH 65536
int swe_nh_dg1d_run_batch(const swe_nh_dg1d_config* cfgs, int32_t nch, double t0, int32_t nsteps,
                          double* h, double* hu, double* hw, double* p, int32_t* status,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif
